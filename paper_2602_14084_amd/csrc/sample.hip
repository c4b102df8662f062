// sample.hip -- edge-sampling estimator (Algorithms "Baseline Edge Sampling" and
// "Improved Edge Local Search", Section 6.2), the vertex-sampling estimator (Algorithm
// "Baseline Vertex Sampling", Section 6.1), per-edge and per-vertex local counts, and the
// histogram-to-count / estimate finalisation shared with the batch path.
//
// Local search of a sampled edge e = (a, b): nothing if |d_e| < c (Lemma 2); else the
// Absolute-Edge-Order prefix (|d| >= c) of the shorter row is streamed and each
// neighbour is looked up in the other row. That mirrors the improved local search, whose
// cost is the pruned degree of the cheaper endpoint (Theorem 6.3). The estimator groups a
// pass of draws by the looked-up endpoint first (counting sort: count, scan, scatter) so a
// group's row is staged once (walk_common.h).
//
// Vertex sampling reuses that machinery: the local count at a sampled vertex q is every
// triangle containing q (the plain count its unbiasedness proof assumes), and each such
// triangle {q, u, w} is found exactly twice among the edge local counts of q's edges,
// through (q, u) and through (q, w). So a sampled vertex becomes the edge records of its
// Lemma-2 prefix (edges with |d| < c close no classified triangle), the records go through
// the grouped edge sampler, and the world's histogram is halved exactly at the end.
#include <algorithm>

#include "walk_common.h"

using namespace utri_dev;

namespace {

inline int blocks_for(int64_t n) { return (int)((n + TPB - 1) / TPB); }

__global__ void k_symlen(const int64_t* __restrict__ off, const double* __restrict__ dd, int64_t n,
                         double c, int32_t* __restrict__ len) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int64_t a = off[v], b = off[v + 1];
    int64_t lo = a, hi = b;
    if (c > 0.0) {
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (fabs(dd[mid]) >= c) lo = mid + 1; else hi = mid;
        }
    } else {
        lo = b;
    }
    len[v] = (int32_t)(lo - a);
}

// Draw t of the pass: world t / k, index t % k. Returns false when the draw cannot close a
// triangle (|d_e| < cmin or an empty prefix).
__device__ __forceinline__ bool pass_draw(const SampleParams& sp, const SampleGraph& G,
                                          const int32_t* __restrict__ slen, int64_t t, int64_t& e,
                                          int32_t& world, int32_t& y) {
    if (sp.vrec) {
        const int64_t r = sp.vrec[t];
        e = r & 0xFFFFFFFFll;
        world = (int32_t)(r >> 32);
    } else {
        const uint64_t seed = sp.seed_dev ? *sp.seed_dev : sp.seed;
        world = (int32_t)(t / sp.k);
        const int64_t i = t - (int64_t)world * sp.k;
        e = utri_sample_edge(seed, (uint32_t)world, (uint64_t)i, G.m);
    }
    if (fabs(G.e_d[e]) < sp.cmin) return false;
    int32_t x;
    int lx;
    draw_ends(G, slen, e, x, y, lx);
    return lx > 0;
}

// When every active lane of the wave has the same group (the records of one sampled hub
// vertex), one atomic serves them all; otherwise each lane does its own. Returns the
// lane's slot offset from the value the atomic returned (for counting, unused).
__device__ __forceinline__ int group_slot(int32_t* cnt, int32_t y, bool act, bool consume) {
    const uint64_t am = __ballot(act);
    if (am == 0) return 0;
    const int lead = __ffsll((long long)am) - 1;
    const int32_t y0 = __shfl(y, lead);
    const uint64_t same = __ballot(act && y == y0);
    if (same == am) {
        const int nact = __popcll(am);
        const int rank = __popcll(am & ((1ull << utri_lane()) - 1ull));
        int base = 0;
        if (utri_lane() == lead) base = consume ? atomicSub(&cnt[y0], nact) : atomicAdd(&cnt[y0], nact);
        base = __shfl(base, lead);
        return base - 1 - rank;  // consume: slots base-1, base-2, ... in lane order
    }
    if (!act) return 0;
    return consume ? atomicSub(&cnt[y], 1) - 1 : atomicAdd(&cnt[y], 1);
}

// Lanes past the pass end take part in the wave-wide steps as inactive lanes.
__global__ void k_s_count(SampleParams sp, SampleGraph G, const int32_t* __restrict__ slen,
                          int32_t* __restrict__ cnt) {
    const int64_t t = sp.t0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t e = 0;
    int32_t world = 0, y = 0;
    const bool act = t < sp.t1 && pass_draw(sp, G, slen, t, e, world, y);
    (void)group_slot(cnt, y, act, false);
}

// Each draw takes a distinct slot of its group (the count is consumed downwards).
__global__ void k_s_scatter(SampleParams sp, SampleGraph G, const int32_t* __restrict__ slen,
                            int32_t* __restrict__ cnt, int64_t* __restrict__ rec) {
    const int64_t t = sp.t0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t e = 0;
    int32_t world = 0, y = 0;
    const bool act = t < sp.t1 && pass_draw(sp, G, slen, t, e, world, y);
    const int slot = group_slot(cnt, y, act, true);
    if (act) rec[sp.goff[y] + slot] = e | ((int64_t)world << 32);
}

// Items per group: ceil(draws / chunk), as work-group items when the probed prefix fits a
// work-group table but not a wave table, as wave items when it fits a wave table, and as
// hub items (work-group items probing the global table) when it fits neither.
__global__ void k_s_icount(const int64_t* __restrict__ goff, const int32_t* __restrict__ slen,
                           int64_t n, int chunk, int32_t* __restrict__ cb, int32_t* __restrict__ cw,
                           int32_t* __restrict__ ch) {
    const int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= n) return;
    const int64_t c = goff[y + 1] - goff[y];
    const int32_t ns = (int32_t)((c + chunk - 1) / chunk);
    const int L = slen[y];
    cb[y] = (L > SCAP && L <= SCAPH) ? ns : 0;
    cw[y] = L <= SCAP ? ns : 0;
    ch[y] = L > SCAPH ? ns : 0;
}

__global__ void k_s_ifill(const int32_t* __restrict__ cb, const int32_t* __restrict__ cw,
                          const int32_t* __restrict__ ch, const int64_t* __restrict__ ob,
                          const int64_t* __restrict__ ow, const int64_t* __restrict__ oh, int64_t n,
                          int64_t wave_base, int64_t hub_base, int64_t* __restrict__ items) {
    const int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= n) return;
    for (int q = 0; q < cb[y]; q++) items[ob[y] + q] = y | ((int64_t)q << 32);
    for (int q = 0; q < cw[y]; q++) items[wave_base + ow[y] + q] = y | ((int64_t)q << 32);
    for (int q = 0; q < ch[y]; q++) items[hub_base + oh[y] + q] = y | ((int64_t)q << 32);
}

__global__ void __launch_bounds__(TPB) k_sample(SampleParams sp, SampleGraph G,
                                                const int32_t* __restrict__ slen) {
    __shared__ SampleLds S;
    thresh_stage(sp.cvals, sp.nt);
    sample_groups(sp, G, slen, S);
}

// one wave per listed edge: out[i][j][0/1] = local counts at threshold j (original order)
__global__ void __launch_bounds__(TPB) k_edge_local(SampleGraph G, const double* __restrict__ cv,
                                                    const int32_t* __restrict__ order, int nt,
                                                    const int64_t* __restrict__ eids, int64_t k,
                                                    int64_t* __restrict__ out) {
    __shared__ unsigned long long hist[WPB][2][NB];
    const int wib = threadIdx.x / UTRI_WAVE;
    const int lane = utri_lane();
    const int64_t gw = (int64_t)blockIdx.x * WPB + wib;
    const int64_t W = (int64_t)gridDim.x * WPB;
    thresh_stage(cv, nt);
    for (int64_t q = gw; q < k; q += W) {
        for (int t = lane; t < 2 * NB; t += UTRI_WAVE) hist[wib][t / NB][t % NB] = 0;
        utri_wave_sync();
        const int64_t e = eids[q];
        const double de = G.e_d[e];
        const int32_t a = G.inv[G.e_lo[e]], b = G.inv[G.e_hi[e]];
        const int64_t la = G.s_off[a + 1] - G.s_off[a], lb = G.s_off[b + 1] - G.s_off[b];
        const bool ax = (la < lb) || (la == lb && a < b);
        const int32_t x = ax ? a : b, y = ax ? b : a;
        const int64_t lx = ax ? la : lb;
        const int64_t xoff = G.s_off[x], hoff = G.h_off[y];
        const int lg = hbuckets_lg(G, y);
        for (int64_t j = lane; j < lx; j += UTRI_WAVE) {
            const int32_t w = G.s_adj[xoff + j];
            const int64_t sl = sym_lookup(G.h_tab, hoff, lg, w);
            if (sl >= 0) {
                const double s = utri_tri_s(de, G.s_d[xoff + j], sym_d(G.h_tab, sl));
                bool bal;
                const int bin = thresh_bin(s, bal);
                if (bin > 0) atomicAdd(&hist[wib][bal ? 0 : 1][bin], 1ull);
            }
        }
        utri_wave_sync();
        // suffix sums: a triangle in bin k is classified at sorted thresholds 0..k-1
        for (int js = lane; js < nt; js += UTRI_WAVE) {
            unsigned long long cb = 0, cu = 0;
            for (int bin = js + 1; bin <= nt; bin++) { cb += hist[wib][0][bin]; cu += hist[wib][1][bin]; }
            const int jo = order[js];
            out[(q * nt + jo) * 2] = (int64_t)cb;
            out[(q * nt + jo) * 2 + 1] = (int64_t)cu;
        }
        utri_wave_sync();
    }
}

// Vertex draw t = world * k + i: the sampled vertex (new id) and its prefix length.
__global__ void k_v_draw(uint64_t seed, int64_t k, int64_t T, int64_t n,
                         const int32_t* __restrict__ inv, const int32_t* __restrict__ slen,
                         int32_t* __restrict__ vq, int32_t* __restrict__ vlen) {
    UTRI_FOR_GRID(t, T) {
        const int32_t world = (int32_t)(t / k);
        const int64_t i = t - (int64_t)world * k;
        const int32_t q = inv[utri_sample_vertex(seed, (uint32_t)world, (uint64_t)i, n)];
        vq[t] = q;
        vlen[t] = slen[q];
    }
}

// One wave per vertex draw writes the edge records of the vertex's prefix.
__global__ void __launch_bounds__(TPB) k_v_expand(const int32_t* __restrict__ vq,
                                                  const int32_t* __restrict__ vlen,
                                                  const int64_t* __restrict__ voff, int64_t T,
                                                  int64_t k, const int64_t* __restrict__ s_off,
                                                  const int32_t* __restrict__ s_eid,
                                                  int64_t* __restrict__ vrec) {
    const int64_t W = (int64_t)gridDim.x * WPB;
    for (int64_t t = (int64_t)blockIdx.x * WPB + threadIdx.x / UTRI_WAVE; t < T; t += W) {
        const int64_t base = s_off[vq[t]], o = voff[t];
        const int64_t wtag = (t / k) << 32;
        const int L = vlen[t];
        for (int j = utri_lane(); j < L; j += UTRI_WAVE) vrec[o + j] = (int64_t)s_eid[base + j] | wtag;
    }
}

// One wave per listed vertex q (new id): the edge local counts of every edge (q, u) of
// q's prefix at the smallest threshold, summed in LDS; out = half the sums (each
// triangle at q is found through both of its edges at q).
__global__ void __launch_bounds__(TPB) k_vertex_local(SampleGraph G, const int32_t* __restrict__ slen,
                                                      const double* __restrict__ cv,
                                                      const int32_t* __restrict__ order, int nt,
                                                      const int64_t* __restrict__ vids, int64_t k,
                                                      int64_t* __restrict__ out) {
    __shared__ unsigned long long hist[WPB][2][NB];
    const int wib = threadIdx.x / UTRI_WAVE;
    const int lane = utri_lane();
    const int64_t gw = (int64_t)blockIdx.x * WPB + wib;
    const int64_t W = (int64_t)gridDim.x * WPB;
    thresh_stage(cv, nt);
    for (int64_t qi = gw; qi < k; qi += W) {
        for (int t = lane; t < 2 * NB; t += UTRI_WAVE) hist[wib][t / NB][t % NB] = 0;
        utri_wave_sync();
        const int32_t q = G.inv[vids[qi]];
        const int64_t qoff = G.s_off[q];
        const int lq = slen[q];
        for (int a = 0; a < lq; a++) {
            const int32_t u = G.s_adj[qoff + a];
            const double de = G.s_d[qoff + a];
            const int lu = slen[u];
            // stream the shorter prefix, look its entries up in the other row's table
            const bool qx = (lq < lu) || (lq == lu && q < u);
            const int32_t y = qx ? u : q;
            const int64_t xoff = G.s_off[qx ? q : u];
            const int lx = qx ? lq : lu;
            const int64_t hoff = G.h_off[y];
            const int lg = hbuckets_lg(G, y);
            for (int j = lane; j < lx; j += UTRI_WAVE) {
                const int64_t sl = sym_lookup(G.h_tab, hoff, lg, G.s_adj[xoff + j]);
                if (sl >= 0) {
                    const double s = utri_tri_s(de, G.s_d[xoff + j], sym_d(G.h_tab, sl));
                    bool bal;
                    const int bin = thresh_bin(s, bal);
                    if (bin > 0) atomicAdd(&hist[wib][bal ? 0 : 1][bin], 1ull);
                }
            }
        }
        utri_wave_sync();
        for (int js = lane; js < nt; js += UTRI_WAVE) {
            unsigned long long cb = 0, cu = 0;
            for (int bin = js + 1; bin <= nt; bin++) { cb += hist[wib][0][bin]; cu += hist[wib][1][bin]; }
            const int jo = order[js];
            out[(qi * nt + jo) * 2] = (int64_t)(cb / 2);
            out[(qi * nt + jo) * 2 + 1] = (int64_t)(cu / 2);
        }
        utri_wave_sync();
    }
}

// s of each listed triangle (original ids) from the per-row tables, and a key whose
// ascending order is ascending s (descending s when desc); -0 and +0 get one key so they
// tie, as their values do.
__global__ void k_topk_keys(SampleGraph G, const int32_t* __restrict__ tri, int64_t N, int desc,
                            double* __restrict__ sv, uint64_t* __restrict__ key,
                            uint32_t* __restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int32_t a = G.inv[tri[3 * i]], b = G.inv[tri[3 * i + 1]], c = G.inv[tri[3 * i + 2]];
    const int64_t ab = sym_lookup(G.h_tab, G.h_off[a], hbuckets_lg(G, a), b);
    const int64_t ac = sym_lookup(G.h_tab, G.h_off[a], hbuckets_lg(G, a), c);
    const int64_t bc = sym_lookup(G.h_tab, G.h_off[b], hbuckets_lg(G, b), c);
    // the listed triples are triangles, so every lookup hits
    const double s = utri_tri_s(ab >= 0 ? sym_d(G.h_tab, ab) : 0.0,
                                ac >= 0 ? sym_d(G.h_tab, ac) : 0.0,
                                bc >= 0 ? sym_d(G.h_tab, bc) : 0.0);
    sv[i] = s;
    uint64_t u = (uint64_t)__double_as_longlong(s == 0.0 ? 0.0 : s);
    u = (u >> 63) ? ~u : (u | (1ull << 63));
    key[i] = desc ? ~u : u;
    idx[i] = (uint32_t)i;
}

__global__ void k_topk_gather(const int32_t* __restrict__ tri, const double* __restrict__ sv,
                              const uint32_t* __restrict__ idx, int64_t r,
                              int32_t* __restrict__ out_tri, double* __restrict__ out_s) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= r) return;
    const int64_t j = idx[i];
    out_tri[3 * i] = tri[3 * j];
    out_tri[3 * i + 1] = tri[3 * j + 1];
    out_tri[3 * i + 2] = tri[3 * j + 2];
    out_s[i] = sv[j];
}

// hist [rows][2][nt+1] -> counts [rows][nt][2] (threshold order given by `order`) and
// est [rows][nt][2] = ((double)count * (double)num) / (3.0 * (double)k), where count is
// the suffix sum of the bins divided by div (2 for vertex sampling, exact: every triangle
// is counted twice there).
__global__ void k_finalize(const unsigned long long* __restrict__ hist, int rows, int nt,
                           const int32_t* __restrict__ order, int64_t m, int64_t k, int div,
                           int64_t* __restrict__ counts, double* __restrict__ est) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)rows * nt * 2) return;
    const int cls = (int)(t & 1);
    const int js = (int)((t >> 1) % nt);
    const int64_t r = (t >> 1) / nt;
    const unsigned long long* h = hist + (r * 2 + cls) * (nt + 1);
    unsigned long long c = 0;
    for (int bin = js + 1; bin <= nt; bin++) c += h[bin];
    c /= (unsigned long long)div;
    const int jo = order ? order[js] : js;
    const int64_t o = (r * nt + jo) * 2 + cls;
    if (counts) counts[o] = (int64_t)c;
    if (est) est[o] = ((double)c * (double)m) / (3.0 * (double)k);
}

}  // namespace

int utri_sym_prepare(utri_graph* g, double c_rows, hipStream_t s, int32_t** slen) {
    void* p;
    UTRI_TRY(utri_scratch(g, SCR_SLEN, sizeof(int32_t) * (size_t)(g->n + 1), &p));
    *slen = (int32_t*)p;
    if (g->n == 0) return UTRI_OK;
    hipLaunchKernelGGL(k_symlen, dim3(blocks_for(g->n)), dim3(TPB), 0, s, g->s_off, g->s_d, g->n,
                       c_rows, (int32_t*)p);
    UTRI_HIP_TRY(hipGetLastError());
    return UTRI_OK;
}

static SampleGraph sample_graph(utri_graph* g) {
    return SampleGraph{g->m, g->e_lo, g->e_hi, g->e_d, g->inv, g->s_off, g->s_adj, g->s_d,
                       g->h_off, g->h_tab};
}

int utri_sample_prepare(utri_graph* g, SampleParams& sp, const int32_t* slen, int64_t t0,
                        int64_t t1, hipStream_t s) {
    const int64_t n = g->n;
    const int64_t draws = t1 - t0;
    // items of one list: at most ceil(c / chunk) <= c / chunk + 1 per non-empty group
    const int64_t bound = draws / sp.chunk + std::min<int64_t>(n, draws) + 1;
    void *pc, *po, *pr, *pic, *pio, *pit, *pq;
    UTRI_TRY(utri_scratch(g, SCR_SCNT, sizeof(int32_t) * (size_t)(n + 2), &pc));
    UTRI_TRY(utri_scratch(g, SCR_SOFF, sizeof(int64_t) * (size_t)(n + 1), &po));
    UTRI_TRY(utri_scratch(g, SCR_SREC, sizeof(int64_t) * (size_t)(draws + 1), &pr));
    UTRI_TRY(utri_scratch(g, SCR_SICNT, sizeof(int32_t) * (size_t)(3 * n), &pic));
    UTRI_TRY(utri_scratch(g, SCR_SIOFF, sizeof(int64_t) * (size_t)(3 * n), &pio));
    UTRI_TRY(utri_scratch(g, SCR_SITEMS, sizeof(int64_t) * (size_t)(3 * bound), &pit));
    UTRI_TRY(utri_scratch(g, SCR_SQ, sizeof(int64_t) * 16, &pq));
    int32_t* cnt = (int32_t*)pc;
    int64_t* goff = (int64_t*)po;
    int32_t* cb = (int32_t*)pic;
    int32_t* cw = cb + n;
    int32_t* ch = cw + n;
    int64_t* ob = (int64_t*)pio;
    int64_t* ow = ob + n;
    int64_t* oh = ow + n;
    int64_t* q = (int64_t*)pq;
    sp.t0 = t0;
    sp.t1 = t1;
    sp.rec = (const int64_t*)pr;
    sp.goff = goff;
    sp.items = (const int64_t*)pit;
    sp.nitems = q;
    sp.wave_base = bound;
    sp.hub_base = 2 * bound;
    sp.qctr = (unsigned long long*)(q + 4);  // q[4, 14)
    UTRI_TRY(utri_fill_u64(cnt, 0, (n + 2) / 2, s));
    UTRI_TRY(utri_fill_u64(q, 0, 16, s));
    const SampleGraph G = sample_graph(g);
    if (draws > 0) {
        hipLaunchKernelGGL(k_s_count, dim3(blocks_for(draws)), dim3(TPB), 0, s, sp, G, slen, cnt);
        UTRI_HIP_TRY(hipGetLastError());
    }
    UTRI_TRY(utri_scan_i32(g, cnt, goff, n, goff + n, s));
    if (draws > 0) {
        hipLaunchKernelGGL(k_s_scatter, dim3(blocks_for(draws)), dim3(TPB), 0, s, sp, G, slen, cnt,
                           (int64_t*)pr);
        UTRI_HIP_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(k_s_icount, dim3(blocks_for(n)), dim3(TPB), 0, s, (const int64_t*)goff, slen,
                       n, sp.chunk, cb, cw, ch);
    UTRI_HIP_TRY(hipGetLastError());
    UTRI_TRY(utri_scan_i32(g, cb, ob, n, q, s));
    UTRI_TRY(utri_scan_i32(g, cw, ow, n, q + 1, s));
    UTRI_TRY(utri_scan_i32(g, ch, oh, n, q + 2, s));
    hipLaunchKernelGGL(k_s_ifill, dim3(blocks_for(n)), dim3(TPB), 0, s, (const int32_t*)cb,
                       (const int32_t*)cw, (const int32_t*)ch, (const int64_t*)ob,
                       (const int64_t*)ow, (const int64_t*)oh, n, bound, 2 * bound, (int64_t*)pit);
    UTRI_HIP_TRY(hipGetLastError());
    return UTRI_OK;
}

int utri_sample_launch(utri_graph* g, const SampleParams& sp, const int32_t* slen, hipStream_t s) {
    if (g->m == 0 || sp.t1 <= sp.t0) return UTRI_OK;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sample, TPB, 0) != hipSuccess || nb < 1)
        nb = 4;
    const int blocks = g->num_cu * std::min(nb, g->sample_blocks_per_cu);
    hipLaunchKernelGGL(k_sample, dim3(blocks), dim3(TPB), 0, s, sp, sample_graph(g), slen);
    UTRI_HIP_TRY(hipGetLastError());
    return UTRI_OK;
}

int utri_edge_local_launch(utri_graph* g, const double* cvals, const int32_t* order, int nt,
                           const int64_t* eids, int64_t k, int64_t* out, hipStream_t s) {
    if (k <= 0) return UTRI_OK;
    const int blocks = (int)std::min<int64_t>((int64_t)g->num_cu * 8, (k + WPB - 1) / WPB);
    hipLaunchKernelGGL(k_edge_local, dim3(blocks), dim3(TPB), 0, s, sample_graph(g), cvals, order,
                       nt, eids, k, out);
    UTRI_HIP_TRY(hipGetLastError());
    return UTRI_OK;
}

int utri_finalize_launch(const unsigned long long* hist, int rows, int nt, const int32_t* order,
                         int64_t m, int64_t k, int64_t* counts_out, double* est_out,
                         hipStream_t s, int div) {
    const int64_t tot = (int64_t)rows * nt * 2;
    if (tot == 0) return UTRI_OK;
    hipLaunchKernelGGL(k_finalize, dim3(blocks_for(tot)), dim3(TPB), 0, s, hist, rows, nt, order,
                       m, k > 0 ? k : 1, div, counts_out, est_out);
    UTRI_HIP_TRY(hipGetLastError());
    return UTRI_OK;
}

int utri_vertex_prepare(utri_graph* g, SampleParams& sp, const int32_t* slen, hipStream_t s,
                        int64_t* n_records) {
    const int64_t T = (int64_t)sp.worlds * sp.k;
    void *pq, *pl, *po, *pr;
    UTRI_TRY(utri_scratch(g, SCR_VQ, sizeof(int32_t) * (size_t)T, &pq));
    UTRI_TRY(utri_scratch(g, SCR_VLEN, sizeof(int32_t) * (size_t)T, &pl));
    UTRI_TRY(utri_scratch(g, SCR_VOFF, sizeof(int64_t) * (size_t)(T + 1), &po));
    int32_t* vq = (int32_t*)pq;
    int32_t* vlen = (int32_t*)pl;
    int64_t* voff = (int64_t*)po;
    hipLaunchKernelGGL(k_v_draw, dim3(utri_grid(T, TPB)), dim3(TPB), 0, s, sp.seed, sp.k, T, g->n,
                       (const int32_t*)g->inv, slen, vq, vlen);
    UTRI_HIP_TRY(hipGetLastError());
    UTRI_TRY(utri_scan_i32(g, vlen, voff, T, voff + T, s));
    int64_t R = 0;
    UTRI_HIP_TRY(hipMemcpyAsync(&R, voff + T, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    UTRI_HIP_TRY(hipStreamSynchronize(s));
    UTRI_TRY(utri_scratch(g, SCR_VREC, sizeof(int64_t) * (size_t)(R + 1), &pr));
    if (R > 0) {
        const int blocks = (int)std::min<int64_t>((int64_t)g->num_cu * 16, (T + WPB - 1) / WPB);
        hipLaunchKernelGGL(k_v_expand, dim3(blocks), dim3(TPB), 0, s, (const int32_t*)vq,
                           (const int32_t*)vlen, (const int64_t*)voff, T, sp.k,
                           (const int64_t*)g->s_off, (const int32_t*)g->s_eid, (int64_t*)pr);
        UTRI_HIP_TRY(hipGetLastError());
    }
    sp.vrec = (const int64_t*)pr;
    *n_records = R;
    return UTRI_OK;
}

int utri_vertex_local_launch(utri_graph* g, const double* cvals, const int32_t* order, int nt,
                             const int64_t* vids, int64_t k, int64_t* out, hipStream_t s) {
    if (k <= 0) return UTRI_OK;
    int32_t* slen;
    double cmin = 0.0;
    UTRI_HIP_TRY(hipMemcpyAsync(&cmin, cvals, sizeof(double), hipMemcpyDeviceToHost, s));
    UTRI_HIP_TRY(hipStreamSynchronize(s));
    UTRI_TRY(utri_sym_prepare(g, cmin, s, &slen));
    const int blocks = (int)std::min<int64_t>((int64_t)g->num_cu * 8, (k + WPB - 1) / WPB);
    hipLaunchKernelGGL(k_vertex_local, dim3(blocks), dim3(TPB), 0, s, sample_graph(g),
                       (const int32_t*)slen, cvals, order, nt, vids, k, out);
    UTRI_HIP_TRY(hipGetLastError());
    return UTRI_OK;
}

int utri_topk_keys_launch(utri_graph* g, const int32_t* tri, int64_t N, int desc, double* sv,
                          uint64_t* key, uint32_t* idx, hipStream_t s) {
    if (N <= 0) return UTRI_OK;
    hipLaunchKernelGGL(k_topk_keys, dim3(blocks_for(N)), dim3(TPB), 0, s, sample_graph(g), tri, N,
                       desc, sv, key, idx);
    UTRI_HIP_TRY(hipGetLastError());
    return UTRI_OK;
}

int utri_topk_gather_launch(const int32_t* tri, const double* sv, const uint32_t* idx, int64_t r,
                            int32_t* out_tri, double* out_s, hipStream_t s) {
    if (r <= 0) return UTRI_OK;
    hipLaunchKernelGGL(k_topk_gather, dim3(blocks_for(r)), dim3(TPB), 0, s, tri, sv, idx, r,
                       out_tri, out_s);
    UTRI_HIP_TRY(hipGetLastError());
    return UTRI_OK;
}
