// walk.hip -- the triangle walk: forward edge iteration over the degree-oriented graph
// (Algorithm "Baseline UBTE/UBTC", Section 4) with the probability pruning of Section 5.
//
// For every oriented edge u -> v and every w in N+(u) ∩ N+(v) the triangle (u, v, w)
// is visited exactly once (Node Order, Section 4). Rows are stored in Absolute Edge
// Order, so Lemma 2 (every triangle through an edge with |d| < c is unclassifiable)
// reduces each row to a prefix of length len[x]; the optional Lemma-3 cut shortens the
// target row N+(v) further, per pair, to entries with |d_vw| * |d_uv| * max|d_u.| >= c.
//
// GPU mapping (one wave64 per work item, persistent grid):
//   item = (u, chunk): the chunk's slice of N+(u) (at most CAP entries) is staged in an
//   LDS open-addressing table (neighbour -> position). The wave then walks the target
//   rows N+(v), v in N+(u), one row at a time: v, its row start and length are
//   broadcast into scalar registers and the row is streamed coalesced, 64 entries per
//   step, each lane probing one w in the table. Only hits read d values. The classify,
//   count, histogram, fixed-point, enumeration and statistics epilogues are selected at
//   compile time.
#include <algorithm>

#include "walk_common.h"

using namespace utri_dev;

namespace {

inline int blocks_for(int64_t n) { return (int)((n + TPB - 1) / TPB); }

__global__ void k_rowlen(const int64_t* __restrict__ off, const double* __restrict__ dd,
                         int64_t n, double c, int cap, int32_t* __restrict__ len,
                         int32_t* __restrict__ icnt) {
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
    int32_t L = (int32_t)(lo - a);
    len[v] = L;
    if (icnt) icnt[v] = (L >= 2) ? (L + cap - 1) / cap : 0;
}

__global__ void k_items(const int32_t* __restrict__ icnt, const int64_t* __restrict__ ioff,
                        int64_t n, int64_t* __restrict__ items) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int c = icnt[v];
    int64_t o = ioff[v];
    for (int k = 0; k < c; k++) items[o + k] = ((int64_t)k << 32) | (int64_t)v;
}

struct WalkLaneState {
    uint64_t nb = 0, nu = 0;       // COUNT / ENUM_COUNT
    uint64_t tri = 0;              // EXPECTED / STATS
    uint64_t slo = 0;              // EXPECTED: sum of low 32 bits of each fixed-point term
    int64_t shi = 0;               // EXPECTED: sum of the terms shifted right by 32
    uint64_t wt = 0, wt_all = 0;   // STATS: streamed target elements (first chunk / all)
};

// Process one work item. `it` is the item's index in the items array.
template <int MODE>
__device__ void walk_item(const WalkParams& wp, const int64_t* __restrict__ o_off,
                          const int32_t* __restrict__ o_adj, const double* __restrict__ o_d,
                          const int32_t* __restrict__ len, const int32_t* __restrict__ perm,
                          int64_t item, int64_t it, WalkLds& L, HistLds* H,
                          WalkLaneState& st) {
    const int lane = utri_lane();
    const int u = (int)(item & 0xFFFFFFFF);
    const int chunk = (int)(item >> 32);
    const int64_t ou = o_off[u];
    const int Lu = len[u];
    const int cb = chunk * CAP;
    const int cl = min(CAP, Lu - cb);
    int lg = 1;
    while ((1 << lg) < 2 * cl) lg++;
    const int size = 1 << lg;
    const uint32_t mask = (uint32_t)(size - 1);

    // stage the chunk of N+(u) as (neighbour -> position) in the wave's LDS table
    for (int i = lane; i < size; i += UTRI_WAVE) L.key[i] = -1;
    utri_wave_sync();
    for (int j = lane; j < cl; j += UTRI_WAVE) {
        const int32_t w = o_adj[ou + cb + j];
        uint32_t h = utri_hash32(w, lg);
        for (;;) {
            const int old = atomicCAS(&L.key[h], -1, w);
            if (old == -1) { L.pos[h] = (uint16_t)j; break; }
            h = (h + 1) & mask;
        }
    }
    utri_wave_sync();

    const double dmax_chunk = fabs(o_d[ou + cb]);
    const int32_t pu = (MODE == WALK_ENUM_FILL) ? perm[u] : 0;
    int64_t run_b = 0, run_u = 0;
    if (MODE == WALK_ENUM_FILL) {
        run_b = wp.off_b[it];
        run_u = wp.off_u[it];
    }

    for (int i0 = 0; i0 < Lu; i0 += UTRI_WAVE) {
        // lane i holds v = N+(u)[i0 + i], its row start, kept length and d_uv
        const int i = i0 + lane;
        int lv = 0, v = 0;
        int64_t ov = 0;
        double duv = 0.0;
        if (i < Lu) {
            v = o_adj[ou + i];
            duv = o_d[ou + i];
            ov = o_off[v];
            lv = len[v];
            if (wp.lemma3 && lv > 0) {
                // Lemma 3: keep w only if |d_vw| * (|d_uv| * max|d_uw|) >= c (with slack)
                const double P = __dmul_rn(fabs(duv), dmax_chunk);
                int a = 0, b = lv;
                while (a < b) {
                    const int mid = (a + b) >> 1;
                    if (__dmul_rn(fabs(o_d[ov + mid]), P) >= wp.c_l3) a = mid + 1; else b = mid;
                }
                lv = a;
            }
            if (MODE == WALK_STATS) {
                st.wt_all += (uint64_t)lv;
                if (chunk == 0) st.wt += (uint64_t)lv;
            }
        }
        const int nv = min(UTRI_WAVE, Lu - i0);
        for (int s_i = 0; s_i < nv; s_i++) {
            const int lvs = bcast_i32(lv, s_i);
            if (lvs == 0) continue;
            const int64_t ovs = bcast_i64(ov, s_i);
            const double duvs = bcast_f64(duv, s_i);
            const int32_t pv = (MODE == WALK_ENUM_FILL) ? perm[bcast_i32(v, s_i)] : 0;
            for (int j0 = 0; j0 < lvs; j0 += UTRI_WAVE) {
                const int j = j0 + lane;
                bool is_b = false, is_u = false;
                int32_t tw = 0;
                if (j < lvs) {
                    const int32_t w = o_adj[ovs + j];
                    uint32_t h = utri_hash32(w, lg);
                    int hit = -1;
                    for (;;) {
                        const int k = L.key[h];
                        if (k == w) { hit = L.pos[h]; break; }
                        if (k == -1) break;
                        h = (h + 1) & mask;
                    }
                    if (hit >= 0) {
                        const double dvw = o_d[ovs + j];
                        const double duw = o_d[ou + cb + hit];
                        if (MODE == WALK_STATS) {
                            st.tri++;
                        } else {
                            const double s = utri_tri_s(duvs, duw, dvw);
                            if (MODE == WALK_COUNT || MODE == WALK_ENUM_COUNT) {
                                if (s <= -wp.c) st.nb++;
                                else if (s > wp.c) st.nu++;
                            } else if (MODE == WALK_HIST) {
                                bool bal;
                                const int bin = utri_bin_of(s, wp.cvals, wp.nt, bal);
                                if (bin > 0) atomicAdd(&H->hist[bal ? 0 : 1][bin], 1ull);
                            } else if (MODE == WALK_EXPECTED) {
                                const int64_t t = utri_fix62(s);
                                st.tri++;
                                st.slo += (uint64_t)(uint32_t)(t & 0xFFFFFFFFll);
                                st.shi += (t >> 32);
                            } else if (MODE == WALK_ENUM_FILL) {
                                is_b = (s <= -wp.c) && (wp.which & UTRI_BAL);
                                is_u = (s > wp.c) && (wp.which & UTRI_UNBAL);
                                tw = w;
                            }
                        }
                    }
                }
                if (MODE == WALK_ENUM_FILL) {
                    const uint64_t mb = __ballot(is_b);
                    const uint64_t mu = __ballot(is_u);
                    if (is_b || is_u) {
                        int32_t a = pu, b = pv, c = perm[tw], t;
                        if (b < a) { t = a; a = b; b = t; }
                        if (c < b) { t = b; b = c; c = t; }
                        if (b < a) { t = a; a = b; b = t; }
                        const uint64_t lt = __lanemask_lt();
                        int32_t* dst;
                        int64_t slot;
                        if (is_b) { dst = wp.out_bal; slot = run_b + __popcll(mb & lt); }
                        else      { dst = wp.out_unbal; slot = run_u + __popcll(mu & lt); }
                        dst[3 * slot] = a;
                        dst[3 * slot + 1] = b;
                        dst[3 * slot + 2] = c;
                    }
                    run_b += __popcll(mb);
                    run_u += __popcll(mu);
                }
            }
        }
    }
    if (MODE == WALK_ENUM_COUNT) {
        const uint64_t item_nb = utri_wave_sum_u64(st.nb);
        const uint64_t item_nu = utri_wave_sum_u64(st.nu);
        if (lane == 0) {
            wp.cnt_b[it] = (int64_t)item_nb;
            wp.cnt_u[it] = (int64_t)item_nu;
        }
        st.nb = st.nu = 0;
    }
    utri_wave_sync();
}

template <int MODE>
__device__ void walk_flush(const WalkParams& wp, HistLds* H, WalkLaneState& st) {
    const int lane = utri_lane();
    if (MODE == WALK_COUNT) {
        const uint64_t b = utri_wave_sum_u64(st.nb), u = utri_wave_sum_u64(st.nu);
        if (lane == 0) {
            if (b) atomicAdd(&wp.acc[0], (unsigned long long)b);
            if (u) atomicAdd(&wp.acc[1], (unsigned long long)u);
        }
    } else if (MODE == WALK_EXPECTED) {
        // lane value = shi * 2^32 + slo as a 128-bit two's complement number
        uint64_t lo = ((uint64_t)st.shi << 32);
        uint64_t hi = (uint64_t)(st.shi >> 32);
        const uint64_t s2 = lo + st.slo;
        hi += (s2 < lo) ? 1ull : 0ull;
        lo = s2;
        const uint64_t tri = utri_wave_sum_u64(st.tri);
        utri_wave_sum_u128(lo, hi);
        if (lane == 0) {
            if (tri) atomicAdd(&wp.acc[0], (unsigned long long)tri);
            utri_atomic_add_u128(&wp.acc[1], lo, hi);
        }
    } else if (MODE == WALK_STATS) {
        const uint64_t a = utri_wave_sum_u64(st.tri), b = utri_wave_sum_u64(st.wt),
                       c = utri_wave_sum_u64(st.wt_all);
        if (lane == 0) {
            atomicAdd(&wp.acc[0], (unsigned long long)a);
            atomicAdd(&wp.acc[1], (unsigned long long)b);
            atomicAdd(&wp.acc[2], (unsigned long long)c);
        }
    } else if (MODE == WALK_HIST) {
        utri_wave_sync();
        for (int q = lane; q < 2 * NB; q += UTRI_WAVE) {
            const int cls = q / NB, bin = q % NB;
            const unsigned long long v = H->hist[cls][bin];
            if (v && bin <= wp.nt) atomicAdd(&wp.acc[cls * (wp.nt + 1) + bin], v);
        }
    }
}

template <int MODE>
__global__ void __launch_bounds__(TPB) k_walk(WalkParams wp, const int64_t* __restrict__ o_off,
                                              const int32_t* __restrict__ o_adj,
                                              const double* __restrict__ o_d,
                                              const int32_t* __restrict__ len,
                                              const int32_t* __restrict__ perm,
                                              const int64_t* __restrict__ items,
                                              const int64_t* __restrict__ n_items_dev) {
    __shared__ WalkLds lds[WPB];
    __shared__ HistLds hlds[MODE == WALK_HIST ? WPB : 1];
    const int wib = threadIdx.x / UTRI_WAVE;
    WalkLds& L = lds[wib];
    HistLds* H = &hlds[MODE == WALK_HIST ? wib : 0];
    if (MODE == WALK_HIST) {
        for (int q = utri_lane(); q < 2 * NB; q += UTRI_WAVE) H->hist[q / NB][q % NB] = 0;
        utri_wave_sync();
    }
    const int64_t nitems = *n_items_dev;
    const int64_t gw = (int64_t)blockIdx.x * WPB + wib;
    const int64_t W = (int64_t)gridDim.x * WPB;
    WalkLaneState st;
    for (int64_t q = gw; q < nitems; q += W) {
        const int64_t it = nitems - 1 - q;  // heaviest vertices (highest ids) first
        walk_item<MODE>(wp, o_off, o_adj, o_d, len, perm, items[it], it, L, H, st);
    }
    walk_flush<MODE>(wp, H, st);
}

// Fused batch: walk items (threshold histogram of every triangle at the smallest
// threshold) followed by edge-sampling units, in one persistent launch.
__global__ void __launch_bounds__(TPB) k_batch(WalkParams wp, const int64_t* __restrict__ o_off,
                                               const int32_t* __restrict__ o_adj,
                                               const double* __restrict__ o_d,
                                               const int32_t* __restrict__ len,
                                               const int32_t* __restrict__ perm,
                                               const int64_t* __restrict__ items,
                                               const int64_t* __restrict__ n_items_dev,
                                               SampleParams sp, SampleGraph G,
                                               const int32_t* __restrict__ slen, int64_t units) {
    __shared__ WalkLds lds[WPB];
    __shared__ HistLds hlds[WPB];
    __shared__ SegLds slds[WPB];
    const int wib = threadIdx.x / UTRI_WAVE;
    WalkLds& L = lds[wib];
    HistLds* H = &hlds[wib];
    for (int q = utri_lane(); q < 2 * NB; q += UTRI_WAVE) H->hist[q / NB][q % NB] = 0;
    utri_wave_sync();
    const int64_t nitems = (wp.acc != nullptr) ? *n_items_dev : 0;
    const int64_t gw = (int64_t)blockIdx.x * WPB + wib;
    const int64_t W = (int64_t)gridDim.x * WPB;
    const int64_t upw = (sp.k + sp.chunk - 1) / sp.chunk;  // units per world
    WalkLaneState st;
    for (int64_t q = gw; q < nitems + units; q += W) {
        if (q < nitems) {
            const int64_t it = nitems - 1 - q;
            walk_item<WALK_HIST>(wp, o_off, o_adj, o_d, len, perm, items[it], it, L, H, st);
        } else {
            const int64_t u = q - nitems;
            const int32_t world = (int32_t)(u / upw);
            const int64_t part = u % upw;
            const int64_t i0 = part * sp.chunk;
            const int64_t i1 = std::min<int64_t>(sp.k, i0 + sp.chunk);
            sample_unit(sp, G, slen, world, i0, i1, slds[wib]);
        }
    }
    if (wp.acc != nullptr) walk_flush<WALK_HIST>(wp, H, st);
}

}  // namespace

int utri_walk_prepare(utri_graph* g, double c_rows, int cap, hipStream_t s, int64_t** items,
                      int64_t** n_items_dev, int32_t** len) {
    (void)cap;
    const int64_t n = g->n;
    void *plen, *picnt, *pioff, *pitems, *pn;
    UTRI_TRY(utri_scratch(g, SCR_LEN, sizeof(int32_t) * (size_t)(n + 1), &plen));
    UTRI_TRY(utri_scratch(g, SCR_ICNT, sizeof(int32_t) * (size_t)(n + 1), &picnt));
    UTRI_TRY(utri_scratch(g, SCR_IOFF, sizeof(int64_t) * (size_t)(n + 1), &pioff));
    const int64_t bound = std::min<int64_t>(g->m, n + g->m / CAP + 1) + 1;
    UTRI_TRY(utri_scratch(g, SCR_ITEMS, sizeof(int64_t) * (size_t)bound, &pitems));
    UTRI_TRY(utri_scratch(g, SCR_NITEMS, sizeof(int64_t) * 4, &pn));
    *items = (int64_t*)pitems;
    *n_items_dev = (int64_t*)pn;
    *len = (int32_t*)plen;
    UTRI_TRY(utri_fill_u64(pn, 0, 1, s));
    if (n == 0) return UTRI_OK;
    hipLaunchKernelGGL(k_rowlen, dim3(blocks_for(n)), dim3(TPB), 0, s, g->o_off, g->o_d, n,
                       c_rows, CAP, (int32_t*)plen, (int32_t*)picnt);
    UTRI_HIP_TRY(hipGetLastError());
    UTRI_TRY(utri_scan_i32(g, (const int32_t*)picnt, (int64_t*)pioff, n, (int64_t*)pn, s));
    hipLaunchKernelGGL(k_items, dim3(blocks_for(n)), dim3(TPB), 0, s, (const int32_t*)picnt,
                       (const int64_t*)pioff, n, (int64_t*)pitems);
    UTRI_HIP_TRY(hipGetLastError());
    return UTRI_OK;
}

int utri_walk_items_bound(utri_graph* g) {
    return (int)std::min<int64_t>(g->m, g->n + g->m / CAP + 1);
}

template <int MODE>
static void launch_walk(utri_graph* g, int blocks, const WalkParams& wp, const int32_t* len,
                        const int64_t* items, const int64_t* n_items_dev, hipStream_t s) {
    hipLaunchKernelGGL(k_walk<MODE>, dim3(blocks), dim3(TPB), 0, s, wp, g->o_off, g->o_adj,
                       g->o_d, len, g->perm, items, n_items_dev);
}

int utri_walk_launch(utri_graph* g, int mode, const WalkParams& wp, const int64_t* items,
                     const int64_t* n_items_dev, const int32_t* len, int64_t n_items_host_bound,
                     hipStream_t s) {
    (void)n_items_host_bound;
    if (g->n == 0 || g->m == 0) return UTRI_OK;
    const int blocks = g->num_cu * g->walk_blocks_per_cu;
    switch (mode) {
        case WALK_COUNT: launch_walk<WALK_COUNT>(g, blocks, wp, len, items, n_items_dev, s); break;
        case WALK_HIST: launch_walk<WALK_HIST>(g, blocks, wp, len, items, n_items_dev, s); break;
        case WALK_EXPECTED: launch_walk<WALK_EXPECTED>(g, blocks, wp, len, items, n_items_dev, s); break;
        case WALK_ENUM_COUNT: launch_walk<WALK_ENUM_COUNT>(g, blocks, wp, len, items, n_items_dev, s); break;
        case WALK_ENUM_FILL: launch_walk<WALK_ENUM_FILL>(g, blocks, wp, len, items, n_items_dev, s); break;
        case WALK_STATS: launch_walk<WALK_STATS>(g, blocks, wp, len, items, n_items_dev, s); break;
        default: return UTRI_E_INVALID;
    }
    UTRI_HIP_TRY(hipGetLastError());
    return UTRI_OK;
}

int utri_batch_launch(utri_graph* g, const WalkParams& wp, const int64_t* items,
                      const int64_t* n_items_dev, const int32_t* len, int64_t n_items_bound,
                      const SampleParams& sp, const int32_t* slen, hipStream_t s) {
    (void)n_items_bound;
    if (g->n == 0 || g->m == 0) return UTRI_OK;
    const int64_t units = (sp.hist != nullptr && sp.k > 0)
                              ? (int64_t)sp.worlds * ((sp.k + sp.chunk - 1) / sp.chunk) : 0;
    SampleGraph G{g->m, g->e_lo, g->e_hi, g->e_d, g->inv, g->s_off, g->s_adj, g->s_d, g->h_off,
                  g->h_slot};
    const int blocks = g->num_cu * g->walk_blocks_per_cu;
    hipLaunchKernelGGL(k_batch, dim3(blocks), dim3(TPB), 0, s, wp, g->o_off, g->o_adj, g->o_d,
                       len, g->perm, items, n_items_dev, sp, G, slen, units);
    UTRI_HIP_TRY(hipGetLastError());
    return UTRI_OK;
}
