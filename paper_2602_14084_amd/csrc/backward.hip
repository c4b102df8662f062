// backward.hip -- per-edge gradient of the expected balanced count.
//
// E = sum over triangles of P_bal = (1 - d_e d_f d_g)/2 (Section 3 four-term sum in
// product form, d = 1 - 2 P+). With dd_e/dp_e = -2, dE/dp_e = sum over the triangles
// (e, f, g) through e of d_f * d_g.
//
// Every triangle u < v < w (Node Order) is found by two walks over the degree-oriented
// rows O(.) and hands each of its edges the product of the other two d values:
//   * pass A, the forward walk's order: O(u) is staged in an LDS table with one
//     accumulator per entry and O(v) is streamed for every v in O(u). A hit w adds
//     d_uw * d_vw to the row sum of (u, v), reduced over the wave when the row ends and
//     added to v's entry, and d_uv * d_vw to w's entry, the edge (u, w);
//   * pass B, middle vertex first: O(v) is staged likewise and O(u) is streamed for every
//     in-neighbour u of v (an entry x < v of the symmetric row N(v)). A hit w adds
//     d_uv * d_uw to w's entry, the edge (v, w).
// The two passes stream sum_u |O(u)| (|O(u)| + |I(u)|) = sum_e min(deg) entries, the
// edge-centric cost, and every probe is an LDS bucket read (no hub tables in global
// memory). An entry's sum has one writer, the wave or work-group that staged the row.
// Rows longer than one table are cut into chunks and in-neighbour lists into ranges of the
// symmetric row; each (chunk, range) item writes its own slice of a partial-sum array and
// a final pass adds the slices of every oriented edge and rounds once. Each product is
// rounded to FP64, then summed exactly in 2^-62 fixed point (as two 64-bit half sums), so
// the result does not depend on the order and no atomics touch global memory.
#include <algorithm>

#include "walk_common.h"

using namespace utri_dev;

namespace {

#ifndef UTRI_GRAD_CAP
#define UTRI_GRAD_CAP 128       // longest row staged by one wave
#endif
#ifndef UTRI_GRAD_SLOTS
#define UTRI_GRAD_SLOTS 4       // wave-table slots per staged entry
#endif
#ifndef UTRI_GRAD_CAPH
#define UTRI_GRAD_CAPH 512      // row chunk staged by one work-group
#endif
#ifndef UTRI_GRAD_SLOTS_WG
#define UTRI_GRAD_SLOTS_WG 4    // work-group-table slots per staged entry
#endif
#ifndef UTRI_GRAD_SPAN
#define UTRI_GRAD_SPAN 256      // symmetric-row positions scanned by one pass-B item
#endif
constexpr int GCAP = UTRI_GRAD_CAP;
constexpr int GSL = UTRI_GRAD_SLOTS;
constexpr int GCAPH = UTRI_GRAD_CAPH;
constexpr int GSLH = UTRI_GRAD_SLOTS_WG;
constexpr int GSPAN = UTRI_GRAD_SPAN;
constexpr int GGROUP = 4;  // wave items taken per queue grab
static_assert((GCAP & (GCAP - 1)) == 0 && (GCAPH & (GCAPH - 1)) == 0 && GCAP <= GCAPH &&
                  GCAPH <= 65536 && (GSL & (GSL - 1)) == 0 && (GSLH & (GSLH - 1)) == 0 &&
                  GCAP * GSL >= 8 && GSPAN % UTRI_WAVE == 0,
              "table sizes are powers of two; item ranges are whole strips");

// An oriented row has at most sqrt(2m) < 2^16 entries (its entries have at least its own
// degree), so a row has at most 128 chunks; a symmetric row has fewer than 2^23 ranges.
// Pass-B work-group items pack (vertex, range, chunk) as 32 + 24 + 8 bits.
constexpr int RANGE_SHIFT = 32, CHUNK_SHIFT = 56;

struct GWaveLds {
    alignas(16) int32_t key[GCAP * GSL];
    uint16_t pos[GCAP * GSL];
    unsigned long long lo[GCAP];  // per entry: sum of the low 32 bits of its terms
    unsigned long long hi[GCAP];  // per entry: sum of the terms shifted right by 32
};
struct GBlockLds {
    alignas(16) int32_t key[GCAPH * GSLH];
    uint16_t pos[GCAPH * GSLH];
    unsigned long long lo[GCAPH];
    unsigned long long hi[GCAPH];
};
union GShared {
    GWaveLds wave[WPB];
    GBlockLds block;
};

struct GradParams {
    const int64_t* o_off;
    const int32_t* o_adj;      // packed words: id in the low bits
    const double* o_d;
    const int32_t* o_eid;
    const int64_t* s_off;
    const int32_t* s_adj;
    const double* s_d;
    uint32_t idmask;
    const int64_t* pa_off;     // [n+1] pass-A slices: chunks x |O(u)| entries per source u
    const int64_t* pb_off;     // [n+1] pass-B slices: ranges x |O(v)| entries per middle v
    ulonglong2* pa;            // (low-half sum, high-half sum) per entry and slice
    ulonglong2* pb;
    const int64_t* items;      // A-wave | A-block | B-wave | B-block item lists
    int64_t n_aw, n_ab, n_bw, n_bb;
    unsigned long long* qctr;  // four work-queue counters, zeroed per launch
    double* grad;
    int64_t n;
};

// The staged row (or chunk) of one item.
struct GTab {
    const int32_t* key;
    const uint16_t* pos;
    int lg;
    uint32_t mask;
    unsigned long long* lo;
    unsigned long long* hi;
    int64_t src;  // position of the staged entries in o_adj / o_d
};

__device__ __forceinline__ int64_t fix_prod(double a, double b) {
    return utri_fix62(__dmul_rn(a, b));
}

// Stream the oriented row [ovs, ovs + lvs) and handle every entry found in the table.
// Pass A (row O(v), dpair = d_uv): adds d_uw * d_vw to the lane's row sum and
// d_uv * d_vw to the hit entry. Pass B (row O(u), dpair = d_uv): adds d_uv * d_uw to the
// hit entry. Lanes past the row end are masked off and their results dropped.
template <bool PASS_A, int UNR>
__device__ __forceinline__ void g_stream(const GradParams& P, const GTab& T, int64_t ovs, int lvs,
                                         double dpair, uint64_t& slo, int64_t& shi) {
    static_assert(UNR * UTRI_WAVE <= UTRI_ROW_PAD, "row streams stay inside the padding");
    const int lane = utri_lane();
    const char* rowb = (const char*)((const uint32_t*)P.o_adj + ovs);
    const double* rowd = P.o_d + ovs;
    for (int j0 = 0; j0 < lvs; j0 += UNR * UTRI_WAVE) {
        uint32_t pw[UNR];
        const char* lb = rowb + (((uint32_t)(j0 + lane)) << 2);
#pragma unroll
        for (int k = 0; k < UNR; k++)
            pw[k] = (j0 + k * UTRI_WAVE + lane < lvs) ? *(const uint32_t*)(lb + k * 4 * UTRI_WAVE) : 0u;
#pragma unroll
        for (int k = 0; k < UNR; k++) {
            // strips past the row end hold no entries (wave-uniform exit)
            if (k > 0 && j0 + k * UTRI_WAVE >= lvs) break;
            const int j = j0 + k * UTRI_WAVE + lane;
            int h;
            const int kk = bucket_find(T.key, T.lg, T.mask, pw[k] & P.idmask, P.idmask, h);
            if (j < lvs && kk != 0) {
                const int hit = T.pos[h];
                const double dx = rowd[j];
                if (PASS_A) {
                    const int64_t t1 = fix_prod(P.o_d[T.src + hit], dx);
                    slo += (uint64_t)(uint32_t)(t1 & 0xFFFFFFFFll);
                    shi += t1 >> 32;
                }
                const int64_t t2 = fix_prod(dpair, dx);
                atomicAdd(&T.lo[hit], (unsigned long long)(uint32_t)(t2 & 0xFFFFFFFFll));
                atomicAdd(&T.hi[hit], (unsigned long long)(t2 >> 32));
            }
        }
    }
}

template <bool PASS_A>
__device__ __forceinline__ void g_stream_any(const GradParams& P, const GTab& T, int64_t ovs,
                                             int lvs, double dpair, uint64_t& slo, int64_t& shi) {
    if (lvs > 2 * UTRI_WAVE) g_stream<PASS_A, 4>(P, T, ovs, lvs, dpair, slo, shi);
    else if (lvs > UTRI_WAVE) g_stream<PASS_A, 2>(P, T, ovs, lvs, dpair, slo, shi);
    else if (lvs > 0) g_stream<PASS_A, 1>(P, T, ovs, lvs, dpair, slo, shi);
}

// Clear the table and the accumulators of a chunk of cl entries staged at o_adj[src].
__device__ __forceinline__ GTab g_clear(int64_t src, int cl, int32_t* key, uint16_t* pos,
                                        unsigned long long* lo, unsigned long long* hi, int slots,
                                        int tid, int nthreads) {
    const int lg = table_lg(cl, slots);
    const int nbk = 1 << lg;
    for (int i = tid; i < 4 * nbk; i += nthreads) key[i] = 0;
    for (int i = tid; i < cl; i += nthreads) { lo[i] = 0; hi[i] = 0; }
    return GTab{key, pos, lg, (uint32_t)(nbk - 1), lo, hi, src};
}

// Pass A over a chunk [cb, cb + cl) of O(u): the rows v = O(u)[i] with (i mod 64) % nparts
// == part are this wave's. A row sum whose entry is in the chunk goes to its accumulator;
// otherwise it is the item's own slice entry and is stored directly (also when zero).
__device__ __forceinline__ void g_pass_a_rows(const GradParams& P, const GTab& T, int64_t ou, int L,
                                              int cb, int cl, ulonglong2* slice, int part,
                                              int nparts) {
    const int lane = utri_lane();
    for (int i0 = 0; i0 < L; i0 += UTRI_WAVE) {
        const int i = i0 + lane;
        int64_t ov = 0;
        int lv = 0;
        double duv = 0.0;
        if (i < L) {
            const int32_t v = (int32_t)((uint32_t)P.o_adj[ou + i] & P.idmask);
            duv = P.o_d[ou + i];
            ov = P.o_off[v];
            lv = (int)(P.o_off[v + 1] - ov);
        }
        const int nv = min(UTRI_WAVE, L - i0);
        for (int si = part; si < nv; si += nparts) {
            uint64_t slo = 0;
            int64_t shi = 0;
            g_stream_any<true>(P, T, bcast_i64(ov, si), bcast_i32(lv, si), bcast_f64(duv, si), slo,
                               shi);
            const uint64_t l = utri_wave_sum_u64(slo);
            const uint64_t h = utri_wave_sum_u64((uint64_t)shi);
            if (lane == 0) {
                const int iv = i0 + si;
                if (iv >= cb && iv < cb + cl) {
                    if (l | h) {
                        atomicAdd(&T.lo[iv - cb], (unsigned long long)l);
                        atomicAdd(&T.hi[iv - cb], (unsigned long long)h);
                    }
                } else {
                    slice[iv] = make_ulonglong2(l, h);
                }
            }
        }
    }
}

// Pass B over range `range` of the symmetric row N(v): the in-neighbours u < v found there
// whose rank in their 64-position group is part mod nparts are this wave's.
__device__ __forceinline__ void g_pass_b_rows(const GradParams& P, const GTab& T, int32_t v, int range,
                                              int part, int nparts) {
    const int64_t sv = P.s_off[v];
    const int D = (int)(P.s_off[v + 1] - sv);
    const int pb = range * GSPAN;
    const int pe = min(D, pb + GSPAN);
    for (int g0 = pb; g0 < pe; g0 += UTRI_WAVE) {
        const int p = g0 + utri_lane();
        int32_t x = 0;
        bool in = false;
        if (p < pe) {
            x = P.s_adj[sv + p];
            in = x < v;
        }
        int64_t ou = 0;
        int lu = 0;
        double duv = 0.0;
        if (in) {
            ou = P.o_off[x];
            lu = (int)(P.o_off[x + 1] - ou);
            duv = P.s_d[sv + p];
        }
        uint64_t mask = __ballot(in);
        for (int r = 0; mask; r++) {
            const int si = __builtin_ctzll(mask);
            mask &= mask - 1;
            if (r % nparts != part) continue;
            uint64_t slo = 0;
            int64_t shi = 0;
            g_stream_any<false>(P, T, bcast_i64(ou, si), bcast_i32(lu, si), bcast_f64(duv, si), slo,
                                shi);
        }
    }
}

__device__ void g_item_a_block(const GradParams& P, int64_t item, GBlockLds& B) {
    const int wib = threadIdx.x / UTRI_WAVE;
    const int32_t u = (int32_t)(item & 0xFFFFFFFF);
    const int chunk = (int)(item >> 32);
    const int64_t ou = P.o_off[u];
    const int L = (int)(P.o_off[u + 1] - ou);
    const int cb = chunk * GCAPH;
    const int cl = min(GCAPH, L - cb);
    __syncthreads();  // the previous item is flushed
    const GTab T = g_clear(ou + cb, cl, B.key, B.pos, B.lo, B.hi, GSLH, threadIdx.x, TPB);
    __syncthreads();
    stage_table(P.o_adj, ou + cb, cl, B.key, B.pos, T.lg, threadIdx.x, TPB, P.idmask);
    __syncthreads();
    ulonglong2* slice = P.pa + P.pa_off[u] + (int64_t)chunk * L;
    g_pass_a_rows(P, T, ou, L, cb, cl, slice, wib, WPB);
    __syncthreads();
    for (int q = threadIdx.x; q < cl; q += TPB) slice[cb + q] = make_ulonglong2(B.lo[q], B.hi[q]);
}

__device__ void g_item_b_block(const GradParams& P, int64_t item, GBlockLds& B) {
    const int wib = threadIdx.x / UTRI_WAVE;
    const int32_t v = (int32_t)(item & 0xFFFFFFFF);
    const int range = (int)((item >> RANGE_SHIFT) & 0xFFFFFF);
    const int chunk = (int)((uint64_t)item >> CHUNK_SHIFT);
    const int64_t ov = P.o_off[v];
    const int L = (int)(P.o_off[v + 1] - ov);
    const int cb = chunk * GCAPH;
    const int cl = min(GCAPH, L - cb);
    __syncthreads();  // the previous item is flushed
    const GTab T = g_clear(ov + cb, cl, B.key, B.pos, B.lo, B.hi, GSLH, threadIdx.x, TPB);
    __syncthreads();
    stage_table(P.o_adj, ov + cb, cl, B.key, B.pos, T.lg, threadIdx.x, TPB, P.idmask);
    __syncthreads();
    g_pass_b_rows(P, T, v, range, wib, WPB);
    __syncthreads();
    ulonglong2* slice = P.pb + P.pb_off[v] + (int64_t)range * L;
    for (int q = threadIdx.x; q < cl; q += TPB) slice[cb + q] = make_ulonglong2(B.lo[q], B.hi[q]);
}

__device__ void g_item_a_wave(const GradParams& P, int32_t u, GWaveLds& W) {
    const int lane = utri_lane();
    const int64_t ou = P.o_off[u];
    const int L = (int)(P.o_off[u + 1] - ou);
    const GTab T = g_clear(ou, L, W.key, W.pos, W.lo, W.hi, GSL, lane, UTRI_WAVE);
    utri_wave_sync();
    stage_table(P.o_adj, ou, L, W.key, W.pos, T.lg, lane, UTRI_WAVE, P.idmask);
    utri_wave_sync();
    ulonglong2* slice = P.pa + P.pa_off[u];
    g_pass_a_rows(P, T, ou, L, 0, L, slice, 0, 1);
    utri_wave_sync();
    for (int q = lane; q < L; q += UTRI_WAVE) slice[q] = make_ulonglong2(W.lo[q], W.hi[q]);
    utri_wave_sync();  // read before the next item clears the accumulators
}

__device__ void g_item_b_wave(const GradParams& P, int64_t item, GWaveLds& W) {
    const int lane = utri_lane();
    const int32_t v = (int32_t)(item & 0xFFFFFFFF);
    const int range = (int)(item >> RANGE_SHIFT);
    const int64_t ov = P.o_off[v];
    const int L = (int)(P.o_off[v + 1] - ov);
    const GTab T = g_clear(ov, L, W.key, W.pos, W.lo, W.hi, GSL, lane, UTRI_WAVE);
    utri_wave_sync();
    stage_table(P.o_adj, ov, L, W.key, W.pos, T.lg, lane, UTRI_WAVE, P.idmask);
    utri_wave_sync();
    g_pass_b_rows(P, T, v, range, 0, 1);
    utri_wave_sync();
    ulonglong2* slice = P.pb + P.pb_off[v] + (int64_t)range * L;
    for (int q = lane; q < L; q += UTRI_WAVE) slice[q] = make_ulonglong2(W.lo[q], W.hi[q]);
    utri_wave_sync();  // read before the next item clears the accumulators
}

// Persistent grid, four atomic work queues, heaviest items (highest ids) first:
// A work-group items, B work-group items, then A and B wave items, GGROUP per grab.
__global__ void __launch_bounds__(TPB) k_grad2(GradParams P) {
    __shared__ GShared S;
    __shared__ int64_t s_q;
    const int wib = threadIdx.x / UTRI_WAVE;
    const int lane = utri_lane();
    const int64_t* it_aw = P.items;
    const int64_t* it_ab = it_aw + P.n_aw;
    const int64_t* it_bw = it_ab + P.n_ab;
    const int64_t* it_bb = it_bw + P.n_bw;
    for (;;) {
        if (threadIdx.x == 0) s_q = (int64_t)atomicAdd(&P.qctr[0], 1ull);
        __syncthreads();
        const int64_t q = s_q;
        __syncthreads();
        if (q >= P.n_ab) break;
        g_item_a_block(P, it_ab[P.n_ab - 1 - q], S.block);
    }
    for (;;) {
        if (threadIdx.x == 0) s_q = (int64_t)atomicAdd(&P.qctr[1], 1ull);
        __syncthreads();
        const int64_t q = s_q;
        __syncthreads();
        if (q >= P.n_bb) break;
        g_item_b_block(P, it_bb[P.n_bb - 1 - q], S.block);
    }
    __syncthreads();  // the work-group table is no longer read; the wave tables reuse it
    for (;;) {
        int64_t base = 0;
        if (lane == 0) base = (int64_t)atomicAdd(&P.qctr[2], (unsigned long long)GGROUP);
        base = bcast_i64(base, 0);
        if (base >= P.n_aw) break;
        const int64_t end = base + GGROUP < P.n_aw ? base + GGROUP : P.n_aw;
        for (int64_t q = base; q < end; q++)
            g_item_a_wave(P, (int32_t)it_aw[P.n_aw - 1 - q], S.wave[wib]);
    }
    for (;;) {
        int64_t base = 0;
        if (lane == 0) base = (int64_t)atomicAdd(&P.qctr[3], (unsigned long long)GGROUP);
        base = bcast_i64(base, 0);
        if (base >= P.n_bw) break;
        const int64_t end = base + GGROUP < P.n_bw ? base + GGROUP : P.n_bw;
        for (int64_t q = base; q < end; q++) g_item_b_wave(P, it_bw[P.n_bw - 1 - q], S.wave[wib]);
    }
}

// Per vertex x (L = |O(x)|, D = deg x): pass-A items (one wave item for 2 <= L <= CAP,
// else ceil(L / CAPH) work-group chunks), pass-B items (ceil(D / SPAN) ranges when x has
// an out- and an in-neighbour, times the chunks for L > CAP) and the slice sizes.
__global__ void k_g_counts(const int64_t* __restrict__ o_off, const int64_t* __restrict__ s_off,
                           int64_t n, int32_t* __restrict__ c_aw, int32_t* __restrict__ c_ab,
                           int32_t* __restrict__ c_bw, int32_t* __restrict__ c_bb,
                           int64_t* __restrict__ sz_a, int64_t* __restrict__ sz_b) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int64_t L = o_off[x + 1] - o_off[x];
    const int64_t D = s_off[x + 1] - s_off[x];
    const int64_t nch = L > GCAP ? (L + GCAPH - 1) / GCAPH : 1;
    const int64_t nr = (L >= 1 && D > L) ? (D + GSPAN - 1) / GSPAN : 0;
    c_aw[x] = (L >= 2 && L <= GCAP) ? 1 : 0;
    c_ab[x] = L > GCAP ? (int32_t)nch : 0;
    c_bw[x] = L <= GCAP ? (int32_t)nr : 0;
    c_bb[x] = L > GCAP ? (int32_t)(nr * nch) : 0;
    sz_a[x] = L >= 2 ? nch * L : 0;
    sz_b[x] = nr * L;
}

__global__ void k_g_items(const int64_t* __restrict__ o_off, const int32_t* __restrict__ c_aw,
                          const int32_t* __restrict__ c_ab, const int32_t* __restrict__ c_bw,
                          const int32_t* __restrict__ c_bb, const int64_t* __restrict__ f_aw,
                          const int64_t* __restrict__ f_ab, const int64_t* __restrict__ f_bw,
                          const int64_t* __restrict__ f_bb, int64_t n, int64_t b_ab,
                          int64_t b_bw, int64_t b_bb, int64_t* __restrict__ items) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    if (c_aw[x]) items[f_aw[x]] = x;
    for (int c = 0; c < c_ab[x]; c++) items[b_ab + f_ab[x] + c] = x | ((int64_t)c << 32);
    for (int r = 0; r < c_bw[x]; r++) items[b_bw + f_bw[x] + r] = x | ((int64_t)r << RANGE_SHIFT);
    if (c_bb[x]) {
        const int64_t L = o_off[x + 1] - o_off[x];
        const int nch = (int)((L + GCAPH - 1) / GCAPH);
        const int nr = c_bb[x] / nch;
        int64_t o = b_bb + f_bb[x];
        for (int r = 0; r < nr; r++)
            for (int c = 0; c < nch; c++)
                items[o++] = x | ((int64_t)r << RANGE_SHIFT) | ((int64_t)c << CHUNK_SHIFT);
    }
}

// One wave per vertex x: add the pass-A and pass-B slices of every entry of O(x) and
// store the rounded value at the entry's edge id.
__global__ void __launch_bounds__(TPB) k_g_final(GradParams P) {
    const int64_t x = (int64_t)blockIdx.x * WPB + threadIdx.x / UTRI_WAVE;
    if (x >= P.n) return;
    const int64_t ox = P.o_off[x];
    const int L = (int)(P.o_off[x + 1] - ox);
    if (L == 0) return;
    const int64_t a0 = P.pa_off[x], b0 = P.pb_off[x];
    const int na = (int)((P.pa_off[x + 1] - a0) / L);
    const int nr = (int)((P.pb_off[x + 1] - b0) / L);
    for (int q = utri_lane(); q < L; q += UTRI_WAVE) {
        uint64_t l = 0, h = 0;
        for (int c = 0; c < na; c++) {
            const ulonglong2 t = P.pa[a0 + (int64_t)c * L + q];
            l += t.x;
            h += t.y;
        }
        for (int r = 0; r < nr; r++) {
            const ulonglong2 t = P.pb[b0 + (int64_t)r * L + q];
            l += t.x;
            h += t.y;
        }
        // value = h * 2^32 + l as a 128-bit two's complement number
        uint64_t lo = h << 32;
        uint64_t hi = (uint64_t)((int64_t)h >> 32);
        const uint64_t s2 = lo + l;
        hi += (s2 < lo) ? 1ull : 0ull;
        lo = s2;
        P.grad[P.o_eid[ox + q]] = utri_i128_to_double((int64_t)hi, lo) * 0x1p-62;
    }
}

template <class K>
int grad_blocks_per_cu(utri_graph* g, K kernel) {
    if (g->walk_blocks_per_cu > 0) return g->walk_blocks_per_cu;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, TPB, 0) != hipSuccess || nb < 1)
        nb = 4;
    return nb;
}

inline unsigned nblocks(int64_t count) { return (unsigned)((count + TPB - 1) / TPB); }

}  // namespace

int utri_grad_launch(utri_graph* g, double* grad, hipStream_t s) {
    if (g->m == 0) return UTRI_OK;
    const int64_t n = g->n;
    void *pc, *po, *pz, *pq;
    UTRI_TRY(utri_scratch(g, SCR_GCNT, sizeof(int32_t) * (size_t)(4 * n), &pc));
    UTRI_TRY(utri_scratch(g, SCR_GOFF, sizeof(int64_t) * (size_t)(6 * n + 2), &po));
    UTRI_TRY(utri_scratch(g, SCR_GSZ, sizeof(int64_t) * (size_t)(2 * n), &pz));
    UTRI_TRY(utri_scratch(g, SCR_GQ, sizeof(int64_t) * 16, &pq));
    int32_t* c_aw = (int32_t*)pc;
    int32_t* c_ab = c_aw + n;
    int32_t* c_bw = c_ab + n;
    int32_t* c_bb = c_bw + n;
    int64_t* f_aw = (int64_t*)po;
    int64_t* f_ab = f_aw + n;
    int64_t* f_bw = f_ab + n;
    int64_t* f_bb = f_bw + n;
    int64_t* pa_off = f_bb + n;        // n + 1
    int64_t* pb_off = pa_off + n + 1;  // n + 1
    int64_t* sz_a = (int64_t*)pz;
    int64_t* sz_b = sz_a + n;
    int64_t* tot = (int64_t*)pq;       // [0, 4): item counts
    unsigned long long* qctr = (unsigned long long*)(tot + 8);
    hipLaunchKernelGGL(k_g_counts, dim3(nblocks(n)), dim3(TPB), 0, s, g->o_off, g->s_off, n, c_aw,
                       c_ab, c_bw, c_bb, sz_a, sz_b);
    UTRI_HIP_TRY(hipGetLastError());
    UTRI_TRY(utri_scan_i32(g, c_aw, f_aw, n, tot + 0, s));
    UTRI_TRY(utri_scan_i32(g, c_ab, f_ab, n, tot + 1, s));
    UTRI_TRY(utri_scan_i32(g, c_bw, f_bw, n, tot + 2, s));
    UTRI_TRY(utri_scan_i32(g, c_bb, f_bb, n, tot + 3, s));
    UTRI_TRY(utri_scan_i64(g, sz_a, pa_off, n, pa_off + n, s));
    UTRI_TRY(utri_scan_i64(g, sz_b, pb_off, n, pb_off + n, s));
    // item counts and slice totals depend on the degrees only: read them once per graph
    if (g->grad_sizes[0] < 0) {
        int64_t h[6];
        UTRI_HIP_TRY(hipMemcpyAsync(h, tot, sizeof(int64_t) * 4, hipMemcpyDeviceToHost, s));
        UTRI_HIP_TRY(hipMemcpyAsync(h + 4, pa_off + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        UTRI_HIP_TRY(hipMemcpyAsync(h + 5, pb_off + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        UTRI_HIP_TRY(hipStreamSynchronize(s));
        for (int i = 0; i < 6; i++) g->grad_sizes[i] = h[i];
    }
    const int64_t* gs = g->grad_sizes;
    const int64_t n_items = gs[0] + gs[1] + gs[2] + gs[3];
    void *pi, *pp;
    UTRI_TRY(utri_scratch(g, SCR_GITEMS, sizeof(int64_t) * (size_t)(n_items + 1), &pi));
    UTRI_TRY(utri_scratch(g, SCR_GPART, sizeof(ulonglong2) * (size_t)(gs[4] + gs[5] + 1), &pp));
    hipLaunchKernelGGL(k_g_items, dim3(nblocks(n)), dim3(TPB), 0, s, g->o_off, (const int32_t*)c_aw,
                       (const int32_t*)c_ab, (const int32_t*)c_bw, (const int32_t*)c_bb,
                       (const int64_t*)f_aw, (const int64_t*)f_ab, (const int64_t*)f_bw,
                       (const int64_t*)f_bb, n, gs[0], gs[0] + gs[1], gs[0] + gs[1] + gs[2],
                       (int64_t*)pi);
    UTRI_HIP_TRY(hipGetLastError());
    UTRI_TRY(utri_fill_u64(qctr, 0, 4, s));
    GradParams P;
    P.o_off = g->o_off;
    P.o_adj = g->o_adj;
    P.o_d = g->o_d;
    P.o_eid = g->o_eid;
    P.s_off = g->s_off;
    P.s_adj = g->s_adj;
    P.s_d = g->s_d;
    P.idmask = g->idmask;
    P.pa_off = pa_off;
    P.pb_off = pb_off;
    P.pa = (ulonglong2*)pp;
    P.pb = (ulonglong2*)pp + gs[4];
    P.items = (const int64_t*)pi;
    P.n_aw = gs[0];
    P.n_ab = gs[1];
    P.n_bw = gs[2];
    P.n_bb = gs[3];
    P.qctr = qctr;
    P.grad = grad;
    P.n = n;
    const int blocks = g->num_cu * grad_blocks_per_cu(g, k_grad2);
    hipLaunchKernelGGL(k_grad2, dim3(blocks), dim3(TPB), 0, s, P);
    UTRI_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_g_final, dim3((unsigned)((n + WPB - 1) / WPB)), dim3(TPB), 0, s, P);
    UTRI_HIP_TRY(hipGetLastError());
    return UTRI_OK;
}
