// backward.hip -- per-edge gradient of the expected balanced count.
//
// E = sum over triangles of P_bal = (1 - d_e d_f d_g)/2 (Section 3 four-term sum in
// product form, d = 1 - 2 P+). With dd_e/dp_e = -2, dE/dp_e = sum over the triangles
// (e, f, g) through e of d_f * d_g.
//
// Edge-centric re-walk grouped by owner. Edge (x, y) with x < y in Node Order (so
// deg x <= deg y) is owned by y: its triangles are the w of N(x) that are also in N(y),
// found by streaming N(x) (cost deg x = min(deg x, deg y)) and probing a table of N(y).
// The owner's row is prepared once for many of its edges:
//   * deg y <= CAPW: an exact LDS hash table of one wave (one item per owner);
//   * deg y <= CAPB: an exact LDS hash table of one work-group, its waves splitting the
//     owner's edges;
//   * hubs: the row does not fit in LDS. Each work-group item (a range of the hub's row
//     positions) builds a blocked Bloom filter of N(y) in LDS; streamed entries that pass
//     it (the hits and a few percent of false positives) are confirmed 64 at a time in
//     the row's global hash table. Hub items are queued per XCD (work-group index mod 8,
//     the hardware's round-robin placement), so the one or two hubs an XCD works through
//     at a time keep their tables in its L2.
// Each product d_xw * d_yw is rounded to FP64 and added exactly in 2^-62 fixed point in
// lane registers, reduced over the wave once per edge and rounded once: the result does
// not depend on which lane found which triangle. Every edge has one writer and no
// atomics touch the result.
#include <algorithm>

#include "walk_common.h"

using namespace utri_dev;

namespace {

#ifndef UTRI_GRAD_CAPW
#define UTRI_GRAD_CAPW 256
#endif
#ifndef UTRI_GRAD_CAPB
#define UTRI_GRAD_CAPB 2048
#endif
#ifndef UTRI_GRAD_FILTER_WORDS
#define UTRI_GRAD_FILTER_WORDS 5632
#endif
constexpr int GCAPW = UTRI_GRAD_CAPW;  // longest owner row staged by one wave
constexpr int GCAPB = UTRI_GRAD_CAPB;  // longest owner row staged by one work-group
constexpr int GFW = UTRI_GRAD_FILTER_WORDS;  // 32-bit words of a hub row's LDS filter
#ifndef UTRI_GRAD_HUB_SPAN
#define UTRI_GRAD_HUB_SPAN 128
#endif
// Row positions per hub item (a multiple of 64). Small items put every work-group of an
// XCD on the same one or two hubs, so their global tables stay in that XCD's L2; the
// filter is rebuilt per item (a few microseconds against ~100 strips of work).
constexpr int GSPAN = UTRI_GRAD_HUB_SPAN;
static_assert(GSPAN % UTRI_WAVE == 0, "hub items cover whole 64-position chunks");
constexpr int NXCD = 8;                // hub work queues (one per XCD)
constexpr int GGROUP = 4;              // wave owners taken per queue grab
constexpr int GQCAP = 2 * UTRI_WAVE;   // filter-passing entries a wave holds back
static_assert(GCAPW <= GCAPB && GCAPB <= 32768, "LDS row positions are 16-bit");

struct GWaveLds {
    int32_t key[2 * GCAPW];
    uint16_t pos[2 * GCAPW];
};
struct GBlockLds {
    int32_t key[2 * GCAPB];
    uint16_t pos[2 * GCAPB];
};
// Entries of a streamed row that passed a hub filter, waiting to be confirmed 64 at a
// time in the hub's global table (so the global probes run on full waves).
struct GQueue {
    int32_t w[GQCAP];  // vertex id
    int32_t j[GQCAP];  // position in the streamed row
};
struct GHubLds {
    uint32_t filt[GFW];
    GQueue q[WPB];
};
union GShared {
    GWaveLds wave[WPB];
    GBlockLds block;
    GHubLds hub;
};

struct GradParams {
    const int64_t* s_off;
    const int32_t* s_adj;
    const double* s_d;
    const int32_t* s_eid;
    const int64_t* h_off;      // symmetric-row hash tables (slot = id << 32 | position)
    const uint64_t* h_slot;
    double* grad;
    const int64_t* items;      // [0, n) wave owners, [n, 2n) work-group owners, [2n, ...) hub items
    const int64_t* cnt;        // device: # wave owners, # work-group owners, # hub items
    unsigned long long* qctr;  // [0] work-group owners, [1, 9) hub queues, [9] wave owners
    int64_t n;
};

struct LdsTab {
    const int32_t* key;
    const uint16_t* pos;
    int lg;
    uint32_t mask;
};
struct HubTab {
    const uint64_t* slot;  // the row's global table, ~0 = empty slot
    int lg;
    uint32_t mask;
    const uint32_t* filt;  // LDS blocked Bloom filter of the row
    GQueue* q;             // the wave's queue of filter-passing entries
};

// Filter word and the two bits of id w (both bits in one word: one LDS read per test).
struct FilterKey {
    uint32_t word, bits;
};
__device__ __forceinline__ FilterKey filter_key(int32_t w) {
    const uint32_t x = (uint32_t)w * 0x9E3779B1u;
    const uint32_t y = (x ^ (x >> 15)) * 0x2C1B3C6Du;
    return {__umulhi(x, (uint32_t)GFW), (1u << (y >> 27)) | (1u << ((y >> 22) & 31u))};
}

__device__ __forceinline__ void acc_term(uint64_t& slo, int64_t& shi, double a, double b) {
    const int64_t t = utri_fix62(__dmul_rn(a, b));
    slo += (uint64_t)(uint32_t)(t & 0xFFFFFFFFll);
    shi += t >> 32;
}

// Reduce the lanes' fixed-point partial sums of one edge and store the rounded value.
__device__ __forceinline__ void grad_store(double* __restrict__ grad, int32_t eid, uint64_t slo,
                                           int64_t shi) {
    const uint64_t l = utri_wave_sum_u64(slo);
    const int64_t h = (int64_t)utri_wave_sum_u64((uint64_t)shi);
    if (utri_lane() == 0) {
        // value = h * 2^32 + l as a 128-bit two's complement number
        uint64_t lo = (uint64_t)h << 32;
        uint64_t hi = (uint64_t)(h >> 32);
        const uint64_t s2 = lo + l;
        hi += (s2 < lo) ? 1ull : 0ull;
        lo = s2;
        grad[eid] = utri_i128_to_double((int64_t)hi, lo) * 0x1p-62;
    }
}

// Stream N(x) = s_adj[xoff, xoff + lx) and add d_xw * d_yw for every w found in the
// owner's LDS table. Lanes past the row end re-load its last entry and drop the result;
// all UNR loads are issued before any probe.
template <int UNR>
__device__ __forceinline__ void grad_row(const GradParams& P, const LdsTab& LT,
                                         const double* __restrict__ yd, int64_t xoff, int lx,
                                         uint64_t& slo, int64_t& shi) {
    const int lane = utri_lane();
    const int32_t* rowp = P.s_adj + xoff;
    const double* rowd = P.s_d + xoff;
    for (int j0 = 0; j0 < lx; j0 += UNR * UTRI_WAVE) {
        int32_t w[UNR];
#pragma unroll
        for (int k = 0; k < UNR; k++) w[k] = rowp[min(j0 + k * UTRI_WAVE + lane, lx - 1)];
#pragma unroll
        for (int k = 0; k < UNR; k++) {
            const int j = j0 + k * UTRI_WAVE + lane;
            uint32_t h = utri_hash32(w[k], LT.lg);
            int kk = LT.key[h];
            while (kk != -1 && kk != w[k]) {
                h = (h + 1) & LT.mask;
                kk = LT.key[h];
            }
            if (j < lx && kk != -1) acc_term(slo, shi, rowd[j], yd[LT.pos[h]]);
        }
    }
}

// Confirm queue entries [base, base + cnt) (cnt <= 64, one per lane) in the hub's global
// table and add the products of the hits.
__device__ __forceinline__ void hub_confirm(const HubTab& HT, const double* __restrict__ rowd,
                                            const double* __restrict__ yd, int base, int cnt,
                                            uint64_t& slo, int64_t& shi) {
    const int lane = utri_lane();
    if (lane < cnt) {
        const int32_t w = HT.q->w[base + lane];
        const int j = HT.q->j[base + lane];
        uint32_t h = utri_hash32(w, HT.lg);
        uint64_t sl = HT.slot[h];
        while (sl != ~0ull && (int32_t)(sl >> 32) != w) {
            h = (h + 1) & HT.mask;
            sl = HT.slot[h];
        }
        if (sl != ~0ull) acc_term(slo, shi, rowd[j], yd[(uint32_t)(sl & 0xFFFFFFFFull)]);
    }
    utri_wave_sync();  // the entries are read before later ones overwrite them
}

// Hub variant: entries that pass the LDS filter are appended to the wave's queue, and
// every full 64 of them are confirmed together; the rest at the end of the row.
template <int UNR>
__device__ __forceinline__ void grad_row_hub(const GradParams& P, const HubTab& HT,
                                             const double* __restrict__ yd, int64_t xoff, int lx,
                                             uint64_t& slo, int64_t& shi) {
    const int lane = utri_lane();
    const int32_t* rowp = P.s_adj + xoff;
    const double* rowd = P.s_d + xoff;
    const uint64_t lt = __lanemask_lt();
    int qn = 0;  // queued entries (wave-uniform, < 64 between strips)
    for (int j0 = 0; j0 < lx; j0 += UNR * UTRI_WAVE) {
        int32_t w[UNR];
#pragma unroll
        for (int k = 0; k < UNR; k++) w[k] = rowp[min(j0 + k * UTRI_WAVE + lane, lx - 1)];
#pragma unroll
        for (int k = 0; k < UNR; k++) {
            const int j = j0 + k * UTRI_WAVE + lane;
            const FilterKey fk = filter_key(w[k]);
            const bool pass = (j < lx) && (HT.filt[fk.word] & fk.bits) == fk.bits;
            const uint64_t M = __ballot(pass);
            if (pass) {
                const int r = qn + __popcll(M & lt);
                HT.q->w[r] = w[k];
                HT.q->j[r] = j;
            }
            qn += __popcll(M);
            utri_wave_sync();
            if (qn >= UTRI_WAVE) {
                qn -= UTRI_WAVE;
                hub_confirm(HT, rowd, yd, qn, UTRI_WAVE, slo, shi);
            }
        }
    }
    if (qn > 0) hub_confirm(HT, rowd, yd, 0, qn, slo, shi);
}

template <bool HUB>
__device__ __forceinline__ void grad_row_any(const GradParams& P, const LdsTab& LT,
                                             const HubTab& HT, const double* __restrict__ yd,
                                             int64_t xoff, int lx, uint64_t& slo, int64_t& shi) {
    if (HUB) {
        if (lx > 2 * UTRI_WAVE) grad_row_hub<4>(P, HT, yd, xoff, lx, slo, shi);
        else if (lx > UTRI_WAVE) grad_row_hub<2>(P, HT, yd, xoff, lx, slo, shi);
        else grad_row_hub<1>(P, HT, yd, xoff, lx, slo, shi);
    } else {
        if (lx > 2 * UTRI_WAVE) grad_row<4>(P, LT, yd, xoff, lx, slo, shi);
        else if (lx > UTRI_WAVE) grad_row<2>(P, LT, yd, xoff, lx, slo, shi);
        else grad_row<1>(P, LT, yd, xoff, lx, slo, shi);
    }
}

// Positions [p0, p0 + 64) of the owner row N(y): every x < y there is an owned edge.
// The wave takes the owned edges whose rank in the chunk is `part` mod `nparts`.
template <bool HUB>
__device__ __forceinline__ void owner_chunk(const GradParams& P, int32_t y, int64_t yoff, int D,
                                            int p0, const LdsTab& LT, const HubTab& HT, int part,
                                            int nparts) {
    const int p = p0 + utri_lane();
    int32_t x = 0, eid = 0;
    int64_t xoff = 0;
    int lx = 0;
    bool owned = false;
    if (p < D) {
        x = P.s_adj[yoff + p];
        owned = x < y;
    }
    if (owned) {
        xoff = P.s_off[x];
        lx = (int)(P.s_off[x + 1] - xoff);
        eid = P.s_eid[yoff + p];
    }
    uint64_t mask = __ballot(owned);
    const double* yd = P.s_d + yoff;
    for (int r = 0; mask; r++) {
        const int si = __builtin_ctzll(mask);
        mask &= mask - 1;
        if (r % nparts != part) continue;
        uint64_t slo = 0;
        int64_t shi = 0;
        grad_row_any<HUB>(P, LT, HT, yd, bcast_i64(xoff, si), bcast_i32(lx, si), slo, shi);
        grad_store(P.grad, bcast_i32(eid, si), slo, shi);
    }
}

__device__ __forceinline__ int grad_table_lg(int cl) {
    int lg = 1;
    while ((1 << lg) < 2 * cl) lg++;
    return lg;
}

// Insert row positions [0, D) of `row` into a 2^lg-slot LDS table; `tid` / `nthreads`
// are the caller's lanes (one wave or one work-group).
__device__ __forceinline__ void grad_stage(const int32_t* __restrict__ row, int D, int32_t* key,
                                           uint16_t* pos, int lg, int tid, int nthreads) {
    const uint32_t mask = (1u << lg) - 1u;
    for (int j = tid; j < D; j += nthreads) {
        const int32_t w = row[j];
        uint32_t h = utri_hash32(w, lg);
        for (;;) {
            const int old = atomicCAS(&key[h], -1, w);
            if (old == -1) { pos[h] = (uint16_t)j; break; }
            h = (h + 1) & mask;
        }
    }
}

__device__ void grad_wave_owner(const GradParams& P, int32_t y, GWaveLds& L) {
    const int lane = utri_lane();
    const int64_t yoff = P.s_off[y];
    const int D = (int)(P.s_off[y + 1] - yoff);
    const int lg = grad_table_lg(D);
    const int size = 1 << lg;
    for (int i = lane; i < size; i += UTRI_WAVE) L.key[i] = -1;
    utri_wave_sync();
    grad_stage(P.s_adj + yoff, D, L.key, L.pos, lg, lane, UTRI_WAVE);
    utri_wave_sync();
    const LdsTab T{L.key, L.pos, lg, (uint32_t)(size - 1)};
    for (int p0 = 0; p0 < D; p0 += UTRI_WAVE) owner_chunk<false>(P, y, yoff, D, p0, T, HubTab{}, 0, 1);
    utri_wave_sync();  // probes done before the next owner clears the table
}

__device__ void grad_block_owner(const GradParams& P, int32_t y, GBlockLds& B) {
    const int wib = threadIdx.x / UTRI_WAVE;
    const int64_t yoff = P.s_off[y];
    const int D = (int)(P.s_off[y + 1] - yoff);
    const int lg = grad_table_lg(D);
    const int size = 1 << lg;
    __syncthreads();  // the previous owner's probes are done
    for (int i = threadIdx.x; i < size; i += TPB) B.key[i] = -1;
    __syncthreads();
    grad_stage(P.s_adj + yoff, D, B.key, B.pos, lg, threadIdx.x, TPB);
    __syncthreads();
    const LdsTab T{B.key, B.pos, lg, (uint32_t)(size - 1)};
    for (int p0 = 0; p0 < D; p0 += UTRI_WAVE)
        owner_chunk<false>(P, y, yoff, D, p0, T, HubTab{}, wib, WPB);
}

// Work-group item of a hub row: positions [chunk * GSPAN, chunk * GSPAN + GSPAN) of N(y).
// The filter of N(y) is rebuilt only when the work-group moves to another hub.
__device__ void grad_hub_item(const GradParams& P, int64_t item, GHubLds& HL, int32_t& cur) {
    const int wib = threadIdx.x / UTRI_WAVE;
    const int32_t y = (int32_t)(item & 0xFFFFFFFF);
    const int chunk = (int)(item >> 32);
    const int64_t yoff = P.s_off[y];
    const int D = (int)(P.s_off[y + 1] - yoff);
    if (y != cur) {
        __syncthreads();  // the previous hub's probes are done
        for (int i = threadIdx.x; i < GFW; i += TPB) HL.filt[i] = 0u;
        __syncthreads();
        for (int j = threadIdx.x; j < D; j += TPB) {
            const FilterKey fk = filter_key(P.s_adj[yoff + j]);
            atomicOr(&HL.filt[fk.word], fk.bits);
        }
        __syncthreads();
        cur = y;
    }
    const int64_t hoff = P.h_off[y];
    const int64_t size = P.h_off[y + 1] - hoff;  // a power of two
    const int lg = 63 - __builtin_clzll((unsigned long long)size);
    const HubTab T{P.h_slot + hoff, lg, (uint32_t)(size - 1), HL.filt, &HL.q[wib]};
    const int pb = chunk * GSPAN;
    const int pe = min(D, pb + GSPAN);
    for (int p0 = pb; p0 < pe; p0 += UTRI_WAVE)
        owner_chunk<true>(P, y, yoff, pe, p0, LdsTab{}, T, wib, WPB);
}

// Persistent grid, three phases per work-group, each fed by atomic work queues:
// work-group owners (longest rows first), hub items (own XCD's queue, then the others'),
// wave owners (longest rows first, GGROUP per grab).
__global__ void __launch_bounds__(TPB) k_grad(GradParams P) {
    __shared__ GShared S;
    __shared__ int64_t s_q;
    const int wib = threadIdx.x / UTRI_WAVE;
    const int lane = utri_lane();
    const int64_t nw = P.cnt[0], nb = P.cnt[1], nh = P.cnt[2];
    for (;;) {
        if (threadIdx.x == 0) s_q = (int64_t)atomicAdd(&P.qctr[0], 1ull);
        __syncthreads();
        const int64_t q = s_q;
        __syncthreads();
        if (q >= nb) break;
        grad_block_owner(P, (int32_t)P.items[P.n + nb - 1 - q], S.block);
    }
    const int xcd = (int)(blockIdx.x % NXCD);
    int32_t cur = -1;  // hub whose filter is in LDS (the union was just used by tables)
    for (int qq = 0; qq < NXCD; qq++) {
        const int q = (xcd + qq) % NXCD;
        const int64_t a = nh * q / NXCD, b = nh * (q + 1) / NXCD;
        for (;;) {
            if (threadIdx.x == 0) s_q = (int64_t)atomicAdd(&P.qctr[1 + q], 1ull);
            __syncthreads();
            const int64_t t = s_q;
            __syncthreads();
            if (a + t >= b) break;
            grad_hub_item(P, P.items[2 * P.n + (nh - 1 - (a + t))], S.hub, cur);  // largest first
        }
    }
    __syncthreads();  // the filter is no longer read; the wave tables reuse its memory
    for (;;) {
        int64_t base = 0;
        if (lane == 0) base = (int64_t)atomicAdd(&P.qctr[1 + NXCD], (unsigned long long)GGROUP);
        base = bcast_i64(base, 0);
        if (base >= nw) break;
        const int64_t end = base + GGROUP < nw ? base + GGROUP : nw;
        for (int64_t q = base; q < end; q++)
            grad_wave_owner(P, (int32_t)P.items[nw - 1 - q], S.wave[wib]);
    }
}

// Owner class of every vertex: wave (1 <= deg <= CAPW), work-group (deg <= CAPB), or
// hub with ceil(deg / GSPAN) items.
__global__ void k_grad_rows(const int64_t* __restrict__ s_off, int64_t n, int32_t* __restrict__ wcnt,
                            int32_t* __restrict__ bcnt, int32_t* __restrict__ hcnt) {
    const int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= n) return;
    const int64_t D = s_off[y + 1] - s_off[y];
    wcnt[y] = (D >= 1 && D <= GCAPW) ? 1 : 0;
    bcnt[y] = (D > GCAPW && D <= GCAPB) ? 1 : 0;
    hcnt[y] = D > GCAPB ? (int32_t)((D + GSPAN - 1) / GSPAN) : 0;
}

__global__ void k_grad_items(const int32_t* __restrict__ wcnt, const int32_t* __restrict__ bcnt,
                             const int32_t* __restrict__ hcnt, const int64_t* __restrict__ woff,
                             const int64_t* __restrict__ boff, const int64_t* __restrict__ hoff,
                             int64_t n, int64_t* __restrict__ items) {
    const int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= n) return;
    if (wcnt[y]) items[woff[y]] = y;
    if (bcnt[y]) items[n + boff[y]] = y;
    const int c = hcnt[y];
    const int64_t o = 2 * n + hoff[y];
    for (int k = 0; k < c; k++) items[o + k] = ((int64_t)k << 32) | y;
}

template <class K>
int grad_blocks_per_cu(utri_graph* g, K kernel) {
    if (g->walk_blocks_per_cu > 0) return g->walk_blocks_per_cu;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, TPB, 0) != hipSuccess || nb < 1)
        nb = 4;
    return nb;
}

}  // namespace

int utri_grad_launch(utri_graph* g, double* grad, hipStream_t s) {
    if (g->m == 0) return UTRI_OK;
    const int64_t n = g->n;
    // hub items: ceil(deg / GSPAN) for each of the (< 2m / CAPB) hub rows
    const int64_t hb = 2 * g->m / GSPAN + 2 * g->m / GCAPB + 2;
    void *pc, *po, *pi, *pq;
    UTRI_TRY(utri_scratch(g, SCR_GCNT, sizeof(int32_t) * (size_t)(3 * n), &pc));
    UTRI_TRY(utri_scratch(g, SCR_GOFF, sizeof(int64_t) * (size_t)(3 * n), &po));
    UTRI_TRY(utri_scratch(g, SCR_GITEMS, sizeof(int64_t) * (size_t)(2 * n + hb), &pi));
    UTRI_TRY(utri_scratch(g, SCR_GQ, sizeof(int64_t) * 16, &pq));
    UTRI_TRY(utri_fill_u64(pq, 0, 16, s));
    int32_t* wcnt = (int32_t*)pc;
    int32_t* bcnt = wcnt + n;
    int32_t* hcnt = bcnt + n;
    int64_t* woff = (int64_t*)po;
    int64_t* boff = woff + n;
    int64_t* hoff = boff + n;
    int64_t* cnt = (int64_t*)pq;
    const int nblk = (int)((n + TPB - 1) / TPB);
    hipLaunchKernelGGL(k_grad_rows, dim3(nblk), dim3(TPB), 0, s, g->s_off, n, wcnt, bcnt, hcnt);
    UTRI_HIP_TRY(hipGetLastError());
    UTRI_TRY(utri_scan_i32(g, wcnt, woff, n, cnt, s));
    UTRI_TRY(utri_scan_i32(g, bcnt, boff, n, cnt + 1, s));
    UTRI_TRY(utri_scan_i32(g, hcnt, hoff, n, cnt + 2, s));
    hipLaunchKernelGGL(k_grad_items, dim3(nblk), dim3(TPB), 0, s, (const int32_t*)wcnt,
                       (const int32_t*)bcnt, (const int32_t*)hcnt, (const int64_t*)woff,
                       (const int64_t*)boff, (const int64_t*)hoff, n, (int64_t*)pi);
    UTRI_HIP_TRY(hipGetLastError());
    GradParams P;
    P.s_off = g->s_off;
    P.s_adj = g->s_adj;
    P.s_d = g->s_d;
    P.s_eid = g->s_eid;
    P.h_off = g->h_off;
    P.h_slot = g->h_slot;
    P.grad = grad;
    P.items = (const int64_t*)pi;
    P.cnt = cnt;
    P.qctr = (unsigned long long*)(cnt + 4);
    P.n = n;
    const int blocks = g->num_cu * grad_blocks_per_cu(g, k_grad);
    hipLaunchKernelGGL(k_grad, dim3(blocks), dim3(TPB), 0, s, P);
    UTRI_HIP_TRY(hipGetLastError());
    return UTRI_OK;
}
