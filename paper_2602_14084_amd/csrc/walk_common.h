// walk_common.h -- the LDS bucket tables (hash, staging, probe) shared by the walk and the
// gradient passes, per-wave LDS layouts, and the edge-sampling work unit shared by the
// sampler kernels and the fused batch kernel.
#pragma once

#include "utri_internal.h"

namespace utri_dev {

constexpr int TPB = 256;
constexpr int WPB = TPB / UTRI_WAVE;
#ifndef UTRI_WALK_CAP
#define UTRI_WALK_CAP 128
#endif
#ifndef UTRI_WALK_SLOTS
#define UTRI_WALK_SLOTS 8
#endif
constexpr int CAP = UTRI_WALK_CAP;  // longest source row staged by one wave
constexpr int SLOTS = UTRI_WALK_SLOTS;  // wave-table slots per staged entry (load factor 1/SLOTS)
constexpr int HS = SLOTS * CAP;     // LDS table slots, in buckets of 4
// a table for cl <= CAP entries has the least power-of-two bucket count with 4 * buckets
// >= SLOTS * cl (at least 2 buckets): with powers of two that is at most HS slots
static_assert((CAP & (CAP - 1)) == 0 && (SLOTS & (SLOTS - 1)) == 0 && SLOTS * CAP >= 8,
              "table sizes are powers of two");
constexpr int NB = 65;         // histogram bins (nt + 1 <= 65)

// Bucket of w in a table of 2^lg buckets (lg >= 1): its low bits. Vertex ids are ranks in
// (degree, mixed id) order, so within a degree class they follow no input pattern, and the
// few vertices of distinct high degrees have consecutive ids, which land in distinct
// buckets; a multiplicative hash would cost two more instructions per probe.
__device__ __forceinline__ uint32_t walk_hash(int32_t w, int lg) {
    return (uint32_t)w & ((1u << lg) - 1u);
}

// Stage `cl` source entries starting at o_adj[base] into an open-addressing table of
// 2^lg buckets of 4 slots; `tid` / `nthreads` are the caller's lanes (one wave or one
// work-group). Each entry takes the first free slot of the first bucket (from its home
// bucket on) that has one; slots are claimed in order, so a bucket's slots fill in order.
__device__ __forceinline__ void stage_table(const int32_t* __restrict__ o_adj, int64_t base, int cl,
                                            int32_t* key, uint16_t* pos, int lg, int tid,
                                            int nthreads, uint32_t idmask) {
    const uint32_t mask = (1u << lg) - 1u;
    for (int j = tid; j < cl; j += nthreads) {
        // the key is the packed word (id and d code); its id is at least 1, so it is
        // never 0, the empty marker and the probe's not-found value
        const int32_t pw = o_adj[base + j];
        uint32_t b = walk_hash((int32_t)((uint32_t)pw & idmask), lg);
        for (;;) {
            int s = 0;
            while (s < 4 && atomicCAS(&key[4 * b + s], 0, pw) != 0) s++;
            if (s < 4) { pos[4 * b + s] = (uint16_t)j; break; }
            b = (b + 1) & mask;
        }
    }
}

// log2 of the bucket count of a table for cl entries: 4 * 2^lg >= slots * cl, 2^lg >= 2
__device__ __forceinline__ int table_lg(int cl, int slots) {
    int lg = 1;
    while ((4 << lg) < slots * cl) lg++;
    return lg;
}

// Find packed key with id w in a table of 2^lg buckets of 4 slots (mask = 2^lg - 1):
// linear probe over buckets until the key or a bucket with an empty slot. Empty slots hold
// 0, whose id part (vertex 0, the lowest rank) is in no oriented row, so it never matches
// w; slots of a bucket fill in order, so its last slot tells whether the bucket is full.
// Returns the key (0 if absent) and its slot in h.
__device__ __forceinline__ int bucket_find(const int32_t* key, int lg, uint32_t mask, uint32_t w,
                                           uint32_t idmask, int& h) {
    uint32_t b = walk_hash((int32_t)w, lg);
    int kk;
    for (;;) {
        const int4 kv = *reinterpret_cast<const int4*>(key + 4 * b);
        const bool f0 = ((uint32_t)kv.x & idmask) == w;
        const bool f1 = ((uint32_t)kv.y & idmask) == w;
        const bool f2 = ((uint32_t)kv.z & idmask) == w;
        const bool f3 = ((uint32_t)kv.w & idmask) == w;
        kk = f0 ? kv.x : f1 ? kv.y : f2 ? kv.z : f3 ? kv.w : 0;
        h = 4 * (int)b + (f0 ? 0 : f1 ? 1 : f2 ? 2 : 3);
        // keep the results in registers here: otherwise the compiler carries the four
        // match flags out of the loop as scalar lane masks
        asm volatile("" : "+v"(kk), "+v"(h));
        if (kk != 0 || kv.w == 0) break;
        b = (b + 1) & mask;
    }
    return kk;
}

// LDS of one wave of the walk: the staged source chunk as an open-addressing table of
// 4-slot buckets (one 16-byte LDS read per bucket)
struct WalkLds {
    alignas(16) int32_t key[HS];
    uint16_t pos[HS];
};

struct HistLds {
    unsigned long long hist[2][NB];
};

// ------------------------------------------------------------------ threshold bins
//
// The bin of a triangle value s is the number of sorted thresholds c_j it passes
// (balanced: c_j <= -s for s <= 0; unbalanced: c_j < s for s > 0). A work-group stages the
// thresholds in LDS with a grid over [0, 1]: cell g = min(floor(key * TG), TG - 1) of
// key = |s|, and base[g] = the number of thresholds below cell g (negative ones, or whose
// own cell is smaller), all of which key passes; only the thresholds in key's own cell
// (none or one for thresholds spread over [0, 1]) are compared. The result equals a
// binary search over the thresholds, comparison for comparison.
constexpr int TG = 512;
static_assert(NB - 1 <= 255, "base counts are bytes");
struct ThreshLds {
    double c[NB];
    uint8_t base[TG + 1];
};
__shared__ ThreshLds thr_lds;

__device__ __forceinline__ int thresh_cell(double x) {
    return x < 0.0 ? -1 : min((int)(x * (double)TG), TG - 1);
}

// All threads of the work-group call this (it synchronises the work-group).
__device__ inline void thresh_stage(const double* __restrict__ cv, int nt) {
    for (int j = threadIdx.x; j < nt; j += blockDim.x) thr_lds.c[j] = cv[j];
    __syncthreads();
    for (int g = threadIdx.x; g <= TG; g += blockDim.x) {
        int cnt = 0;
        for (int j = 0; j < nt; j++) cnt += thresh_cell(thr_lds.c[j]) < g ? 1 : 0;
        thr_lds.base[g] = (uint8_t)cnt;
    }
    __syncthreads();
}

__device__ __forceinline__ int thresh_bin(double s, bool& bal) {
    bal = (s <= 0.0);
    const double key = bal ? -s : s;
    const int g = thresh_cell(key);
    int b = thr_lds.base[g];
    const int e = thr_lds.base[g + 1];
    while (b < e && (bal ? thr_lds.c[b] <= key : thr_lds.c[b] < key)) b++;
    return b;
}

// wave-uniform broadcast of lane `src` (src must be wave-uniform)
__device__ inline int bcast_i32(int x, int src) { return __builtin_amdgcn_readlane(x, src); }
__device__ inline int64_t bcast_i64(int64_t x, int src) {
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)x, src);
    const int hi = __builtin_amdgcn_readlane((int)((uint64_t)x >> 32), src);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}
__device__ inline double bcast_f64(double x, int src) {
    return __longlong_as_double(bcast_i64(__double_as_longlong(x), src));
}

struct SampleGraph {
    int64_t m;
    const int32_t* e_lo;
    const int32_t* e_hi;
    const double* e_d;
    const int32_t* inv;
    const int64_t* s_off;
    const int32_t* s_adj;
    const double* s_d;
    const int64_t* h_off;
    const uint32_t* h_tab;
};

__device__ inline int log2_size(int64_t size) {
    int lg = 0;
    while ((1ll << lg) < size) lg++;
    return lg;
}

// log2 of the bucket count of row y's global table
__device__ inline int hbuckets_lg(const SampleGraph& G, int32_t y) {
    return log2_size((G.h_off[y + 1] - G.h_off[y]) / UTRI_HB);
}

// Keys of bucket b (two 16-byte words) of the table at slot offset hoff.
__device__ __forceinline__ const uint4* hbucket_ptr(const uint32_t* __restrict__ htab, int64_t hoff,
                                                    uint32_t b) {
    return (const uint4*)(htab + ((hoff >> 3) + (int64_t)b) * UTRI_HB_WORDS);
}

// d of the edge to the neighbour in slot sl (a slot index from sym_lookup).
__device__ __forceinline__ double sym_d(const uint32_t* __restrict__ htab, int64_t sl) {
    return reinterpret_cast<const double*>(htab)[utri_hd_index(sl)];
}

// Slot of w in the symmetric row whose table (2^lgb buckets) starts at slot hoff, or -1.
// A bucket whose last slot is empty ends the search (slots fill in order).
__device__ inline int64_t sym_lookup(const uint32_t* __restrict__ htab, int64_t hoff, int lgb,
                                     int32_t w) {
    const uint32_t mask = (1u << lgb) - 1u;
    uint32_t b = utri_hbucket(w, lgb);
    for (;;) {
        const uint4* p = hbucket_ptr(htab, hoff, b);
        const uint4 k0 = p[0], k1 = p[1];
        const int s = utri_hmatch(k0, k1, w);
        if (s >= 0) return hoff + (int64_t)b * UTRI_HB + s;
        if (k1.w == 0xFFFFFFFFu) return -1;
        b = (b + 1) & mask;
    }
}

// ------------------------------------------------------------------ grouped edge sampling
//
// A sampled edge e = (x, y) with |d_e| >= cmin streams the Absolute-Edge-Order prefix
// (|d| >= cmin) of the endpoint with the shorter prefix, x, and looks every entry up in
// the other endpoint's row, y; each triangle found is classified and binned by threshold
// into the draw's histogram, added to hist[world][2][nt+1] when the draw ends. Draws are
// grouped by y beforehand (a counting sort), so a group stages y's prefix once: in the LDS
// of one wave (<= SCAP entries) or of one work-group (<= SCAPH), else y's global hash
// table is probed while the group's draws keep it in cache.

#ifndef UTRI_SAMPLE_CAP
#define UTRI_SAMPLE_CAP 128
#endif
#ifndef UTRI_SAMPLE_CAPH
#define UTRI_SAMPLE_CAPH 1024
#endif
constexpr int SCAP = UTRI_SAMPLE_CAP;    // probed-row prefixes staged by one wave
constexpr int SCAPH = UTRI_SAMPLE_CAPH;  // probed-row prefixes staged by one work-group
constexpr int SSL = 4;                   // table slots per staged entry (load factor 1/4)
static_assert((SCAP & (SCAP - 1)) == 0 && (SCAPH & (SCAPH - 1)) == 0 && SCAP <= SCAPH &&
                  SCAPH <= 65536,
              "table sizes are powers of two; positions are 16-bit");

// Hub groups probe y's global table; a one-hash bit filter of y's prefix, in the LDS that
// the work-group tables use otherwise (SF_BITS bits), sends only the entries whose bit is
// set there to the table.
#ifndef UTRI_SAMPLE_FILTER
#define UTRI_SAMPLE_FILTER 1
#endif
constexpr uint32_t SF_BITS = (uint32_t)SCAPH * SSL * 48;  // key and pos arrays: 6 bytes per slot
__device__ __forceinline__ uint32_t sample_filter_bit(int32_t w) {
    return __umulhi((uint32_t)w * 0x9E3779B1u, SF_BITS);
}

struct SampleWaveLds {
    alignas(16) int32_t key[SCAP * SSL];  // neighbour id + 1 (0 = empty)
    uint16_t pos[SCAP * SSL];
    uint32_t rh[2][NB];                   // histogram of the current draw
};
struct SampleBlockLds {
    alignas(16) int32_t key[SCAPH * SSL];
    uint16_t pos[SCAPH * SSL];
    uint32_t rh[WPB][2][NB];
};
union SampleLds {
    SampleWaveLds wave[WPB];
    SampleBlockLds block;
};

// Stage the first cl entries of the symmetric row at s_adj[base] with keys id + 1.
__device__ __forceinline__ void stage_sym(const int32_t* __restrict__ s_adj, int64_t base, int cl,
                                          int32_t* key, uint16_t* pos, int lg, int tid,
                                          int nthreads) {
    const uint32_t mask = (1u << lg) - 1u;
    for (int j = tid; j < cl; j += nthreads) {
        const int32_t w1 = s_adj[base + j] + 1;
        uint32_t b = walk_hash(w1, lg);
        for (;;) {
            int s = 0;
            while (s < 4 && atomicCAS(&key[4 * b + s], 0, w1) != 0) s++;
            if (s < 4) { pos[4 * b + s] = (uint16_t)j; break; }
            b = (b + 1) & mask;
        }
    }
}

// Endpoints of edge e: x has the shorter prefix (ties by id), lx its length.
__device__ __forceinline__ void draw_ends(const SampleGraph& G, const int32_t* __restrict__ slen,
                                          int64_t e, int32_t& x, int32_t& y, int& lx) {
    const int32_t a = G.inv[G.e_lo[e]], b = G.inv[G.e_hi[e]];
    const int la = slen[a], lb = slen[b];
    const bool ax = (la < lb) || (la == lb && a < b);
    x = ax ? a : b;
    y = ax ? b : a;
    lx = ax ? la : lb;
}

// Stream x's prefix [sx, sx + lx) against y's staged prefix (or y's global table) and bin
// the triangles into rh. UNR strips of loads (and, for global tables, their first table
// slots) are in flight before any is used; lanes past the row end re-load its last entry
// and drop the result.
template <bool GLOBAL_TABLE, int UNR>
__device__ __forceinline__ void draw_row(const SampleParams& sp, const SampleGraph& G,
                                         const int32_t* key, const uint16_t* pos, int lg,
                                         uint32_t mask, int64_t hoff, int64_t sy, int64_t sx,
                                         int lx, double de, uint32_t (*rh)[NB]) {
    const int lane = utri_lane();
    for (int j0 = 0; j0 < lx; j0 += UNR * UTRI_WAVE) {
        int32_t w[UNR];
        double dx[UNR];  // loaded with the ids: the row's lines are read for the hits anyway
#pragma unroll
        for (int k = 0; k < UNR; k++) {
            const int64_t j = sx + min(j0 + k * UTRI_WAVE + lane, lx - 1);
            w[k] = G.s_adj[j];
            dx[k] = G.s_d[j];
        }
        bool hit[UNR];
        double dy[UNR];
        if (GLOBAL_TABLE) {
            // lg: log2 of the bucket count; a hit reads d from the slot; key: the filter
            const uint32_t gm = (1u << lg) - 1u;
            uint32_t b[UNR];
            uint4 k0[UNR], k1[UNR];
#pragma unroll
            for (int k = 0; k < UNR; k++) {
                b[k] = utri_hbucket(w[k], lg);
                bool cand = true;
#if UTRI_SAMPLE_FILTER
                const uint32_t fb = sample_filter_bit(w[k]);
                cand = ((reinterpret_cast<const uint32_t*>(key)[fb >> 5] >> (fb & 31u)) & 1u) != 0u;
#endif
                // an all-empty bucket matches nothing and ends the search
                k0[k] = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
                k1[k] = k0[k];
                if (cand) {
                    const uint4* p = hbucket_ptr(G.h_tab, hoff, b[k]);
                    k0[k] = p[0];
                    k1[k] = p[1];
                }
            }
#pragma unroll
            for (int k = 0; k < UNR; k++) {
                int s = utri_hmatch(k0[k], k1[k], w[k]);
                while (s < 0 && k1[k].w != 0xFFFFFFFFu) {
                    b[k] = (b[k] + 1) & gm;
                    const uint4* p = hbucket_ptr(G.h_tab, hoff, b[k]);
                    k0[k] = p[0];
                    k1[k] = p[1];
                    s = utri_hmatch(k0[k], k1[k], w[k]);
                }
                hit[k] = s >= 0;
                dy[k] = hit[k] ? sym_d(G.h_tab, hoff + (int64_t)b[k] * UTRI_HB + s) : 0.0;
            }
        } else {
#pragma unroll
            for (int k = 0; k < UNR; k++) {
                int h;
                const int kk = bucket_find(key, lg, mask, (uint32_t)w[k] + 1u, 0xFFFFFFFFu, h);
                hit[k] = kk != 0;
                dy[k] = hit[k] ? G.s_d[sy + pos[h]] : 0.0;
            }
        }
#pragma unroll
        for (int k = 0; k < UNR; k++) {
            const int j = j0 + k * UTRI_WAVE + lane;
            if (j < lx && hit[k]) {
                const double s = utri_tri_s(de, dx[k], dy[k]);
                bool bal;
                const int bin = thresh_bin(s, bal);
                if (bin > 0) atomicAdd(&rh[bal ? 0 : 1][bin], 1u);
            }
        }
    }
}

template <bool GLOBAL_TABLE>
__device__ __forceinline__ void draw_row_any(const SampleParams& sp, const SampleGraph& G,
                                             const int32_t* key, const uint16_t* pos, int lg,
                                             uint32_t mask, int64_t hoff, int64_t sy, int64_t sx,
                                             int lx, double de, uint32_t (*rh)[NB]) {
    if (lx > 2 * UTRI_WAVE)
        draw_row<GLOBAL_TABLE, 4>(sp, G, key, pos, lg, mask, hoff, sy, sx, lx, de, rh);
    else if (lx > UTRI_WAVE)
        draw_row<GLOBAL_TABLE, 2>(sp, G, key, pos, lg, mask, hoff, sy, sx, lx, de, rh);
    else
        draw_row<GLOBAL_TABLE, 1>(sp, G, key, pos, lg, mask, hoff, sy, sx, lx, de, rh);
}

// Add the draw's histogram to its world's and clear it.
__device__ __forceinline__ void draw_flush(const SampleParams& sp, int32_t world, uint32_t (*rh)[NB]) {
    utri_wave_sync();
    const int nb = sp.nt + 1;
    for (int q = utri_lane(); q < 2 * nb; q += UTRI_WAVE) {
        const int cls = q / nb, bin = q % nb;
        const uint32_t v = rh[cls][bin];
        if (v) {
            atomicAdd(&sp.hist[((int64_t)world * 2 + cls) * nb + bin], (unsigned long long)v);
            rh[cls][bin] = 0;
        }
    }
    utri_wave_sync();
}

// The draws [r0, r1) of group y whose index is part mod nparts, 64 loaded at a time.
template <bool GLOBAL_TABLE>
__device__ __forceinline__ void group_draws(const SampleParams& sp, const SampleGraph& G,
                                            const int32_t* __restrict__ slen, int32_t y, int64_t r0,
                                            int64_t r1, const int32_t* key, const uint16_t* pos,
                                            int lg, uint32_t mask, int64_t hoff, uint32_t (*rh)[NB],
                                            int part, int nparts) {
    const int lane = utri_lane();
    const int64_t sy = G.s_off[y];
    for (int64_t b0 = r0; b0 < r1; b0 += UTRI_WAVE) {
        const int64_t r = b0 + lane;
        int64_t sx = 0;
        int lx = 0;
        double de = 0.0;
        int32_t world = 0;
        if (r < r1) {
            const int64_t rec = sp.rec[r];
            const int64_t e = rec & 0xFFFFFFFFll;
            world = (int32_t)(rec >> 32);
            int32_t x, yy;
            draw_ends(G, slen, e, x, yy, lx);
            de = G.e_d[e];
            sx = G.s_off[x];
        }
        const int nr = (int)min((int64_t)UTRI_WAVE, r1 - b0);
        for (int si = part; si < nr; si += nparts) {
            draw_row_any<GLOBAL_TABLE>(sp, G, key, pos, lg, mask, hoff, sy, bcast_i64(sx, si),
                                       bcast_i32(lx, si), bcast_f64(de, si), rh);
            draw_flush(sp, bcast_i32(world, si), rh);
        }
    }
}

// One group item: draws [sub * chunk, sub * chunk + chunk) of group y. Work-group items
// split the draws over the four waves and stage y's prefix in the work-group table
// (SCAP < prefix <= SCAPH) or, for longer prefixes, probe y's global hash table; wave
// items stage it in the wave's table (prefix <= SCAP).
__device__ inline void sample_item(const SampleParams& sp, const SampleGraph& G,
                                   const int32_t* __restrict__ slen, int64_t item, bool block,
                                   SampleLds& S) {
    const int wib = threadIdx.x / UTRI_WAVE;
    const int lane = utri_lane();
    const int32_t y = (int32_t)(item & 0xFFFFFFFF);
    const int64_t sub = item >> 32;
    const int Ly = slen[y];
    const int64_t r0 = sp.goff[y] + sub * sp.chunk;
    const int64_t r1 = min(sp.goff[y + 1], r0 + (int64_t)sp.chunk);
    if (block && Ly > SCAPH) {
        SampleBlockLds& B = S.block;
        const int64_t hoff = G.h_off[y];
        const int hlg = hbuckets_lg(G, y);
        __syncthreads();  // the previous item's flushes are done
        for (int q = threadIdx.x; q < WPB * 2 * NB; q += TPB) (&B.rh[0][0][0])[q] = 0;
        uint32_t* bits = reinterpret_cast<uint32_t*>(B.key);
#if UTRI_SAMPLE_FILTER
        for (int i = threadIdx.x; i < (int)(SF_BITS / 32); i += TPB) bits[i] = 0u;
        __syncthreads();
        const int64_t sy = G.s_off[y];
        for (int j = threadIdx.x; j < Ly; j += TPB) {
            const uint32_t fb = sample_filter_bit(G.s_adj[sy + j]);
            atomicOr(&bits[fb >> 5], 1u << (fb & 31u));
        }
#endif
        __syncthreads();
        group_draws<true>(sp, G, slen, y, r0, r1, (const int32_t*)bits, nullptr, hlg, 0, hoff,
                          B.rh[wib], wib, WPB);
        return;
    }
    if (block) {
        SampleBlockLds& B = S.block;
        const int lg = table_lg(Ly, SSL);
        const int nbk = 1 << lg;
        __syncthreads();  // the previous item's probes are done
        for (int i = threadIdx.x; i < 4 * nbk; i += TPB) B.key[i] = 0;
        for (int q = threadIdx.x; q < WPB * 2 * NB; q += TPB) (&B.rh[0][0][0])[q] = 0;
        __syncthreads();
        stage_sym(G.s_adj, G.s_off[y], Ly, B.key, B.pos, lg, threadIdx.x, TPB);
        __syncthreads();
        group_draws<false>(sp, G, slen, y, r0, r1, B.key, B.pos, lg, (uint32_t)(nbk - 1), 0,
                           B.rh[wib], wib, WPB);
        return;
    }
    SampleWaveLds& W = S.wave[wib];
    for (int q = lane; q < 2 * NB; q += UTRI_WAVE) (&W.rh[0][0])[q] = 0;
    const int lg = table_lg(Ly, SSL);
    const int nbk = 1 << lg;
    for (int i = lane; i < 4 * nbk; i += UTRI_WAVE) W.key[i] = 0;
    utri_wave_sync();
    stage_sym(G.s_adj, G.s_off[y], Ly, W.key, W.pos, lg, lane, UTRI_WAVE);
    utri_wave_sync();
    group_draws<false>(sp, G, slen, y, r0, r1, W.key, W.pos, lg, (uint32_t)(nbk - 1), 0, W.rh, 0,
                       1);
    utri_wave_sync();  // probes done before the next item clears the table
}

// All group items of a pass, heaviest groups (highest ids) first: hub items from eight
// queues, one per XCD (work-group index mod 8, the hardware's round-robin placement), so
// each XCD works through its own few hubs and keeps their tables in its L2; then the other
// work-group items (one queue); then wave items in groups of four.
__device__ inline void sample_groups(const SampleParams& sp, const SampleGraph& G,
                                     const int32_t* __restrict__ slen, SampleLds& S) {
    __shared__ int64_t s_qs;
    const int64_t nb = sp.nitems[0], nw = sp.nitems[1], nh = sp.nitems[2];
    const int xcd = (int)(blockIdx.x % 8);
    for (int qq = 0; qq < 8; qq++) {
        const int q8 = (xcd + qq) % 8;
        const int64_t a = nh * q8 / 8, b = nh * (q8 + 1) / 8;
        for (;;) {
            if (threadIdx.x == 0) s_qs = (int64_t)atomicAdd(&sp.qctr[2 + q8], 1ull);
            __syncthreads();
            const int64_t t = s_qs;
            __syncthreads();
            if (a + t >= b) break;
            sample_item(sp, G, slen, sp.items[sp.hub_base + nh - 1 - (a + t)], true, S);
        }
    }
    for (;;) {
        if (threadIdx.x == 0) s_qs = (int64_t)atomicAdd(&sp.qctr[0], 1ull);
        __syncthreads();
        const int64_t q = s_qs;
        __syncthreads();
        if (q >= nb) break;
        sample_item(sp, G, slen, sp.items[nb - 1 - q], true, S);
    }
    __syncthreads();  // the work-group table is no longer read; the wave tables reuse it
    for (;;) {
        int64_t base = 0;
        if (utri_lane() == 0) base = (int64_t)atomicAdd(&sp.qctr[1], 4ull);
        base = bcast_i64(base, 0);
        if (base >= nw) break;
        const int64_t end = base + 4 < nw ? base + 4 : nw;
        for (int64_t q = base; q < end; q++)
            sample_item(sp, G, slen, sp.items[sp.wave_base + nw - 1 - q], false, S);
    }
}

}  // namespace utri_dev
