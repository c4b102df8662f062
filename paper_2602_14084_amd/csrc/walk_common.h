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

#ifndef UTRI_WALK_HASH24
#define UTRI_WALK_HASH24 0         // 1: full-rate 24-bit multiplicative hash; 0: 32-bit
#endif

// bucket of w in a table of 2^lg buckets (lg >= 1)
__device__ __forceinline__ uint32_t walk_hash(int32_t w, int lg) {
#if UTRI_WALK_HASH24
    // the 24-bit multiplier runs at full rate (the 32-bit one at quarter rate); ids above
    // 2^24 fold their high bits in. __umul24 returns a signed int: shift the unsigned value
    const uint32_t x = (uint32_t)w ^ ((uint32_t)w >> 24);
    return (uint32_t)__umul24(x, 0x9E3779u) >> (32 - lg);
#else
    return utri_hash32(w, lg);
#endif
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

// LDS of one wave of a flattened strip loop (sampler, backward)
struct SegLds {
    int32_t end[UTRI_WAVE];       // inclusive prefix of segment lengths
    int64_t xoff[UTRI_WAVE];      // start of the streamed row of each segment
    int64_t yoff[UTRI_WAVE];      // start of the probe-side row
    int64_t hoff[UTRI_WAVE];      // start of the probe-side table
    int32_t hlg[UTRI_WAVE];       // log2 size of the probe-side table
    double dseg[UTRI_WAVE];       // d of the segment's own edge
    unsigned long long shist[2][NB];
};

__device__ inline int seg_search(const int32_t* end, int f) {
    // smallest index i with end[i] > f (end is non-decreasing and end[63] > f)
    int lo = 0, hi = UTRI_WAVE - 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (end[mid] > f) hi = mid; else lo = mid + 1;
    }
    return lo;
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
    const uint64_t* h_slot;
};

// position of w in the symmetric row whose table starts at hoff with 2^lg slots, or -1
__device__ inline int64_t sym_lookup(const uint64_t* __restrict__ h_slot, int64_t hoff, int lg,
                                     int32_t w) {
    const uint32_t mask = (1u << lg) - 1u;
    uint32_t h = utri_hash32(w, lg);
    for (;;) {
        const uint64_t sl = h_slot[hoff + h];
        if (sl == ~0ull) return -1;
        if ((int32_t)(sl >> 32) == w) return (int64_t)(uint32_t)(sl & 0xFFFFFFFFull);
        h = (h + 1) & mask;
    }
}

__device__ inline int log2_size(int64_t size) {
    int lg = 0;
    while ((1ll << lg) < size) lg++;
    return lg;
}

// One work unit of the edge-sampling estimator: samples [i_begin, i_end) of `world`.
// Each sampled edge e = (a, b) with |d_e| >= cmin streams the Absolute-Edge-Order
// prefix (|d| >= cmin) of its shorter row and probes the other row's hash table; the
// triangles found are classified and binned by threshold into the wave's histogram,
// which is added to hist[world][2][nt+1] at the end of the unit.
__device__ inline void sample_unit(const SampleParams& sp, const SampleGraph& G,
                                   const int32_t* __restrict__ slen, int32_t world,
                                   int64_t i_begin, int64_t i_end, SegLds& L) {
    const int lane = utri_lane();
    for (int q = lane; q < 2 * NB; q += UTRI_WAVE) L.shist[q / NB][q % NB] = 0;
    utri_wave_sync();
    const uint64_t seed = sp.seed_dev ? *sp.seed_dev : sp.seed;
    for (int64_t i0 = i_begin; i0 < i_end; i0 += UTRI_WAVE) {
        const int64_t i = i0 + lane;
        int work = 0;
        int64_t xoff = 0, yoff = 0, hoff = 0;
        int lg = 0;
        double de = 0.0;
        if (i < i_end) {
            const int64_t e = utri_sample_edge(seed, (uint32_t)world, (uint64_t)i, G.m);
            de = G.e_d[e];
            if (fabs(de) >= sp.cmin) {
                const int32_t a = G.inv[G.e_lo[e]], b = G.inv[G.e_hi[e]];
                const int la = slen[a], lb = slen[b];
                const bool ax = (la < lb) || (la == lb && a < b);
                const int32_t x = ax ? a : b, y = ax ? b : a;
                work = ax ? la : lb;
                xoff = G.s_off[x];
                yoff = G.s_off[y];
                hoff = G.h_off[y];
                lg = log2_size(G.h_off[y + 1] - hoff);
            }
        }
        const int incl = (int)utri_wave_incl_scan((int64_t)work);
        const int total = __shfl(incl, UTRI_WAVE - 1, UTRI_WAVE);
        L.end[lane] = incl;
        L.xoff[lane] = xoff;
        L.yoff[lane] = yoff;
        L.hoff[lane] = hoff;
        L.hlg[lane] = lg;
        L.dseg[lane] = de;
        utri_wave_sync();
        for (int f0 = 0; f0 < total; f0 += UTRI_WAVE) {
            const int f = f0 + lane;
            if (f < total) {
                const int sg = seg_search(L.end, f);
                const int start = sg ? L.end[sg - 1] : 0;
                const int64_t px = L.xoff[sg] + (f - start);
                const int32_t w = G.s_adj[px];
                const int64_t py = sym_lookup(G.h_slot, L.hoff[sg], L.hlg[sg], w);
                if (py >= 0) {
                    const double s = utri_tri_s(L.dseg[sg], G.s_d[px], G.s_d[L.yoff[sg] + py]);
                    bool bal;
                    const int bin = utri_bin_of(s, sp.cvals, sp.nt, bal);
                    if (bin > 0) atomicAdd(&L.shist[bal ? 0 : 1][bin], 1ull);
                }
            }
        }
        utri_wave_sync();
    }
    for (int q = lane; q < 2 * NB; q += UTRI_WAVE) {
        const int cls = q / NB, bin = q % NB;
        const unsigned long long v = L.shist[cls][bin];
        if (v && bin <= sp.nt)
            atomicAdd(&sp.hist[((int64_t)world * 2 + cls) * (sp.nt + 1) + bin], v);
    }
    utri_wave_sync();
}

}  // namespace utri_dev
