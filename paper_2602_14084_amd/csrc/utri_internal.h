// utri_internal.h -- shared declarations of the HIP library (not part of the ABI).
//
// Data layout in HBM (all device memory, owned by the graph handle):
//   canonical edges, edge-id order      e_lo/e_hi int32 [m], e_p/e_d f64 [m]
//   vertex relabelling                  perm (new -> original) / inv int32 [n]
//       new ids rank vertices by degree, ties by a fixed bijective mix of the id: the
//       Node Order of Section 4 with another tie-break (any strict order by degree
//       visits each triangle once).
//   symmetric rows, new ids             s_off int64 [n+1], s_adj int32 [2m],
//       each row in Absolute Edge Order  s_d f64 [2m], s_eid int32 [2m]
//       (|d| descending, then neighbour id ascending; Section 5), so the entries
//       with |d| >= c of any row form a prefix.
//   per-row bucketed hash tables        h_off int64 [n+1] (slots), h_tab u32 [4 * sum]:
//       buckets of 8 slots, 128 bytes each: the keys (neighbour id, ~0 = empty; 32
//       bytes), each slot's d of the edge to that neighbour (64 bytes), 32 bytes of
//       padding; slots fill in order; size = pow2 >= max(3*deg, 8), a load factor of at
//       most 1/3, so a lookup almost always reads one bucket.
//   oriented rows u -> v (v > u)        o_off int64 [n+1], o_adj int32 [m],
//       same Absolute Edge Order         o_d f64 [m], o_eid int32 [m]
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "utri.h"

#define UTRI_WAVE 64
// readable entries the oriented id array carries past its last row: a row stream loads
// whole groups of up to 8 strips of 64 without clamping to the row end
#define UTRI_ROW_PAD 512
// most sampler draws grouped per pass (records of 8 bytes each)
#define UTRI_SAMPLE_PASS (1ll << 27)

// A dispatch's work-item count (blocks x threads) must stay below 2^32: one-dimensional
// launches over arrays that can be longer than that (enumerated triangles, sign masks,
// caller-sized draws) cap their grid here and their kernels stride over the rest.
constexpr int64_t UTRI_MAX_GRID_BLOCKS = (int64_t)1 << 20;
inline unsigned utri_grid(int64_t n, int tpb) {
    int64_t b = (n + tpb - 1) / tpb;
    if (b < 1) b = 1;
    return (unsigned)(b < UTRI_MAX_GRID_BLOCKS ? b : UTRI_MAX_GRID_BLOCKS);
}
#define UTRI_FOR_GRID(i, n)                                                  \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
         i += (int64_t)gridDim.x * blockDim.x)

// ------------------------------------------------------------------ error plumbing

#define UTRI_HIP_TRY(expr)                                 \
    do {                                                   \
        hipError_t _e = (expr);                            \
        if (_e != hipSuccess) {                            \
            utri_note_hip_error(_e, #expr, __FILE__, __LINE__); \
            return (_e == hipErrorOutOfMemory) ? UTRI_E_NOMEM : UTRI_E_HIP; \
        }                                                  \
    } while (0)

#define UTRI_TRY(expr)                 \
    do {                               \
        int _rc = (expr);              \
        if (_rc != UTRI_OK) return _rc; \
    } while (0)

void utri_note_hip_error(hipError_t e, const char* what, const char* file, int line);

// device error flag bits
enum : uint32_t {
    UTRI_FLAG_BAD_ID = 1u,
    UTRI_FLAG_BAD_P = 2u,
    UTRI_FLAG_CONFLICT = 4u,
};

// scratch buffers kept by a handle between calls (grown on demand)
enum UtriScratch {
    SCR_TEMP = 0,     // rocPRIM temporary storage
    SCR_LEN,          // int32 [2n+2] row prefix lengths at c (oriented, then symmetric)
    SCR_SLEN,         // int32 [n] row prefix lengths at c (symmetric)
    SCR_ICNT,         // int32 [n] items per vertex
    SCR_IOFF,         // int64 [n] item offsets
    SCR_ITEMS,        // int64 [items]
    SCR_NITEMS,       // int64 [4] item count and friends
    SCR_ACC,          // u64 accumulators of a query
    SCR_CVALS,        // f64 [64] sorted thresholds
    SCR_ICNT2,        // int64 [items][2] per-item counts (enumeration)
    SCR_IOFF2,        // int64 [items][2] per-item offsets (enumeration)
    SCR_SORT_A,       // enumeration sort buffers
    SCR_SORT_B,
    SCR_SORT_C,
    SCR_SORT_D,
    SCR_HIST,         // u64 [worlds][2][nt+1]
    SCR_BATCH_T,      // f64 [64] thresholds of the captured batch
    SCR_ORDER,        // int32 [64] original position of each sorted threshold
    SCR_OUT,          // int64 small device results
    SCR_SEED,         // u64 seed of the captured batch
    SCR_HIST2,        // u64 walk histogram of the batch
    SCR_GCNT,         // int32 [4n] gradient items per vertex (four lists)
    SCR_GOFF,         // int64 [6n+2] gradient item offsets and partial-slice offsets
    SCR_GSZ,          // int64 [2n] gradient partial-slice sizes
    SCR_GITEMS,       // int64 gradient items
    SCR_GQ,           // int64 [16] gradient item counts and work-queue counters
    SCR_GPART,        // gradient partial sums (pairs of 64-bit half sums)
    SCR_SCNT,         // int32 [n+2] sampler draws per probed endpoint
    SCR_SOFF,         // int64 [n+1] sampler group offsets
    SCR_SREC,         // int64 sampler draw records of one pass
    SCR_SICNT,        // int32 [3n] sampler items per group (work-group, wave, hub)
    SCR_SIOFF,        // int64 [3n] sampler item offsets
    SCR_SITEMS,       // int64 sampler items
    SCR_SQ,           // int64 [16] sampler item counts and work-queue counters
    SCR_VQ,           // int32 [worlds * k] sampled vertices (new ids)
    SCR_VLEN,         // int32 [worlds * k] their Lemma-2 prefix lengths
    SCR_VOFF,         // int64 [worlds * k + 1] offsets of their edge records
    SCR_VREC,         // int64 edge records of the sampled vertices: edge | world << 32
    SCR_TOPK_TRI,     // int32 [N][3] top-k candidates (enumerated at the found threshold)
    SCR_TOPK_S,       // f64 [N] their s values
    SCR_TOPK_KEY,     // u64 [2N] sort keys
    SCR_TOPK_IDX,     // u32 [2N] sort values
    SCR_SIGN_MASK,    // u32 [m][worlds / 32] negative-sign masks of the sign worlds
    SCR_SIGN_CNT,     // u64 [worlds] balanced triangles per sign world
    SCR_TUNE,         // f64 estimates written by the autotuner's sampler trials
    SCR_RINFO,        // uint2 [n] (row start, kept length) of each vertex at the query's c
    SCR_COUNT
};

// Run-time launch parameters of the triangle walk (the autotuner's search space; every
// value gives the same results):
//   pr    partners (symmetric-row entries) per work item, a multiple of 64;
//   cap   longest kept row staged in one wave's table (longer rows go to work-groups),
//         a power of two <= 128;
//   caph  entries per work-group table chunk, a power of two in [cap, 2048];
//   unr   most row loads in flight per lane (1, 2, 4 or 8);
//   shorter_min  the walk streams the shorter kept row of each edge when the plain
//         forward iteration would stream at least this many ids per kept edge.
struct WalkTune {
    int32_t pr = 1024;
    int32_t cap = 128;
    int32_t caph = 2048;
    int32_t unr = 8;
    int64_t shorter_min = 320;
    bool operator==(const WalkTune& o) const {
        return pr == o.pr && cap == o.cap && caph == o.caph && unr == o.unr &&
               shorter_min == o.shorter_min;
    }
};

// Longest work-group table chunk of the sign-world walk (its work-groups keep a smaller
// table so that more of them fit a compute unit).
constexpr int UTRI_SIGN_WALK_CHUNK = 1024;

struct UtriBatchGraph {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    std::vector<double> cvals;
    int nt = 0;
    int64_t k = 0;
    int32_t worlds = 0;
    int64_t* exact = nullptr;
    double* est = nullptr;
    // the graph holds raw pointers to the handle's scratch buffers and bakes in its launch
    // shape: it is replayed only while neither has changed since capture
    uint64_t scr_gen = 0;
    int walk_blocks_per_cu = 0, sample_chunk = 0, walk_order = 0;
    int64_t sample_pass = 0;
    WalkTune walk_tune;
};

// Per-item counts of an enumeration (in SCR_ICNT2, offsets in SCR_IOFF2) that a
// utri_enumerate call left behind when it returned UTRI_E_CAPACITY, with everything they
// depend on; the next call of the same query with enough capacity fills from them once.
struct EnumTicket {
    bool valid = false;
    double c = 0.0;
    int method = 0, which = 0, walk_order = 0;
    WalkTune walk_tune;
    uint64_t scr_gen = 0, rows_gen = 0;
    int64_t nb = 0, nu = 0;
};

struct utri_graph {
    int device = 0;
    int num_cu = 256;
    int64_t n = 0, m = 0;
    int64_t self_loops = 0, dups = 0, max_deg = 0, max_out = 0;

    int32_t *e_lo = nullptr, *e_hi = nullptr;
    double *e_p = nullptr, *e_d = nullptr;
    int32_t *perm = nullptr, *inv = nullptr;
    int32_t* deg_new = nullptr;  // degree of each new id (ascending)

    int64_t* s_off = nullptr;
    int32_t* s_adj = nullptr;
    double* s_d = nullptr;
    int32_t* s_eid = nullptr;
    int32_t* s_row = nullptr;    // row of each symmetric entry

    int64_t* h_off = nullptr;
    uint32_t* h_tab = nullptr;   // UTRI_HB_WORDS words per bucket (utri_hkey_index)
    int64_t h_total = 0;

    int64_t* o_off = nullptr;
    int32_t* o_adj = nullptr;    // packed: id | q(|d|) << idbits | sign(d) << 31
    double* o_d = nullptr;
    int32_t* o_eid = nullptr;
    // Oriented-row packing. Ids take the low `idbits` bits; when at least three bits are
    // left, bits idbits .. idbits + mb - 1 hold q = min(floor(|d| * 2^mb), 2^mb - 1), so |d|
    // lies in [q, q + 1] * 2^-mb, and bit 31 holds sign(d). Ids are at least 1 (vertex 0
    // has the lowest rank and is in no oriented row), so a packed word is never 0.
    int idbits = 31;
    int code_mb = 0;             // magnitude bits of the code, 0 = no code
    uint32_t idmask = 0x7FFFFFFFu;

    uint32_t* d_flags = nullptr;
    void* rinfo_cur = nullptr;   // the last walk preparation's per-vertex (row start, length)

    void* scr[SCR_COUNT] = {};
    size_t scr_bytes[SCR_COUNT] = {};
    uint64_t scr_gen = 0;  // bumped whenever a scratch buffer is reallocated
    uint64_t rows_gen = 0; // bumped whenever the rows (and their d) are rebuilt
    EnumTicket enum_ticket;
    // No-allocation mode (set for the duration of one call): scratch slots are carved from
    // this caller-owned device arena instead of hipMalloc; a request that does not fit is
    // UTRI_E_CAPACITY.
    char* arena = nullptr;
    size_t arena_bytes = 0, arena_used = 0;
    void* arena_slot[SCR_COUNT] = {};
    size_t arena_slot_bytes[SCR_COUNT] = {};

    // launch shape (set by the autotuner, else defaults)
    int walk_blocks_per_cu = 0;     // 0: the kernel's resident occupancy
    int sample_blocks_per_cu = 8;
    int sample_chunk = 128;         // draws per sampler group item
    int64_t sample_pass = UTRI_SAMPLE_PASS;  // draws grouped per sampler pass
    uint32_t sign_flush_at = 65535;          // sign-world counter additions between flushes
    int walk_order = 0;                      // UTRI_ORDER_*: row streamed per kept edge
    WalkTune walk_tune;                      // walk work-chunk and tile sizes

    // gradient: item counts of its four lists and partial-slice totals (they depend on the
    // degrees only), -1 = not read yet
    int64_t grad_sizes[6] = {-1, -1, -1, -1, -1, -1};

    // event timing of the counting walk kernel (utri_timing)
    int timing = 0;
    double timing_ms = 0.0;
    int64_t timing_launches = 0;
    hipEvent_t tev0 = nullptr, tev1 = nullptr;

    UtriBatchGraph batch;
};

int utri_scratch(utri_graph* g, int slot, size_t bytes, void** out);
int utri_build_rows(utri_graph* g, hipStream_t s);

// ------------------------------------------------------------------ device helpers

// Canonical FP64 decision, the library's own copy:
//   d = 1.0 - 2.0*p, c = 2.0*t - 1.0, three d sorted ascending, s = (x*y)*z.
__host__ __device__ inline double utri_d_of_p(double p) { return 1.0 - 2.0 * p; }
__host__ __device__ inline double utri_c_of_t(double t) { return 2.0 * t - 1.0; }

__device__ inline double utri_tri_s(double a, double b, double c) {
    double lo = fmin(a, b), hi = fmax(a, b);
    double x = fmin(lo, c);          // smallest
    double z = fmax(hi, c);          // largest
    double y = fmax(lo, fmin(hi, c));  // middle
    double xy = __dmul_rn(x, y);
    return __dmul_rn(xy, z);
}

// nearest multiple of 2^-62 (ties to even) of |x| <= 1, as an integer
__device__ inline int64_t utri_fix62(double x) {
    return (int64_t)rint(x * 0x1p62);
}

// correctly rounded conversion of a two's complement 128-bit integer (hi:lo) to double
__host__ __device__ inline double utri_u64_to_double_rn(uint64_t v) {
    // the product is exact and the single addition rounds once
    double h = (double)(uint32_t)(v >> 32) * 4294967296.0;
    double l = (double)(uint32_t)(v & 0xFFFFFFFFull);
    return h + l;
}

__host__ __device__ inline double utri_i128_to_double(int64_t hi, uint64_t lo) {
    bool neg = hi < 0;
    uint64_t uhi = (uint64_t)hi, ulo = lo;
    if (neg) {
        ulo = ~ulo + 1ull;
        uhi = ~uhi + (ulo == 0 ? 1ull : 0ull);
    }
    double r;
    if (uhi == 0) {
        r = utri_u64_to_double_rn(ulo);
    } else {
        int lz = 0;
        while (!((uhi << lz) & 0x8000000000000000ull)) lz++;
        int sh = 64 - lz;  // shift right by sh bits to fit 64 bits
        uint64_t v = (sh == 64) ? uhi : ((uhi << (64 - sh)) | (ulo >> sh));
        uint64_t lost = (sh == 64) ? ulo : (ulo << (64 - sh));
        if (lost) v |= 1ull;  // sticky bit below the rounding position (v has 64 significant bits)
        r = utri_u64_to_double_rn(v);
        r = ldexp(r, sh);
    }
    return neg ? -r : r;
}

__device__ inline uint32_t utri_hash32(int32_t key, int lg) {
    return ((uint32_t)key * 0x9E3779B1u) >> (32 - lg);
}

// Per-row global tables: slots per bucket and the table size for a row of deg entries.
constexpr int UTRI_HB = 8;
__host__ __device__ inline int64_t utri_htable_slots(int64_t deg) {
    if (deg <= 0) return 0;
    int64_t size = UTRI_HB;
    while (size < 3 * deg) size <<= 1;
    return size;
}

// A bucket takes 128 bytes of h_tab: its 8 keys, then their d values, then 32 bytes of
// padding. The d of the first four slots, which hold the entries of all but crowded
// buckets (slots fill in order), lie in the keys' 64-byte sector, so a hit reads no other
// sector. Slot sl, counted like h_off, is slot sl % 8 of bucket sl / 8.
constexpr int UTRI_HB_WORDS = 32;  // 32-bit words per bucket
__host__ __device__ inline int64_t utri_hkey_index(int64_t sl) {
    return (sl >> 3) * UTRI_HB_WORDS + (sl & 7);
}
__host__ __device__ inline int64_t utri_hd_index(int64_t sl) {  // in 8-byte words
    return (sl >> 3) * (UTRI_HB_WORDS / 2) + 4 + (sl & 7);
}

// Home bucket of key in a table of 2^lgb buckets (lgb >= 0).
__device__ inline uint32_t utri_hbucket(int32_t key, int lgb) {
    return lgb > 0 ? utri_hash32(key, lgb) : 0u;
}

// Slot of key among the 8 keys of a bucket (two 16-byte words), or -1.
__device__ __forceinline__ int utri_hmatch(const uint4& a, const uint4& b, int32_t key) {
    const uint32_t k = (uint32_t)key;
    int s = -1;
    s = a.x == k ? 0 : s;
    s = a.y == k ? 1 : s;
    s = a.z == k ? 2 : s;
    s = a.w == k ? 3 : s;
    s = b.x == k ? 4 : s;
    s = b.y == k ? 5 : s;
    s = b.z == k ? 6 : s;
    s = b.w == k ? 7 : s;
    return s;
}

__device__ inline void utri_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int utri_lane() { return (int)(threadIdx.x & (UTRI_WAVE - 1)); }

// inclusive prefix sum over the 64 lanes of a wave
__device__ inline int64_t utri_wave_incl_scan(int64_t v) {
    const int lane = utri_lane();
#pragma unroll
    for (int d = 1; d < UTRI_WAVE; d <<= 1) {
        int64_t o = __shfl_up(v, d, UTRI_WAVE);
        if (lane >= d) v += o;
    }
    return v;
}

__device__ inline uint64_t utri_wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int d = UTRI_WAVE / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, UTRI_WAVE);
    return v;
}

// 128-bit sum over the wave of (hi:lo) pairs, exact modulo 2^128
__device__ inline void utri_wave_sum_u128(uint64_t& lo, uint64_t& hi) {
#pragma unroll
    for (int d = UTRI_WAVE / 2; d >= 1; d >>= 1) {
        uint64_t olo = __shfl_xor(lo, d, UTRI_WAVE);
        uint64_t ohi = __shfl_xor(hi, d, UTRI_WAVE);
        uint64_t s = lo + olo;
        hi = hi + ohi + (s < lo ? 1ull : 0ull);
        lo = s;
    }
}

// exact 128-bit atomic accumulation into (acc[0] = lo, acc[1] = hi)
__device__ inline void utri_atomic_add_u128(unsigned long long* acc, uint64_t lo, uint64_t hi) {
    unsigned long long old = atomicAdd(&acc[0], (unsigned long long)lo);
    uint64_t carry = ((uint64_t)old + lo < (uint64_t)old) ? 1ull : 0ull;
    if (hi + carry) atomicAdd(&acc[1], (unsigned long long)(hi + carry));
}

// Philox4x32-10 block (Salmon, Moraes, Dror, Shaw, SC'11): multipliers 0xD2511F53 and
// 0xCD9E8D57, Weyl key increments 0x9E3779B9 and 0xBB67AE85, ten rounds.
__device__ inline void utri_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                   uint32_t k1, uint32_t* out) {
#pragma unroll
    for (int r = 0; r < 10; r++) {
        uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// index in [0, range) drawn by sample i of world w: the high 64 bits of (x1:x0) * range
// for the Philox block with counter (i_lo, i_hi, 0, 0) and key (seed_lo ^ w, seed_hi)
__device__ inline int64_t utri_draw_index(uint64_t seed, uint32_t world, uint64_t i, int64_t range) {
    uint32_t x[4];
    utri_philox((uint32_t)i, (uint32_t)(i >> 32), 0u, 0u, (uint32_t)seed ^ world,
                (uint32_t)(seed >> 32), x);
    uint64_t x64 = ((uint64_t)x[1] << 32) | (uint64_t)x[0];
    return (int64_t)__umul64hi(x64, (uint64_t)range);
}

// edge drawn by sample i of world w (edge sampling) and vertex (vertex sampling)
__device__ inline int64_t utri_sample_edge(uint64_t seed, uint32_t world, uint64_t i, int64_t m) {
    return utri_draw_index(seed, world, i, m);
}
__device__ inline int64_t utri_sample_vertex(uint64_t seed, uint32_t world, uint64_t i, int64_t n) {
    return utri_draw_index(seed, world, i, n);
}

// ------------------------------------------------------------------ kernels (host launchers)

// per-query preparation of the oriented walk
int utri_walk_prepare(utri_graph* g, double c_rows, int lemma3, hipStream_t s, int64_t** items,
                      int64_t** n_items_dev, int32_t** len);

enum WalkMode {
    WALK_COUNT = 0,
    WALK_HIST = 1,
    WALK_EXPECTED = 2,
    WALK_ENUM_COUNT = 3,
    WALK_ENUM_FILL = 4,
    WALK_STATS = 5,  // acc[0] = hash hits, acc[1] = target elements (first chunk), acc[2] = all streamed
    WALK_SIGN = 6,   // wcount[w] += balanced triangles of sign world w
};

struct WalkParams {
    double c = 0.0;          // decision threshold (COUNT / ENUM)
    int lemma3 = 0;
    double c_l3 = 0.0;       // c * (1 - 2^-50) for the Lemma-3 cut
    const double* cvals = nullptr;  // HIST: sorted thresholds
    int nt = 0;
    unsigned long long* acc = nullptr;  // COUNT [2], HIST [2][nt+1], EXPECTED [3]
    int64_t* cnt_b = nullptr;           // ENUM_COUNT [items] balanced per item
    int64_t* cnt_u = nullptr;           // ENUM_COUNT [items] unbalanced per item
    const int64_t* off_b = nullptr;     // ENUM_FILL [items] output offsets
    const int64_t* off_u = nullptr;
    int32_t* out_bal = nullptr;
    int32_t* out_unbal = nullptr;
    int which = UTRI_BOTH;
    int64_t lb = 0;                     // first enumeration slot of the heavy items (set at launch)
    unsigned long long* qctr = nullptr; // two work-queue counters, zeroed per launch
    // oriented-row packing (set at launch from the graph)
    uint32_t idmask = 0x7FFFFFFFu;
    int idbits = 31;
    int mb = 0;
    // SIGN: per-edge negative-sign masks [m][ww] (bit b of word j: world 32 j + b), the
    // oriented rows' edge ids, and the per-world counters
    const int32_t* o_eid = nullptr;
    const uint32_t* masks = nullptr;
    int ww = 0;
    unsigned long long* wcount = nullptr;
    uint32_t sign_flush_at = 65535;  // additions between counter flushes (<= 2^16 - 1)
    // symmetric rows: the partner lists of the walk items (set at launch), and the kept
    // prefix length of each vertex's symmetric row
    const int64_t* s_off = nullptr;
    const int32_t* s_adj = nullptr;
    const double* s_d = nullptr;
    const int32_t* s_eid = nullptr;
    const int32_t* slen = nullptr;
    int order = 0;                      // UTRI_ORDER_* (set at launch)
    WalkTune tune;                      // work-chunk and tile sizes (set at launch)
    const int32_t* o_adj = nullptr;     // packed oriented rows (set at launch)
};

// Negative-sign masks of `ww` words per edge (worlds 32 ww) for the sign-world walk.
int utri_sign_masks_launch(utri_graph* g, uint64_t seed, int ww, uint32_t* masks, hipStream_t s);

int utri_walk_launch(utri_graph* g, int mode, const WalkParams& wp, const int64_t* items,
                     const int64_t* n_items_dev, const int32_t* len, int64_t n_items_host_bound,
                     hipStream_t s);

struct SampleParams {
    const double* cvals = nullptr;  // sorted thresholds, nt of them
    int nt = 0;
    double cmin = 0.0;
    uint64_t seed = 0;
    const uint64_t* seed_dev = nullptr;  // if set, the seed is read from device memory
    int64_t k = 0;
    int32_t worlds = 0;
    int chunk = 128;                // draws per group item
    unsigned long long* hist = nullptr;  // [worlds][2][nt+1]
    // vertex sampling: draw t is the edge record vrec[t] (edge | world << 32) of a sampled
    // vertex's prefix instead of a Philox-drawn edge
    const int64_t* vrec = nullptr;
    // draws of one pass grouped by the probed endpoint (set by utri_sample_prepare)
    int64_t t0 = 0, t1 = 0;              // flat draw range [t0, t1), t = world * k + i
    const int64_t* rec = nullptr;        // edge | world << 32, grouped by probed endpoint
    const int64_t* goff = nullptr;       // [n+1] group offsets into rec
    const int64_t* items = nullptr;      // work-group, wave and hub items: y | sub << 32
    const int64_t* nitems = nullptr;     // device: # work-group, # wave, # hub items
    int64_t wave_base = 0;               // first wave item in items
    int64_t hub_base = 0;                // first hub item in items
    unsigned long long* qctr = nullptr;  // ten work-queue counters, zeroed per pass
};

int utri_sym_prepare(utri_graph* g, double c_rows, hipStream_t s, int32_t** slen);
// Group the draws [t0, t1) by probed endpoint and build the pass's items into sp.
int utri_sample_prepare(utri_graph* g, SampleParams& sp, const int32_t* slen, int64_t t0,
                        int64_t t1, hipStream_t s);
int utri_sample_launch(utri_graph* g, const SampleParams& sp, const int32_t* slen, hipStream_t s);
// Vertex sampling: draw the worlds * k vertices, expand each into the edge records of its
// Lemma-2 prefix (sp.vrec) and return their number (one host synchronisation).
int utri_vertex_prepare(utri_graph* g, SampleParams& sp, const int32_t* slen, hipStream_t s,
                        int64_t* n_records);
int utri_vertex_local_launch(utri_graph* g, const double* cvals, const int32_t* order, int nt,
                             const int64_t* vids, int64_t k, int64_t* out, hipStream_t s);
// Top-k: s of each listed triangle with its sort key (ascending s, or descending when
// desc), then the first r entries of the sorted order.
int utri_topk_keys_launch(utri_graph* g, const int32_t* tri, int64_t N, int desc, double* sv,
                          uint64_t* key, uint32_t* idx, hipStream_t s);
int utri_topk_gather_launch(const int32_t* tri, const double* sv, const uint32_t* idx, int64_t r,
                            int32_t* out_tri, double* out_s, hipStream_t s);
int utri_batch_launch(utri_graph* g, const WalkParams& wp, const int64_t* items,
                      const int64_t* n_items_dev, const int32_t* len, int64_t n_items_bound,
                      const SampleParams& sp, const int32_t* slen, hipStream_t s);
int utri_finalize_launch(const unsigned long long* hist, int rows, int nt, const int32_t* order,
                         int64_t m, int64_t k, int64_t* counts_out, double* est_out,
                         hipStream_t s, int div = 1);
int utri_edge_local_launch(utri_graph* g, const double* cvals, const int32_t* order, int nt,
                           const int64_t* eids, int64_t k, int64_t* out, hipStream_t s);
int64_t utri_walk_items_bound(utri_graph* g);
// Whether run-time walk launch parameters fit the compiled table geometry.
bool utri_walk_tune_ok(const WalkTune& t);
// Ids the plain forward iteration streams per kept edge at the last prepared query.
int utri_walk_plain_ratio(utri_graph* g, hipStream_t s, double* ratio);
// Upper bound of the scratch bytes one counting query requests (row prefixes, work items,
// counters, scan partials, accumulators), with `align` bytes of padding per buffer.
int64_t utri_count_scratch_bound(const utri_graph* g, int64_t align);
int utri_grad_launch(utri_graph* g, double* grad, hipStream_t s);

// generic helpers
int utri_fill_u64(void* p, uint64_t v, int64_t count, hipStream_t s);
int utri_exclusive_scan_i32_to_i64(utri_graph* g, const int32_t* in, int64_t* out, int64_t n,
                                   hipStream_t s);
int utri_exclusive_scan_i64(utri_graph* g, const int64_t* in, int64_t* out, int64_t n,
                            hipStream_t s);
// graph-capture-safe exclusive scans (kernels only); *total optional, device memory
int utri_scan_i32(utri_graph* g, const int32_t* in, int64_t* out, int64_t n, int64_t* total,
                  hipStream_t s);
int utri_scan_i64(utri_graph* g, const int64_t* in, int64_t* out, int64_t n, int64_t* total,
                  hipStream_t s);
int utri_load_internal(const int64_t* src, const int64_t* dst, const double* p, int64_t m_in,
                       int64_t n, int ptr_kind, hipStream_t s, utri_graph** out);
int utri_set_p_internal(utri_graph* g, const double* p, int ptr_kind, hipStream_t s);
void utri_free_graph_internal(utri_graph* g);
