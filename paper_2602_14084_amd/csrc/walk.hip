// walk.hip -- the triangle walk: forward edge iteration over the degree-oriented graph
// (Algorithm "Baseline UBTE/UBTC", Section 4) with the probability pruning of Section 5.
//
// For every oriented edge u -> v and every w in N+(u) ∩ N+(v) the triangle (u, v, w)
// is visited exactly once (Node Order, Section 4). Rows are stored in Absolute Edge
// Order, so Lemma 2 (every triangle through an edge with |d| < c is unclassifiable)
// reduces each row to a prefix of length len[x]; the optional Lemma-3 cut shortens the
// streamed row further, per pair, to the entries whose |d| times |d| of the pair's edge
// times the largest |d| of the staged row (chunk) is at least c.
//
// Which row is streamed: for the oriented edge u -> v the triangles are the w in
// N+(u) ∩ N+(v), and the intersection can be taken by staging either row as a hash table
// and streaming the other through it. When the kept rows are long (see stream_shorter)
// the walk streams the shorter kept row (ties: N+(v), the plain forward iteration), which
// on R-MAT s23 streams 2.5x fewer ids than always streaming N+(v); otherwise it streams
// N+(v). A work item is a vertex x with its kept row N+(x) staged and a range of its kept
// symmetric row as partners y: y's row N+(y) is streamed through the table when the edge
// {x, y} is streamed from x's side (see k_items).
//
// GPU mapping (persistent grid, two phases per work-group, atomic work queues):
//   * long staged rows (len > cap): one work-group per item (x, chunk of caph entries,
//     partner range); the chunk of N+(x) is staged in a work-group LDS table and the
//     work-group's waves take the partners round-robin (on R-MAT s23 these items carry
//     98% of the streamed ids);
//   * other staged rows: one wave per item, the row staged in the wave's own table.
//   cap (at most CAP = 128), caph (at most CAPH = 2048), the partners per item, the loads
//   in flight and the shorter-row crossover are run-time launch parameters (WalkTune) that
//   the autotuner picks per graph; the defaults are 128, 2048, 1024, 8 and 320.
//   A table is open addressing over buckets of four slots with two parallel arrays: the
//   staged ids (0 = empty) and, per slot, a word holding the entry's d code, its position
//   in the row and a presence bit. A probe reads one bucket of each with two 16-byte LDS
//   loads from one address and selects the matching slot's word with four compares; at
//   the tables' load (at most two entries per bucket on average, one for rows up to half
//   the capacity) almost every probe ends in its home bucket. A streamed row is read with
//   buffer loads whose descriptor spans exactly the row, so lanes past its end get 0 (an
//   id in no table) without a bounds test; each lane has up to eight loads in flight.
//   Hits are classified from the d codes (staged word and streamed word) with two 24-bit
//   products against per-row integer thresholds; only the few the codes leave undecided
//   read the exact d values. The classify, count, histogram, fixed-point, enumeration,
//   sign-world and statistics epilogues are selected at compile time.
//
// Sign worlds (possible-world Monte-Carlo of E): every triangle's three edge ids go to a
// per-wave LDS queue; a full queue is drained with lanes over world words (world
// 32 j + b is bit b of mask word j): the balanced worlds of a triangle are the zero bits
// of the XOR of its three negative-sign masks, added into per-lane bit-sliced counters
// (SIGN_K bit planes in registers) that are flushed to the per-world totals when they
// could overflow and when the wave ends.
#include <algorithm>

#include "walk_common.h"

using namespace utri_dev;

namespace {

#ifndef UTRI_WALK_CAPH
#define UTRI_WALK_CAPH 2048
#endif
#ifndef UTRI_WALK_WAVE_LG
#define UTRI_WALK_WAVE_LG 7
#endif
constexpr int CAPH = UTRI_WALK_CAPH;  // most entries of one work-group table chunk
constexpr int NW_MAX = 8;             // enumeration slots per heavy item (one per wave)
constexpr int WAVE_LG = UTRI_WALK_WAVE_LG;  // wave tables: 2^WAVE_LG buckets of 4 slots
static_assert(CAP <= (4 << WAVE_LG), "wave tables hold CAP entries");
static_assert(CAPH < 32768, "positions are 15-bit in the table words");

#ifndef UTRI_WALK_NW
#define UTRI_WALK_NW 8             // waves per work-group of the counting walks
#endif
#ifndef UTRI_WALK_LGH
#define UTRI_WALK_LGH 10           // log2 of the work-group table's buckets
#endif
#ifndef UTRI_WALK_UNR_MAX
#define UTRI_WALK_UNR_MAX 8        // loads in flight per lane on long streamed rows
#endif
#ifndef UTRI_WALK_SHORTER
#define UTRI_WALK_SHORTER 1        // 1: each edge streams the shorter kept row; 0: always N+(v)
#endif

// Launch geometry of a walk kernel: NW waves per work-group, a work-group table of 2^LGH
// buckets and wave tables of 2^WLG buckets, four slots per bucket.
template <int NW_, int LGH_, int WLG_>
struct Geom {
    static constexpr int NW = NW_;
    static constexpr int TPBW = NW_ * UTRI_WAVE;
    static constexpr int LGH = LGH_;
    static constexpr int WLG = WLG_;
};
using GeomWalk = Geom<UTRI_WALK_NW, UTRI_WALK_LGH, WAVE_LG>;  // the standalone walks
using GeomBatch = Geom<WPB, 10, 7>;  // the fused batch (the sampler's block size)
static_assert(UTRI_WALK_NW <= NW_MAX && WPB <= NW_MAX, "enumeration slots");

inline int blocks_for(int64_t n) { return (int)((n + TPB - 1) / TPB); }

// A table keeps, per slot, the staged id (0 = empty) and a word: sign of d_uw in bit 31,
// QB = 15 magnitude bits of |d_uw| (floor(|d_uw| * 2^15), at most 2^15 - 1, from the exact
// d at staging) in bits 16..30, a presence bit (bit 15, so a word is never 0) and the
// entry's position in the staged chunk in bits 0..14.
constexpr int QB = 15;
constexpr uint32_t W_PRESENT = 1u << 15;
constexpr uint32_t W_POS = (1u << 15) - 1u;

template <class G>
struct WaveTab {
    alignas(16) uint32_t key[4 << G::WLG];
    alignas(16) uint32_t word[4 << G::WLG];
};
template <class G>
struct BlockTab {
    alignas(16) uint32_t key[4 << G::LGH];
    alignas(16) uint32_t word[4 << G::LGH];
};
template <class G>
union WalkShared {
    WaveTab<G> wave[G::NW];
    BlockTab<G> block;
};

// Table of a staged chunk: key array (its word array follows at WOFF slots), bucket mask,
// where the staged entries sit in o_adj / o_d, perm[u] (enumeration) and the chunk index.
struct TabRef {
    const uint32_t* key;
    uint32_t bmask;
    int64_t src_base;
    int32_t pu;
    int chunk;
};

// log2 of the bucket count for cl staged entries: 2^lg >= 2 cl (at most two entries per
// bucket of four on average), at least 2 buckets, at most 2^max_lg
__device__ __forceinline__ int tab_lg(int cl, int max_lg) {
    int lg = 1;
    while (lg < max_lg && (1 << lg) < 2 * cl) lg++;
    return lg;
}

// Clear the first 2^lg buckets of a table (keys and words).
template <int WOFF>
__device__ __forceinline__ void tab_clear(uint32_t* key, int lg, int tid, int nth) {
    const int n4 = 1 << lg;  // buckets = uint4 stores per array
    uint4* k4 = reinterpret_cast<uint4*>(key);
    uint4* w4 = reinterpret_cast<uint4*>(key + WOFF);
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    for (int i = tid; i < n4; i += nth) {
        k4[i] = z;
        w4[i] = z;
    }
}

// Stage cl entries o_adj[base ..] / o_d[base ..] (ids of at least 1) into a table of
// bmask + 1 buckets: each entry takes the first free slot from its home bucket (its id's
// low bits: ids rank vertices by degree with ties broken by a mixed id, so they spread
// over the buckets) onwards; slots of a bucket fill in order, so a bucket whose last key
// is 0 has room and ends a probe.
template <int WOFF>
__device__ __forceinline__ void tab_stage(uint32_t* key, const int32_t* __restrict__ o_adj,
                                          const double* __restrict__ o_d, int64_t base, int cl,
                                          uint32_t bmask, int tid, int nth, uint32_t idmask) {
    for (int j = tid; j < cl; j += nth) {
        const uint32_t pw = (uint32_t)o_adj[base + j];
        const uint32_t id = pw & idmask;
        const double d = o_d[base + j];
        // floor (exact: a power-of-two scaling), |d| = 1 clamped into the top code
        const uint32_t q = min((uint32_t)(fabs(d) * (double)(1u << QB)), (1u << QB) - 1u);
        const uint32_t word = (d < 0.0 ? 0x80000000u : 0u) | (q << 16) | W_PRESENT | (uint32_t)j;
        uint32_t b = id & bmask;
        for (;;) {
            int s = 0;
            while (s < 4 && atomicCAS(&key[4 * b + s], 0u, id) != 0u) s++;
            if (s < 4) {
                key[WOFF + 4 * b + s] = word;
                break;
            }
            b = (b + 1) & bmask;
        }
    }
}

// The word of id w, 0 if absent. Lanes past a streamed row's end probe w = 0, which only
// matches empty slots, whose words are 0. tab_bucket looks in one bucket (full: its last
// slot is taken, so w may lie further on).
template <int WOFF>
__device__ __forceinline__ uint32_t tab_bucket(const uint32_t* key, uint32_t b, uint32_t w,
                                               bool& full) {
    const uint4 k = *reinterpret_cast<const uint4*>(key + 4 * b);
    const uint4 d = *reinterpret_cast<const uint4*>(key + WOFF + 4 * b);
    uint32_t r = (k.w == w) ? d.w : 0u;
    r = (k.z == w) ? d.z : r;
    r = (k.y == w) ? d.y : r;
    r = (k.x == w) ? d.x : r;
    full = k.w != 0u;
    return r;
}

template <int WOFF>
__device__ __forceinline__ uint32_t tab_find(const uint32_t* key, uint32_t bmask, uint32_t w) {
    uint32_t b = w & bmask;
    bool full;
    uint32_t r = tab_bucket<WOFF>(key, b, w, full);
    // a full bucket without w sends the lane on to the next one (rare: the tables hold at
    // most half an entry per bucket)
    if (__builtin_expect(r == 0u && full, 0)) {
        do {
            b = (b + 1) & bmask;
            r = tab_bucket<WOFF>(key, b, w, full);
        } while (r == 0u && full);
    }
    return r;
}

// Items. Every vertex x with a kept oriented row of len >= 2 stages (chunks of) N+(x) as a
// table and streams, for each partner y (a kept neighbour of x, in ranges of pr entries of
// the symmetric row), the kept row N+(y) through it. Each kept edge {x, y} is streamed
// from exactly one side: the shorter kept row goes through the longer one's table (ties:
// the row of the higher-ranked end through the lower one's table, as in the plain forward
// iteration). Either way w runs over N+(u) ∩ N+(v) for the oriented edge u -> v, so the
// triangles visited are those of Section 4, once each. Item word: vertex in bits 0-30,
// table chunk in bits 32-42, partner range in bits 43-63.
//   light items: 2 <= len <= cap, one per partner range;
//   heavy items: len > cap, one per (chunk of caph entries, partner range).
__host__ __device__ inline int64_t item_word(int64_t v, int64_t chunk, int64_t range) {
    return (int64_t)(((uint64_t)range << 43) | ((uint64_t)chunk << 32) | (uint64_t)v);
}
__device__ inline int item_vertex(int64_t it) { return (int)(it & 0x7FFFFFFF); }
__device__ inline int item_chunk(int64_t it) { return (int)(((uint64_t)it >> 32) & 0x7FF); }
__device__ inline int item_range(int64_t it) { return (int)((uint64_t)it >> 43); }
constexpr int64_t MAX_CHUNKS = 2048;
__host__ __device__ inline int partner_ranges(int32_t sl, int pr) {
    return sl > pr ? (int)(((int64_t)sl + pr - 1) / pr) : 1;
}

// Streaming the shorter row pays when the rows the plain forward iteration streams are
// long: it then skips most of their strips, while scanning both ends' symmetric rows for
// partners costs about the same per edge either way. When the plain iteration would
// stream fewer than tune.shorter_min ids per kept edge on average, and for the sign-world
// walk (whose mask reads follow the staged row), items stream N+(v) for the v of their
// own row (only the first partner range of an item has work then).
// The two totals are accumulated in KEPT_SLOTS slot pairs, 128 bytes apart, after the
// four item counters (atomics on one address serialise).
constexpr int KEPT_SLOTS = 64;
constexpr int KEPT_STRIDE = 16;  // int64 per slot pair
constexpr int NITEMS_WORDS = 4 + KEPT_SLOTS * KEPT_STRIDE;

template <int MODE>
__device__ inline bool stream_shorter(const WalkParams& wp, const int64_t* n_items_dev) {
    if (!UTRI_WALK_SHORTER || MODE == WALK_SIGN || wp.order == UTRI_ORDER_PLAIN) return false;
    if (wp.order == UTRI_ORDER_SHORTER) return true;
    int64_t kept = 0, plain = 0;
    for (int i = 0; i < KEPT_SLOTS; i++) {
        kept += n_items_dev[4 + i * KEPT_STRIDE];
        plain += n_items_dev[5 + i * KEPT_STRIDE];
    }
    return (double)plain >= (double)wp.tune.shorter_min * (double)kept;
}

// Bounds of the two item lists (a kept symmetric row of sl entries has at most
// 1 + sl / pr ranges; the symmetric rows hold 2m entries).
inline int64_t chunks_bound(const utri_graph* g) {
    const int64_t caph = g->walk_tune.caph;
    return (g->max_out + caph - 1) / caph + 1;
}
inline int64_t light_bound(const utri_graph* g) {
    return std::min<int64_t>(g->n, g->m / 2) + 2 * g->m / g->walk_tune.pr + 1;
}
inline int64_t heavy_bound(const utri_graph* g) {
    const WalkTune& t = g->walk_tune;
    return g->m / t.caph + g->m / t.cap + chunks_bound(g) * (g->m / t.cap + 2 * g->m / t.pr + 1) + 2;
}

}  // namespace

// Whether run-time launch parameters fit the compiled table geometry.
bool utri_walk_tune_ok(const WalkTune& t) {
    const auto pow2 = [](int64_t x) { return x > 0 && (x & (x - 1)) == 0; };
    return t.pr >= UTRI_WAVE && t.pr <= (1 << 20) && t.pr % UTRI_WAVE == 0 && pow2(t.cap) &&
           t.cap >= 8 && t.cap <= CAP && pow2(t.caph) && t.caph >= std::max(t.cap, 256) &&
           t.caph <= CAPH &&
           (t.unr == 1 || t.unr == 2 || t.unr == 4 || t.unr == 8) && t.shorter_min >= 0 &&
           t.shorter_min <= ((int64_t)1 << 40);
}

namespace {

// Kept prefixes at c of the oriented row (len) and of the symmetric row (slen) of each
// vertex, and its light and heavy item counts. Over the slot pairs, kept[.][0] sums to the
// kept oriented edges and kept[.][1] to the sum over v of (kept in-edges of v) * len(v):
// the ids the plain forward iteration would stream.
__device__ __forceinline__ int32_t kept_prefix(const int64_t* __restrict__ off,
                                               const double* __restrict__ dd, int64_t v, double c) {
    const int64_t a = off[v], b = off[v + 1];
    int64_t lo = a, hi = b;
    if (c > 0.0) {
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (fabs(dd[mid]) >= c) lo = mid + 1; else hi = mid;
        }
    } else {
        lo = b;
    }
    return (int32_t)(lo - a);
}

// Also writes rinfo[v] = (start of N+(v) in o_adj, kept length | q << 16): what a partner
// scan reads about each partner, in one 8-byte load (m < 2^31, so row starts fit 32 bits,
// and an oriented row has fewer than 2^16 entries); q = floor(|d| * 2^16) of the kept
// row's last entry, a lower bound of every kept |d| that lets the Lemma-3 cut skip the
// row end's exact d when the bound already keeps the whole row.
__global__ void k_rowlen(const int64_t* __restrict__ off, const double* __restrict__ dd,
                         const int64_t* __restrict__ soff, const double* __restrict__ sd,
                         int64_t n, double c, int32_t* __restrict__ len,
                         int32_t* __restrict__ slen, int32_t* __restrict__ lcnt,
                         int32_t* __restrict__ hcnt, unsigned long long* __restrict__ kept,
                         uint2* __restrict__ rinfo, int cap, int caph, int pr, int lemma3) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t L = 0, SL = 0;
    if (v < n) {
        L = kept_prefix(off, dd, v, c);
        SL = kept_prefix(soff, sd, v, c);
    }
    // one atomic per work-group for each total, into one of KEPT_SLOTS slot pairs
    __shared__ uint64_t part[2][TPB / UTRI_WAVE];
    const uint64_t tl = utri_wave_sum_u64((uint64_t)L);
    const uint64_t tw = utri_wave_sum_u64((uint64_t)(SL - L) * (uint64_t)L);
    if (utri_lane() == 0) {
        part[0][threadIdx.x / UTRI_WAVE] = tl;
        part[1][threadIdx.x / UTRI_WAVE] = tw;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t a = 0, b = 0;
        for (int i = 0; i < TPB / UTRI_WAVE; i++) { a += part[0][i]; b += part[1][i]; }
        unsigned long long* k = kept + (blockIdx.x % KEPT_SLOTS) * KEPT_STRIDE;
        if (a) atomicAdd(&k[0], (unsigned long long)a);
        if (b) atomicAdd(&k[1], (unsigned long long)b);
    }
    if (v >= n) return;
    len[v] = L;
    slen[v] = SL;
    uint32_t q = 0;
    if (lemma3 && L > 0) q = min((uint32_t)(fabs(dd[off[v] + L - 1]) * 65536.0), 65535u);
    rinfo[v] = make_uint2((uint32_t)off[v], (uint32_t)L | (q << 16));
    const int nr = partner_ranges(SL, pr);
    lcnt[v] = (L >= 2 && L <= cap) ? nr : 0;
    hcnt[v] = (L > cap) ? ((L + caph - 1) / caph) * nr : 0;
}

__global__ void k_items(const int32_t* __restrict__ lcnt, const int32_t* __restrict__ hcnt,
                        const int32_t* __restrict__ slen, const int64_t* __restrict__ loff,
                        const int64_t* __restrict__ hoff, int64_t n, int64_t hbase,
                        int64_t* __restrict__ items, int pr) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int nl = lcnt[v];
    for (int r = 0; r < nl; r++) items[loff[v] + r] = item_word(v, 0, r);
    const int nh = hcnt[v];
    if (nh == 0) return;
    const int nr = partner_ranges(slen[v], pr);
    const int64_t o = hbase + hoff[v];
    for (int k = 0; k < nh; k++) items[o + k] = item_word(v, k / nr, k % nr);
}

constexpr int SIGN_K = 16;   // bit planes of the sign-world counters (flush before 2^16)
constexpr int SIGN_Q = 128;  // triangles queued per wave

struct WalkLaneState {
    uint64_t nb = 0, nu = 0;       // COUNT / ENUM_COUNT
    uint32_t nb32 = 0, nu32 = 0;   // COUNT / ENUM_COUNT within one item: balanced, classified
    uint64_t tri = 0;              // EXPECTED / STATS
    uint64_t slo = 0;              // EXPECTED: sum of low 32 bits of each fixed-point term
    int64_t shi = 0;               // EXPECTED: sum of the terms shifted right by 32
    uint64_t wt = 0, wt_all = 0;   // STATS: streamed target elements (first chunk / all)
    uint32_t bs[SIGN_K] = {};      // SIGN: bit planes of this lane's 32 world counters
    uint32_t npass = 0;            // SIGN: additions since the last flush (wave-uniform)
    int qn = 0;                    // SIGN: queued triangles (wave-uniform)
    int dn = 0;                    // COUNT / ENUM_*: hits queued (wave-uniform)
};

// SIGN: per-wave queue of triangles as their three edge ids
struct SignQueue {
    int32_t e[3][SIGN_Q];
};
constexpr int SIGN_NW = 4;  // waves per work-group of the sign-world walk
__shared__ SignQueue sign_q[SIGN_NW];

// Add this lane's 32 counters into the per-world totals and clear them.
__device__ __forceinline__ void sign_flush(const WalkParams& wp, WalkLaneState& st) {
    const int wd = utri_lane() % wp.ww;
    for (int b = 0; b < 32; b++) {
        uint32_t v = 0;
#pragma unroll
        for (int i = 0; i < SIGN_K; i++) v |= ((st.bs[i] >> b) & 1u) << i;
        if (v) atomicAdd(&wp.wcount[wd * 32 + b], (unsigned long long)v);
    }
#pragma unroll
    for (int i = 0; i < SIGN_K; i++) st.bs[i] = 0;
    st.npass = 0;
}

// Count the queued triangles into the lanes' counters and empty the queue. Lane l takes
// word l % ww of triangle l / ww of each group of 64 / ww triangles.
__device__ __forceinline__ void sign_drain(const WalkParams& wp, WalkLaneState& st) {
    SignQueue& Q = sign_q[threadIdx.x / UTRI_WAVE];
    const int lane = utri_lane();
    const int ww = wp.ww;
    const int tp = UTRI_WAVE / ww;
    const int ti = lane / ww, wd = lane % ww;
    utri_wave_sync();
    for (int b0 = 0; b0 < st.qn; b0 += tp) {
        const int t = b0 + ti;
        uint32_t c = 0;
        if (t < st.qn) {
            const uint32_t x = wp.masks[(int64_t)Q.e[0][t] * ww + wd] ^
                               wp.masks[(int64_t)Q.e[1][t] * ww + wd] ^
                               wp.masks[(int64_t)Q.e[2][t] * ww + wd];
            c = ~x;  // worlds with an even number of negative edges
        }
        // ripple-carry add of the 32 one-bit values into the bit planes
#pragma unroll
        for (int i = 0; i < SIGN_K; i++) {
            if (__ballot(c != 0) == 0) break;
            const uint32_t carry = st.bs[i] & c;
            st.bs[i] ^= c;
            c = carry;
        }
        if (++st.npass >= wp.sign_flush_at) sign_flush(wp, st);
    }
    st.qn = 0;
    utri_wave_sync();
}

// Per-row integer thresholds of the code decision. With A = |d_uv|, qb the 15-bit code of
// |d_uw| (table word) and qc the mb-bit code of |d_vw| (streamed word), |s| lies in
// [A * P0, A * P1] * 2^-(15 + mb) with P0 = qb * qc and P1 = (qb + 1) * (qc + 1). With
// K = c * 2^(15 + mb) / A:
//   P0 >= khi = floor(K (1 + 2^-40)) + 1   =>  |s| > c  (balanced if s < 0, else unbalanced)
//   P1 <= klo = floor(K (1 - 2^-40))       =>  |s| < c  (neither)
// The 2^-40 margins exceed the roundings of K and the 2^-51 gap between the real product
// and the FP64 s of the exact rule, so exact ties always go to the exact rule. A = 0 rows
// are left to the exact rule. rsign holds sign(d_uv) in bit 31, so bit 31 of (table word
// ^ streamed word ^ rsign) is sign(s).
struct CodeRow {
    uint32_t khi, klo, rsign;
};

__device__ __forceinline__ CodeRow code_row(const WalkParams& wp, double duv) {
    CodeRow r;
    const double a = fabs(duv);
    r.rsign = duv < 0.0 ? 0x80000000u : 0u;
    if (!(a > 0.0) || wp.mb == 0) {
        r.khi = 0xFFFFFFFFu;
        r.klo = 0u;
        return r;
    }
    const double K = ldexp(wp.c, QB + wp.mb) / a;
    const double hi = floor(K * (1.0 + 0x1p-40)) + 1.0;
    const double lo = floor(K * (1.0 - 0x1p-40));
    r.khi = hi >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)hi;
    r.klo = lo >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)lo;
    return r;
}

// Hits the codes leave undecided (counting walks): queued per wave as (position of d_vw in
// o_d, staged position | partner slot << 15) and decided by the exact rule in batches, so
// a wave waits for their d loads once per batch instead of once per strip. The queue is
// drained between partner rows once it holds more than DQ_DRAIN entries and whenever the
// partners' d values (registers of the current batch of 64 partners) are about to change;
// a strip whose hits do not fit decides them at once.
constexpr int DQ_CAP = 96;
constexpr int DQ_DRAIN = 48;
struct DeferQueue {
    uint32_t vw[DQ_CAP];
    uint32_t ps[DQ_CAP];
};
__shared__ DeferQueue defer_q[NW_MAX];

// Decide the queued hits exactly and count them; duv_lanes: d_xy of the batch's partners
// on their lanes, src_base: position of the staged chunk in o_d.
__device__ __forceinline__ void defer_drain(const WalkParams& wp, const double* __restrict__ o_d,
                                            int64_t src_base, double duv_lanes, WalkLaneState& st) {
    DeferQueue& Q = defer_q[threadIdx.x / UTRI_WAVE];
    utri_wave_sync();
    for (int e0 = 0; e0 < st.dn; e0 += UTRI_WAVE) {
        const int e = e0 + utri_lane();
        const bool live = e < st.dn;
        const uint32_t ps = live ? Q.ps[e] : 0u;
        const uint32_t vw = live ? Q.vw[e] : 0u;
        const double duv = __shfl(duv_lanes, (int)(ps >> 15), UTRI_WAVE);
        if (live) {
            const double s = utri_tri_s(duv, o_d[src_base + (ps & W_POS)], o_d[vw]);
            st.nb32 += (s <= -wp.c) ? 1u : 0u;
            st.nu32 += (s <= -wp.c || s > wp.c) ? 1u : 0u;
        }
    }
    st.dn = 0;
    utri_wave_sync();
}

// The fill walk queues its hits per wave, in probe order, as (id of w, its class) or, for
// a hit the codes leave undecided, (position of d_vw, class 3), and writes them in
// batches: a wave waits for the permutation loads of its triangles' third vertex (and the
// d loads of the undecided ones) once per batch instead of once per strip. Written in
// queue order, the lists keep the order in which the strips were probed. Queue words:
// vw = id of w or position of d_vw; ps = staged position | partner slot << 15 |
// class << 21 (1 balanced, 2 unbalanced, 3 undecided).
constexpr uint32_t FQ_BAL = 1u, FQ_UNBAL = 2u, FQ_UND = 3u;
// A full queue is drained 64 entries at a time (the rest move to the front), so every
// batch but an item's last fills the wave. 120 entries keep the fill walk's work-group
// within a quarter of the LDS.
constexpr int FQ_CAP = 120;
struct FillQueue {
    uint32_t vw[FQ_CAP];
    uint32_t ps[FQ_CAP];
};
__shared__ FillQueue fill_q[NW_MAX];

// pv_lanes / duv_lanes: original id of y and d_xy of the batch's partners on their lanes;
// all: drain every entry (else the first 64 when there are that many).
__device__ __forceinline__ void fill_drain(const WalkParams& wp, const double* __restrict__ o_d,
                                           const int32_t* __restrict__ perm, int64_t src_base,
                                           int32_t pu, int32_t pv_lanes, double duv_lanes,
                                           WalkLaneState& st, int64_t& run_b, int64_t& run_u,
                                           bool all) {
    FillQueue& Q = fill_q[threadIdx.x / UTRI_WAVE];
    utri_wave_sync();
    const int take = (all || st.dn < UTRI_WAVE) ? st.dn : UTRI_WAVE;
    for (int e0 = 0; e0 < take; e0 += UTRI_WAVE) {
        const int e = e0 + utri_lane();
        const bool live = e < take;
        const uint32_t ps = live ? Q.ps[e] : 0u;
        const uint32_t vw = live ? Q.vw[e] : 0u;
        const int si = (int)((ps >> 15) & 63u);
        const uint32_t cls = ps >> 21;
        const double duv = __shfl(duv_lanes, si, UTRI_WAVE);
        const int32_t pv = __shfl(pv_lanes, si, UTRI_WAVE);
        bool is_b = cls == FQ_BAL, is_u = cls == FQ_UNBAL;
        uint32_t w = vw;
        if (cls == FQ_UND) {
            // the exact FP64 rule reads d_uw and d_vw
            w = (uint32_t)wp.o_adj[vw] & wp.idmask;
            const double s = utri_tri_s(duv, o_d[src_base + (ps & W_POS)], o_d[vw]);
            is_b = s <= -wp.c && (wp.which & UTRI_BAL);
            is_u = s > wp.c && (wp.which & UTRI_UNBAL);
        }
        const uint64_t mb_ = __ballot(is_b);
        const uint64_t mu_ = __ballot(is_u);
        if (is_b || is_u) {
            int32_t a = pu, b = pv, c = perm[w], t;
            if (b < a) { t = a; a = b; b = t; }
            if (c < b) { t = b; b = c; c = t; }
            if (b < a) { t = a; a = b; b = t; }
            const uint64_t lt = __lanemask_lt();
            int32_t* dst;
            int64_t slot;
            if (is_b) { dst = wp.out_bal; slot = run_b + __popcll(mb_ & lt); }
            else      { dst = wp.out_unbal; slot = run_u + __popcll(mu_ & lt); }
            dst[3 * slot] = a;
            dst[3 * slot + 1] = b;
            dst[3 * slot + 2] = c;
        }
        run_b += __popcll(mb_);
        run_u += __popcll(mu_);
    }
    // the entries left (at most FQ_CAP - 64) move to the front
    const int rest = st.dn - take;
    if (rest > 0) {
        const int e = utri_lane();
        uint32_t ps = 0u, vw = 0u;
        if (e < rest) { ps = Q.ps[take + e]; vw = Q.vw[take + e]; }
        utri_wave_sync();
        if (e < rest) { Q.ps[e] = ps; Q.vw[e] = vw; }
    }
    st.dn = rest;
    utri_wave_sync();
}

// Stream the kept target row [ovs, ovs + lvs) of v, probing every entry in the table.
// Row entries are packed words (id in the low idbits bits, mb-bit d code above, sign(d)
// in bit 31); table words carry the staged entry's code and position. si: the partner's
// slot in its batch of 64 (deferred hits); duv_lanes: the batch's d_xy on their lanes.
#ifndef UTRI_WALK_CODES
#define UTRI_WALK_CODES 1
#endif

// A buffer descriptor spanning exactly the kept row [ovs, ovs + lvs) of o_adj: loads at or
// past its end return 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const WalkParams& wp, int64_t ovs,
                                                           int lvs) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)(wp.o_adj + ovs), (short)0, lvs * 4,
                                             0x00020000);
}

template <int UNR>
__device__ __forceinline__ void load_strips(__amdgpu_buffer_rsrc_t rs, int j0, uint32_t (&pw)[UNR]) {
    const int lane = utri_lane();
#pragma unroll
    for (int k = 0; k < UNR; k++)
        pw[k] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, (j0 + k * UTRI_WAVE + lane) * 4,
                                                               0, 0);
}

// Probe the UNR loaded strips pw (row positions j0 + 64 k + lane) of the row [ovs, ovs + lvs)
// and apply the mode's epilogue to every hit.
template <int MODE, int UNR, int WOFF>
__device__ __forceinline__ void probe_strips(const WalkParams& wp, const double* __restrict__ o_d,
                                             const int32_t* __restrict__ perm, const TabRef& R,
                                             const uint32_t (&pw)[UNR], int j0, int64_t ovs,
                                             int lvs, double duvs, int32_t pv, const CodeRow& cr,
                                             int si, double duv_lanes, HistLds* H,
                                             WalkLaneState& st, int64_t& run_b, int64_t& run_u) {
    const int lane = utri_lane();
    constexpr bool kCoded = UTRI_WALK_CODES && (MODE == WALK_COUNT || MODE == WALK_ENUM_COUNT ||
                                                MODE == WALK_ENUM_FILL);
    constexpr bool kDefer = MODE == WALK_COUNT || MODE == WALK_ENUM_COUNT;
    const uint32_t qm = (1u << wp.mb) - 1u;
    const double* rowd = o_d + ovs;
    {
#pragma unroll
        for (int k = 0; k < UNR; k++) {
            // strips past the row end hold no entries (wave-uniform exit)
            if (k > 0 && j0 + k * UTRI_WAVE >= lvs) break;
            const int j = j0 + k * UTRI_WAVE + lane;
            const uint32_t w = pw[k] & wp.idmask;
            const uint32_t r = tab_find<WOFF>(R.key, R.bmask, w);
            const bool found = r != 0u;
            if (kDefer) {
                // classified hits are counted as (classified, of which s < 0: balanced); the
                // undecided ones are queued for the exact rule
                const uint32_t qb = __builtin_amdgcn_ubfe(r, 16, QB);
                const uint32_t qc = __builtin_amdgcn_ubfe(pw[k], wp.idbits, wp.mb);
                const uint32_t p0 = __umul24(qb, qc);
                const uint32_t t1 = p0 + qb + qc;  // (qb + 1)(qc + 1) - 1
                // khi >= 1, so an absent w (r = 0, qb = 0) is never classified
                const bool ccls = p0 >= cr.khi;
                const bool bal = ccls && (int32_t)(r ^ pw[k] ^ cr.rsign) < 0;
                st.nb32 += bal ? 1u : 0u;
                st.nu32 += ccls ? 1u : 0u;
                const bool und = found && !ccls && t1 >= cr.klo;
                const uint64_t um = __builtin_amdgcn_ballot_w64(und);
                if (um) {
                    // this lane's bit of the ballot (keeps und itself out of the branch)
                    const bool mine = (um >> lane) & 1ull;
                    const int nq = __popcll(um);
                    if (st.dn + nq <= DQ_CAP) {
                        if (mine) {
                            DeferQueue& Q = defer_q[threadIdx.x / UTRI_WAVE];
                            const int slot = st.dn + __popcll(um & __lanemask_lt());
                            Q.vw[slot] = (uint32_t)(ovs + j);
                            Q.ps[slot] = (r & W_POS) | ((uint32_t)si << 15);
                        }
                        st.dn += nq;
                    } else if (mine) {
                        const double s = utri_tri_s(duvs, o_d[R.src_base + (r & W_POS)], rowd[j]);
                        const uint32_t c = (s <= -wp.c || s > wp.c) ? 1u : 0u;
                        st.nb32 += (s <= -wp.c) ? 1u : 0u;
                        st.nu32 += c;
                    }
                }
            } else if (MODE == WALK_ENUM_FILL) {
                // pv: the partners' original ids on their lanes (see fill_drain)
                uint32_t cls = found ? FQ_UND : 0u;
                if (kCoded) {
                    const uint32_t qb = (r >> 16) & ((1u << QB) - 1u);
                    const uint32_t qc = (pw[k] >> wp.idbits) & qm;
                    const uint32_t p0 = __umul24(qb, qc);
                    const uint32_t t1 = p0 + qb + qc;  // (qb + 1)(qc + 1) - 1
                    const bool neg = (int32_t)(r ^ pw[k] ^ cr.rsign) < 0;
                    if (p0 >= cr.khi)
                        cls = !found ? 0u : neg ? ((wp.which & UTRI_BAL) ? FQ_BAL : 0u)
                                                : ((wp.which & UTRI_UNBAL) ? FQ_UNBAL : 0u);
                    else if (t1 < cr.klo)
                        cls = 0u;
                }
                const uint64_t qm_ = __ballot(cls != 0u);
                if (qm_) {
                    const int nq = __popcll(qm_);
                    if (st.dn + nq > FQ_CAP)
                        fill_drain(wp, o_d, perm, R.src_base, R.pu, pv, duv_lanes, st, run_b,
                                   run_u, false);
                    if (cls) {
                        FillQueue& Q = fill_q[threadIdx.x / UTRI_WAVE];
                        const int slot = st.dn + __popcll(qm_ & __lanemask_lt());
                        Q.vw[slot] = cls == FQ_UND ? (uint32_t)(ovs + j) : w;
                        Q.ps[slot] = (r & W_POS) | ((uint32_t)si << 15) | (cls << 21);
                    }
                    st.dn += nq;
                }
            } else if (MODE == WALK_STATS) {
                if (found) st.tri++;
            } else if (MODE == WALK_SIGN) {
                // queue this strip's triangles (pv carries the edge id of u -> v)
                const uint64_t hm = __ballot(found);
                if (hm) {
                    if (found) {
                        SignQueue& Q = sign_q[threadIdx.x / UTRI_WAVE];
                        const int slot = st.qn + __popcll(hm & __lanemask_lt());
                        Q.e[0][slot] = pv;
                        Q.e[1][slot] = wp.o_eid[R.src_base + (r & W_POS)];
                        Q.e[2][slot] = wp.o_eid[ovs + j];
                    }
                    st.qn += __popcll(hm);
                    if (st.qn >= SIGN_Q - UTRI_WAVE) sign_drain(wp, st);
                }
            } else if (found) {
                const double s = utri_tri_s(duvs, o_d[R.src_base + (r & W_POS)], rowd[j]);
                if (MODE == WALK_HIST) {
                    bool bal;
                    const int bin = thresh_bin(s, bal);
                    if (bin > 0) atomicAdd(&H->hist[bal ? 0 : 1][bin], 1ull);
                } else if (MODE == WALK_EXPECTED) {
                    const int64_t t = utri_fix62(s);
                    st.tri++;
                    st.slo += (uint64_t)(uint32_t)(t & 0xFFFFFFFFll);
                    st.shi += (t >> 32);
                }
            }
        }
    }
}

// Stream the kept target row [ovs, ovs + lvs) of v, UNR strips of loads in flight. q3 > 0
// (a row the Lemma-3 cut may shorten, see load_partners) stops the stream after the first
// batch of strips whose last entry has code q with q + 1 <= q3: that entry, and every later
// one (the row is in |d| order), fails the cut, and the triangles of the entries that fail
// it are unclassifiable, streamed or not. (Checking after every strip instead cuts more but
// was slower on R-MAT s23.)
template <int MODE, int UNR, int WOFF, bool L3>
__device__ __forceinline__ void stream_row(const WalkParams& wp, const double* __restrict__ o_d,
                                           const int32_t* __restrict__ perm, const TabRef& R,
                                           int64_t ovs, int lvs, double duvs, int32_t pv,
                                           const CodeRow& cr, int si, double duv_lanes, int q3,
                                           HistLds* H, WalkLaneState& st, int64_t& run_b,
                                           int64_t& run_u) {
    const __amdgpu_buffer_rsrc_t rs = row_rsrc(wp, ovs, lvs);
    int covered = lvs;
    for (int j0 = 0; j0 < lvs; j0 += UNR * UTRI_WAVE) {
        uint32_t pw[UNR];
        load_strips<UNR>(rs, j0, pw);  // all UNR loads are issued before any probe
        probe_strips<MODE, UNR, WOFF>(wp, o_d, perm, R, pw, j0, ovs, lvs, duvs, pv, cr, si,
                                      duv_lanes, H, st, run_b, run_u);
        if (L3 && q3 > 0 && j0 + UNR * UTRI_WAVE < lvs) {
            const uint32_t wl = (uint32_t)__builtin_amdgcn_readlane((int)pw[UNR - 1], UTRI_WAVE - 1);
            if ((int)((wl >> wp.idbits) & ((1u << wp.mb) - 1u)) + 1 <= q3) {
                covered = j0 + UNR * UTRI_WAVE;
                break;
            }
        }
    }
    if (MODE == WALK_STATS && utri_lane() == 0) {
        st.wt_all += (uint64_t)covered;
        if (R.chunk == 0) st.wt += (uint64_t)covered;
    }
}

template <int MODE, int WOFF, bool L3>
__device__ __forceinline__ void stream_any(const WalkParams& wp, const double* __restrict__ o_d,
                                           const int32_t* __restrict__ perm, const TabRef& R,
                                           int64_t ovs, int lvs, double duvs, int32_t pv,
                                           const CodeRow& cr, int si, double duv_lanes, int q3,
                                           HistLds* H, WalkLaneState& st, int64_t& run_b,
                                           int64_t& run_u) {
#if UTRI_WALK_UNR_MAX >= 8
    // the sign-world walk keeps its counter planes in registers, and the fill walk its
    // queue drain's: eight loads ahead would spill them
    if (MODE != WALK_SIGN && MODE != WALK_ENUM_FILL && lvs > 4 * UTRI_WAVE && wp.tune.unr >= 8)
        stream_row<MODE, 8, WOFF, L3>(wp, o_d, perm, R, ovs, lvs, duvs, pv, cr, si, duv_lanes, q3, H, st,
                                  run_b, run_u);
    else
#endif
    if (lvs > 2 * UTRI_WAVE && wp.tune.unr >= 4)
        stream_row<MODE, 4, WOFF, L3>(wp, o_d, perm, R, ovs, lvs, duvs, pv, cr, si, duv_lanes, q3, H, st,
                                  run_b, run_u);
    else if (lvs > UTRI_WAVE && wp.tune.unr >= 2)
        stream_row<MODE, 2, WOFF, L3>(wp, o_d, perm, R, ovs, lvs, duvs, pv, cr, si, duv_lanes, q3, H, st,
                                  run_b, run_u);
    else
        stream_row<MODE, 1, WOFF, L3>(wp, o_d, perm, R, ovs, lvs, duvs, pv, cr, si, duv_lanes, q3, H, st,
                                  run_b, run_u);
}

// Load, on lane l, partner y = entry sb + i0 + l * nparts + part of the kept symmetric row
// of x (np entries in this item's range; the waves of a work-group take every nparts-th
// partner) with the start of N+(y), the kept length of N+(y) this item streams (0 when the
// edge {x, y} is streamed from y's side, see k_items), d_xy and the edge id (sign worlds).
// PV: bit 0 = partners from the symmetric row (the shorter-row order), bit 1 = the
// Lemma-3 cut is applied (its code is compiled only into the kernels that use it).
template <int MODE, int PV>
__device__ __forceinline__ void load_partners(const WalkParams& wp, const int32_t* __restrict__ o_adj,
                                              const double* __restrict__ o_d,
                                              const uint2* __restrict__ rinfo, int x, int Lx,
                                              int64_t sb, int np, int i0, int part, int nparts,
                                              double dmax_chunk, int& y, int64_t& oy, int& ly,
                                              double& dxy, int32_t& exy, CodeRow& cr) {
    constexpr bool shorter = (PV & 1) != 0;
    const int i = i0 + utri_lane() * nparts + part;
    ly = 0; y = 0; oy = 0; dxy = 0.0; exy = 0;
    cr.khi = 0xFFFFFFFFu; cr.klo = 0u; cr.rsign = 0u;
    if (i < np) {
        // shorter: entry of x's kept symmetric row; else: entry of N+(x) itself
        y = shorter ? wp.s_adj[sb + i] : (int)((uint32_t)o_adj[sb + i] & wp.idmask);
        const uint2 ri = rinfo[y];
        const int L = (int)(ri.y & 0xFFFFu);
        const bool mine = !shorter || ((y > x) ? (L <= Lx) : (L < Lx));
        if (mine && L > 0) {
            dxy = shorter ? wp.s_d[sb + i] : o_d[sb + i];
            oy = (int64_t)ri.x;
            ly = L;
            if (PV & 2) {
                // Lemma 3 keeps w only if |d_yw| * P >= c (with slack), P = |d_xy| *
                // max|d_xw|. The row is in |d| order, so nothing is cut when its last entry
                // passes, and it passes when the lower bound of its |d| does (rounding is
                // monotonic). Otherwise ly carries, in bits 16 up, the code limit q3: an
                // entry with code q (|d| <= (q + 1) 2^-mb) and q + 1 <= q3 fails the cut,
                // since q3 <= c / P 2^mb - 2 keeps (q + 1) 2^-mb P below c by far more than
                // the rounding of the product; c / P 2^mb is taken in FP32 with a hardware
                // reciprocal, whose relative error (about 2^-21 in all) moves it by less
                // than one of the two units of margin (a P too small for the margin gives
                // q3 = 2^mb, and then every entry's |d| P <= P fails).
                const double P = __dmul_rn(fabs(dxy), dmax_chunk);
                const double lb = (double)(ri.y >> 16) * 0x1p-16;
                if (__dmul_rn(lb, P) < wp.c_l3) {
                    const float qf = __builtin_amdgcn_rcpf((float)P) * (float)wp.c_l3 *
                                     (float)(1 << wp.mb);
                    const float qd = floorf(qf) - 2.0f;
                    const int q3 = qd >= (float)(1 << wp.mb) ? (1 << wp.mb) : (qd > 0.0f ? (int)qd : 0);
                    ly |= q3 << 16;
                }
            }
            cr = code_row(wp, dxy);
            if (MODE == WALK_SIGN) exy = shorter ? wp.s_eid[sb + i] : wp.o_eid[sb + i];
        }
    }
}

// Counting walks: the partner rows of a batch that are at most one strip long are laid end
// to end and probed 64 entries per strip, instead of one strip (and one round of per-row
// broadcasts) each: at s23, t = 0.8, a third of the streamed rows are shorter than 64
// entries. Lane l of packed strip k takes position P = 64 k + l of the concatenation; its
// row is the partner r with the last start pre_r <= P (a binary search over the lanes'
// exclusive prefix sums of the lengths), and the row's start and code thresholds come from
// lane r. Undecided hits go to the deferred queue with r as their partner slot, like those
// of whole strips. Rows this short are one strip long, so the Lemma-3 cut, which acts only
// between batches of strips, never shortens them.
template <int WOFF>
__device__ __forceinline__ void walk_packed_rows(const WalkParams& wp, const double* __restrict__ o_d,
                                                 const TabRef& R, int lv, int64_t ov, double duv,
                                                 const CodeRow& cr, int nv, WalkLaneState& st) {
    const int lane = utri_lane();
    const int lvs = lv & 0xFFFF;
    const int my_len = (lane < nv && lvs > 0 && lvs <= UTRI_WAVE) ? lvs : 0;
    // inclusive prefix of the lengths over the lanes
    int inc = my_len;
#pragma unroll
    for (int d = 1; d < UTRI_WAVE; d <<= 1) {
        const int o = __shfl_up(inc, d, UTRI_WAVE);
        if (lane >= d) inc += o;
    }
    const int pre = inc - my_len;  // exclusive
    const int total = __shfl(inc, UTRI_WAVE - 1, UTRI_WAVE);
    // (a lane with an empty row shares its start with the next lane, so the search below
    // never ends on one: for P < total the last lane with pre_r <= P has P < pre_r + len_r)
    for (int base = 0; base < total; base += UTRI_WAVE) {
        const int P = base + lane;
        const bool act = P < total;
        // si: the last lane with pre_si <= P, whose row holds position P
        int si = 0;
#pragma unroll
        for (int step = UTRI_WAVE / 2; step >= 1; step >>= 1) {
            if (__shfl(pre, si + step, UTRI_WAVE) <= P) si += step;
        }
        const int64_t pos = __shfl(ov, si, UTRI_WAVE) + (P - __shfl(pre, si, UTRI_WAVE));
        const uint32_t pw = act ? (uint32_t)wp.o_adj[pos] : 0u;
        const uint32_t w = pw & wp.idmask;
        const uint32_t r = tab_find<WOFF>(R.key, R.bmask, w);
        const bool found = r != 0u;
        const uint32_t khi = (uint32_t)__shfl((int)cr.khi, si, UTRI_WAVE);
        const uint32_t klo = (uint32_t)__shfl((int)cr.klo, si, UTRI_WAVE);
        const uint32_t rsign = (uint32_t)__shfl((int)cr.rsign, si, UTRI_WAVE);
        const uint32_t qb = __builtin_amdgcn_ubfe(r, 16, QB);
        const uint32_t qc = __builtin_amdgcn_ubfe(pw, wp.idbits, wp.mb);
        const uint32_t p0 = __umul24(qb, qc);
        const uint32_t t1 = p0 + qb + qc;  // (qb + 1)(qc + 1) - 1
        // khi >= 1, so an absent w (r = 0, qb = 0) is never classified
        const bool ccls = p0 >= khi;
        const bool bal = ccls && (int32_t)(r ^ pw ^ rsign) < 0;
        st.nb32 += bal ? 1u : 0u;
        st.nu32 += ccls ? 1u : 0u;
        const bool und = found && !ccls && t1 >= klo;
        const uint64_t um = __builtin_amdgcn_ballot_w64(und);
        if (um) {
            const bool mine = (um >> lane) & 1ull;
            const int nq = __popcll(um);
            if (st.dn + nq <= DQ_CAP) {
                if (mine) {
                    DeferQueue& Q = defer_q[threadIdx.x / UTRI_WAVE];
                    const int qs = st.dn + __popcll(um & __lanemask_lt());
                    Q.vw[qs] = (uint32_t)pos;
                    Q.ps[qs] = (r & W_POS) | ((uint32_t)si << 15);
                }
                st.dn += nq;
            } else {
                // every lane takes part in the shuffle (a lane shut off by a branch would
                // hand its neighbours nothing); those with an undecided hit decide it now
                const double duv_r = __shfl(duv, si, UTRI_WAVE);
                if (mine) {
                    const double s = utri_tri_s(duv_r, o_d[R.src_base + (r & W_POS)], o_d[pos]);
                    st.nb32 += (s <= -wp.c) ? 1u : 0u;
                    st.nu32 += (s <= -wp.c || s > wp.c) ? 1u : 0u;
                }
            }
        }
        if (st.dn > DQ_DRAIN) defer_drain(wp, o_d, R.src_base, duv, st);
    }
}

#ifndef UTRI_WALK_MIN_WAVES
#define UTRI_WALK_MIN_WAVES 8      // waves per SIMD the register allocation must allow
#endif

// Stream every partner row of one partner range of an item through the staged table;
// partner p goes to the wave with p % nparts == part, which loads its own partners 64 at a
// time.
template <int MODE, int PV, int WOFF>
__device__ __forceinline__ void walk_partners(const WalkParams& wp, const int32_t* __restrict__ o_adj,
                                              const double* __restrict__ o_d,
                                              const uint2* __restrict__ rinfo,
                                              const int32_t* __restrict__ perm, const TabRef& R,
                                              int u, int Lu, int64_t sb, int np, double dmax_chunk,
                                              int part, int nparts, HistLds* H, WalkLaneState& st,
                                              int64_t& run_b, int64_t& run_u) {
    for (int i0 = 0; i0 < np; i0 += UTRI_WAVE * nparts) {
        int v, lv;
        int64_t ov;
        double duv;
        int32_t euv;
        CodeRow cr;
        load_partners<MODE, PV>(wp, o_adj, o_d, rinfo, u, Lu, sb, np, i0, part, nparts,
                                     dmax_chunk, v, ov, lv, duv, euv, cr);
        // this wave's partners in the batch: i0 + part + nparts * si < np
        const int nv = min(UTRI_WAVE, (np - i0 - part + nparts - 1) / nparts);
        // fill: the partners' original ids on their lanes (fill_drain reads them by slot)
        const int32_t pvl = (MODE == WALK_ENUM_FILL && lv != 0) ? perm[v] : 0;
        constexpr bool kPack = MODE == WALK_COUNT || MODE == WALK_ENUM_COUNT;
        if (kPack) walk_packed_rows<WOFF>(wp, o_d, R, lv, ov, duv, cr, nv, st);
        // lane by lane (a loop over the set bits of a ballot made the sign-world walk slower
        // and the others no faster)
        for (int si = 0; si < nv; si++) {
            const int lvm = bcast_i32(lv, si);
            const int lvs = lvm & 0xFFFF;
            if (lvs == 0 || (kPack && lvs <= UTRI_WAVE)) continue;
            const int32_t pv = (MODE == WALK_ENUM_FILL) ? pvl
                               : (MODE == WALK_SIGN) ? bcast_i32(euv, si) : 0;
            const CodeRow crs{(uint32_t)bcast_i32((int)cr.khi, si),
                              (uint32_t)bcast_i32((int)cr.klo, si),
                              (uint32_t)bcast_i32((int)cr.rsign, si)};
            stream_any<MODE, WOFF, (PV & 2) != 0>(wp, o_d, perm, R, bcast_i64(ov, si), lvs,
                                                  bcast_f64(duv, si), pv, crs, si, duv,
                                                  (int)((uint32_t)lvm >> 16), H, st, run_b, run_u);
            if ((MODE == WALK_COUNT || MODE == WALK_ENUM_COUNT) && st.dn > DQ_DRAIN)
                defer_drain(wp, o_d, R.src_base, duv, st);
        }
        // deferred hits use this batch's d_xy
        if ((MODE == WALK_COUNT || MODE == WALK_ENUM_COUNT) && st.dn > 0)
            defer_drain(wp, o_d, R.src_base, duv, st);
        if (MODE == WALK_ENUM_FILL && st.dn > 0)
            fill_drain(wp, o_d, perm, R.src_base, R.pu, pvl, duv, st, run_b, run_u, true);
    }
}

// Wave item: vertex u with 2 <= len <= cap, N+(u) staged in the wave's own table, and
// one range of its partners.
template <int MODE, int PV, class G>
__device__ void walk_item_wave(const WalkParams& wp, const int64_t* __restrict__ o_off,
                               const int32_t* __restrict__ o_adj, const double* __restrict__ o_d,
                               const int32_t* __restrict__ len, const uint2* __restrict__ rinfo,
                               const int32_t* __restrict__ perm, int64_t item, int64_t it,
                               WaveTab<G>& L, HistLds* H, WalkLaneState& st) {
    constexpr bool shorter = (PV & 1) != 0;
    constexpr int WOFF = 4 << G::WLG;
    const int lane = utri_lane();
    const int u = item_vertex(item);
    const int rg = item_range(item);
    const int64_t ou = o_off[u];
    const int Lu = len[u];
    const int pr = wp.tune.pr;
    const int64_t sb = shorter ? wp.s_off[u] + (int64_t)rg * pr : ou;
    const int np = shorter ? min(pr, wp.slen[u] - rg * pr) : (rg == 0 ? Lu : 0);
    if (np <= 0) return;  // (the enumeration slots start zeroed)
    const int lg = tab_lg(Lu, G::WLG);
    tab_clear<WOFF>(L.key, lg, lane, UTRI_WAVE);
    utri_wave_sync();
    tab_stage<WOFF>(L.key, o_adj, o_d, ou, Lu, (1u << lg) - 1u, lane, UTRI_WAVE, wp.idmask);
    utri_wave_sync();
    const TabRef R{L.key, (1u << lg) - 1u, ou, (MODE == WALK_ENUM_FILL) ? perm[u] : 0, 0};
    const double dmax_chunk = fabs(o_d[ou]);
    int64_t run_b = 0, run_u = 0;
    if (MODE == WALK_ENUM_FILL) { run_b = wp.off_b[it]; run_u = wp.off_u[it]; }
    walk_partners<MODE, PV, WOFF>(wp, o_adj, o_d, rinfo, perm, R, u, Lu, sb, np, dmax_chunk,
                                       0, 1, H, st, run_b, run_u);
    // an item counts at most its candidates per lane, far below 2^32; the counting walks
    // keep (balanced, classified) per lane
    st.nb += st.nb32;
    st.nu += (MODE == WALK_COUNT || MODE == WALK_ENUM_COUNT) ? st.nu32 - st.nb32 : st.nu32;
    st.nb32 = st.nu32 = 0;
    if (MODE == WALK_ENUM_COUNT) {
        const uint64_t nb = utri_wave_sum_u64(st.nb), nu = utri_wave_sum_u64(st.nu);
        if (lane == 0) { wp.cnt_b[it] = (int64_t)nb; wp.cnt_u[it] = (int64_t)nu; }
        st.nb = st.nu = 0;
    }
    utri_wave_sync();
}

// Work-group item: chunk `chunk` (caph entries) of a long source row, one shared table,
// target rows split round-robin over the waves. Enumeration slots are per wave.
template <int MODE, int PV, class G>
__device__ void walk_item_block(const WalkParams& wp, const int64_t* __restrict__ o_off,
                                const int32_t* __restrict__ o_adj, const double* __restrict__ o_d,
                                const int32_t* __restrict__ len, const uint2* __restrict__ rinfo,
                                const int32_t* __restrict__ perm, int64_t item, int64_t hq,
                                BlockTab<G>& B, HistLds* H, WalkLaneState& st) {
    constexpr bool shorter = (PV & 1) != 0;
    constexpr int WOFF = 4 << G::LGH;
    const int lane = utri_lane();
    const int wib = threadIdx.x / UTRI_WAVE;
    const int u = item_vertex(item);
    const int chunk = item_chunk(item);
    const int rg = item_range(item);
    const int64_t ou = o_off[u];
    const int Lu = len[u];
    const int pr = wp.tune.pr;
    const int64_t sb = shorter ? wp.s_off[u] + (int64_t)rg * pr : ou;
    const int np = shorter ? min(pr, wp.slen[u] - rg * pr) : (rg == 0 ? Lu : 0);
    if (np <= 0) return;  // work-group uniform (the enumeration slots start zeroed)
    const int cb = chunk * wp.tune.caph;
    const int cl = min(wp.tune.caph, Lu - cb);
    const int lg = tab_lg(cl, G::LGH);
    __syncthreads();  // the previous item's probes are done
    tab_clear<WOFF>(B.key, lg, threadIdx.x, G::TPBW);
    __syncthreads();
    tab_stage<WOFF>(B.key, o_adj, o_d, ou + cb, cl, (1u << lg) - 1u, threadIdx.x, G::TPBW,
                    wp.idmask);
    __syncthreads();
    const TabRef R{B.key, (1u << lg) - 1u, ou + cb, (MODE == WALK_ENUM_FILL) ? perm[u] : 0, chunk};
    const double dmax_chunk = fabs(o_d[ou + cb]);
    const int64_t slot = wp.lb + NW_MAX * hq + wib;
    int64_t run_b = 0, run_u = 0;
    if (MODE == WALK_ENUM_FILL) { run_b = wp.off_b[slot]; run_u = wp.off_u[slot]; }
    walk_partners<MODE, PV, WOFF>(wp, o_adj, o_d, rinfo, perm, R, u, Lu, sb, np, dmax_chunk,
                                       wib, G::NW, H, st, run_b, run_u);
    // an item counts at most its candidates per lane, far below 2^32; the counting walks
    // keep (balanced, classified) per lane
    st.nb += st.nb32;
    st.nu += (MODE == WALK_COUNT || MODE == WALK_ENUM_COUNT) ? st.nu32 - st.nb32 : st.nu32;
    st.nb32 = st.nu32 = 0;
    if (MODE == WALK_ENUM_COUNT) {
        const uint64_t nb = utri_wave_sum_u64(st.nb), nu = utri_wave_sum_u64(st.nu);
        if (lane == 0) { wp.cnt_b[slot] = (int64_t)nb; wp.cnt_u[slot] = (int64_t)nu; }
        st.nb = st.nu = 0;
    }
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
    } else if (MODE == WALK_SIGN) {
        if (st.qn > 0) sign_drain(wp, st);
        sign_flush(wp, st);
    } else if (MODE == WALK_HIST) {
        utri_wave_sync();
        for (int q = lane; q < 2 * NB; q += UTRI_WAVE) {
            const int cls = q / NB, bin = q % NB;
            const unsigned long long v = H->hist[cls][bin];
            if (v && bin <= wp.nt) atomicAdd(&wp.acc[cls * (wp.nt + 1) + bin], v);
        }
    }
}

// Both phases of the walk for one work-group: heavy items cooperatively, then light
// items one per wave. Heaviest rows (highest ids) go first in both lists; work queues:
// qctr[0] hands out heavy items to work-groups, qctr[1] light items to waves in groups of
// four.
template <int MODE, int PV, class G>
__device__ void walk_phases(const WalkParams& wp, const int64_t* __restrict__ o_off,
                            const int32_t* __restrict__ o_adj, const double* __restrict__ o_d,
                            const int32_t* __restrict__ len, const uint2* __restrict__ rinfo,
                            const int32_t* __restrict__ perm, const int64_t* __restrict__ items,
                            int64_t nl, int64_t nh, WalkShared<G>& S, HistLds* H,
                            WalkLaneState& st) {
    const int wib = threadIdx.x / UTRI_WAVE;
    __shared__ int64_t s_q;
    for (;;) {
        if (threadIdx.x == 0) s_q = (int64_t)atomicAdd(&wp.qctr[0], 1ull);
        __syncthreads();
        const int64_t q = s_q;
        __syncthreads();
        if (q >= nh) break;
        const int64_t hq = nh - 1 - q;
        walk_item_block<MODE, PV, G>(wp, o_off, o_adj, o_d, len, rinfo, perm,
                                          items[wp.lb + hq], hq, S.block, H, st);
    }
    __syncthreads();  // the work-group table is no longer read; the wave tables reuse it
    constexpr int QGROUP = 4;
    for (;;) {
        int64_t base = 0;
        if (utri_lane() == 0) base = (int64_t)atomicAdd(&wp.qctr[1], (unsigned long long)QGROUP);
        base = bcast_i64(base, 0);
        if (base >= nl) break;
        const int64_t end = base + QGROUP < nl ? base + QGROUP : nl;
        for (int64_t q = base; q < end; q++) {
            const int64_t it = nl - 1 - q;
            walk_item_wave<MODE, PV, G>(wp, o_off, o_adj, o_d, len, rinfo, perm, items[it],
                                             it, S.wave[wib], H, st);
        }
    }
}

// Geometry of each walk kernel: the sign-world walk keeps its counter planes in registers
// (about 96 VGPRs, five waves per SIMD), so it runs four-wave work-groups with a smaller
// work-group table (chunks of at most UTRI_SIGN_WALK_CHUNK entries), which fill those five
// wave slots; the other walks run eight waves per group within 64 VGPRs.
template <int MODE>
struct WalkGeom {
    using G = GeomWalk;
    static constexpr int MIN_WAVES = UTRI_WALK_MIN_WAVES;
};
template <>
struct WalkGeom<WALK_SIGN> {
    using G = Geom<SIGN_NW, 9, WAVE_LG>;
    static constexpr int MIN_WAVES = 1;
    static_assert(2 * (1 << G::LGH) >= UTRI_SIGN_WALK_CHUNK, "chunks fit the table");
};

// L3: the kernel of the Lemma-3 queries (its cut's code is compiled only here, so the
// other kernels keep their registers).
template <int MODE, bool L3>
__global__ void __launch_bounds__(WalkGeom<MODE>::G::TPBW, WalkGeom<MODE>::MIN_WAVES) k_walk(WalkParams wp,
                                                          const int64_t* __restrict__ o_off,
                                                          const int32_t* __restrict__ o_adj,
                                                          const double* __restrict__ o_d,
                                                          const int32_t* __restrict__ len,
                                                          const uint2* __restrict__ rinfo,
                                                          const int32_t* __restrict__ perm,
                                                          const int64_t* __restrict__ items,
                                                          const int64_t* __restrict__ n_items_dev) {
    using G = typename WalkGeom<MODE>::G;
    __shared__ WalkShared<G> S;
    __shared__ HistLds hlds[MODE == WALK_HIST ? G::NW : 1];
    const int wib = threadIdx.x / UTRI_WAVE;
    HistLds* H = &hlds[MODE == WALK_HIST ? wib : 0];
    if (MODE == WALK_HIST) {
        for (int q = utri_lane(); q < 2 * NB; q += UTRI_WAVE) H->hist[q / NB][q % NB] = 0;
        thresh_stage(wp.cvals, wp.nt);
    }
    WalkLaneState st;
    // both partner sources as their own code (the choice is uniform over the launch)
    constexpr int PL = L3 ? 2 : 0;
    const int64_t nl = n_items_dev[0], nh = n_items_dev[1];
    if (stream_shorter<MODE>(wp, n_items_dev))
        walk_phases<MODE, PL | 1, G>(wp, o_off, o_adj, o_d, len, rinfo, perm, items, nl, nh, S, H,
                                     st);
    else
        walk_phases<MODE, PL, G>(wp, o_off, o_adj, o_d, len, rinfo, perm, items, nl, nh, S, H, st);
    walk_flush<MODE>(wp, H, st);
}

// Fused batch: the walk (threshold histogram of every triangle at the smallest
// threshold) followed by the grouped edge-sampling items of the first pass, in one
// persistent launch.
__global__ void __launch_bounds__(TPB) k_batch(WalkParams wp, const int64_t* __restrict__ o_off,
                                               const int32_t* __restrict__ o_adj,
                                               const double* __restrict__ o_d,
                                               const int32_t* __restrict__ len,
                                               const uint2* __restrict__ rinfo,
                                               const int32_t* __restrict__ perm,
                                               const int64_t* __restrict__ items,
                                               const int64_t* __restrict__ n_items_dev,
                                               SampleParams sp, SampleGraph SG,
                                               const int32_t* __restrict__ slen) {
    using G = GeomBatch;
    static_assert(G::TPBW == TPB, "the batch shares the sampler's block size");
    // the walk's tables and the sampler's tables are used one after the other
    union BatchLds {
        WalkShared<G> walk;
        SampleLds samp;
    };
    __shared__ BatchLds S;
    __shared__ HistLds hlds[WPB];
    const int wib = threadIdx.x / UTRI_WAVE;
    HistLds* H = &hlds[wib];
    for (int q = utri_lane(); q < 2 * NB; q += UTRI_WAVE) H->hist[q / NB][q % NB] = 0;
    // the walk and the sampler share the thresholds
    if (wp.acc != nullptr) thresh_stage(wp.cvals, wp.nt);
    else thresh_stage(sp.cvals, sp.nt);
    WalkLaneState st;
    if (wp.acc != nullptr) {
        // (the batch walk counts with Lemma 2 only)
        const int64_t nl = n_items_dev[0], nh = n_items_dev[1];
        if (stream_shorter<WALK_HIST>(wp, n_items_dev))
            walk_phases<WALK_HIST, 1, G>(wp, o_off, o_adj, o_d, len, rinfo, perm, items, nl, nh,
                                         S.walk, H, st);
        else
            walk_phases<WALK_HIST, 0, G>(wp, o_off, o_adj, o_d, len, rinfo, perm, items, nl, nh,
                                         S.walk, H, st);
        walk_flush<WALK_HIST>(wp, H, st);
    }
    __syncthreads();  // the walk's tables are no longer read; the sampler's reuse them
    if (sp.hist != nullptr && sp.t1 > sp.t0) sample_groups(sp, SG, slen, S.samp);
}

}  // namespace

int utri_walk_prepare(utri_graph* g, double c_rows, int lemma3, hipStream_t s, int64_t** items,
                      int64_t** n_items_dev, int32_t** len) {
    const int64_t n = g->n;
    const int64_t lb = light_bound(g), hb = heavy_bound(g);
    void *plen, *pcnt, *poff, *pitems, *pn, *pri;
    // oriented prefixes in [0, n], symmetric prefixes in [n + 1, 2n + 1]
    UTRI_TRY(utri_scratch(g, SCR_LEN, sizeof(int32_t) * (size_t)(2 * n + 2), &plen));
    UTRI_TRY(utri_scratch(g, SCR_ICNT, sizeof(int32_t) * (size_t)(2 * n + 2), &pcnt));
    UTRI_TRY(utri_scratch(g, SCR_IOFF, sizeof(int64_t) * (size_t)(2 * n + 2), &poff));
    UTRI_TRY(utri_scratch(g, SCR_ITEMS, sizeof(int64_t) * (size_t)(lb + hb), &pitems));
    // [0] light items, [1] heavy items, [2..3] work-queue counters, then the slot pairs of
    // the kept oriented edges and of the ids the plain forward iteration would stream
    UTRI_TRY(utri_scratch(g, SCR_NITEMS, sizeof(int64_t) * NITEMS_WORDS, &pn));
    // per vertex: (row start, kept length) for the partner scans
    UTRI_TRY(utri_scratch(g, SCR_RINFO, sizeof(uint2) * (size_t)std::max<int64_t>(n, 1), &pri));
    *items = (int64_t*)pitems;
    *n_items_dev = (int64_t*)pn;
    *len = (int32_t*)plen;
    g->rinfo_cur = pri;
    UTRI_TRY(utri_fill_u64(pn, 0, NITEMS_WORDS, s));
    if (n == 0) return UTRI_OK;
    int32_t* lcnt = (int32_t*)pcnt;
    int32_t* hcnt = lcnt + n;
    int64_t* loff = (int64_t*)poff;
    int64_t* hoff = loff + n;
    if (chunks_bound(g) > MAX_CHUNKS) return UTRI_E_RANGE;  // the item word's chunk field
    int32_t* slen = (int32_t*)plen + n + 1;
    hipLaunchKernelGGL(k_rowlen, dim3(blocks_for(n)), dim3(TPB), 0, s, g->o_off, g->o_d, g->s_off,
                       g->s_d, n, c_rows, (int32_t*)plen, slen, lcnt, hcnt,
                       (unsigned long long*)pn + 4, (uint2*)pri, g->walk_tune.cap,
                       g->walk_tune.caph, g->walk_tune.pr, lemma3);
    UTRI_HIP_TRY(hipGetLastError());
    UTRI_TRY(utri_scan_i32(g, lcnt, loff, n, (int64_t*)pn, s));
    UTRI_TRY(utri_scan_i32(g, hcnt, hoff, n, (int64_t*)pn + 1, s));
    hipLaunchKernelGGL(k_items, dim3(blocks_for(n)), dim3(TPB), 0, s, (const int32_t*)lcnt,
                       (const int32_t*)hcnt, (const int32_t*)slen, (const int64_t*)loff,
                       (const int64_t*)hoff, n, lb, (int64_t*)pitems, g->walk_tune.pr);
    UTRI_HIP_TRY(hipGetLastError());
    return UTRI_OK;
}

// Ids the plain forward iteration streams per kept oriented edge at the last prepared
// query (the ratio the shorter-row crossover is compared with); waits for the stream.
int utri_walk_plain_ratio(utri_graph* g, hipStream_t s, double* ratio) {
    void* pn;
    UTRI_TRY(utri_scratch(g, SCR_NITEMS, sizeof(int64_t) * NITEMS_WORDS, &pn));
    int64_t h[NITEMS_WORDS];
    UTRI_HIP_TRY(hipMemcpyAsync(h, pn, sizeof(h), hipMemcpyDeviceToHost, s));
    UTRI_HIP_TRY(hipStreamSynchronize(s));
    int64_t kept = 0, plain = 0;
    for (int i = 0; i < KEPT_SLOTS; i++) {
        kept += h[4 + i * KEPT_STRIDE];
        plain += h[5 + i * KEPT_STRIDE];
    }
    *ratio = kept > 0 ? (double)plain / (double)kept : 0.0;
    return UTRI_OK;
}

// Graph-dependent fields of a launch: enumeration slot base, row packing, symmetric rows
// and their kept prefixes (stored after the oriented ones).
static void set_launch_fields(utri_graph* g, WalkParams& wp, const int32_t* len) {
    wp.lb = light_bound(g);
    wp.order = g->walk_order;
    wp.tune = g->walk_tune;
    wp.s_off = g->s_off;
    wp.s_adj = g->s_adj;
    wp.s_d = g->s_d;
    wp.s_eid = g->s_eid;
    wp.slen = len ? len + g->n + 1 : nullptr;
    wp.o_adj = g->o_adj;
    wp.idmask = g->idmask;
    wp.idbits = g->idbits;
    wp.mb = g->code_mb;
}

int64_t utri_count_scratch_bound(const utri_graph* g, int64_t align) {
    const int64_t n = g->n;
    const int64_t scan_blocks = (n + 1023) / 1024 + 1;  // the scans' block partials
    const int64_t bytes[] = {
        4 * (2 * n + 2),                          // oriented and symmetric prefixes
        4 * (2 * n + 2),                          // light and heavy item counts
        8 * (2 * n + 2),                          // their offsets
        8 * (light_bound(g) + heavy_bound(g)),    // work items
        8 * (int64_t)NITEMS_WORDS,                // item counts, queues, kept totals
        8 * std::max<int64_t>(n, 1),              // row starts and kept lengths
        8 * scan_blocks,                          // scan partials
        8 * 4,                                    // class counters
    };
    int64_t tot = 0;
    for (int64_t b : bytes) tot += b + align;
    return tot;
}

// Slots of the per-item enumeration arrays: one per light item, NW_MAX per heavy item.
int64_t utri_walk_items_bound(utri_graph* g) { return light_bound(g) + NW_MAX * heavy_bound(g); }

// Work-groups per CU for a kernel: the resident occupancy (so no second, partial round of
// work-groups trails the items), unless a tuned value is set.
template <class K>
static int blocks_per_cu(utri_graph* g, K kernel, int tpb) {
    if (g->walk_blocks_per_cu > 0) return g->walk_blocks_per_cu;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, tpb, 0) != hipSuccess || nb < 1)
        nb = 2;
    return nb;
}

template <int MODE, bool L3>
static void launch_walk_k(utri_graph* g, const WalkParams& wp, const int32_t* len,
                          const int64_t* items, const int64_t* n_items_dev, hipStream_t s) {
    const int tpb = WalkGeom<MODE>::G::TPBW;
    const int blocks = g->num_cu * blocks_per_cu(g, k_walk<MODE, L3>, tpb);
    hipLaunchKernelGGL((k_walk<MODE, L3>), dim3(blocks), dim3(tpb), 0, s, wp, g->o_off, g->o_adj,
                       g->o_d, len, (const uint2*)g->rinfo_cur, g->perm, items, n_items_dev);
}

// The Lemma-3 cut runs in the threshold walks of PRUNED_L3 queries on graphs with row codes
// (at c = 0 it cuts nothing).
template <int MODE>
static void launch_walk(utri_graph* g, const WalkParams& wp, const int32_t* len,
                        const int64_t* items, const int64_t* n_items_dev, hipStream_t s) {
    constexpr bool kL3 = MODE == WALK_COUNT || MODE == WALK_HIST || MODE == WALK_ENUM_COUNT ||
                         MODE == WALK_ENUM_FILL || MODE == WALK_STATS;
    if (kL3 && wp.lemma3 && wp.mb > 0 && wp.c > 0.0)
        launch_walk_k<MODE, kL3>(g, wp, len, items, n_items_dev, s);
    else
        launch_walk_k<MODE, false>(g, wp, len, items, n_items_dev, s);
}

int utri_walk_launch(utri_graph* g, int mode, const WalkParams& wp_in, const int64_t* items,
                     const int64_t* n_items_dev, const int32_t* len, int64_t n_items_host_bound,
                     hipStream_t s) {
    (void)n_items_host_bound;
    if (g->n == 0 || g->m == 0) return UTRI_OK;
    WalkParams wp = wp_in;
    set_launch_fields(g, wp, len);
    // the work-queue counters live after the two item counts and restart at every launch
    wp.qctr = (unsigned long long*)(const_cast<int64_t*>(n_items_dev) + 2);
    UTRI_TRY(utri_fill_u64(wp.qctr, 0, 2, s));
    switch (mode) {
        case WALK_COUNT: launch_walk<WALK_COUNT>(g, wp, len, items, n_items_dev, s); break;
        case WALK_HIST: launch_walk<WALK_HIST>(g, wp, len, items, n_items_dev, s); break;
        case WALK_EXPECTED: launch_walk<WALK_EXPECTED>(g, wp, len, items, n_items_dev, s); break;
        case WALK_ENUM_COUNT: launch_walk<WALK_ENUM_COUNT>(g, wp, len, items, n_items_dev, s); break;
        case WALK_ENUM_FILL: launch_walk<WALK_ENUM_FILL>(g, wp, len, items, n_items_dev, s); break;
        case WALK_STATS: launch_walk<WALK_STATS>(g, wp, len, items, n_items_dev, s); break;
        case WALK_SIGN: launch_walk<WALK_SIGN>(g, wp, len, items, n_items_dev, s); break;
        default: return UTRI_E_INVALID;
    }
    UTRI_HIP_TRY(hipGetLastError());
    return UTRI_OK;
}

int utri_batch_launch(utri_graph* g, const WalkParams& wp_in, const int64_t* items,
                      const int64_t* n_items_dev, const int32_t* len, int64_t n_items_bound,
                      const SampleParams& sp, const int32_t* slen, hipStream_t s) {
    (void)n_items_bound;
    if (g->n == 0 || g->m == 0) return UTRI_OK;
    WalkParams wp = wp_in;
    set_launch_fields(g, wp, len);
    wp.qctr = (unsigned long long*)(const_cast<int64_t*>(n_items_dev) + 2);
    UTRI_TRY(utri_fill_u64(wp.qctr, 0, 2, s));
    SampleGraph G{g->m, g->e_lo, g->e_hi, g->e_d, g->inv, g->s_off, g->s_adj, g->s_d, g->h_off,
                  g->h_tab};
    const int blocks = g->num_cu * blocks_per_cu(g, k_batch, TPB);
    hipLaunchKernelGGL(k_batch, dim3(blocks), dim3(TPB), 0, s, wp, g->o_off, g->o_adj, g->o_d,
                       len, (const uint2*)g->rinfo_cur, g->perm, items, n_items_dev, sp, G, slen);
    UTRI_HIP_TRY(hipGetLastError());
    return UTRI_OK;
}

namespace {

// Thread per (edge, mask word): 8 Philox blocks of 4 worlds each; bit 4 r + q of word j
// is world 32 j + 4 r + q, set when the edge is negative there (u >= P+ * 2^32).
__global__ void k_sign_masks(const double* __restrict__ e_p, int64_t m, uint64_t seed, int ww,
                             uint32_t* __restrict__ masks) {
    UTRI_FOR_GRID(t, m * ww) {
        const int64_t e = t / ww;
        const int j = (int)(t - e * ww);
        const double th = e_p[e] * 4294967296.0;
        uint32_t mk = 0;
        for (int r = 0; r < 8; r++) {
            uint32_t x[4];
            utri_philox((uint32_t)e, (uint32_t)(8 * j + r), 1u, 0u, (uint32_t)seed,
                        (uint32_t)(seed >> 32), x);
#pragma unroll
            for (int q = 0; q < 4; q++) mk |= ((double)x[q] < th ? 0u : 1u) << (4 * r + q);
        }
        masks[t] = mk;
    }
}

}  // namespace

int utri_sign_masks_launch(utri_graph* g, uint64_t seed, int ww, uint32_t* masks, hipStream_t s) {
    const int64_t tot = g->m * ww;
    if (tot == 0) return UTRI_OK;
    hipLaunchKernelGGL(k_sign_masks, dim3(utri_grid(tot, TPB)), dim3(TPB), 0, s, (const double*)g->e_p,
                       g->m, seed, ww, masks);
    UTRI_HIP_TRY(hipGetLastError());
    return UTRI_OK;
}
