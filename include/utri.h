/*
 * utri.h -- C ABI of libutri: exact counting and enumeration of uncertain balanced
 * and unbalanced triangles, the expected balanced count and its per-edge gradient,
 * and the edge-sampling estimator, on MI355X (gfx950).
 *
 * Model (arXiv 2602.14084, Section 3): an undirected graph whose edges all exist,
 * each with a probability P+(e) in [0,1] that its sign is positive, signs
 * independent. A triangle is balanced when it has an odd number of '+' edges; its
 * probability of being balanced is the four-term sum of Section 3, equal to
 * P_bal = (1 - s)/2 with s = d1*d2*d3 and d = 1 - 2*P+. At a threshold t in [0.5, 1]
 * (the paper assumes t >= 0.5) a triangle is
 *   uncertain balanced   iff P_bal   >= t   (Definition "Uncertain Balanced Triangle")
 *   uncertain unbalanced iff P_unbal >  t   (Definition "Uncertain Unbalanced Triangle").
 * Decisions are taken in FP64 as: d = 1.0 - 2.0*p; c = 2.0*t - 1.0; the three d of a
 * triangle sorted ascending by value; s = (x*y)*z, each product rounded (no fused
 * multiply-add); balanced iff s <= -c, unbalanced iff s > c. Counts are exact
 * integers; a result depends on the graph and t only, never on thread scheduling.
 *
 * Conventions shared by every call:
 *  - Return value: UTRI_OK (0) or a negative utri_status. No call aborts or exits.
 *  - Vertex ids are 0..n-1 with n < 2^31; the canonical graph has m < 2^31 edges.
 *    Canonical edge e is (lo[e], hi[e]) with lo < hi; edge ids are ranks in
 *    ascending (lo, hi) order. Self-loops are dropped and counted; an exact
 *    duplicate (either orientation, same P+) is merged and counted; a duplicate
 *    with a different P+ is UTRI_E_CONFLICT (an edge has one P+, Section 3).
 *  - hip_stream is a hipStream_t (NULL = the legacy default stream). Every kernel
 *    of a call is enqueued on it. Calls that return scalars through host pointers
 *    (counts, E, sizes) wait for that stream before returning; calls whose outputs
 *    are device arrays return as soon as the work is enqueued.
 *  - Buffers passed in are owned by the caller and are not retained after the call
 *    returns. The handle owns every device copy it makes. A handle must not be used
 *    from two host threads or two streams at the same time.
 *  - Device pointers must be device memory of the current HIP device.
 */
#ifndef UTRI_H
#define UTRI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct utri_graph utri_graph;

typedef enum {
    UTRI_OK = 0,
    UTRI_E_INVALID = -1,   /* bad argument: NULL pointer, id out of range, P+ NaN or outside [0,1], t outside [0.5,1] */
    UTRI_E_CONFLICT = -2,  /* the same undirected edge given twice with different P+ */
    UTRI_E_CAPACITY = -3,  /* an enumeration output buffer is too small; sizes are still reported */
    UTRI_E_NOMEM = -4,     /* device or host allocation failed */
    UTRI_E_HIP = -5,       /* a HIP runtime call failed */
    UTRI_E_RANGE = -6      /* n or m does not fit the int32 ids of the library */
} utri_status;

/* Search methods (both give identical results). */
enum {
    UTRI_PLAIN = 0,      /* forward edge iteration over every triangle (Algorithm "Baseline UBTE/UBTC", Section 4) */
    UTRI_PRUNED = 1,     /* rows cut to |d| >= c before the walk (Lemma 2, Section 5) */
    UTRI_PRUNED_L3 = 2   /* PRUNED plus a per-edge cut |d_vw| * |d_uv| * max|d_u.| >= c (Lemma 3, Section 5) */
};

/* Which classes to count or list (Section 3: "balanced and/or unbalanced"). */
enum { UTRI_BAL = 1, UTRI_UNBAL = 2, UTRI_BOTH = 3 };

/* Pointer kinds for inputs / outputs that may live on either side. */
enum { UTRI_HOST_PTR = 0, UTRI_DEVICE_PTR = 1 };

/* Sampling schemes: edge sampling (Section 6.2) and vertex sampling (Section 6.1) with the
 * improved local searches, and the same estimators with the baseline local search (no
 * Lemma-2 pruning: every neighbour is searched), which give identical estimates. */
enum { UTRI_SAMPLE_EDGE = 0, UTRI_SAMPLE_VERTEX = 1, UTRI_SAMPLE_EDGE_PLAIN = 2,
       UTRI_SAMPLE_VERTEX_PLAIN = 3 };

/*
 * Build a graph handle (Definition "Uncertain Signed Graph", Section 3).
 * src, dst: int64 [m_in] endpoint ids in [0, n); p: FP64 [m_in] P+ of each input edge.
 * ptr_kind says whether the three arrays are host or device memory.
 * Preprocessing (kept for every later query, as the paper pre-sorts its data,
 * Section 7): canonical sorted edge list, symmetric adjacency with rows in
 * Absolute Edge Order (|d| descending, then neighbour id; Definitions "Absolute Edge
 * Value" / "Absolute Edge Order", Section 5), per-row hash tables, and the degree
 * orientation of Definition "Node Order" (Section 4) with vertices relabelled by it.
 * Errors: UTRI_E_INVALID (NULL with m_in > 0, id out of range, bad P+),
 * UTRI_E_CONFLICT, UTRI_E_RANGE (n >= 2^31, m_in >= 2^31 or m >= 2^31), UTRI_E_NOMEM,
 * UTRI_E_HIP.
 * On error *out is NULL.
 */
int utri_graph_load(const int64_t* src, const int64_t* dst, const double* p, int64_t m_in,
                    int64_t n, int ptr_kind, void* hip_stream, utri_graph** out);

/* Release a handle and all its device memory. NULL is accepted. */
int utri_graph_free(utri_graph* g);

/* Sizes of the canonical graph. Any output pointer may be NULL. */
int utri_graph_info(const utri_graph* g, int64_t* n, int64_t* m, int64_t* self_loops_dropped,
                    int64_t* dups_merged, int64_t* max_deg);

/* Canonical edges in edge-id order: lo, hi int32 [m], p FP64 [m] (host or device per
 * ptr_kind; any may be NULL). These ids index the gradient and the sampler. */
int utri_graph_edges(const utri_graph* g, int32_t* lo, int32_t* hi, double* p, int ptr_kind,
                     void* hip_stream);

/* Replace every P+ (FP64 [m] in edge-id order, host or device). The topology is kept;
 * rows are re-sorted into Absolute Edge Order for the new values.
 * Errors: UTRI_E_INVALID for NaN or values outside [0,1] (the handle keeps its old P+). */
int utri_graph_set_p(utri_graph* g, const double* p, int ptr_kind, void* hip_stream);

/*
 * Counting problem (Definition "The Uncertain Balanced/Unbalanced Triangle Counting
 * Problem", Section 3) at threshold t in [0.5, 1].
 * out[0] = number of uncertain balanced triangles, out[1] = unbalanced (host int64 [2]);
 * a class not selected by `which` is reported as 0. method: UTRI_PLAIN / UTRI_PRUNED /
 * UTRI_PRUNED_L3. Waits for the stream.
 */
int utri_count(utri_graph* g, double t, int method, int which, int64_t out[2], void* hip_stream);

/*
 * utri_count without any device allocation, for callers that cannot allocate (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc). Same arguments,
 * results and errors as utri_count. Its scratch (row prefixes, work items, counters) lives
 * in a file-scope device array of UTRI_NOALLOC_SCRATCH_MB MiB that each GPU the library
 * runs on holds until the process ends; the call makes no hipMalloc, hipFree or other
 * allocating call. A graph whose query needs more scratch than that (about
 * 16 * (2n + 2) + 8 * work items bytes, n <= ~1.5 M vertices at R-MAT density) returns
 * UTRI_E_CAPACITY before any work is enqueued; UTRI_E_INVALID also when the current HIP
 * device is not the handle's. Every call on a GPU shares that GPU's array (the call
 * clears what must start at zero): calls that overlap on one GPU, from any thread,
 * stream or handle, race. Waits for the stream.
 */
#define UTRI_NOALLOC_SCRATCH_MB 64
int utri_count_noalloc(utri_graph* g, double t, int method, int which, int64_t out[2],
                       void* hip_stream);

/* Counts at nt thresholds (any order, 1 <= nt <= 64) from one walk at the smallest
 * one: out host int64 [nt][2]. Waits for the stream. */
int utri_count_batch(utri_graph* g, const double* t, int nt, int method, int64_t* out,
                     void* hip_stream);

/*
 * Enumeration problem (Section 3) at t. bal / unbal: device int32 [cap][3] triples of
 * original vertex ids, each triple sorted ascending. out_counts (host int64 [2]) gets
 * the full list sizes. sorted = 1 sorts each list lexicographically; sorted = 0 leaves
 * it in a deterministic walk order. A class not selected by `which` is neither
 * written nor counted. The call counts first (one walk) and then fills (a second). If a
 * list exceeds its capacity nothing is written and UTRI_E_CAPACITY is returned with the
 * sizes filled in, so the caller can retry: the handle then keeps the per-item counts of
 * that query, and the next utri_enumerate on it with the same t, method and which, while
 * the graph's P+, walk order and tuning are unchanged, fills from them without counting
 * again (once; any other outcome forgets them). Probing with capacities 0 and retrying
 * at the reported sizes therefore costs one counting walk and one fill.
 * Sorting a list of 2^32 triangles or more returns UTRI_E_RANGE (the unsorted list is
 * written).
 * Waits for the stream.
 */
int utri_enumerate(utri_graph* g, double t, int method, int which, int32_t* bal, int64_t cap_b,
                   int32_t* unbal, int64_t cap_u, int64_t out_counts[2], int sorted,
                   void* hip_stream);

/*
 * Expected number of balanced triangles E = sum over all triangles of P_bal (Section 3
 * four-term sum) = (T - sum s)/2. The sum of s is exact in 128-bit fixed point (each s
 * rounded to a multiple of 2^-62, ties to even) and E = (T*2^62 - S) * 2^-63 is
 * rounded once, so E does not depend on summation order. E: host double. Waits.
 */
int utri_expected(utri_graph* g, double* E, void* hip_stream);

/*
 * Gradient dE/dP+(e) for every edge: the sum over triangles (e, f, g) of d_f * d_g
 * (derivative of (1 - d_e d_f d_g)/2 with dd/dp = -2), each product rounded to FP64,
 * summed in the same fixed point and rounded once. grad: device FP64 [m] in edge-id
 * order. Each edge's sum is produced by one owner; no global atomics.
 */
int utri_expected_grad(utri_graph* g, double* grad, void* hip_stream);

/*
 * Local counts of Algorithm "Improved Edge Local Search" (Section 6.2): for each listed
 * edge id, the uncertain balanced / unbalanced triangles through it at each threshold.
 * eids: device int64 [k]; out: device int64 [k][nt][2]; 1 <= nt <= 64, t any order.
 */
int utri_edge_local(utri_graph* g, const double* t, int nt, const int64_t* eids, int64_t k,
                    int64_t* out, void* hip_stream);

/*
 * Local counts of the vertex-sampling framework (Algorithm "Baseline Vertex Sampling",
 * Section 6.1): for each listed vertex, every uncertain balanced / unbalanced triangle
 * containing it, at each threshold (the plain local count that the framework's
 * unbiasedness proof assumes; the improved vertex local search as printed counts some
 * triangles twice and misses others). vids: device int64 [k], original vertex ids in
 * [0, n) (UTRI_E_INVALID otherwise); out: device int64 [k][nt][2]; 1 <= nt <= 64.
 */
int utri_vertex_local(utri_graph* g, const double* t, int nt, const int64_t* vids, int64_t k,
                      int64_t* out, void* hip_stream);

/*
 * Possible-world Monte-Carlo of the expected balanced count (the possible-world model of
 * Section 3: every edge independently positive with probability P+). Sign world w of
 * edge e uses Philox4x32-10 with key (seed_lo, seed_hi) and counter (e, w / 4, 1, 0):
 * word w % 4 = u, the edge is positive iff u < P+(e) * 2^32. A triangle is balanced in
 * a world iff it has an even number of negative edges. counts: device int64 [worlds],
 * the balanced triangles of each world (their mean estimates E without bias; the exact
 * E is utri_expected). worlds: 32, 64, 128, 256, 512 or 1024 (UTRI_E_INVALID
 * otherwise). Needs 4 * m * worlds / 32 bytes of device scratch. Waits for the stream.
 */
int utri_sign_worlds(utri_graph* g, int32_t worlds, uint64_t seed, int64_t* counts,
                     void* hip_stream);

/*
 * Top-k search (Section 5, "Adaption to Top-k Search"): which = UTRI_BAL gives the k
 * triangles with the highest P_bal among those with P_bal >= 1/2 (the smallest
 * s = d1 d2 d3), UTRI_UNBAL the k with the highest P_unbal among those with P_unbal > 1/2
 * (the largest s); ties in s are broken by the sorted id triple, lexicographically.
 * tri: device int32 [k][3] original ids sorted within each triple, in rank order;
 * s: device FP64 [k], the canonical s of each (P_bal = (1 - s)/2); *count (host) = the
 * number written, min(k, #qualifying triangles). The threshold is tightened as the
 * paper describes, on the GPU by counting at 64 thresholds per walk (from t = 1
 * downwards, so every walk prunes with Lemma 2) until the class count at the largest
 * threshold still holding k triangles is small, then those candidates are enumerated,
 * valued and sorted. Errors: UTRI_E_INVALID for k < 0, another `which`, or missing
 * outputs. Waits for the stream.
 */
int utri_topk(utri_graph* g, int64_t k, int which, int32_t* tri, double* s, int64_t* count,
              void* hip_stream);

/*
 * Sampling estimators, `worlds` independent replicates of k uniform draws (with
 * replacement) each. Draw i of replicate w is Philox4x32-10 (Salmon et al., SC'11) with
 * key (seed_lo ^ w, seed_hi) and counter (i_lo, i_hi, 0, 0), mapped to the high 64 bits
 * of (x1:x0) * range.
 *  - UTRI_SAMPLE_EDGE (Algorithm "Baseline Edge Sampling" with the improved local
 *    search, Section 6.2): range m, est = m * (sum of edge local counts) / (3k);
 *  - UTRI_SAMPLE_VERTEX (Algorithm "Baseline Vertex Sampling", Section 6.1, with the
 *    plain vertex local count of utri_vertex_local): range n, est = n * (sum of vertex
 *    local counts) / (3k). Needs one host synchronisation to size its edge records.
 * est: device FP64 [worlds][nt][2], computed as ((double)sum * (double)range) /
 * (3.0 * (double)k). UTRI_SAMPLE_EDGE_PLAIN / UTRI_SAMPLE_VERTEX_PLAIN run the same
 * draws with the baseline local search (the paper's eBase / vBase), for comparison.
 * Errors: UTRI_E_INVALID for another scheme, k <= 0, worlds <= 0, or
 * an empty range (m = 0 for edges, n = 0 for vertices).
 */
int utri_sample(utri_graph* g, const double* t, int nt, int64_t k, int32_t worlds, uint64_t seed,
                int scheme, double* est, void* hip_stream);

/*
 * Batched queries in one persistent launch: exact counts at nt thresholds (one walk at
 * the smallest, binned by s) together with `worlds` replicates of the edge-sampling
 * estimator at the same thresholds. exact: device int64 [nt][2]; est: device FP64
 * [worlds][nt][2] (either may be NULL to skip that part). use_graph = 1 captures the
 * launch sequence into a hipGraph on the first call with a given shape and replays it
 * afterwards (t and seed are re-read from device buffers on every replay).
 */
int utri_batch(utri_graph* g, const double* t, int nt, int64_t k, int32_t worlds, uint64_t seed,
               int64_t* exact, double* est, int use_graph, void* hip_stream);

/*
 * Launch parameters of the walk and the sampler (the work-chunk and tile sizes of the
 * kernels that run Sections 4-6; no value changes any result), as int64 in this order:
 *   UTRI_TUNE_WALK_BLOCKS_PER_CU  walk work-groups per compute unit, 0 = the kernel's
 *                                 resident occupancy (default 0; 0..64);
 *   UTRI_TUNE_SAMPLE_CHUNK        draws per sampler group item (default 128; a multiple
 *                                 of 64 in 64..4096);
 *   UTRI_TUNE_WALK_PARTNERS       neighbours (partner rows) per walk work item (default
 *                                 1024; a multiple of 64 in 64..2^20);
 *   UTRI_TUNE_WALK_LIGHT_CAP      longest kept row staged by one wavefront, longer rows
 *                                 go to work-groups (default 128; a power of two, 8..128);
 *   UTRI_TUNE_WALK_CHUNK          row entries per work-group table chunk (default 2048; a
 *                                 power of two, at least 256 and the light cap, at most
 *                                 2048);
 *   UTRI_TUNE_WALK_UNROLL         row loads in flight per lane (default 8; 1, 2, 4, 8);
 *   UTRI_TUNE_WALK_SHORTER_MIN    under UTRI_ORDER_AUTO the walk streams the shorter kept
 *                                 row of each edge when the plain forward iteration would
 *                                 stream at least this many ids per kept edge (default
 *                                 320; 0..2^40).
 * utri_get_tuning writes the handle's current values to out (host int64
 * [UTRI_TUNE_COUNT]); utri_set_tuning validates all of in (host) and applies them to later
 * calls on g, or changes nothing and returns UTRI_E_INVALID.
 */
enum {
    UTRI_TUNE_WALK_BLOCKS_PER_CU = 0,
    UTRI_TUNE_SAMPLE_CHUNK = 1,
    UTRI_TUNE_WALK_PARTNERS = 2,
    UTRI_TUNE_WALK_LIGHT_CAP = 3,
    UTRI_TUNE_WALK_CHUNK = 4,
    UTRI_TUNE_WALK_UNROLL = 5,
    UTRI_TUNE_WALK_SHORTER_MIN = 6,
    UTRI_TUNE_COUNT = 7
};
int utri_get_tuning(utri_graph* g, int64_t out[UTRI_TUNE_COUNT]);
int utri_set_tuning(utri_graph* g, const int64_t in[UTRI_TUNE_COUNT]);

/*
 * Autotuner: picks the launch parameters above for this graph by timing the pruned
 * count at t (coordinate descent: work-groups per CU, partners per item, chunk size,
 * light cap, loads in flight, each over a few values, then the shorter-row crossover
 * moved so that t's query takes the faster of the two row orders) and the sampler at t
 * (draws per group item), and keeps the fastest for later calls on g. If cache_path is
 * not NULL and the file holds a choice for this graph shape (n, m, max degree), that
 * choice is applied without timing; otherwise the new choice is appended to it as one
 * JSON line. Handles created while the environment variable UTRI_TUNE_CACHE names such a
 * file start from its choice. Results never depend on these parameters.
 */
int utri_autotune(utri_graph* g, double t, const char* cache_path, void* hip_stream);

/*
 * Which row the triangle walk streams for each kept oriented edge u -> v (Section 4 visits
 * the w in N+(u) ∩ N+(v); any of these orders visits every triangle once, so results do
 * not depend on it). UTRI_ORDER_AUTO (the default) streams the shorter of the two kept
 * rows when the plain forward iteration would stream at least 320 ids per kept edge on
 * average, else N+(v); UTRI_ORDER_PLAIN always streams N+(v); UTRI_ORDER_SHORTER always
 * streams the shorter row (the sign-world walk always streams N+(v)). Applies to later
 * calls on g. Returns UTRI_E_INVALID for another value.
 */
enum { UTRI_ORDER_AUTO = 0, UTRI_ORDER_PLAIN = 1, UTRI_ORDER_SHORTER = 2 };
int utri_set_walk_order(utri_graph* g, int order);

/*
 * Work figures of one counting walk at t (the units the cost analysis of Theorem 5.1,
 * Section 5, sums over): out (host int64 [5]) =
 *   [0] m_c: oriented edges kept (sum of the kept oriented-row prefixes),
 *   [1] sum over kept oriented edges u -> v of the kept length of the row the walk
 *       streams for it: the shorter of N+(u) and N+(v) (N+(v) on ties) when that pays
 *       (the kept rows are long on average), else N+(v),
 *   [2] candidate triangles (streamed entries found in the staged row),
 *   [3] row entries actually streamed (a row is streamed once per chunk of a staged
 *       row longer than one work-group table),
 *   [4] work items. Waits for the stream.
 */
int utri_walk_stats(utri_graph* g, double t, int method, int64_t out[5], void* hip_stream);

/*
 * Event timing of the counting walk kernel launched by utri_count, recorded with HIP
 * events on the stream the kernel runs on. enable = 1 resets and starts recording,
 * 0 stops, any other value only reads. *ms and *launches (either may be NULL) return
 * the accumulated kernel time and the number of timed launches.
 */
int utri_timing(utri_graph* g, int enable, double* ms, int64_t* launches);

/* Human-readable text for a status code. */
const char* utri_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* UTRI_H */
