/*
 * oracle.c -- plain, slow CPU reference for counting, enumerating, the expected
 * balanced count, its gradient and the edge-sampling estimator of uncertain
 * balanced / unbalanced triangles (arXiv 2602.14084).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the library's product path may call,
 * link or load this file: only the tests, the smoke check and the benchmark's
 * CPU baseline use it. It shares no code with the HIP library; the two meet only
 * at the seeded input generators.
 *
 * How each function follows the paper:
 *  - orc_load: the uncertain signed graph of Definition "Uncertain Signed Graph"
 *    (Section 3): undirected, one P+ in [0,1] per edge. Self-loops and repeated
 *    edges are removed as the experiments section says of its datasets; a
 *    repeated edge with a different P+ is rejected, since an edge has one P+.
 *  - orc_count / orc_enumerate: the counting and enumeration problems of Section 3
 *    over every triangle, with the decisions of Definitions "Uncertain Balanced
 *    Triangle" (balanced with probability >= t) and "Uncertain Unbalanced
 *    Triangle" (unbalanced with probability > t). Triangles are listed by a plain
 *    node-iterator with hash sets: every pair of higher-ranked neighbours of a
 *    vertex is probed. Vertices are ranked by (degree, splitmix64(id)), a tie-break
 *    deliberately unlike the library's (degree, id) Node Order.
 *  - orc_enumerate_digest / orc_hash_triples: the same enumeration reduced to an
 *    order-free digest of each list (sum and xor of a hash of each sorted id triple)
 *    plus a hash-selected spot sample, for graphs whose lists are too long to hold.
 *    The lists are sets (Section 3), so an order-free digest is what can be compared.
 *  - The decision uses P_bal = (1 - s)/2 with s = d1*d2*d3 and d = 1 - 2*P+.
 *    This is the paper's four-term sum for P_bal (Section 3) in product form:
 *    P_bal >= t  <=>  s <= -(2t - 1),  P_unbal = 1 - P_bal > t  <=>  s > 2t - 1.
 *    In FP64: d = 1.0 - 2.0*p, c = 2.0*t - 1.0 (exact for t in [0.5, 1]), the three
 *    d values sorted ascending by value and s = (x*y)*z, no fused multiply-add.
 *  - orc_expected: E = sum over triangles of P_bal = (T - sum s)/2. The sum of s is
 *    kept exactly in 128-bit fixed point, each term rounded to the nearest
 *    multiple of 2^-62 (ties to even); E = (T*2^62 - S) * 2^-63 rounded once.
 *  - orc_grad: dE/dP+(e) for e = (a, b) is the sum over common neighbours w of
 *    d(a,w)*d(b,w) (differentiate (1 - d_e d_f d_g)/2 with dd_e/dp_e = -2); each
 *    product is rounded to FP64, summed in the same 2^-62 fixed point, rounded once.
 *  - orc_edge_local: the local count of Algorithm "Improved Edge Local Search"
 *    (Section 6.2): every triangle through the query edge, classified at t.
 *    Its pruning only skips triangles that cannot be classified, so the plain
 *    local count is the same number.
 *  - orc_sample: Algorithm "Baseline Edge Sampling" (Section 6.2) with exactly k
 *    uniform draws with replacement; the estimate is m * (sum of local counts)
 *    / (3k), the final value of the running mean. Draw i of world w uses
 *    Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with key
 *    (seed_lo ^ w, seed_hi) and counter (i_lo, i_hi, 0, 0); the edge index is the
 *    high 64 bits of (x1:x0) * m.
 *  - orc_vertex_local: the local count that the vertex-sampling framework (Section
 *    6.1) needs, taken as its plain definition: every triangle containing the query
 *    vertex, classified at t. (The improved vertex local search as printed counts
 *    some triangles twice and misses others; the unbiasedness proof assumes the
 *    plain count, which is what this computes.)
 *  - orc_topk: the top-k search of Section 5 ("Adaption to Top-k Search"), taken as
 *    its plain result: among the uncertain balanced triangles at t = 1/2 (P_bal >= 1/2,
 *    s <= 0) the k with the highest P_bal, i.e. the smallest s; among the unbalanced ones
 *    (P_unbal > 1/2, s > 0) the k with the largest s. Ties in s are broken by the sorted
 *    id triple, lexicographically; fewer than k qualifying triangles give all of them.
 *  - orc_sign_worlds: possible-world Monte-Carlo of the expected balanced count. The
 *    model of Section 3 makes every edge independently positive with probability
 *    P+(e); world w draws each edge's sign from Philox4x32-10 with key (seed_lo,
 *    seed_hi) and counter (e, w / 4, 1, 0), word w % 4 = u, positive iff
 *    u < P+(e) * 2^32. A triangle is balanced in a world iff it has an even number of
 *    negative edges; counts[w] is the number of balanced triangles of world w, whose
 *    mean over worlds estimates E = sum of P_bal without bias.
 *  - orc_sample_vertices: Algorithm "Baseline Vertex Sampling" (Section 6.1) with
 *    exactly k uniform draws with replacement; the estimate is n * (sum of local
 *    counts) / (3k). Vertex draw i of world w is the Philox block of edge draw i of
 *    world w, mapped to the high 64 bits of (x1:x0) * n.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum {
    ORC_OK = 0,
    ORC_E_INVALID = -1,
    ORC_E_CONFLICT = -2,
    ORC_E_CAPACITY = -3,
    ORC_E_NOMEM = -4,
    ORC_E_RANGE = -6
};

typedef struct {
    int64_t n, m;
    int32_t *lo, *hi;   /* canonical edges (lo < hi) sorted by (lo, hi); edge id = index */
    double *p, *d;      /* P+(e) and d(e) = 1 - 2 P+(e) */
    int64_t *off;       /* adjacency offsets, [n+1] */
    int32_t *nbr;       /* neighbour ids, ascending within a vertex, [2m] */
    int32_t *eid;       /* edge id of each adjacency entry, [2m] */
    int64_t *hoff;      /* hash set offsets, [n+1]; each size is 0 or a power of two */
    int32_t *hkey;      /* neighbour id, or -1 for an empty slot */
    int32_t *hval;      /* edge id stored with the key */
    int64_t *rank;      /* position of each vertex in (degree, splitmix64(id)) order */
    int64_t self_loops, dups, max_deg;
} orc_graph;

static uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
}

/* ---------------------------------------------------------------- decision */

static double orc_d(double p) { return 1.0 - 2.0 * p; }
static double orc_c(double t) { return 2.0 * t - 1.0; }

/* s = (x*y)*z over the three d values sorted ascending by value. */
static double orc_s(double a, double b, double c) {
    double t;
    if (b < a) { t = a; a = b; b = t; }
    if (c < b) { t = b; b = c; c = t; }
    if (b < a) { t = a; a = b; b = t; }
    volatile double xy = a * b;  /* two separate roundings, never fused */
    return xy * c;
}

/* 1 = uncertain balanced (P_bal >= t), 2 = uncertain unbalanced (P_unbal > t), 0 = neither. */
static int orc_classify(double s, double cthr) {
    if (s <= -cthr) return 1;
    if (s > cthr) return 2;
    return 0;
}

/* nearest multiple of 2^-62, ties to even, as an integer (|x| <= 1). */
static int64_t orc_fix62(double x) {
    return (int64_t)nearbyint(x * 0x1p62);
}

/* ---------------------------------------------------------------- loading */

typedef struct { uint64_t key; double p; } orc_kp;

static int cmp_kp(const void* a, const void* b) {
    const orc_kp* x = (const orc_kp*)a;
    const orc_kp* y = (const orc_kp*)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return 0;
}

typedef struct { int32_t nbr, eid; } orc_ne;

static int cmp_ne(const void* a, const void* b) {
    const orc_ne* x = (const orc_ne*)a;
    const orc_ne* y = (const orc_ne*)b;
    return (x->nbr > y->nbr) - (x->nbr < y->nbr);
}

static const int64_t* g_sort_deg;
static const uint64_t* g_sort_mix;

static int cmp_rank(const void* a, const void* b) {
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    if (g_sort_deg[x] != g_sort_deg[y]) return g_sort_deg[x] < g_sort_deg[y] ? -1 : 1;
    if (g_sort_mix[x] != g_sort_mix[y]) return g_sort_mix[x] < g_sort_mix[y] ? -1 : 1;
    return 0;
}

void orc_free(orc_graph* g) {
    if (!g) return;
    free(g->lo); free(g->hi); free(g->p); free(g->d);
    free(g->off); free(g->nbr); free(g->eid);
    free(g->hoff); free(g->hkey); free(g->hval); free(g->rank);
    free(g);
}

static uint32_t hslot(int32_t key, uint64_t mask) {
    return (uint32_t)(splitmix64((uint64_t)(uint32_t)key) & mask);
}

/* edge id of (a, b), or -1 when a and b are not adjacent */
static int32_t orc_find(const orc_graph* g, int32_t a, int32_t b) {
    int64_t base = g->hoff[a];
    uint64_t size = (uint64_t)(g->hoff[a + 1] - base);
    if (size == 0) return -1;
    uint64_t mask = size - 1;
    uint64_t h = hslot(b, mask);
    for (;;) {
        int32_t k = g->hkey[base + h];
        if (k == b) return g->hval[base + h];
        if (k == -1) return -1;
        h = (h + 1) & mask;
    }
}

int orc_load(int64_t n, int64_t m_in, const int64_t* src, const int64_t* dst, const double* p,
             orc_graph** out) {
    *out = NULL;
    if (n < 0 || m_in < 0) return ORC_E_INVALID;
    if (n >= ((int64_t)1 << 31)) return ORC_E_RANGE;
    if (m_in > 0 && (!src || !dst || !p)) return ORC_E_INVALID;
    for (int64_t i = 0; i < m_in; i++) {
        if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) return ORC_E_INVALID;
        if (!(p[i] >= 0.0 && p[i] <= 1.0)) return ORC_E_INVALID; /* NaN fails both */
    }
    orc_graph* g = (orc_graph*)calloc(1, sizeof(orc_graph));
    if (!g) return ORC_E_NOMEM;
    g->n = n;
    orc_kp* kp = (orc_kp*)malloc(sizeof(orc_kp) * (size_t)(m_in > 0 ? m_in : 1));
    if (!kp) { orc_free(g); return ORC_E_NOMEM; }
    int64_t k = 0;
    for (int64_t i = 0; i < m_in; i++) {
        int64_t a = src[i], b = dst[i];
        if (a == b) { g->self_loops++; continue; }
        int64_t lo = a < b ? a : b, hi = a < b ? b : a;
        kp[k].key = ((uint64_t)lo << 32) | (uint64_t)hi;
        kp[k].p = p[i];
        k++;
    }
    qsort(kp, (size_t)k, sizeof(orc_kp), cmp_kp);
    int64_t m = 0;
    for (int64_t i = 0; i < k; i++) {
        if (m > 0 && kp[m - 1].key == kp[i].key) {
            if (kp[m - 1].p != kp[i].p) { free(kp); orc_free(g); return ORC_E_CONFLICT; }
            g->dups++;
            continue;
        }
        kp[m++] = kp[i];
    }
    if (m >= ((int64_t)1 << 31)) { free(kp); orc_free(g); return ORC_E_RANGE; }
    g->m = m;
    size_t ms = (size_t)(m > 0 ? m : 1);
    g->lo = (int32_t*)malloc(sizeof(int32_t) * ms);
    g->hi = (int32_t*)malloc(sizeof(int32_t) * ms);
    g->p = (double*)malloc(sizeof(double) * ms);
    g->d = (double*)malloc(sizeof(double) * ms);
    g->off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    g->nbr = (int32_t*)malloc(sizeof(int32_t) * 2 * ms);
    g->eid = (int32_t*)malloc(sizeof(int32_t) * 2 * ms);
    g->hoff = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    g->rank = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!g->lo || !g->hi || !g->p || !g->d || !g->off || !g->nbr || !g->eid || !g->hoff ||
        !g->rank) {
        free(kp); orc_free(g); return ORC_E_NOMEM;
    }
    for (int64_t e = 0; e < m; e++) {
        g->lo[e] = (int32_t)(kp[e].key >> 32);
        g->hi[e] = (int32_t)(kp[e].key & 0xFFFFFFFFu);
        g->p[e] = kp[e].p;
        g->d[e] = orc_d(kp[e].p);
    }
    free(kp);
    /* adjacency by counting, then each row sorted by neighbour id */
    for (int64_t e = 0; e < m; e++) { g->off[g->lo[e] + 1]++; g->off[g->hi[e] + 1]++; }
    for (int64_t v = 0; v < n; v++) g->off[v + 1] += g->off[v];
    int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!cur) { orc_free(g); return ORC_E_NOMEM; }
    for (int64_t v = 0; v < n; v++) cur[v] = g->off[v];
    for (int64_t e = 0; e < m; e++) {
        int32_t a = g->lo[e], b = g->hi[e];
        g->nbr[cur[a]] = b; g->eid[cur[a]] = (int32_t)e; cur[a]++;
        g->nbr[cur[b]] = a; g->eid[cur[b]] = (int32_t)e; cur[b]++;
    }
    free(cur);
    g->max_deg = 0;
    for (int64_t v = 0; v < n; v++) {
        int64_t dv = g->off[v + 1] - g->off[v];
        if (dv > g->max_deg) g->max_deg = dv;
        if (dv > 1) {
            orc_ne* tmp = (orc_ne*)malloc(sizeof(orc_ne) * (size_t)dv);
            if (!tmp) { orc_free(g); return ORC_E_NOMEM; }
            for (int64_t j = 0; j < dv; j++) {
                tmp[j].nbr = g->nbr[g->off[v] + j];
                tmp[j].eid = g->eid[g->off[v] + j];
            }
            qsort(tmp, (size_t)dv, sizeof(orc_ne), cmp_ne);
            for (int64_t j = 0; j < dv; j++) {
                g->nbr[g->off[v] + j] = tmp[j].nbr;
                g->eid[g->off[v] + j] = tmp[j].eid;
            }
            free(tmp);
        }
    }
    /* open-addressing hash set per vertex: size = smallest power of two >= 2*deg */
    for (int64_t v = 0; v < n; v++) {
        int64_t dv = g->off[v + 1] - g->off[v];
        int64_t size = 0;
        if (dv > 0) { size = 1; while (size < 2 * dv) size <<= 1; }
        g->hoff[v + 1] = g->hoff[v] + size;
    }
    int64_t htot = g->hoff[n];
    g->hkey = (int32_t*)malloc(sizeof(int32_t) * (size_t)(htot > 0 ? htot : 1));
    g->hval = (int32_t*)malloc(sizeof(int32_t) * (size_t)(htot > 0 ? htot : 1));
    if (!g->hkey || !g->hval) { orc_free(g); return ORC_E_NOMEM; }
    for (int64_t i = 0; i < htot; i++) g->hkey[i] = -1;
    for (int64_t v = 0; v < n; v++) {
        int64_t base = g->hoff[v];
        uint64_t size = (uint64_t)(g->hoff[v + 1] - base);
        if (!size) continue;
        for (int64_t j = g->off[v]; j < g->off[v + 1]; j++) {
            uint64_t h = hslot(g->nbr[j], size - 1);
            while (g->hkey[base + h] != -1) h = (h + 1) & (size - 1);
            g->hkey[base + h] = g->nbr[j];
            g->hval[base + h] = g->eid[j];
        }
    }
    /* rank by (degree, splitmix64(id)) */
    int64_t* degs = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    uint64_t* mix = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!degs || !mix || !order) { free(degs); free(mix); free(order); orc_free(g); return ORC_E_NOMEM; }
    for (int64_t v = 0; v < n; v++) {
        degs[v] = g->off[v + 1] - g->off[v];
        mix[v] = splitmix64((uint64_t)v);
        order[v] = v;
    }
    g_sort_deg = degs;
    g_sort_mix = mix;
    qsort(order, (size_t)n, sizeof(int64_t), cmp_rank);
    for (int64_t i = 0; i < n; i++) g->rank[order[i]] = i;
    free(degs); free(mix); free(order);
    *out = g;
    return ORC_OK;
}

void orc_info(const orc_graph* g, int64_t* n, int64_t* m, int64_t* self_loops, int64_t* dups,
              int64_t* max_deg) {
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (self_loops) *self_loops = g->self_loops;
    if (dups) *dups = g->dups;
    if (max_deg) *max_deg = g->max_deg;
}

void orc_edges(const orc_graph* g, int32_t* lo, int32_t* hi, double* p) {
    for (int64_t e = 0; e < g->m; e++) {
        if (lo) lo[e] = g->lo[e];
        if (hi) hi[e] = g->hi[e];
        if (p) p[e] = g->p[e];
    }
}

/* ---------------------------------------------------------------- node iterator */

/* Visit every triangle once, from its lowest-ranked vertex u. The callback gets the
 * three vertex ids and the three edge ids (uv, uw, vw). */
typedef void (*orc_visit_fn)(void* ctx, int tid, int32_t u, int32_t v, int32_t w,
                             int32_t euv, int32_t euw, int32_t evw);

static int orc_node_iterate_list(const orc_graph* g, const int64_t* list, int64_t nlist,
                                 orc_visit_fn fn, void* ctx);

static int orc_node_iterate(const orc_graph* g, orc_visit_fn fn, void* ctx, int nthreads_hint) {
    (void)nthreads_hint;
    return orc_node_iterate_list(g, NULL, g->n, fn, ctx);
}

/* Node iterator over the listed vertices (all vertices when list is NULL). */
static int orc_node_iterate_list(const orc_graph* g, const int64_t* list, int64_t nlist,
                                 orc_visit_fn fn, void* ctx) {
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    int64_t cap = g->max_deg > 0 ? g->max_deg : 1;
    int32_t* hv = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap * (size_t)nt);
    int32_t* he = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap * (size_t)nt);
    if (!hv || !he) { free(hv); free(he); return ORC_E_NOMEM; }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t iu = 0; iu < nlist; iu++) {
        const int64_t u = list ? list[iu] : iu;
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        int32_t* H = hv + (size_t)tid * (size_t)cap;
        int32_t* HE = he + (size_t)tid * (size_t)cap;
        int64_t h = 0;
        for (int64_t j = g->off[u]; j < g->off[u + 1]; j++) {
            int32_t v = g->nbr[j];
            if (g->rank[v] > g->rank[u]) { H[h] = v; HE[h] = g->eid[j]; h++; }
        }
        for (int64_t i = 0; i < h; i++) {
            for (int64_t j = i + 1; j < h; j++) {
                int32_t evw = orc_find(g, H[i], H[j]);
                if (evw >= 0) fn(ctx, tid, (int32_t)u, H[i], H[j], HE[i], HE[j], evw);
            }
        }
    }
    free(hv); free(he);
    return ORC_OK;
}

static int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int orc_num_threads(void) { return orc_threads(); }

/* Use n OpenMP threads from now on (n >= 1); returns the count in effect. */
int orc_set_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#endif
    return orc_threads();
}

/* Work of the node iterator, in hash probes: C(h, 2) for a vertex with h higher-ranked
 * neighbours. out[0] = over the listed vertices, out[1] = over all vertices (so a timed
 * run over the listed vertices scales to the whole graph by out[1] / out[0]). */
int orc_probe_work(const orc_graph* g, const int64_t* us, int64_t k, int64_t out[2]) {
    int64_t tot = 0, part = 0;
    for (int64_t u = 0; u < g->n; u++) {
        int64_t h = 0;
        for (int64_t j = g->off[u]; j < g->off[u + 1]; j++)
            if (g->rank[g->nbr[j]] > g->rank[u]) h++;
        tot += h * (h - 1) / 2;
    }
    for (int64_t i = 0; i < k; i++) {
        if (us[i] < 0 || us[i] >= g->n) return ORC_E_INVALID;
        int64_t u = us[i], h = 0;
        for (int64_t j = g->off[u]; j < g->off[u + 1]; j++)
            if (g->rank[g->nbr[j]] > g->rank[u]) h++;
        part += h * (h - 1) / 2;
    }
    out[0] = part;
    out[1] = tot;
    return ORC_OK;
}

typedef struct { int64_t v[8]; } orc_pad; /* one cache line of counters per thread */

typedef struct {
    const orc_graph* g;
    const double* c;  /* thresholds c_j = 2 t_j - 1 */
    int nt;
    int64_t* cnt;     /* [threads][nt][2] */
} count_ctx;

static void count_visit(void* vctx, int tid, int32_t u, int32_t v, int32_t w, int32_t euv,
                        int32_t euw, int32_t evw) {
    (void)u; (void)v; (void)w;
    count_ctx* cx = (count_ctx*)vctx;
    const double* d = cx->g->d;
    double s = orc_s(d[euv], d[euw], d[evw]);
    for (int j = 0; j < cx->nt; j++) {
        int k = orc_classify(s, cx->c[j]);
        if (k) cx->cnt[((size_t)tid * cx->nt + j) * 2 + (k - 1)]++;
    }
}

static int check_t(double t) { return (t >= 0.5 && t <= 1.0) ? ORC_OK : ORC_E_INVALID; }

/* counts[j][0] = |B^t_j|, counts[j][1] = |U^t_j| for every threshold t_j */
int orc_count_multi(const orc_graph* g, const double* t, int nt, int64_t* counts) {
    if (nt <= 0) return ORC_E_INVALID;
    double* c = (double*)malloc(sizeof(double) * (size_t)nt);
    if (!c) return ORC_E_NOMEM;
    for (int j = 0; j < nt; j++) {
        if (check_t(t[j])) { free(c); return ORC_E_INVALID; }
        c[j] = orc_c(t[j]);
    }
    int th = orc_threads();
    count_ctx cx = {g, c, nt, (int64_t*)calloc((size_t)th * nt * 2, sizeof(int64_t))};
    if (!cx.cnt) { free(c); return ORC_E_NOMEM; }
    int rc = orc_node_iterate(g, count_visit, &cx, th);
    for (int j = 0; j < nt; j++) {
        counts[2 * j] = counts[2 * j + 1] = 0;
        for (int q = 0; q < th; q++) {
            counts[2 * j] += cx.cnt[((size_t)q * nt + j) * 2];
            counts[2 * j + 1] += cx.cnt[((size_t)q * nt + j) * 2 + 1];
        }
    }
    free(cx.cnt); free(c);
    return rc;
}

int orc_count(const orc_graph* g, double t, int64_t out[2]) {
    return orc_count_multi(g, &t, 1, out);
}

/* Counts of the triangles whose lowest-ranked vertex is listed (a vertex sample of the
 * node iterator; summed over all vertices it is orc_count). */
int orc_count_vertices(const orc_graph* g, double t, const int64_t* us, int64_t k,
                       int64_t out[2]) {
    if (check_t(t)) return ORC_E_INVALID;
    for (int64_t i = 0; i < k; i++)
        if (us[i] < 0 || us[i] >= g->n) return ORC_E_INVALID;
    double c = orc_c(t);
    int th = orc_threads();
    count_ctx cx = {g, &c, 1, (int64_t*)calloc((size_t)th * 2, sizeof(int64_t))};
    if (!cx.cnt) return ORC_E_NOMEM;
    int rc = orc_node_iterate_list(g, us, k, count_visit, &cx);
    out[0] = out[1] = 0;
    for (int q = 0; q < th; q++) { out[0] += cx.cnt[2 * q]; out[1] += cx.cnt[2 * q + 1]; }
    free(cx.cnt);
    return rc;
}

/* ---------------------------------------------------------------- enumeration */

typedef struct { int32_t* buf; int64_t len, cap; } orc_vec;

static int vec_push(orc_vec* v, int32_t a, int32_t b, int32_t c) {
    if (v->len == v->cap) {
        int64_t nc = v->cap ? 2 * v->cap : 1024;
        int32_t* nb = (int32_t*)realloc(v->buf, sizeof(int32_t) * 3 * (size_t)nc);
        if (!nb) return -1;
        v->buf = nb; v->cap = nc;
    }
    v->buf[3 * v->len] = a; v->buf[3 * v->len + 1] = b; v->buf[3 * v->len + 2] = c;
    v->len++;
    return 0;
}

typedef struct {
    const orc_graph* g;
    double c;
    orc_vec* bal;    /* [threads] */
    orc_vec* unbal;  /* [threads] */
    int* fail;       /* [threads] */
} enum_ctx;

static void enum_visit(void* vctx, int tid, int32_t u, int32_t v, int32_t w, int32_t euv,
                       int32_t euw, int32_t evw) {
    enum_ctx* cx = (enum_ctx*)vctx;
    const double* d = cx->g->d;
    int k = orc_classify(orc_s(d[euv], d[euw], d[evw]), cx->c);
    if (!k) return;
    int32_t a = u, b = v, c = w, t;
    if (b < a) { t = a; a = b; b = t; }
    if (c < b) { t = b; b = c; c = t; }
    if (b < a) { t = a; a = b; b = t; }
    orc_vec* dst = (k == 1) ? &cx->bal[tid] : &cx->unbal[tid];
    if (vec_push(dst, a, b, c)) cx->fail[tid] = 1;
}

static int cmp_tri(const void* x, const void* y) {
    const int32_t* a = (const int32_t*)x;
    const int32_t* b = (const int32_t*)y;
    for (int i = 0; i < 3; i++)
        if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    return 0;
}

/* Lists of uncertain balanced and unbalanced triangles at t as id triples sorted
 * within each triple, the lists sorted lexicographically. counts[] always holds the
 * full sizes; ORC_E_CAPACITY when either list does not fit. */
int orc_enumerate(const orc_graph* g, double t, int32_t* bal, int64_t cap_b, int32_t* unbal,
                  int64_t cap_u, int64_t counts[2]) {
    if (check_t(t)) return ORC_E_INVALID;
    int th = orc_threads();
    enum_ctx cx;
    cx.g = g;
    cx.c = orc_c(t);
    cx.bal = (orc_vec*)calloc((size_t)th, sizeof(orc_vec));
    cx.unbal = (orc_vec*)calloc((size_t)th, sizeof(orc_vec));
    cx.fail = (int*)calloc((size_t)th, sizeof(int));
    if (!cx.bal || !cx.unbal || !cx.fail) { free(cx.bal); free(cx.unbal); free(cx.fail); return ORC_E_NOMEM; }
    int rc = orc_node_iterate(g, enum_visit, &cx, th);
    int64_t nb = 0, nu = 0;
    for (int q = 0; q < th; q++) {
        if (cx.fail[q]) rc = ORC_E_NOMEM;
        nb += cx.bal[q].len;
        nu += cx.unbal[q].len;
    }
    counts[0] = nb;
    counts[1] = nu;
    if (rc == ORC_OK && (nb > cap_b || nu > cap_u)) rc = ORC_E_CAPACITY;
    if (rc == ORC_OK) {
        int64_t ib = 0, iu = 0;
        for (int q = 0; q < th; q++) {
            memcpy(bal + 3 * ib, cx.bal[q].buf, sizeof(int32_t) * 3 * (size_t)cx.bal[q].len);
            ib += cx.bal[q].len;
            memcpy(unbal + 3 * iu, cx.unbal[q].buf, sizeof(int32_t) * 3 * (size_t)cx.unbal[q].len);
            iu += cx.unbal[q].len;
        }
        qsort(bal, (size_t)nb, 3 * sizeof(int32_t), cmp_tri);
        qsort(unbal, (size_t)nu, 3 * sizeof(int32_t), cmp_tri);
    }
    for (int q = 0; q < th; q++) { free(cx.bal[q].buf); free(cx.unbal[q].buf); }
    free(cx.bal); free(cx.unbal); free(cx.fail);
    return rc;
}

/* ---------------------------------------------------------------- enumeration digest */

/* Order-free digest of a list of triangles, for lists too long to hold (the enumeration
 * problem of Section 3 lists sets; their order is free). Each triangle is its id triple
 * sorted ascending, a < b < c, hashed as
 *     h(a, b, c) = splitmix64(splitmix64((a << 32) | b) + c)   (mod 2^64);
 * a list's digest is (sum of h mod 2^64, xor of h). A spot sample keeps the triangles
 * whose top `sample_bits` bits of h are zero, a deterministic subset that another
 * implementation can pick out of its own list. */
static uint64_t orc_triple_hash(int32_t a, int32_t b, int32_t c) {
    uint64_t x = splitmix64(((uint64_t)(uint32_t)a << 32) | (uint64_t)(uint32_t)b);
    return splitmix64(x + (uint64_t)(uint32_t)c);
}

static int orc_in_sample(uint64_t h, int sample_bits) {
    if (sample_bits <= 0) return 1;
    if (sample_bits >= 64) return h == 0;
    return (h >> (64 - sample_bits)) == 0;
}

/* Digest (out[0] = sum, out[1] = xor) of n triples tri[n][3], each sorted ascending
 * (ORC_E_INVALID otherwise), and the spot sample (up to cap triples copied to samp,
 * *nsamp = how many qualify). */
int orc_hash_triples(const int32_t* tri, int64_t n, int sample_bits, uint64_t out[2],
                     int32_t* samp, int64_t cap, int64_t* nsamp) {
    uint64_t s = 0, x = 0;
    int64_t ns = 0;
    for (int64_t i = 0; i < n; i++) {
        const int32_t a = tri[3 * i], b = tri[3 * i + 1], c = tri[3 * i + 2];
        if (!(a < b && b < c)) return ORC_E_INVALID;
        const uint64_t h = orc_triple_hash(a, b, c);
        s += h;
        x ^= h;
        if (orc_in_sample(h, sample_bits)) {
            if (ns < cap) { samp[3 * ns] = a; samp[3 * ns + 1] = b; samp[3 * ns + 2] = c; }
            ns++;
        }
    }
    out[0] = s;
    out[1] = x;
    *nsamp = ns;
    return ORC_OK;
}

typedef struct {
    const orc_graph* g;
    double c;
    uint64_t* acc;      /* [threads][8]: sum_b, xor_b, sum_u, xor_u, n_b, n_u (padded) */
    orc_vec* samp_b;    /* [threads] */
    orc_vec* samp_u;
    int sample_bits;
    int* fail;
} digest_ctx;

static void digest_visit(void* vctx, int tid, int32_t u, int32_t v, int32_t w, int32_t euv,
                         int32_t euw, int32_t evw) {
    digest_ctx* cx = (digest_ctx*)vctx;
    const double* d = cx->g->d;
    int k = orc_classify(orc_s(d[euv], d[euw], d[evw]), cx->c);
    if (!k) return;
    int32_t a = u, b = v, c = w, t;
    if (b < a) { t = a; a = b; b = t; }
    if (c < b) { t = b; b = c; c = t; }
    if (b < a) { t = a; a = b; b = t; }
    const uint64_t h = orc_triple_hash(a, b, c);
    uint64_t* A = cx->acc + 8 * (size_t)tid + (k == 1 ? 0 : 2);
    A[0] += h;
    A[1] ^= h;
    cx->acc[8 * (size_t)tid + 4 + (k - 1)]++;
    if (orc_in_sample(h, cx->sample_bits)) {
        orc_vec* dst = (k == 1) ? &cx->samp_b[tid] : &cx->samp_u[tid];
        if (vec_push(dst, a, b, c)) cx->fail[tid] = 1;
    }
}

/* The enumeration at t without storing it: counts[0..1] = list sizes, digest[0..1] =
 * (sum, xor) of the balanced list and digest[2..3] of the unbalanced one (see
 * orc_hash_triples), and each list's spot sample, sorted lexicographically, in
 * samp_b / samp_u (up to cap_b / cap_u triples; ns[0..1] = how many qualify). */
int orc_enumerate_digest(const orc_graph* g, double t, int sample_bits, int64_t counts[2],
                         uint64_t digest[4], int32_t* samp_b, int64_t cap_b, int32_t* samp_u,
                         int64_t cap_u, int64_t ns[2]) {
    if (check_t(t)) return ORC_E_INVALID;
    int th = orc_threads();
    digest_ctx cx;
    cx.g = g;
    cx.c = orc_c(t);
    cx.sample_bits = sample_bits;
    cx.acc = (uint64_t*)calloc((size_t)th * 8, sizeof(uint64_t));
    cx.samp_b = (orc_vec*)calloc((size_t)th, sizeof(orc_vec));
    cx.samp_u = (orc_vec*)calloc((size_t)th, sizeof(orc_vec));
    cx.fail = (int*)calloc((size_t)th, sizeof(int));
    if (!cx.acc || !cx.samp_b || !cx.samp_u || !cx.fail) {
        free(cx.acc); free(cx.samp_b); free(cx.samp_u); free(cx.fail);
        return ORC_E_NOMEM;
    }
    int rc = orc_node_iterate(g, digest_visit, &cx, th);
    for (int i = 0; i < 4; i++) digest[i] = 0;
    counts[0] = counts[1] = 0;
    ns[0] = ns[1] = 0;
    for (int q = 0; q < th; q++) {
        const uint64_t* A = cx.acc + 8 * (size_t)q;
        digest[0] += A[0]; digest[1] ^= A[1];
        digest[2] += A[2]; digest[3] ^= A[3];
        counts[0] += (int64_t)A[4];
        counts[1] += (int64_t)A[5];
        if (cx.fail[q]) rc = ORC_E_NOMEM;
        ns[0] += cx.samp_b[q].len;
        ns[1] += cx.samp_u[q].len;
    }
    if (rc == ORC_OK) {
        int64_t ib = 0, iu = 0;
        for (int q = 0; q < th; q++) {
            for (int64_t i = 0; i < cx.samp_b[q].len; i++, ib++)
                if (ib < cap_b) memcpy(samp_b + 3 * ib, cx.samp_b[q].buf + 3 * i, 3 * sizeof(int32_t));
            for (int64_t i = 0; i < cx.samp_u[q].len; i++, iu++)
                if (iu < cap_u) memcpy(samp_u + 3 * iu, cx.samp_u[q].buf + 3 * i, 3 * sizeof(int32_t));
        }
        qsort(samp_b, (size_t)(ib < cap_b ? ib : cap_b), 3 * sizeof(int32_t), cmp_tri);
        qsort(samp_u, (size_t)(iu < cap_u ? iu : cap_u), 3 * sizeof(int32_t), cmp_tri);
    }
    for (int q = 0; q < th; q++) { free(cx.samp_b[q].buf); free(cx.samp_u[q].buf); }
    free(cx.acc); free(cx.samp_b); free(cx.samp_u); free(cx.fail);
    return rc;
}

/* ---------------------------------------------------------------- expected count */

typedef struct {
    const orc_graph* g;
    __int128* sum;   /* [threads * 4] (padded) */
    int64_t* tri;    /* [threads * 8] (padded) */
} exp_ctx;

static void exp_visit(void* vctx, int tid, int32_t u, int32_t v, int32_t w, int32_t euv,
                      int32_t euw, int32_t evw) {
    (void)u; (void)v; (void)w;
    exp_ctx* cx = (exp_ctx*)vctx;
    const double* d = cx->g->d;
    cx->sum[(size_t)tid * 4] += (__int128)orc_fix62(orc_s(d[euv], d[euw], d[evw]));
    cx->tri[(size_t)tid * 8] += 1;
}

/* E = sum over all triangles of P_bal; also the triangle count T and the fixed-point
 * sum S of s (two's complement, S = s_hi * 2^64 + s_lo). */
int orc_expected(const orc_graph* g, double* E, int64_t* T, uint64_t* s_lo, int64_t* s_hi) {
    int th = orc_threads();
    exp_ctx cx = {g, (__int128*)calloc((size_t)th * 4, sizeof(__int128)),
                  (int64_t*)calloc((size_t)th * 8, sizeof(int64_t))};
    if (!cx.sum || !cx.tri) { free(cx.sum); free(cx.tri); return ORC_E_NOMEM; }
    int rc = orc_node_iterate(g, exp_visit, &cx, th);
    __int128 S = 0;
    int64_t tri = 0;
    for (int q = 0; q < th; q++) { S += cx.sum[(size_t)q * 4]; tri += cx.tri[(size_t)q * 8]; }
    free(cx.sum); free(cx.tri);
    __int128 num = ((__int128)tri << 62) - S;
    if (E) *E = (double)num * 0x1p-63;
    if (T) *T = tri;
    if (s_lo) *s_lo = (uint64_t)S;
    if (s_hi) *s_hi = (int64_t)(S >> 64);
    return rc;
}

/* ---------------------------------------------------------------- per-edge work */

static int check_eids(const orc_graph* g, const int64_t* eids, int64_t k) {
    for (int64_t i = 0; i < k; i++)
        if (eids[i] < 0 || eids[i] >= g->m) return ORC_E_INVALID;
    return ORC_OK;
}

/* dE/dP+(e) for each listed edge id */
int orc_grad(const orc_graph* g, const int64_t* eids, int64_t k, double* out) {
    if (check_eids(g, eids, k)) return ORC_E_INVALID;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < k; i++) {
        int64_t e = eids[i];
        int32_t a = g->lo[e], b = g->hi[e];
        __int128 S = 0;
        for (int64_t j = g->off[a]; j < g->off[a + 1]; j++) {
            int32_t w = g->nbr[j];
            if (w == b) continue;
            int32_t ebw = orc_find(g, b, w);
            if (ebw < 0) continue;
            S += (__int128)orc_fix62(g->d[g->eid[j]] * g->d[ebw]);
        }
        out[i] = (double)S * 0x1p-62;
    }
    return ORC_OK;
}

/* Local expected balanced count of edge e with its P+ replaced by q:
 * L_e(q) = sum over triangles (e, f, g) of P_bal = (1 - s)/2, s = d(q) d_f d_g.
 * Returned exactly as N = cnt * 2^62 - sum fix62(s) (two's complement hi:lo), so
 * L_e(q) = N * 2^-63 and a central difference of L_e is exact up to 2^-63 per term. */
int orc_local_expected(const orc_graph* g, const int64_t* eids, const double* q, int64_t k,
                       int64_t* n_hi, uint64_t* n_lo) {
    if (check_eids(g, eids, k)) return ORC_E_INVALID;
    for (int64_t i = 0; i < k; i++)
        if (!(q[i] >= 0.0 && q[i] <= 1.0)) return ORC_E_INVALID;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < k; i++) {
        int64_t e = eids[i];
        int32_t a = g->lo[e], b = g->hi[e];
        double de = orc_d(q[i]);
        __int128 S = 0, cnt = 0;
        for (int64_t j = g->off[a]; j < g->off[a + 1]; j++) {
            int32_t w = g->nbr[j];
            if (w == b) continue;
            int32_t ebw = orc_find(g, b, w);
            if (ebw < 0) continue;
            S += (__int128)orc_fix62(orc_s(de, g->d[g->eid[j]], g->d[ebw]));
            cnt += 1;
        }
        __int128 N = (cnt << 62) - S;
        n_hi[i] = (int64_t)(N >> 64);
        n_lo[i] = (uint64_t)N;
    }
    return ORC_OK;
}

/* local counts at each threshold: out[i][j][0/1] = (balanced, unbalanced) triangles
 * through edge eids[i] at t_j */
static void edge_local_one(const orc_graph* g, int64_t e, const double* c, int nt, int64_t* out) {
    int32_t a = g->lo[e], b = g->hi[e];
    for (int j = 0; j < nt; j++) out[2 * j] = out[2 * j + 1] = 0;
    for (int64_t q = g->off[a]; q < g->off[a + 1]; q++) {
        int32_t w = g->nbr[q];
        if (w == b) continue;
        int32_t ebw = orc_find(g, b, w);
        if (ebw < 0) continue;
        double s = orc_s(g->d[e], g->d[g->eid[q]], g->d[ebw]);
        for (int j = 0; j < nt; j++) {
            int k = orc_classify(s, c[j]);
            if (k) out[2 * j + (k - 1)]++;
        }
    }
}

int orc_edge_local(const orc_graph* g, const double* t, int nt, const int64_t* eids, int64_t k,
                   int64_t* out) {
    if (nt <= 0 || check_eids(g, eids, k)) return ORC_E_INVALID;
    double* c = (double*)malloc(sizeof(double) * (size_t)nt);
    if (!c) return ORC_E_NOMEM;
    for (int j = 0; j < nt; j++) {
        if (check_t(t[j])) { free(c); return ORC_E_INVALID; }
        c[j] = orc_c(t[j]);
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < k; i++) edge_local_one(g, eids[i], c, nt, out + (size_t)i * nt * 2);
    free(c);
    return ORC_OK;
}

/* ---------------------------------------------------------------- Philox4x32-10 */

/* One Philox4x32 round and key schedule as defined by Salmon et al. (SC'11):
 * multipliers 0xD2511F53 / 0xCD9E8D57, Weyl increments 0x9E3779B9 / 0xBB67AE85. */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* edge index drawn for sample i of world w */
int64_t orc_sample_edge(uint64_t seed, uint32_t world, uint64_t i, int64_t m) {
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(i >> 32), 0u, 0u};
    uint32_t key[2] = {(uint32_t)seed ^ world, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    uint64_t x64 = ((uint64_t)x[1] << 32) | (uint64_t)x[0];
    return (int64_t)(((unsigned __int128)x64 * (unsigned __int128)(uint64_t)m) >> 64);
}

/* Edge-sampling estimator, replayed draw for draw.
 * sums[w][j][0/1]: sum of local balanced / unbalanced counts of world w at t_j;
 * est[w][j][0/1] = (double)sum * (double)m / (3.0 * (double)k). */
int orc_sample(const orc_graph* g, const double* t, int nt, int64_t k, int32_t worlds,
               uint64_t seed, double* est, int64_t* sums) {
    if (nt <= 0 || k <= 0 || worlds <= 0 || g->m <= 0) return ORC_E_INVALID;
    double* c = (double*)malloc(sizeof(double) * (size_t)nt);
    if (!c) return ORC_E_NOMEM;
    for (int j = 0; j < nt; j++) {
        if (check_t(t[j])) { free(c); return ORC_E_INVALID; }
        c[j] = orc_c(t[j]);
    }
    int fail = 0;
#pragma omp parallel
    {
        int64_t* loc = (int64_t*)malloc(sizeof(int64_t) * (size_t)nt * 2);
        if (!loc) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int32_t w = 0; w < worlds; w++) {
            if (!loc) continue;
            int64_t* S = sums + (size_t)w * nt * 2;
            for (int j = 0; j < 2 * nt; j++) S[j] = 0;
            for (int64_t i = 0; i < k; i++) {
                int64_t e = orc_sample_edge(seed, (uint32_t)w, (uint64_t)i, g->m);
                edge_local_one(g, e, c, nt, loc);
                for (int j = 0; j < 2 * nt; j++) S[j] += loc[j];
            }
            for (int j = 0; j < 2 * nt; j++)
                est[(size_t)w * nt * 2 + j] = ((double)S[j] * (double)g->m) / (3.0 * (double)k);
        }
        free(loc);
    }
    free(c);
    return fail ? ORC_E_NOMEM : ORC_OK;
}

/* ---------------------------------------------------------------- vertex sampling */

/* Every triangle {q, u, w} with u < w: u a neighbour of q, w a neighbour of u that is
 * also a neighbour of q. */
static void vertex_local_one(const orc_graph* g, int32_t q, const double* c, int nt, int64_t* out) {
    for (int j = 0; j < nt; j++) out[2 * j] = out[2 * j + 1] = 0;
    for (int64_t a = g->off[q]; a < g->off[q + 1]; a++) {
        int32_t u = g->nbr[a];
        for (int64_t b = g->off[u]; b < g->off[u + 1]; b++) {
            int32_t w = g->nbr[b];
            if (w <= u || w == q) continue;
            int32_t eqw = orc_find(g, q, w);
            if (eqw < 0) continue;
            double s = orc_s(g->d[g->eid[a]], g->d[g->eid[b]], g->d[eqw]);
            for (int j = 0; j < nt; j++) {
                int k = orc_classify(s, c[j]);
                if (k) out[2 * j + (k - 1)]++;
            }
        }
    }
}

int orc_vertex_local(const orc_graph* g, const double* t, int nt, const int64_t* vs, int64_t k,
                     int64_t* out) {
    if (nt <= 0 || k < 0) return ORC_E_INVALID;
    for (int64_t i = 0; i < k; i++)
        if (vs[i] < 0 || vs[i] >= g->n) return ORC_E_INVALID;
    double* c = (double*)malloc(sizeof(double) * (size_t)nt);
    if (!c) return ORC_E_NOMEM;
    for (int j = 0; j < nt; j++) {
        if (check_t(t[j])) { free(c); return ORC_E_INVALID; }
        c[j] = orc_c(t[j]);
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < k; i++)
        vertex_local_one(g, (int32_t)vs[i], c, nt, out + (size_t)i * nt * 2);
    free(c);
    return ORC_OK;
}

/* vertex drawn for sample i of world w (the Philox block of edge draw i of world w) */
int64_t orc_sample_vertex(uint64_t seed, uint32_t world, uint64_t i, int64_t n) {
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(i >> 32), 0u, 0u};
    uint32_t key[2] = {(uint32_t)seed ^ world, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    uint64_t x64 = ((uint64_t)x[1] << 32) | (uint64_t)x[0];
    return (int64_t)(((unsigned __int128)x64 * (unsigned __int128)(uint64_t)n) >> 64);
}

/* Vertex-sampling estimator, replayed draw for draw.
 * sums[w][j][0/1]: sum of local balanced / unbalanced counts of world w at t_j;
 * est[w][j][0/1] = (double)sum * (double)n / (3.0 * (double)k). */
int orc_sample_vertices(const orc_graph* g, const double* t, int nt, int64_t k, int32_t worlds,
                        uint64_t seed, double* est, int64_t* sums) {
    if (nt <= 0 || k <= 0 || worlds <= 0 || g->n <= 0) return ORC_E_INVALID;
    double* c = (double*)malloc(sizeof(double) * (size_t)nt);
    if (!c) return ORC_E_NOMEM;
    for (int j = 0; j < nt; j++) {
        if (check_t(t[j])) { free(c); return ORC_E_INVALID; }
        c[j] = orc_c(t[j]);
    }
    int fail = 0;
#pragma omp parallel
    {
        int64_t* loc = (int64_t*)malloc(sizeof(int64_t) * (size_t)nt * 2);
        if (!loc) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int32_t w = 0; w < worlds; w++) {
            if (!loc) continue;
            int64_t* S = sums + (size_t)w * nt * 2;
            for (int j = 0; j < 2 * nt; j++) S[j] = 0;
            for (int64_t i = 0; i < k; i++) {
                int64_t q = orc_sample_vertex(seed, (uint32_t)w, (uint64_t)i, g->n);
                vertex_local_one(g, (int32_t)q, c, nt, loc);
                for (int j = 0; j < 2 * nt; j++) S[j] += loc[j];
            }
            for (int j = 0; j < 2 * nt; j++)
                est[(size_t)w * nt * 2 + j] = ((double)S[j] * (double)g->n) / (3.0 * (double)k);
        }
        free(loc);
    }
    free(c);
    return fail ? ORC_E_NOMEM : ORC_OK;
}

/* ---------------------------------------------------------------- top-k */

typedef struct { double s; int32_t a, b, c; } orc_st;
typedef struct { orc_st* buf; int64_t len, cap; } orc_stvec;

typedef struct {
    const orc_graph* g;
    int cls;          /* 1 balanced, 2 unbalanced */
    orc_stvec* v;     /* [threads] */
    int* fail;        /* [threads] */
} topk_ctx;

static void topk_visit(void* vctx, int tid, int32_t u, int32_t v, int32_t w, int32_t euv,
                       int32_t euw, int32_t evw) {
    topk_ctx* cx = (topk_ctx*)vctx;
    const double* d = cx->g->d;
    double s = orc_s(d[euv], d[euw], d[evw]);
    if (orc_classify(s, 0.0) != cx->cls) return;
    int32_t a = u, b = v, c = w, t;
    if (b < a) { t = a; a = b; b = t; }
    if (c < b) { t = b; b = c; c = t; }
    if (b < a) { t = a; a = b; b = t; }
    orc_stvec* x = &cx->v[tid];
    if (x->len == x->cap) {
        int64_t nc = x->cap ? 2 * x->cap : 1024;
        orc_st* nb = (orc_st*)realloc(x->buf, sizeof(orc_st) * (size_t)nc);
        if (!nb) { cx->fail[tid] = 1; return; }
        x->buf = nb; x->cap = nc;
    }
    orc_st e = {s, a, b, c};
    x->buf[x->len++] = e;
}

static int cmp_st_tri(const orc_st* x, const orc_st* y) {
    if (x->a != y->a) return x->a < y->a ? -1 : 1;
    if (x->b != y->b) return x->b < y->b ? -1 : 1;
    if (x->c != y->c) return x->c < y->c ? -1 : 1;
    return 0;
}
static int cmp_st_up(const void* p, const void* q) {
    const orc_st *x = (const orc_st*)p, *y = (const orc_st*)q;
    if (x->s != y->s) return x->s < y->s ? -1 : 1;
    return cmp_st_tri(x, y);
}
static int cmp_st_down(const void* p, const void* q) {
    const orc_st *x = (const orc_st*)p, *y = (const orc_st*)q;
    if (x->s != y->s) return x->s > y->s ? -1 : 1;
    return cmp_st_tri(x, y);
}

/* which = 1 (balanced) or 2 (unbalanced). tri [k][3], s [k]; *count = the number
 * returned, min(k, #qualifying triangles). */
int orc_topk(const orc_graph* g, int64_t k, int which, int32_t* tri, double* sv, int64_t* count) {
    if (k < 0 || (which != 1 && which != 2)) return ORC_E_INVALID;
    int th = orc_threads();
    topk_ctx cx;
    cx.g = g;
    cx.cls = which;
    cx.v = (orc_stvec*)calloc((size_t)th, sizeof(orc_stvec));
    cx.fail = (int*)calloc((size_t)th, sizeof(int));
    if (!cx.v || !cx.fail) { free(cx.v); free(cx.fail); return ORC_E_NOMEM; }
    int rc = orc_node_iterate(g, topk_visit, &cx, th);
    int64_t tot = 0;
    for (int q = 0; q < th; q++) {
        if (cx.fail[q]) rc = ORC_E_NOMEM;
        tot += cx.v[q].len;
    }
    orc_st* all = NULL;
    if (rc == ORC_OK && tot > 0) {
        all = (orc_st*)malloc(sizeof(orc_st) * (size_t)tot);
        if (!all) rc = ORC_E_NOMEM;
    }
    if (rc == ORC_OK) {
        int64_t o = 0;
        for (int q = 0; q < th; q++) {
            if (cx.v[q].len) memcpy(all + o, cx.v[q].buf, sizeof(orc_st) * (size_t)cx.v[q].len);
            o += cx.v[q].len;
        }
        if (tot > 0) qsort(all, (size_t)tot, sizeof(orc_st), which == 1 ? cmp_st_up : cmp_st_down);
        int64_t r = tot < k ? tot : k;
        for (int64_t i = 0; i < r; i++) {
            tri[3 * i] = all[i].a; tri[3 * i + 1] = all[i].b; tri[3 * i + 2] = all[i].c;
            sv[i] = all[i].s;
        }
        *count = r;
    }
    free(all);
    for (int q = 0; q < th; q++) free(cx.v[q].buf);
    free(cx.v); free(cx.fail);
    return rc;
}

/* ---------------------------------------------------------------- sign worlds */

/* 1 if edge e (P+ = p) is negative in world w */
int orc_sign_negative(uint64_t seed, int64_t e, int32_t w, double p) {
    uint32_t ctr[4] = {(uint32_t)e, (uint32_t)(w / 4), 1u, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    return (double)x[w % 4] < p * 4294967296.0 ? 0 : 1;
}

typedef struct {
    const orc_graph* g;
    const uint8_t* neg;   /* [m][worlds] */
    int32_t worlds;
    int64_t* cnt;         /* [threads][worlds] */
} sign_ctx;

static void sign_visit(void* vctx, int tid, int32_t u, int32_t v, int32_t w, int32_t euv,
                       int32_t euw, int32_t evw) {
    sign_ctx* cx = (sign_ctx*)vctx;
    (void)u; (void)v; (void)w;
    const int32_t W = cx->worlds;
    const uint8_t* a = cx->neg + (size_t)euv * W;
    const uint8_t* b = cx->neg + (size_t)euw * W;
    const uint8_t* c = cx->neg + (size_t)evw * W;
    int64_t* cnt = cx->cnt + (size_t)tid * W;
    for (int32_t q = 0; q < W; q++)
        if (((a[q] + b[q] + c[q]) & 1) == 0) cnt[q]++;
}

int orc_sign_worlds(const orc_graph* g, int32_t worlds, uint64_t seed, int64_t* counts) {
    if (worlds <= 0) return ORC_E_INVALID;
    uint8_t* neg = (uint8_t*)malloc((size_t)(g->m > 0 ? g->m : 1) * (size_t)worlds);
    int th = orc_threads();
    int64_t* cnt = (int64_t*)calloc((size_t)th * (size_t)worlds, sizeof(int64_t));
    if (!neg || !cnt) { free(neg); free(cnt); return ORC_E_NOMEM; }
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < g->m; e++)
        for (int32_t q = 0; q < worlds; q++)
            neg[(size_t)e * worlds + q] = (uint8_t)orc_sign_negative(seed, e, q, g->p[e]);
    sign_ctx cx = {g, neg, worlds, cnt};
    int rc = orc_node_iterate(g, sign_visit, &cx, th);
    for (int32_t q = 0; q < worlds; q++) {
        int64_t t = 0;
        for (int i = 0; i < th; i++) t += cnt[(size_t)i * worlds + q];
        counts[q] = t;
    }
    free(neg);
    free(cnt);
    return rc;
}
