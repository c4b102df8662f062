// api.hip -- the extern "C" entry points declared in include/utri.h: argument checks,
// threshold ordering, scratch plumbing, stream handling and result read-back. All
// arithmetic of a query runs in the kernels of walk.hip, sample.hip and backward.hip.
#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "utri_internal.h"

namespace {

inline hipStream_t as_stream(void* s) { return (hipStream_t)s; }

inline bool t_ok(double t) { return t >= 0.5 && t <= 1.0; }  // false for NaN

// Sort thresholds ascending; order[j] = original index of the j-th smallest.
int sort_thresholds(const double* t, int nt, std::vector<double>& cvals,
                    std::vector<int32_t>& order) {
    if (!t || nt < 1 || nt > 64) return UTRI_E_INVALID;
    for (int j = 0; j < nt; j++)
        if (!t_ok(t[j])) return UTRI_E_INVALID;
    order.resize(nt);
    for (int j = 0; j < nt; j++) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return t[a] < t[b]; });
    cvals.resize(nt);
    for (int j = 0; j < nt; j++) cvals[j] = utri_c_of_t(t[order[j]]);
    return UTRI_OK;
}

// Upload the sorted thresholds and their order into scratch device buffers.
int upload_thresholds(utri_graph* g, const std::vector<double>& cvals,
                      const std::vector<int32_t>& order, hipStream_t s, double** dc,
                      int32_t** dord) {
    void *pc, *po;
    UTRI_TRY(utri_scratch(g, SCR_CVALS, sizeof(double) * 64, &pc));
    UTRI_TRY(utri_scratch(g, SCR_ORDER, sizeof(int32_t) * 64, &po));
    UTRI_HIP_TRY(hipMemcpyAsync(pc, cvals.data(), sizeof(double) * cvals.size(),
                                hipMemcpyHostToDevice, s));
    UTRI_HIP_TRY(hipMemcpyAsync(po, order.data(), sizeof(int32_t) * order.size(),
                                hipMemcpyHostToDevice, s));
    *dc = (double*)pc;
    *dord = (int32_t*)po;
    return UTRI_OK;
}

int check_graph(const utri_graph* g) { return g ? UTRI_OK : UTRI_E_INVALID; }

// ------------------------------------------------------------------ enumeration sort

__global__ void k_tri_keys(const int32_t* __restrict__ tri, int64_t cnt, unsigned nb,
                           uint64_t* __restrict__ k_lo, uint32_t* __restrict__ k_hi,
                           uint32_t* __restrict__ idx) {
    UTRI_FOR_GRID(i, cnt) {
        k_lo[i] = ((uint64_t)(uint32_t)tri[3 * i + 1] << nb) | (uint64_t)(uint32_t)tri[3 * i + 2];
        k_hi[i] = (uint32_t)tri[3 * i];
        idx[i] = (uint32_t)i;
    }
}

__global__ void k_tri_key_first(const int32_t* __restrict__ tri, const uint32_t* __restrict__ idx,
                                int64_t cnt, uint32_t* __restrict__ k) {
    UTRI_FOR_GRID(i, cnt) k[i] = (uint32_t)tri[3 * (int64_t)idx[i]];
}

__global__ void k_tri_gather(const int32_t* __restrict__ tri, const uint32_t* __restrict__ idx,
                             int64_t cnt, int32_t* __restrict__ out) {
    UTRI_FOR_GRID(i, cnt) {
        const int64_t j = idx[i];
        out[3 * i] = tri[3 * j];
        out[3 * i + 1] = tri[3 * j + 1];
        out[3 * i + 2] = tri[3 * j + 2];
    }
}

__global__ void k_copy_i32(const int32_t* __restrict__ a, int64_t n, int32_t* __restrict__ b) {
    UTRI_FOR_GRID(i, n) b[i] = a[i];
}

inline unsigned nblk(int64_t n) { return utri_grid(n, 256); }

__global__ void k_check_eids(const int64_t* __restrict__ eids, int64_t k, int64_t m,
                             uint32_t* __restrict__ flag) {
    UTRI_FOR_GRID(i, k) if (eids[i] < 0 || eids[i] >= m) atomicOr(flag, 1u);
}

template <class K, class V>
int radix_pairs(utri_graph* g, const K* kin, K* kout, const V* vin, V* vout, int64_t cnt,
                unsigned bits, hipStream_t s) {
    size_t bytes = 0;
    UTRI_HIP_TRY(rocprim::radix_sort_pairs(nullptr, bytes, kin, kout, vin, vout, (size_t)cnt, 0,
                                           bits, s));
    void* tmp;
    UTRI_TRY(utri_scratch(g, SCR_TEMP, bytes, &tmp));
    UTRI_HIP_TRY(rocprim::radix_sort_pairs(tmp, bytes, kin, kout, vin, vout, (size_t)cnt, 0,
                                           bits, s));
    return UTRI_OK;
}

// Lexicographic sort of cnt int32 triples in place (two stable LSD radix passes).
int sort_triples(utri_graph* g, int32_t* tri, int64_t cnt, hipStream_t s) {
    if (cnt <= 1) return UTRI_OK;
    if (cnt > (int64_t)UINT32_MAX) return UTRI_E_RANGE;  // positions are 32-bit sort values
    unsigned nb = 1;
    while (((int64_t)1 << nb) < g->n) nb++;
    void *pa, *pb, *pc, *pd;
    UTRI_TRY(utri_scratch(g, SCR_SORT_A, sizeof(uint64_t) * cnt * 2, &pa));
    UTRI_TRY(utri_scratch(g, SCR_SORT_B, sizeof(uint32_t) * cnt * 2, &pb));
    UTRI_TRY(utri_scratch(g, SCR_SORT_C, sizeof(uint32_t) * cnt * 2, &pc));
    UTRI_TRY(utri_scratch(g, SCR_SORT_D, sizeof(int32_t) * cnt * 3, &pd));
    uint64_t* k64 = (uint64_t*)pa;
    uint32_t* k32 = (uint32_t*)pb;
    uint32_t* idx = (uint32_t*)pc;
    hipLaunchKernelGGL(k_tri_keys, dim3(nblk(cnt)), dim3(256), 0, s, tri, cnt, nb, k64, k32, idx);
    UTRI_HIP_TRY(hipGetLastError());
    UTRI_TRY(radix_pairs(g, k64, k64 + cnt, idx, idx + cnt, cnt, 2 * nb, s));
    hipLaunchKernelGGL(k_tri_key_first, dim3(nblk(cnt)), dim3(256), 0, s, tri, idx + cnt, cnt, k32);
    UTRI_HIP_TRY(hipGetLastError());
    UTRI_TRY(radix_pairs(g, k32, k32 + cnt, idx + cnt, idx, cnt, nb, s));
    int32_t* tmp = (int32_t*)pd;
    hipLaunchKernelGGL(k_tri_gather, dim3(nblk(cnt)), dim3(256), 0, s, tri, idx, cnt, tmp);
    hipLaunchKernelGGL(k_copy_i32, dim3(nblk(3 * cnt)), dim3(256), 0, s, tmp, 3 * cnt, tri);
    UTRI_HIP_TRY(hipGetLastError());
    return UTRI_OK;
}

// ------------------------------------------------------------------ shared query pieces

int walk_prepare_for(utri_graph* g, int method, double c, hipStream_t s, int64_t** items,
                     int64_t** nitems, int32_t** len) {
    const double c_rows = (method == UTRI_PLAIN) ? 0.0 : c;
    return utri_walk_prepare(g, c_rows, (method == UTRI_PRUNED_L3 && c > 0.0) ? 1 : 0, s, items,
                             nitems, len);
}

WalkParams base_params(int method, double c) {
    WalkParams wp;
    wp.c = c;
    wp.lemma3 = (method == UTRI_PRUNED_L3) ? 1 : 0;
    wp.c_l3 = c * (1.0 - 0x1p-50);
    return wp;
}

int count_impl(utri_graph* g, double t, int method, int64_t out[2], hipStream_t s) {
    const double c = utri_c_of_t(t);
    int64_t *items, *nitems;
    int32_t* len;
    UTRI_TRY(walk_prepare_for(g, method, c, s, &items, &nitems, &len));
    void* acc;
    UTRI_TRY(utri_scratch(g, SCR_ACC, sizeof(uint64_t) * 4, &acc));
    UTRI_TRY(utri_fill_u64(acc, 0, 2, s));
    WalkParams wp = base_params(method, c);
    wp.acc = (unsigned long long*)acc;
    if (g->timing) UTRI_HIP_TRY(hipEventRecord(g->tev0, s));
    UTRI_TRY(utri_walk_launch(g, WALK_COUNT, wp, items, nitems, len, 0, s));
    if (g->timing) UTRI_HIP_TRY(hipEventRecord(g->tev1, s));
    uint64_t h[2] = {0, 0};
    UTRI_HIP_TRY(hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, s));
    UTRI_HIP_TRY(hipStreamSynchronize(s));
    if (g->timing) {
        float ms = 0.f;
        UTRI_HIP_TRY(hipEventElapsedTime(&ms, g->tev0, g->tev1));
        g->timing_ms += ms;
        g->timing_launches += 1;
    }
    out[0] = (int64_t)h[0];
    out[1] = (int64_t)h[1];
    return UTRI_OK;
}

// Launch sequence of the batch path (also what gets captured into a hipGraph).
int64_t n_draws(const SampleParams& sp) { return (int64_t)sp.worlds * sp.k; }

// Grouped sampling of draws [t_begin, t_end), one pass of g->sample_pass at a time.
int sample_passes(utri_graph* g, SampleParams& sp, const int32_t* slen, int64_t t_begin,
                  int64_t t_end, hipStream_t s) {
    for (int64_t t0 = t_begin; t0 < t_end; t0 += g->sample_pass) {
        UTRI_TRY(utri_sample_prepare(g, sp, slen, t0, std::min<int64_t>(t_end, t0 + g->sample_pass), s));
        UTRI_TRY(utri_sample_launch(g, sp, slen, s));
    }
    return UTRI_OK;
}

int batch_sequence(utri_graph* g, const double* dc, const int32_t* dord, int nt, double cmin,
                   int64_t k, int32_t worlds, const uint64_t* seed_dev, int64_t* exact,
                   double* est, hipStream_t s) {
    int64_t *items = nullptr, *nitems = nullptr;
    int32_t* len = nullptr;
    int32_t* slen = nullptr;
    void *hw = nullptr, *hs = nullptr;
    WalkParams wp = base_params(UTRI_PRUNED, cmin);
    if (exact) {
        UTRI_TRY(utri_walk_prepare(g, cmin, 0, s, &items, &nitems, &len));
        UTRI_TRY(utri_scratch(g, SCR_HIST2, sizeof(uint64_t) * 2 * (nt + 1), &hw));
        UTRI_TRY(utri_fill_u64(hw, 0, 2 * (nt + 1), s));
        wp.acc = (unsigned long long*)hw;
        wp.cvals = dc;
        wp.nt = nt;
    }
    SampleParams sp;
    if (est && k > 0 && worlds > 0) {
        UTRI_TRY(utri_sym_prepare(g, cmin, s, &slen));
        const size_t nh = (size_t)worlds * 2 * (nt + 1);
        UTRI_TRY(utri_scratch(g, SCR_HIST, sizeof(uint64_t) * nh, &hs));
        UTRI_TRY(utri_fill_u64(hs, 0, (int64_t)nh, s));
        sp.cvals = dc;
        sp.nt = nt;
        sp.cmin = cmin;
        sp.seed_dev = seed_dev;
        sp.k = k;
        sp.worlds = worlds;
        sp.chunk = g->sample_chunk;
        sp.hist = (unsigned long long*)hs;
        UTRI_TRY(utri_sample_prepare(g, sp, slen, 0, std::min<int64_t>(n_draws(sp), g->sample_pass), s));
    }
    if (!items) {
        // no walk part: the kernel still needs a valid (zero) item count
        void* pn;
        UTRI_TRY(utri_scratch(g, SCR_NITEMS, sizeof(int64_t) * 6, &pn));
        nitems = (int64_t*)pn;
    }
    UTRI_TRY(utri_batch_launch(g, wp, items, nitems, len, 0, sp, slen, s));
    // draws beyond the first pass in further launches
    if (sp.hist) UTRI_TRY(sample_passes(g, sp, slen, g->sample_pass, n_draws(sp), s));
    if (exact) UTRI_TRY(utri_finalize_launch((const unsigned long long*)hw, 1, nt, dord, g->m, 1, exact, nullptr, s));
    if (sp.hist) UTRI_TRY(utri_finalize_launch((const unsigned long long*)hs, worlds, nt, dord, g->m, k, nullptr, est, s));
    return UTRI_OK;
}

// ------------------------------------------------------------------ autotune cache

std::string cache_key(const utri_graph* g) {
    char buf[160];
    snprintf(buf, sizeof(buf), "\"n\": %lld, \"m\": %lld, \"max_deg\": %lld", (long long)g->n,
             (long long)g->m, (long long)g->max_deg);
    return buf;
}

// The launch parameters in UTRI_TUNE_* order, and their JSON names in the cache file.
const char* const TUNE_NAMES[UTRI_TUNE_COUNT] = {
    "walk_blocks_per_cu", "sample_chunk", "walk_partners", "walk_light_cap",
    "walk_chunk",         "walk_unroll",  "walk_shorter_min"};

void tune_get(const utri_graph* g, int64_t v[UTRI_TUNE_COUNT]) {
    v[UTRI_TUNE_WALK_BLOCKS_PER_CU] = g->walk_blocks_per_cu;
    v[UTRI_TUNE_SAMPLE_CHUNK] = g->sample_chunk;
    v[UTRI_TUNE_WALK_PARTNERS] = g->walk_tune.pr;
    v[UTRI_TUNE_WALK_LIGHT_CAP] = g->walk_tune.cap;
    v[UTRI_TUNE_WALK_CHUNK] = g->walk_tune.caph;
    v[UTRI_TUNE_WALK_UNROLL] = g->walk_tune.unr;
    v[UTRI_TUNE_WALK_SHORTER_MIN] = g->walk_tune.shorter_min;
}

int tune_set(utri_graph* g, const int64_t v[UTRI_TUNE_COUNT]) {
    const int64_t b = v[UTRI_TUNE_WALK_BLOCKS_PER_CU], c = v[UTRI_TUNE_SAMPLE_CHUNK];
    if (b < 0 || b > 64 || c < 64 || c > 4096 || c % 64 != 0) return UTRI_E_INVALID;
    for (int i = UTRI_TUNE_WALK_PARTNERS; i <= UTRI_TUNE_WALK_UNROLL; i++)
        if (v[i] < 0 || v[i] > (1 << 20)) return UTRI_E_INVALID;
    WalkTune t;
    t.pr = (int32_t)v[UTRI_TUNE_WALK_PARTNERS];
    t.cap = (int32_t)v[UTRI_TUNE_WALK_LIGHT_CAP];
    t.caph = (int32_t)v[UTRI_TUNE_WALK_CHUNK];
    t.unr = (int32_t)v[UTRI_TUNE_WALK_UNROLL];
    t.shorter_min = v[UTRI_TUNE_WALK_SHORTER_MIN];
    if (!utri_walk_tune_ok(t)) return UTRI_E_INVALID;
    g->walk_blocks_per_cu = (int)b;
    g->sample_chunk = (int)c;
    g->walk_tune = t;
    return UTRI_OK;
}

// The cached choice for g's shape in the file at path (the last matching line wins);
// false if there is none or it does not validate.
bool read_cache(const utri_graph* g, const char* path, int64_t v[UTRI_TUNE_COUNT]) {
    if (!path) return false;
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[1024];
    const std::string key = cache_key(g);
    bool found = false;
    while (fgets(line, sizeof(line), f)) {
        if (!strstr(line, key.c_str())) continue;
        int64_t w[UTRI_TUNE_COUNT];
        tune_get(g, w);
        for (int i = 0; i < UTRI_TUNE_COUNT; i++) {
            const std::string name = std::string("\"") + TUNE_NAMES[i] + "\": ";
            if (const char* a = strstr(line, name.c_str())) w[i] = atoll(a + name.size());
        }
        for (int i = 0; i < UTRI_TUNE_COUNT; i++) v[i] = w[i];
        found = true;
    }
    fclose(f);
    return found;
}

void apply_cache(utri_graph* g, const char* path) {
    int64_t v[UTRI_TUNE_COUNT];
    if (read_cache(g, path, v)) (void)tune_set(g, v);  // an invalid line keeps the defaults
}

// ------------------------------------------------------------------ no-allocation counting
//
// utri_count_noalloc runs utri_count's kernels on a file-scope device array instead of the
// handle's hipMalloc'd scratch. In host code `scratch` is only a host-side stand-in for
// the array: its device address is read once per device with hipGetSymbolAddress (each
// GPU holds its own copy) and only that address is ever handed to kernels or copies.

constexpr size_t NOALLOC_BYTES = (size_t)UTRI_NOALLOC_SCRATCH_MB << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
std::mutex g_scratch_mu;

// Device address of this device's copy of `scratch` (looked up once per device).
int noalloc_scratch(int dev, void** out) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return UTRI_E_INVALID;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        UTRI_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return UTRI_E_HIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return UTRI_OK;
}

// Routes the handle's scratch requests into the arena for the lifetime of this object.
struct ArenaScope {
    utri_graph* g;
    ArenaScope(utri_graph* gg, void* base, size_t bytes) : g(gg) {
        g->arena = (char*)base;
        g->arena_bytes = bytes;
        g->arena_used = 0;
        for (int i = 0; i < SCR_COUNT; i++) {
            g->arena_slot[i] = nullptr;
            g->arena_slot_bytes[i] = 0;
        }
    }
    ~ArenaScope() {
        g->arena = nullptr;
        g->arena_bytes = g->arena_used = 0;
    }
};

}  // namespace

extern "C" {

int utri_count_noalloc(utri_graph* g, double t, int method, int which, int64_t out[2],
                       void* hip_stream) {
    UTRI_TRY(check_graph(g));
    if (!out || !t_ok(t)) return UTRI_E_INVALID;
    if (method < UTRI_PLAIN || method > UTRI_PRUNED_L3) return UTRI_E_INVALID;
    if (which < UTRI_BAL || which > UTRI_BOTH) return UTRI_E_INVALID;
    if (utri_count_scratch_bound(g, 256) > (int64_t)NOALLOC_BYTES) return UTRI_E_CAPACITY;
    int dev = -1;
    UTRI_HIP_TRY(hipGetDevice(&dev));
    if (dev != g->device) return UTRI_E_INVALID;
    void* base = nullptr;
    UTRI_TRY(noalloc_scratch(dev, &base));
    int64_t r[2] = {0, 0};
    {
        ArenaScope scope(g, base, NOALLOC_BYTES);
        UTRI_TRY(count_impl(g, t, method, r, as_stream(hip_stream)));
    }
    out[0] = (which & UTRI_BAL) ? r[0] : 0;
    out[1] = (which & UTRI_UNBAL) ? r[1] : 0;
    return UTRI_OK;
}

const char* utri_strerror(int code) {
    switch (code) {
        case UTRI_OK: return "ok";
        case UTRI_E_INVALID: return "invalid argument";
        case UTRI_E_CONFLICT: return "an edge was given twice with different P+";
        case UTRI_E_CAPACITY: return "output capacity too small";
        case UTRI_E_NOMEM: return "out of memory";
        case UTRI_E_HIP: return "HIP runtime error";
        case UTRI_E_RANGE: return "graph too large for 32-bit ids";
        default: return "unknown status";
    }
}

int utri_graph_load(const int64_t* src, const int64_t* dst, const double* p, int64_t m_in,
                    int64_t n, int ptr_kind, void* hip_stream, utri_graph** out) {
    if (!out) return UTRI_E_INVALID;
    *out = nullptr;
    if (n < 0 || m_in < 0) return UTRI_E_INVALID;
    if (ptr_kind != UTRI_HOST_PTR && ptr_kind != UTRI_DEVICE_PTR) return UTRI_E_INVALID;
    if (m_in > 0 && (!src || !dst || !p)) return UTRI_E_INVALID;
    if (n >= ((int64_t)1 << 31)) return UTRI_E_RANGE;
    // the canonical graph has fewer than 2^31 edges, so more input edges than that could
    // only be duplicates; the load's per-input-edge kernels assume it
    if (m_in >= ((int64_t)1 << 31)) return UTRI_E_RANGE;
    utri_graph* g = nullptr;
    int rc = utri_load_internal(src, dst, p, m_in, n, ptr_kind, as_stream(hip_stream), &g);
    if (rc != UTRI_OK) return rc;
    apply_cache(g, getenv("UTRI_TUNE_CACHE"));
    if (const char* e = getenv("UTRI_WALK_BLOCKS_PER_CU")) g->walk_blocks_per_cu = std::max(0, atoi(e));
    if (const char* e = getenv("UTRI_SIGN_FLUSH"))
        g->sign_flush_at = (uint32_t)std::max<long long>(1, std::min<long long>(65535, atoll(e)));
    if (const char* e = getenv("UTRI_SAMPLE_PASS"))
        g->sample_pass = std::max<int64_t>(64, std::min<int64_t>(UTRI_SAMPLE_PASS, atoll(e)));
    *out = g;
    return UTRI_OK;
}

int utri_graph_free(utri_graph* g) {
    if (!g) return UTRI_OK;
    // the handle's own replay stream first; hipFree then waits for the device itself
    if (g->batch.stream) (void)hipStreamSynchronize(g->batch.stream);
    utri_free_graph_internal(g);
    return UTRI_OK;
}

int utri_graph_info(const utri_graph* g, int64_t* n, int64_t* m, int64_t* self_loops_dropped,
                    int64_t* dups_merged, int64_t* max_deg) {
    UTRI_TRY(check_graph(g));
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (self_loops_dropped) *self_loops_dropped = g->self_loops;
    if (dups_merged) *dups_merged = g->dups;
    if (max_deg) *max_deg = g->max_deg;
    return UTRI_OK;
}

int utri_graph_edges(const utri_graph* g, int32_t* lo, int32_t* hi, double* p, int ptr_kind,
                     void* hip_stream) {
    UTRI_TRY(check_graph(g));
    if (ptr_kind != UTRI_HOST_PTR && ptr_kind != UTRI_DEVICE_PTR) return UTRI_E_INVALID;
    hipStream_t s = as_stream(hip_stream);
    const hipMemcpyKind kind = ptr_kind == UTRI_HOST_PTR ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (g->m > 0) {
        if (lo) UTRI_HIP_TRY(hipMemcpyAsync(lo, g->e_lo, sizeof(int32_t) * g->m, kind, s));
        if (hi) UTRI_HIP_TRY(hipMemcpyAsync(hi, g->e_hi, sizeof(int32_t) * g->m, kind, s));
        if (p) UTRI_HIP_TRY(hipMemcpyAsync(p, g->e_p, sizeof(double) * g->m, kind, s));
    }
    if (ptr_kind == UTRI_HOST_PTR) UTRI_HIP_TRY(hipStreamSynchronize(s));
    return UTRI_OK;
}

int utri_graph_set_p(utri_graph* g, const double* p, int ptr_kind, void* hip_stream) {
    UTRI_TRY(check_graph(g));
    if (ptr_kind != UTRI_HOST_PTR && ptr_kind != UTRI_DEVICE_PTR) return UTRI_E_INVALID;
    if (g->m > 0 && !p) return UTRI_E_INVALID;
    return utri_set_p_internal(g, p, ptr_kind, as_stream(hip_stream));
}

int utri_count(utri_graph* g, double t, int method, int which, int64_t out[2], void* hip_stream) {
    UTRI_TRY(check_graph(g));
    if (!out || !t_ok(t)) return UTRI_E_INVALID;
    if (method < UTRI_PLAIN || method > UTRI_PRUNED_L3) return UTRI_E_INVALID;
    if (which < UTRI_BAL || which > UTRI_BOTH) return UTRI_E_INVALID;
    int64_t r[2] = {0, 0};
    UTRI_TRY(count_impl(g, t, method, r, as_stream(hip_stream)));
    out[0] = (which & UTRI_BAL) ? r[0] : 0;
    out[1] = (which & UTRI_UNBAL) ? r[1] : 0;
    return UTRI_OK;
}

int utri_count_batch(utri_graph* g, const double* t, int nt, int method, int64_t* out,
                     void* hip_stream) {
    UTRI_TRY(check_graph(g));
    if (!out) return UTRI_E_INVALID;
    if (method < UTRI_PLAIN || method > UTRI_PRUNED_L3) return UTRI_E_INVALID;
    std::vector<double> cv;
    std::vector<int32_t> order;
    UTRI_TRY(sort_thresholds(t, nt, cv, order));
    hipStream_t s = as_stream(hip_stream);
    double* dc;
    int32_t* dord;
    UTRI_TRY(upload_thresholds(g, cv, order, s, &dc, &dord));
    const double cmin = cv[0];
    int64_t *items, *nitems;
    int32_t* len;
    UTRI_TRY(walk_prepare_for(g, method, cmin, s, &items, &nitems, &len));
    void *acc, *dout;
    UTRI_TRY(utri_scratch(g, SCR_ACC, sizeof(uint64_t) * 2 * (nt + 1), &acc));
    UTRI_TRY(utri_scratch(g, SCR_OUT, sizeof(int64_t) * 2 * nt, &dout));
    UTRI_TRY(utri_fill_u64(acc, 0, 2 * (nt + 1), s));
    WalkParams wp = base_params(method, cmin);
    wp.acc = (unsigned long long*)acc;
    wp.cvals = dc;
    wp.nt = nt;
    UTRI_TRY(utri_walk_launch(g, WALK_HIST, wp, items, nitems, len, 0, s));
    UTRI_TRY(utri_finalize_launch((const unsigned long long*)acc, 1, nt, dord, g->m, 1,
                                  (int64_t*)dout, nullptr, s));
    UTRI_HIP_TRY(hipMemcpyAsync(out, dout, sizeof(int64_t) * 2 * nt, hipMemcpyDeviceToHost, s));
    UTRI_HIP_TRY(hipStreamSynchronize(s));
    return UTRI_OK;
}

int utri_enumerate(utri_graph* g, double t, int method, int which, int32_t* bal, int64_t cap_b,
                   int32_t* unbal, int64_t cap_u, int64_t out_counts[2], int sorted,
                   void* hip_stream) {
    UTRI_TRY(check_graph(g));
    if (!out_counts || !t_ok(t) || cap_b < 0 || cap_u < 0) return UTRI_E_INVALID;
    if (method < UTRI_PLAIN || method > UTRI_PRUNED_L3) return UTRI_E_INVALID;
    if (which < UTRI_BAL || which > UTRI_BOTH) return UTRI_E_INVALID;
    hipStream_t s = as_stream(hip_stream);
    const double c = utri_c_of_t(t);
    int64_t *items, *nitems;
    int32_t* len;
    UTRI_TRY(walk_prepare_for(g, method, c, s, &items, &nitems, &len));
    const int64_t bound = utri_walk_items_bound(g) + 1;
    void *pc, *po, *ptot;
    UTRI_TRY(utri_scratch(g, SCR_ICNT2, sizeof(int64_t) * 2 * bound, &pc));
    UTRI_TRY(utri_scratch(g, SCR_IOFF2, sizeof(int64_t) * 2 * bound, &po));
    UTRI_TRY(utri_scratch(g, SCR_OUT, sizeof(int64_t) * 4, &ptot));
    int64_t* cnt_b = (int64_t*)pc;
    int64_t* cnt_u = cnt_b + bound;
    int64_t* off_b = (int64_t*)po;
    int64_t* off_u = off_b + bound;
    int64_t* tot = (int64_t*)ptot;
    // the counts a call that returned UTRI_E_CAPACITY left for this same query, if any;
    // they are used once
    EnumTicket& tk = g->enum_ticket;
    const bool reuse = tk.valid && tk.c == c && tk.method == method && tk.which == which &&
                       tk.walk_order == g->walk_order && tk.walk_tune == g->walk_tune &&
                       tk.scr_gen == g->scr_gen && tk.rows_gen == g->rows_gen;
    tk.valid = false;
    int64_t nb, nu;
    if (reuse) {
        nb = tk.nb;
        nu = tk.nu;
    } else {
        UTRI_TRY(utri_fill_u64(pc, 0, 2 * bound, s));
        UTRI_TRY(utri_fill_u64(ptot, 0, 4, s));
        WalkParams wp = base_params(method, c);
        wp.cnt_b = cnt_b;
        wp.cnt_u = cnt_u;
        wp.which = which;
        UTRI_TRY(utri_walk_launch(g, WALK_ENUM_COUNT, wp, items, nitems, len, 0, s));
        UTRI_TRY(utri_scan_i64(g, cnt_b, off_b, bound, tot, s));
        UTRI_TRY(utri_scan_i64(g, cnt_u, off_u, bound, tot + 1, s));
        int64_t h[2] = {0, 0};
        UTRI_HIP_TRY(hipMemcpyAsync(h, tot, sizeof(h), hipMemcpyDeviceToHost, s));
        UTRI_HIP_TRY(hipStreamSynchronize(s));
        nb = (which & UTRI_BAL) ? h[0] : 0;
        nu = (which & UTRI_UNBAL) ? h[1] : 0;
    }
    out_counts[0] = nb;
    out_counts[1] = nu;
    if (nb > cap_b || nu > cap_u) {
        tk.valid = true;
        tk.c = c;
        tk.method = method;
        tk.which = which;
        tk.walk_order = g->walk_order;
        tk.walk_tune = g->walk_tune;
        tk.scr_gen = g->scr_gen;
        tk.rows_gen = g->rows_gen;
        tk.nb = nb;
        tk.nu = nu;
        return UTRI_E_CAPACITY;
    }
    if ((nb > 0 && !bal) || (nu > 0 && !unbal)) return UTRI_E_INVALID;
    if (nb == 0 && nu == 0) return UTRI_OK;
    WalkParams wf = base_params(method, c);
    wf.off_b = off_b;
    wf.off_u = off_u;
    wf.out_bal = bal;
    wf.out_unbal = unbal;
    wf.which = which;
    UTRI_TRY(utri_walk_launch(g, WALK_ENUM_FILL, wf, items, nitems, len, 0, s));
    if (sorted) {
        if (nb > 1) UTRI_TRY(sort_triples(g, bal, nb, s));
        if (nu > 1) UTRI_TRY(sort_triples(g, unbal, nu, s));
    }
    UTRI_HIP_TRY(hipStreamSynchronize(s));
    return UTRI_OK;
}

int utri_expected(utri_graph* g, double* E, void* hip_stream) {
    UTRI_TRY(check_graph(g));
    if (!E) return UTRI_E_INVALID;
    hipStream_t s = as_stream(hip_stream);
    int64_t *items, *nitems;
    int32_t* len;
    UTRI_TRY(utri_walk_prepare(g, 0.0, 0, s, &items, &nitems, &len));
    void* acc;
    UTRI_TRY(utri_scratch(g, SCR_ACC, sizeof(uint64_t) * 4, &acc));
    UTRI_TRY(utri_fill_u64(acc, 0, 3, s));
    WalkParams wp;
    wp.acc = (unsigned long long*)acc;
    UTRI_TRY(utri_walk_launch(g, WALK_EXPECTED, wp, items, nitems, len, 0, s));
    uint64_t h[3] = {0, 0, 0};
    UTRI_HIP_TRY(hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, s));
    UTRI_HIP_TRY(hipStreamSynchronize(s));
    // N = T * 2^62 - S, exact in 128 bits; E = N * 2^-63 rounded once
    const unsigned __int128 T = (unsigned __int128)h[0];
    const unsigned __int128 S = ((unsigned __int128)h[2] << 64) | (unsigned __int128)h[1];
    const unsigned __int128 N = (T << 62) - S;
    *E = utri_i128_to_double((int64_t)(uint64_t)(N >> 64), (uint64_t)N) * 0x1p-63;
    return UTRI_OK;
}

int utri_sign_worlds(utri_graph* g, int32_t worlds, uint64_t seed, int64_t* counts,
                     void* hip_stream) {
    UTRI_TRY(check_graph(g));
    if (!counts || worlds < 32 || worlds > 1024 || (worlds & (worlds - 1)) != 0)
        return UTRI_E_INVALID;
    hipStream_t s = as_stream(hip_stream);
    const int ww = worlds / 32;
    void *pm, *pc;
    UTRI_TRY(utri_scratch(g, SCR_SIGN_MASK, sizeof(uint32_t) * (size_t)std::max<int64_t>(1, g->m * ww), &pm));
    UTRI_TRY(utri_scratch(g, SCR_SIGN_CNT, sizeof(uint64_t) * (size_t)worlds, &pc));
    UTRI_TRY(utri_fill_u64(pc, 0, worlds, s));
    UTRI_TRY(utri_sign_masks_launch(g, seed, ww, (uint32_t*)pm, s));
    // the sign-world walk's work-group table holds chunks of at most UTRI_SIGN_WALK_CHUNK
    // entries: its items are cut that way for this call
    struct TuneScope {
        utri_graph* g;
        WalkTune saved;
        ~TuneScope() { g->walk_tune = saved; }
    } scope{g, g->walk_tune};
    g->walk_tune.caph = std::min(g->walk_tune.caph, UTRI_SIGN_WALK_CHUNK);
    int64_t *items, *nitems;
    int32_t* len;
    UTRI_TRY(utri_walk_prepare(g, 0.0, 0, s, &items, &nitems, &len));
    WalkParams wp;
    wp.o_eid = g->o_eid;
    wp.masks = (const uint32_t*)pm;
    wp.ww = ww;
    wp.wcount = (unsigned long long*)pc;
    wp.sign_flush_at = g->sign_flush_at;
    UTRI_TRY(utri_walk_launch(g, WALK_SIGN, wp, items, nitems, len, 0, s));
    UTRI_HIP_TRY(hipMemcpyAsync(counts, pc, sizeof(int64_t) * (size_t)worlds,
                                hipMemcpyDeviceToDevice, s));
    UTRI_HIP_TRY(hipStreamSynchronize(s));
    return UTRI_OK;
}

int utri_expected_grad(utri_graph* g, double* grad, void* hip_stream) {
    UTRI_TRY(check_graph(g));
    if (g->m > 0 && !grad) return UTRI_E_INVALID;
    return utri_grad_launch(g, grad, as_stream(hip_stream));
}

int utri_edge_local(utri_graph* g, const double* t, int nt, const int64_t* eids, int64_t k,
                    int64_t* out, void* hip_stream) {
    UTRI_TRY(check_graph(g));
    if (k < 0 || (k > 0 && (!eids || !out))) return UTRI_E_INVALID;
    std::vector<double> cv;
    std::vector<int32_t> order;
    UTRI_TRY(sort_thresholds(t, nt, cv, order));
    if (k == 0) return UTRI_OK;
    hipStream_t s = as_stream(hip_stream);
    // edge ids come from the caller: check the range before any kernel indexes with them
    UTRI_HIP_TRY(hipMemsetAsync(g->d_flags, 0, sizeof(uint32_t), s));
    hipLaunchKernelGGL(k_check_eids, dim3(nblk(k)), dim3(256), 0, s, eids, k, g->m, g->d_flags);
    UTRI_HIP_TRY(hipGetLastError());
    uint32_t bad = 0;
    UTRI_HIP_TRY(hipMemcpyAsync(&bad, g->d_flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    UTRI_HIP_TRY(hipStreamSynchronize(s));
    if (bad) return UTRI_E_INVALID;
    double* dc;
    int32_t* dord;
    UTRI_TRY(upload_thresholds(g, cv, order, s, &dc, &dord));
    UTRI_TRY(utri_edge_local_launch(g, dc, dord, nt, eids, k, out, s));
    // the threshold buffers are host vectors: wait before they go out of scope
    UTRI_HIP_TRY(hipStreamSynchronize(s));
    return UTRI_OK;
}

int utri_vertex_local(utri_graph* g, const double* t, int nt, const int64_t* vids, int64_t k,
                      int64_t* out, void* hip_stream) {
    UTRI_TRY(check_graph(g));
    if (k < 0 || (k > 0 && (!vids || !out))) return UTRI_E_INVALID;
    std::vector<double> cv;
    std::vector<int32_t> order;
    UTRI_TRY(sort_thresholds(t, nt, cv, order));
    if (k == 0) return UTRI_OK;
    hipStream_t s = as_stream(hip_stream);
    // vertex ids come from the caller: check the range before any kernel indexes with them
    UTRI_HIP_TRY(hipMemsetAsync(g->d_flags, 0, sizeof(uint32_t), s));
    hipLaunchKernelGGL(k_check_eids, dim3(nblk(k)), dim3(256), 0, s, vids, k, g->n, g->d_flags);
    UTRI_HIP_TRY(hipGetLastError());
    uint32_t bad = 0;
    UTRI_HIP_TRY(hipMemcpyAsync(&bad, g->d_flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    UTRI_HIP_TRY(hipStreamSynchronize(s));
    if (bad) return UTRI_E_INVALID;
    double* dc;
    int32_t* dord;
    UTRI_TRY(upload_thresholds(g, cv, order, s, &dc, &dord));
    UTRI_TRY(utri_vertex_local_launch(g, dc, dord, nt, vids, k, out, s));
    UTRI_HIP_TRY(hipStreamSynchronize(s));
    return UTRI_OK;
}

// Thresholds t_j = lo + (hi - lo) * j / 63, j = 0..63 (both ends included), and the class
// counts at each.
static int count_ladder(utri_graph* g, double lo, double hi, int cls, std::vector<double>& ts,
                        std::vector<int64_t>& cnt, void* hip_stream) {
    ts.resize(64);
    for (int j = 0; j < 64; j++) ts[j] = std::min(1.0, std::max(0.5, lo + (hi - lo) * (j / 63.0)));
    ts[63] = hi;
    std::vector<int64_t> out(128);
    UTRI_TRY(utri_count_batch(g, ts.data(), 64, UTRI_PRUNED, out.data(), hip_stream));
    cnt.resize(64);
    for (int j = 0; j < 64; j++) cnt[j] = out[2 * j + cls];
    return UTRI_OK;
}

int utri_topk(utri_graph* g, int64_t k, int which, int32_t* tri, double* sv, int64_t* count,
              void* hip_stream) {
    UTRI_TRY(check_graph(g));
    if (k < 0 || !count || (which != UTRI_BAL && which != UTRI_UNBAL) || (k > 0 && (!tri || !sv)))
        return UTRI_E_INVALID;
    *count = 0;
    if (k == 0 || g->m == 0) return UTRI_OK;
    hipStream_t s = as_stream(hip_stream);
    const int cls = which == UTRI_BAL ? 0 : 1;
    // 1. the largest threshold on a ladder whose class count is still >= k: the candidate
    // set {s <= -c} (balanced) or {s > c} (unbalanced) there holds the top k; bands are
    // tried from t = 1 down, so the walks prune as much as the answer allows (Lemma 2)
    std::vector<double> ts;
    std::vector<int64_t> cnt;
    // bands [0.999, 1], [0.99, 0.999], [0.9, 0.99], [0.5, 0.9]: each walk costs what its
    // lowest threshold prunes, so the answer's own band dominates the total
    const double starts[4] = {0.999, 0.99, 0.9, 0.5};
    double lo = 0.5, hi = 1.0;
    bool found = false;
    for (int b = 0; b < 4 && !found; b++) {
        lo = starts[b];
        hi = b == 0 ? 1.0 : starts[b - 1];
        UTRI_TRY(count_ladder(g, lo, hi, cls, ts, cnt, hip_stream));
        found = cnt[0] >= k;
    }
    double tstar = 0.5;
    int64_t nstar = cnt[0];  // fewer than k qualifying triangles: take them all
    if (found) {
        for (int round = 0; round < 8; round++) {
            int j = 0;
            while (j + 1 < 64 && cnt[j + 1] >= k) j++;
            tstar = ts[j];
            nstar = cnt[j];
            const double nhi = j + 1 < 64 ? ts[j + 1] : hi;
            if (nstar <= 2 * k + 4096 || !(nhi - tstar > 64 * 4e-16 * tstar)) break;
            lo = tstar;
            hi = nhi;
            UTRI_TRY(count_ladder(g, lo, hi, cls, ts, cnt, hip_stream));
        }
    }
    if (nstar == 0) return UTRI_OK;
    // 2. enumerate the candidates at t*, lexicographically sorted
    void *pt, *ps, *pk, *pi;
    UTRI_TRY(utri_scratch(g, SCR_TOPK_TRI, sizeof(int32_t) * 3 * (size_t)nstar, &pt));
    UTRI_TRY(utri_scratch(g, SCR_TOPK_S, sizeof(double) * (size_t)nstar, &ps));
    UTRI_TRY(utri_scratch(g, SCR_TOPK_KEY, sizeof(uint64_t) * 2 * (size_t)nstar, &pk));
    UTRI_TRY(utri_scratch(g, SCR_TOPK_IDX, sizeof(uint32_t) * 2 * (size_t)nstar, &pi));
    int64_t ec[2] = {0, 0};
    int32_t* list = (int32_t*)pt;
    UTRI_TRY(utri_enumerate(g, tstar, UTRI_PRUNED, which, cls == 0 ? list : nullptr,
                            cls == 0 ? nstar : 0, cls == 1 ? list : nullptr, cls == 1 ? nstar : 0,
                            ec, 1, hip_stream));
    const int64_t N = ec[cls];
    if (N != nstar) return UTRI_E_HIP;  // the count and the list disagree: internal error
    // 3. s and keys, a stable sort by key (ties keep the lexicographic order), first k
    uint64_t* key = (uint64_t*)pk;
    uint32_t* idx = (uint32_t*)pi;
    UTRI_TRY(utri_topk_keys_launch(g, list, N, cls, (double*)ps, key, idx, s));
    UTRI_TRY(radix_pairs(g, key, key + N, idx, idx + N, N, 64, s));
    const int64_t r = std::min<int64_t>(k, N);
    UTRI_TRY(utri_topk_gather_launch(list, (const double*)ps, idx + N, r, tri, sv, s));
    UTRI_HIP_TRY(hipStreamSynchronize(s));
    *count = r;
    return UTRI_OK;
}

int utri_sample(utri_graph* g, const double* t, int nt, int64_t k, int32_t worlds, uint64_t seed,
                int scheme, double* est, void* hip_stream) {
    UTRI_TRY(check_graph(g));
    // the baseline schemes are the same estimators without the Lemma-2 pruning of the
    // local search: full rows are searched and every drawn edge is searched
    const bool plain = scheme == UTRI_SAMPLE_EDGE_PLAIN || scheme == UTRI_SAMPLE_VERTEX_PLAIN;
    if (plain) scheme = scheme == UTRI_SAMPLE_EDGE_PLAIN ? UTRI_SAMPLE_EDGE : UTRI_SAMPLE_VERTEX;
    if ((scheme != UTRI_SAMPLE_EDGE && scheme != UTRI_SAMPLE_VERTEX) || k <= 0 || worlds <= 0 || !est)
        return UTRI_E_INVALID;
    if (scheme == UTRI_SAMPLE_EDGE ? g->m == 0 : g->n == 0) return UTRI_E_INVALID;
    std::vector<double> cv;
    std::vector<int32_t> order;
    UTRI_TRY(sort_thresholds(t, nt, cv, order));
    hipStream_t s = as_stream(hip_stream);
    double* dc;
    int32_t* dord;
    UTRI_TRY(upload_thresholds(g, cv, order, s, &dc, &dord));
    const double cprune = plain ? 0.0 : cv[0];
    int32_t* slen;
    UTRI_TRY(utri_sym_prepare(g, cprune, s, &slen));
    const size_t nh = (size_t)worlds * 2 * (nt + 1);
    void* hs;
    UTRI_TRY(utri_scratch(g, SCR_HIST, sizeof(uint64_t) * nh, &hs));
    UTRI_TRY(utri_fill_u64(hs, 0, (int64_t)nh, s));
    SampleParams sp;
    sp.cvals = dc;
    sp.nt = nt;
    sp.cmin = cprune;
    sp.seed = seed;
    sp.k = k;
    sp.worlds = worlds;
    sp.chunk = g->sample_chunk;
    sp.hist = (unsigned long long*)hs;
    if (scheme == UTRI_SAMPLE_EDGE) {
        UTRI_TRY(sample_passes(g, sp, slen, 0, n_draws(sp), s));
        UTRI_TRY(utri_finalize_launch((const unsigned long long*)hs, worlds, nt, dord, g->m, k,
                                      nullptr, est, s));
    } else {
        // every sampled vertex becomes the edge records of its prefix; each triangle at
        // the vertex is counted through both of its edges there, hence the halving
        int64_t R = 0;
        UTRI_TRY(utri_vertex_prepare(g, sp, slen, s, &R));
        if (g->m > 0) UTRI_TRY(sample_passes(g, sp, slen, 0, R, s));
        UTRI_TRY(utri_finalize_launch((const unsigned long long*)hs, worlds, nt, dord, g->n, k,
                                      nullptr, est, s, 2));
    }
    UTRI_HIP_TRY(hipStreamSynchronize(s));
    return UTRI_OK;
}

int utri_batch(utri_graph* g, const double* t, int nt, int64_t k, int32_t worlds, uint64_t seed,
               int64_t* exact, double* est, int use_graph, void* hip_stream) {
    UTRI_TRY(check_graph(g));
    if (est && (k <= 0 || worlds <= 0)) return UTRI_E_INVALID;
    if (g->m == 0 && est) return UTRI_E_INVALID;
    std::vector<double> cv;
    std::vector<int32_t> order;
    UTRI_TRY(sort_thresholds(t, nt, cv, order));
    hipStream_t s = as_stream(hip_stream);
    double* dc;
    int32_t* dord;
    UTRI_TRY(upload_thresholds(g, cv, order, s, &dc, &dord));
    void* pseed;
    UTRI_TRY(utri_scratch(g, SCR_SEED, sizeof(uint64_t), &pseed));
    UTRI_HIP_TRY(hipMemcpyAsync(pseed, &seed, sizeof(uint64_t), hipMemcpyHostToDevice, s));
    const uint64_t* sd = (const uint64_t*)pseed;
    UtriBatchGraph& B = g->batch;
    if (!use_graph) {
        UTRI_TRY(batch_sequence(g, dc, dord, nt, cv[0], k, worlds, sd, exact, est, s));
        UTRI_HIP_TRY(hipStreamSynchronize(s));
        return UTRI_OK;
    }
    // Graphs are captured and replayed on a stream owned by the handle (capture is not
    // allowed on the legacy default stream); events order it after / before `s`.
    if (!B.stream) UTRI_HIP_TRY(hipStreamCreateWithFlags(&B.stream, hipStreamNonBlocking));
    if (!B.ev) UTRI_HIP_TRY(hipEventCreateWithFlags(&B.ev, hipEventDisableTiming));
    UTRI_HIP_TRY(hipEventRecord(B.ev, s));
    UTRI_HIP_TRY(hipStreamWaitEvent(B.stream, B.ev, 0));
    hipStream_t gs = B.stream;
    // a captured graph is reused only with the same shape, outputs, scratch buffers (no
    // reallocation since capture) and launch shape (the autotuner may have changed it)
    const bool same = B.exec && B.nt == nt && B.k == k && B.worlds == worlds && B.exact == exact &&
                      B.est == est && B.cvals == cv && B.scr_gen == g->scr_gen &&
                      B.walk_blocks_per_cu == g->walk_blocks_per_cu &&
                      B.sample_chunk == g->sample_chunk && B.sample_pass == g->sample_pass &&
                      B.walk_order == g->walk_order && B.walk_tune == g->walk_tune;
    if (!same) {
        if (B.exec) { (void)hipGraphExecDestroy(B.exec); B.exec = nullptr; }
        if (B.graph) { (void)hipGraphDestroy(B.graph); B.graph = nullptr; }
        // eager run first: sizes every scratch buffer, so capture records kernels only
        UTRI_TRY(batch_sequence(g, dc, dord, nt, cv[0], k, worlds, sd, exact, est, gs));
        UTRI_HIP_TRY(hipStreamSynchronize(gs));
        UTRI_HIP_TRY(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
        int rc = batch_sequence(g, dc, dord, nt, cv[0], k, worlds, sd, exact, est, gs);
        hipGraph_t gr = nullptr;
        hipError_t e = hipStreamEndCapture(gs, &gr);
        if (rc != UTRI_OK) { if (gr) (void)hipGraphDestroy(gr); return rc; }
        UTRI_HIP_TRY(e);
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
        if (e != hipSuccess) { (void)hipGraphDestroy(gr); UTRI_HIP_TRY(e); }
        B.graph = gr;
        B.exec = ex;
        B.nt = nt;
        B.k = k;
        B.worlds = worlds;
        B.exact = exact;
        B.est = est;
        B.cvals = cv;
        B.scr_gen = g->scr_gen;
        B.walk_blocks_per_cu = g->walk_blocks_per_cu;
        B.sample_chunk = g->sample_chunk;
        B.sample_pass = g->sample_pass;
        B.walk_order = g->walk_order;
        B.walk_tune = g->walk_tune;
    }
    // thresholds and seed are read from device buffers written above on `s`
    UTRI_HIP_TRY(hipGraphLaunch(B.exec, gs));
    UTRI_HIP_TRY(hipEventRecord(B.ev, gs));
    UTRI_HIP_TRY(hipStreamWaitEvent(s, B.ev, 0));
    // thresholds / seed were uploaded from host memory owned by this call
    UTRI_HIP_TRY(hipStreamSynchronize(s));
    return UTRI_OK;
}

int utri_walk_stats(utri_graph* g, double t, int method, int64_t out[5], void* hip_stream) {
    UTRI_TRY(check_graph(g));
    if (!out || !t_ok(t)) return UTRI_E_INVALID;
    if (method < UTRI_PLAIN || method > UTRI_PRUNED_L3) return UTRI_E_INVALID;
    hipStream_t s = as_stream(hip_stream);
    const double c = utri_c_of_t(t);
    int64_t *items, *nitems;
    int32_t* len;
    UTRI_TRY(walk_prepare_for(g, method, c, s, &items, &nitems, &len));
    void *acc, *tmp, *tot;
    UTRI_TRY(utri_scratch(g, SCR_ACC, sizeof(uint64_t) * 4, &acc));
    UTRI_TRY(utri_scratch(g, SCR_IOFF, sizeof(int64_t) * (size_t)(g->n + 1), &tmp));
    UTRI_TRY(utri_scratch(g, SCR_OUT, sizeof(int64_t) * 4, &tot));
    UTRI_TRY(utri_fill_u64(acc, 0, 3, s));
    UTRI_TRY(utri_fill_u64(tot, 0, 1, s));
    // m_c = sum of the kept source-row prefixes (the k_items pass has consumed SCR_IOFF)
    UTRI_TRY(utri_scan_i32(g, len, (int64_t*)tmp, g->n, (int64_t*)tot, s));
    WalkParams wp = base_params(method, c);
    wp.acc = (unsigned long long*)acc;
    UTRI_TRY(utri_walk_launch(g, WALK_STATS, wp, items, nitems, len, 0, s));
    uint64_t h[3] = {0, 0, 0};
    int64_t mc = 0, ni = 0;
    UTRI_HIP_TRY(hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, s));
    UTRI_HIP_TRY(hipMemcpyAsync(&mc, tot, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    UTRI_HIP_TRY(hipMemcpyAsync(&ni, nitems, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    UTRI_HIP_TRY(hipStreamSynchronize(s));
    out[0] = mc;
    out[1] = (int64_t)h[1];
    out[2] = (int64_t)h[0];
    out[3] = (int64_t)h[2];
    out[4] = ni;
    return UTRI_OK;
}

int utri_timing(utri_graph* g, int enable, double* ms, int64_t* launches) {
    UTRI_TRY(check_graph(g));
    if (enable == 1) {
        if (!g->tev0) UTRI_HIP_TRY(hipEventCreate(&g->tev0));
        if (!g->tev1) UTRI_HIP_TRY(hipEventCreate(&g->tev1));
        g->timing = 1;
        g->timing_ms = 0.0;
        g->timing_launches = 0;
    } else if (enable == 0) {
        g->timing = 0;
    }
    if (ms) *ms = g->timing_ms;
    if (launches) *launches = g->timing_launches;
    return UTRI_OK;
}

int utri_set_walk_order(utri_graph* g, int order) {
    UTRI_TRY(check_graph(g));
    if (order < UTRI_ORDER_AUTO || order > UTRI_ORDER_SHORTER) return UTRI_E_INVALID;
    g->walk_order = order;
    return UTRI_OK;
}

int utri_get_tuning(utri_graph* g, int64_t out[UTRI_TUNE_COUNT]) {
    UTRI_TRY(check_graph(g));
    if (!out) return UTRI_E_INVALID;
    tune_get(g, out);
    return UTRI_OK;
}

int utri_set_tuning(utri_graph* g, const int64_t in[UTRI_TUNE_COUNT]) {
    UTRI_TRY(check_graph(g));
    if (!in) return UTRI_E_INVALID;
    return tune_set(g, in);
}

int utri_autotune(utri_graph* g, double t, const char* cache_path, void* hip_stream) {
    UTRI_TRY(check_graph(g));
    if (!t_ok(t)) return UTRI_E_INVALID;
    // a choice cached for this graph shape is taken as it is
    {
        int64_t v[UTRI_TUNE_COUNT];
        if (read_cache(g, cache_path, v) && tune_set(g, v) == UTRI_OK) return UTRI_OK;
    }
    hipStream_t s = as_stream(hip_stream);
    // events are released on every return path
    struct Events {
        hipEvent_t a = nullptr, b = nullptr;
        ~Events() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev;
    UTRI_HIP_TRY(hipEventCreate(&ev.a));
    UTRI_HIP_TRY(hipEventCreate(&ev.b));
    // the counting query at t: one warm-up, then the summed time of three runs
    const auto time_count = [&](float* ms_out) -> int {
        int64_t out[2];
        UTRI_TRY(count_impl(g, t, UTRI_PRUNED, out, s));
        float tot = 0.f;
        for (int r = 0; r < 3; r++) {
            UTRI_HIP_TRY(hipEventRecord(ev.a, s));
            UTRI_TRY(count_impl(g, t, UTRI_PRUNED, out, s));
            UTRI_HIP_TRY(hipEventRecord(ev.b, s));
            UTRI_HIP_TRY(hipEventSynchronize(ev.b));
            float ms = 0.f;
            UTRI_HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
            tot += ms;
        }
        *ms_out = tot;
        return UTRI_OK;
    };
    // coordinate descent over the walk's launch parameters, one at a time in this order,
    // each kept at its fastest value for the rest
    int64_t cur[UTRI_TUNE_COUNT];
    tune_get(g, cur);
    struct Axis {
        int idx;
        std::vector<int64_t> vals;
    };
    // 0 work-groups per CU = the kernel's resident occupancy; more trade tail balance for
    // overhead
    const Axis axes[] = {
        {UTRI_TUNE_WALK_BLOCKS_PER_CU, {0, 2, 3, 8}},
        {UTRI_TUNE_WALK_PARTNERS, {256, 512, 1024, 2048, 4096}},
        {UTRI_TUNE_WALK_CHUNK, {512, 1024, 2048}},
        {UTRI_TUNE_WALK_LIGHT_CAP, {32, 64, 128}},
        {UTRI_TUNE_WALK_UNROLL, {2, 4, 8}},
    };
    for (const Axis& ax : axes) {
        float best = 1e30f;
        int64_t best_v = cur[ax.idx];
        for (int64_t v : ax.vals) {
            int64_t trial[UTRI_TUNE_COUNT];
            for (int i = 0; i < UTRI_TUNE_COUNT; i++) trial[i] = cur[i];
            trial[ax.idx] = v;
            if (tune_set(g, trial) != UTRI_OK) continue;  // e.g. a chunk below the light cap
            float ms = 0.f;
            UTRI_TRY(time_count(&ms));
            if (ms < best) { best = ms; best_v = v; }
        }
        cur[ax.idx] = best_v;
        UTRI_TRY(tune_set(g, cur));
    }
    // the shorter-row crossover: time both orders at t and move the crossover so that this
    // query's ratio (ids the plain order streams per kept edge) takes the faster one
    if (g->walk_order == UTRI_ORDER_AUTO) {
        float ms_short = 0.f, ms_plain = 0.f;
        int64_t trial[UTRI_TUNE_COUNT];
        for (int i = 0; i < UTRI_TUNE_COUNT; i++) trial[i] = cur[i];
        trial[UTRI_TUNE_WALK_SHORTER_MIN] = 0;  // always the shorter row
        UTRI_TRY(tune_set(g, trial));
        UTRI_TRY(time_count(&ms_short));
        double ratio = 0.0;
        UTRI_TRY(utri_walk_plain_ratio(g, s, &ratio));
        trial[UTRI_TUNE_WALK_SHORTER_MIN] = (int64_t)1 << 40;  // never
        UTRI_TRY(tune_set(g, trial));
        UTRI_TRY(time_count(&ms_plain));
        const int64_t def = WalkTune{}.shorter_min;
        const int64_t r = (int64_t)std::min(ratio, 1e12);
        cur[UTRI_TUNE_WALK_SHORTER_MIN] =
            ms_short < ms_plain ? std::min<int64_t>(def, r) : std::max<int64_t>(def, r + 1);
        UTRI_TRY(tune_set(g, cur));
    }
    // draws per sampler group item
    std::vector<double> tv{t};
    const int32_t worlds = 64;
    const int64_t k = 4096;
    void* pest;
    UTRI_TRY(utri_scratch(g, SCR_TUNE, sizeof(double) * worlds * 2, &pest));
    double* est = (double*)pest;
    float best_s = 1e30f;
    int best_c = g->sample_chunk;
    for (int c : {64, 128, 256, 512}) {
        g->sample_chunk = c;
        int rc = utri_sample(g, tv.data(), 1, k, worlds, 12345, UTRI_SAMPLE_EDGE, est, hip_stream);
        if (rc != UTRI_OK) return rc;
        float tot = 0.f;
        for (int r = 0; r < 3; r++) {
            UTRI_HIP_TRY(hipEventRecord(ev.a, s));
            rc = utri_sample(g, tv.data(), 1, k, worlds, 12345, UTRI_SAMPLE_EDGE, est, hip_stream);
            UTRI_HIP_TRY(hipEventRecord(ev.b, s));
            UTRI_HIP_TRY(hipEventSynchronize(ev.b));
            if (rc != UTRI_OK) return rc;
            float ms = 0.f;
            UTRI_HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
            tot += ms;
        }
        if (tot < best_s) { best_s = tot; best_c = c; }
    }
    g->sample_chunk = best_c;
    if (cache_path) {
        FILE* f = fopen(cache_path, "a");
        if (f) {
            int64_t v[UTRI_TUNE_COUNT];
            tune_get(g, v);
            std::string line = "{" + cache_key(g);
            for (int i = 0; i < UTRI_TUNE_COUNT; i++)
                line += std::string(", \"") + TUNE_NAMES[i] + "\": " + std::to_string(v[i]);
            line += "}\n";
            fputs(line.c_str(), f);
            fclose(f);
        }
    }
    return UTRI_OK;
}

}  // extern "C"
