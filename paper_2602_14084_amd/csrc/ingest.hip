// ingest.hip -- graph load: validation, canonical edge list, Node-Order relabelling,
// symmetric rows in Absolute Edge Order, oriented rows, per-row hash tables.
//
// Model: Definition "Uncertain Signed Graph" (Section 3) -- undirected, one P+ per
// edge. Self-loops and repeated edges are removed (the experiments section removes
// them from its datasets). Node Order (Section 4) ranks vertices by (degree, id);
// vertices are relabelled by that rank so an oriented edge u -> v simply has v > u.
// Rows are sorted in Absolute Edge Order (Section 5): |d| descending, then neighbour
// id, so the entries any threshold keeps (Lemma 2) are a prefix of every row.
#include <rocprim/device/device_radix_sort.hpp>

#include <cstdio>
#include <cstdlib>
#include <new>

#include "utri_internal.h"

namespace {

constexpr int TPB = 256;

inline int blocks_for(int64_t n) { return (int)((n + TPB - 1) / TPB); }

inline unsigned bitlen(uint64_t v) {
    unsigned b = 0;
    while (v) { b++; v >>= 1; }
    return b;
}

__global__ void k_canon(const int64_t* __restrict__ src, const int64_t* __restrict__ dst,
                        const double* __restrict__ p, int64_t m_in, int64_t n,
                        uint64_t* __restrict__ key, double* __restrict__ val,
                        uint32_t* __restrict__ flags, unsigned long long* __restrict__ nself) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int self = 0;
    if (i < m_in) {
        int64_t a = src[i], b = dst[i];
        double q = p[i];
        uint32_t f = 0;
        if (a < 0 || a >= n || b < 0 || b >= n) f |= UTRI_FLAG_BAD_ID;
        if (!(q >= 0.0 && q <= 1.0)) f |= UTRI_FLAG_BAD_P;
        if (f) atomicOr(flags, f);
        uint64_t k;
        if (a == b || f) {
            k = ((uint64_t)n << 32) | (uint64_t)n;  // sorts after every real edge
            self = (a == b && !f);
        } else {
            uint64_t lo = (uint64_t)(a < b ? a : b), hi = (uint64_t)(a < b ? b : a);
            k = (lo << 32) | hi;
        }
        key[i] = k;
        val[i] = q;
    }
    uint64_t cnt = utri_wave_sum_u64((uint64_t)self);
    if (utri_lane() == 0 && cnt) atomicAdd(nself, (unsigned long long)cnt);
}

__global__ void k_heads(const uint64_t* __restrict__ key, const double* __restrict__ val,
                        int64_t cnt, uint64_t dropkey, int32_t* __restrict__ head,
                        uint32_t* __restrict__ flags) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    uint64_t k = key[i];
    int h = 0;
    if (k != dropkey) {
        if (i == 0 || key[i - 1] != k) {
            h = 1;
        } else if (val[i - 1] != val[i]) {
            atomicOr(flags, UTRI_FLAG_CONFLICT);
        }
    }
    head[i] = h;
}

__global__ void k_scatter_edges(const uint64_t* __restrict__ key, const double* __restrict__ val,
                                const int32_t* __restrict__ head, const int64_t* __restrict__ pos,
                                int64_t cnt, int32_t* __restrict__ lo, int32_t* __restrict__ hi,
                                double* __restrict__ p, double* __restrict__ d) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt || !head[i]) return;
    int64_t e = pos[i];
    uint64_t k = key[i];
    lo[e] = (int32_t)(k >> 32);
    hi[e] = (int32_t)(k & 0xFFFFFFFFull);
    p[e] = val[i];
    d[e] = utri_d_of_p(val[i]);
}

__global__ void k_degree(const int32_t* __restrict__ lo, const int32_t* __restrict__ hi, int64_t m,
                         int32_t* __restrict__ deg) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    atomicAdd(&deg[lo[e]], 1);
    atomicAdd(&deg[hi[e]], 1);
}

__global__ void k_iota_u32(uint32_t* __restrict__ a, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = (uint32_t)i;
}

// Node-Order sort key of vertex i: degree first; ties by a fixed bijective mix of the id
// (the finaliser of MurmurHash3), so that within a degree class the new ids are in no
// input-dependent pattern and their low bits index the walk's LDS tables directly.
__global__ void k_rank_key(const int32_t* __restrict__ deg, uint64_t* __restrict__ key, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t x = (uint32_t)i;
    x ^= x >> 16;
    x *= 0x85EBCA6Bu;
    x ^= x >> 13;
    x *= 0xC2B2AE35u;
    x ^= x >> 16;
    key[i] = ((uint64_t)(uint32_t)deg[i] << 32) | x;
}

__global__ void k_relabel(const uint32_t* __restrict__ order, const uint64_t* __restrict__ skey,
                          int64_t n, int32_t* __restrict__ perm, int32_t* __restrict__ inv,
                          int32_t* __restrict__ deg_new) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t old = order[i];
    perm[i] = (int32_t)old;
    inv[old] = (int32_t)i;
    deg_new[i] = (int32_t)(skey[i] >> 32);
}

__global__ void k_max_i32(const int32_t* __restrict__ a, int64_t n, unsigned int* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int v = (i < n) ? a[i] : 0;
#pragma unroll
    for (int d = UTRI_WAVE / 2; d >= 1; d >>= 1) v = max(v, __shfl_xor(v, d, UTRI_WAVE));
    if (utri_lane() == 0 && v) atomicMax(out, (unsigned)v);
}

// symmetric entry i: edge i>>1; side 0 = (inv lo -> inv hi), side 1 = (inv hi -> inv lo)
__device__ inline void sym_entry(const int32_t* lo, const int32_t* hi, const int32_t* inv,
                                 uint32_t i, int32_t& row, int32_t& nbr) {
    uint32_t e = i >> 1;
    int32_t a = inv[lo[e]], b = inv[hi[e]];
    if (i & 1u) { row = b; nbr = a; } else { row = a; nbr = b; }
}

__global__ void k_key_nbr(const int32_t* __restrict__ lo, const int32_t* __restrict__ hi,
                          const int32_t* __restrict__ inv, int64_t cnt,
                          uint32_t* __restrict__ key) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    int32_t r, v;
    sym_entry(lo, hi, inv, (uint32_t)i, r, v);
    key[i] = (uint32_t)v;
}

// Absolute Edge Order key: |d| descending. |d| in [0,1], so its bits are at most
// 0x3FF0000000000000 and (that - bits) is ascending in the order we want.
__global__ void k_key_absd(const uint32_t* __restrict__ ord, const double* __restrict__ ed,
                           int64_t cnt, uint64_t* __restrict__ key) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    double a = fabs(ed[ord[i] >> 1]);
    uint64_t bits = (uint64_t)__double_as_longlong(a);
    key[i] = 0x3FF0000000000000ull - bits;
}

__global__ void k_key_row(const uint32_t* __restrict__ ord, const int32_t* __restrict__ lo,
                          const int32_t* __restrict__ hi, const int32_t* __restrict__ inv,
                          int64_t cnt, uint32_t* __restrict__ key) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    int32_t r, v;
    sym_entry(lo, hi, inv, ord[i], r, v);
    key[i] = (uint32_t)r;
}

__global__ void k_gather_sym(const uint32_t* __restrict__ ord, const int32_t* __restrict__ lo,
                             const int32_t* __restrict__ hi, const int32_t* __restrict__ inv,
                             const double* __restrict__ ed, int64_t cnt,
                             int32_t* __restrict__ s_adj, double* __restrict__ s_d,
                             int32_t* __restrict__ s_eid, int32_t* __restrict__ s_row,
                             int32_t* __restrict__ oflag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    uint32_t ent = ord[i];
    int32_t r, v;
    sym_entry(lo, hi, inv, ent, r, v);
    s_adj[i] = v;
    s_d[i] = ed[ent >> 1];
    s_eid[i] = (int32_t)(ent >> 1);
    s_row[i] = r;
    oflag[i] = (v > r) ? 1 : 0;
}

__global__ void k_scatter_oriented(const int32_t* __restrict__ oflag,
                                   const int64_t* __restrict__ opos,
                                   const int32_t* __restrict__ s_adj,
                                   const double* __restrict__ s_d,
                                   const int32_t* __restrict__ s_eid, int64_t cnt,
                                   int32_t* __restrict__ o_adj, double* __restrict__ o_d,
                                   int32_t* __restrict__ o_eid) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt || !oflag[i]) return;
    int64_t j = opos[i];
    o_adj[j] = s_adj[i];
    o_d[j] = s_d[i];
    o_eid[j] = s_eid[i];
}

// Pack a quantized |d| above every oriented-row id and sign(d) into bit 31.
__global__ void k_pack_oriented(int32_t* __restrict__ o_adj, const double* __restrict__ o_d,
                                int64_t m, int idbits, int mb) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const double d = o_d[i];
    const uint32_t qmax = (1u << mb) - 1u;
    // floor (exact: a power-of-two scaling): q <= |d| * 2^mb < q + 1; |d| = 1 maps to
    // 2^mb - 1, whose bucket [q, q + 1] * 2^-mb still holds it
    uint32_t q = (uint32_t)(fabs(d) * (double)(1u << mb));
    if (q > qmax) q = qmax;
    // sign(d) in bit 31 whatever the widths, so one xor of two words gives a product's sign
    const uint32_t sign = d < 0.0 ? 0x80000000u : 0u;
    o_adj[i] = (int32_t)(((uint32_t)o_adj[i]) | (q << idbits) | sign);
}

__global__ void k_oriented_offsets(const int64_t* __restrict__ s_off,
                                   const int64_t* __restrict__ opos,
                                   const int32_t* __restrict__ oflag, int64_t n, int64_t cnt,
                                   int64_t* __restrict__ o_off) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v > n) return;
    if (v < n) {
        int64_t j = s_off[v];
        o_off[v] = (j < cnt) ? opos[j] : (cnt > 0 ? opos[cnt - 1] + oflag[cnt - 1] : 0);
    } else {
        o_off[n] = cnt > 0 ? opos[cnt - 1] + oflag[cnt - 1] : 0;
    }
}

__global__ void k_outdeg(const int64_t* __restrict__ o_off, int64_t n, int32_t* __restrict__ od) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) od[v] = (int32_t)(o_off[v + 1] - o_off[v]);
}

__global__ void k_hsize(const int32_t* __restrict__ deg_new, int64_t n, int64_t* __restrict__ hs) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    hs[v] = utri_htable_slots(deg_new[v]);
}

// Entry i of the symmetric rows takes the first empty slot of the first bucket, from its
// home bucket on, that has one; slots therefore fill in order within a bucket.
__global__ void k_hinsert(const int32_t* __restrict__ s_row, const int32_t* __restrict__ s_adj,
                          const double* __restrict__ s_d, const int64_t* __restrict__ h_off,
                          int64_t cnt, uint32_t* __restrict__ htab) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    const int32_t r = s_row[i];
    const int32_t key = s_adj[i];
    const int64_t base = h_off[r];
    const int64_t nbk = (h_off[r + 1] - base) / UTRI_HB;
    int lgb = 0;
    while ((1ll << lgb) < nbk) lgb++;
    uint32_t b = utri_hbucket(key, lgb);
    for (;;) {
        const int64_t b0 = base + (int64_t)b * UTRI_HB;
        // claim the first slot seen empty; a lost race moves on to the next one
        int q = 0;
        uint32_t* hkey = htab + utri_hkey_index(b0);
        while (q < UTRI_HB && __atomic_load_n(&hkey[q], __ATOMIC_RELAXED) != 0xFFFFFFFFu) q++;
        for (; q < UTRI_HB; q++) {
            if (atomicCAS(&hkey[q], 0xFFFFFFFFu, (uint32_t)key) == 0xFFFFFFFFu) {
                reinterpret_cast<double*>(htab)[utri_hd_index(b0 + q)] = s_d[i];
                return;
            }
        }
        b = (b + 1) & (uint32_t)(nbk - 1);
    }
}

__global__ void k_fill_u64(uint64_t* __restrict__ p, uint64_t v, int64_t n) {
    UTRI_FOR_GRID(i, n) p[i] = v;
}

__global__ void k_set_i64(int64_t* __restrict__ p, int64_t v) { *p = v; }

__global__ void k_widen_i32(const int32_t* __restrict__ in, int64_t* __restrict__ out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i];
}

template <class T>
int dev_alloc(T** p, int64_t count) {
    size_t bytes = sizeof(T) * (size_t)(count > 0 ? count : 1);
    hipError_t e = hipMalloc((void**)p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return e == hipErrorOutOfMemory ? UTRI_E_NOMEM : UTRI_E_HIP;
    }
    return UTRI_OK;
}

struct TmpBuf {
    void* p = nullptr;
    ~TmpBuf() { if (p) (void)hipFree(p); }
};

template <class T>
int tmp_alloc(TmpBuf& b, int64_t count, T** out) {
    int rc = dev_alloc((T**)&b.p, count);
    *out = (T*)b.p;
    return rc;
}

template <class K, class V>
int sort_pairs(utri_graph* g, const K* kin, K* kout, const V* vin, V* vout, int64_t cnt,
               unsigned end_bit, hipStream_t s) {
    if (cnt == 0) return UTRI_OK;
    size_t bytes = 0;
    UTRI_HIP_TRY(rocprim::radix_sort_pairs(nullptr, bytes, kin, kout, vin, vout, (size_t)cnt, 0,
                                           end_bit, s));
    void* tmp;
    UTRI_TRY(utri_scratch(g, SCR_TEMP, bytes, &tmp));
    UTRI_HIP_TRY(rocprim::radix_sort_pairs(tmp, bytes, kin, kout, vin, vout, (size_t)cnt, 0,
                                           end_bit, s));
    return UTRI_OK;
}

}  // namespace

void utri_note_hip_error(hipError_t e, const char* what, const char* file, int line) {
    if (getenv("UTRI_LOG"))
        fprintf(stderr, "[utri] %s failed: %s (%s:%d)\n", what, hipGetErrorString(e), file, line);
}

int utri_scratch(utri_graph* g, int slot, size_t bytes, void** out) {
    if (bytes == 0) bytes = 16;
    if (g->arena) {
        // no-allocation mode: a slot asked for twice in one call keeps its buffer
        if (g->arena_slot[slot] && g->arena_slot_bytes[slot] >= bytes) {
            *out = g->arena_slot[slot];
            return UTRI_OK;
        }
        const size_t off = (g->arena_used + 255) & ~(size_t)255;
        if (off > g->arena_bytes || bytes > g->arena_bytes - off) return UTRI_E_CAPACITY;
        g->arena_slot[slot] = g->arena + off;
        g->arena_slot_bytes[slot] = bytes;
        g->arena_used = off + bytes;
        *out = g->arena_slot[slot];
        return UTRI_OK;
    }
    if (g->scr_bytes[slot] < bytes) {
        if (g->scr[slot]) UTRI_HIP_TRY(hipFree(g->scr[slot]));
        g->scr[slot] = nullptr;
        g->scr_bytes[slot] = 0;
        g->scr_gen++;  // any captured batch graph holding the old address is stale now
        size_t want = bytes + bytes / 8;
        hipError_t e = hipMalloc(&g->scr[slot], want);
        if (e != hipSuccess) {
            g->scr[slot] = nullptr;
            return e == hipErrorOutOfMemory ? UTRI_E_NOMEM : UTRI_E_HIP;
        }
        g->scr_bytes[slot] = want;
    }
    *out = g->scr[slot];
    return UTRI_OK;
}

int utri_fill_u64(void* p, uint64_t v, int64_t count, hipStream_t s) {
    if (count <= 0) return UTRI_OK;
    hipLaunchKernelGGL(k_fill_u64, dim3(utri_grid(count, TPB)), dim3(TPB), 0, s, (uint64_t*)p, v, count);
    UTRI_HIP_TRY(hipGetLastError());
    return UTRI_OK;
}

int utri_exclusive_scan_i64(utri_graph* g, const int64_t* in, int64_t* out, int64_t n,
                            hipStream_t s) {
    return utri_scan_i64(g, in, out, n, nullptr, s);
}

int utri_exclusive_scan_i32_to_i64(utri_graph* g, const int32_t* in, int64_t* out, int64_t n,
                                   hipStream_t s) {
    return utri_scan_i32(g, in, out, n, nullptr, s);
}

// Rebuild every row structure from (e_lo, e_hi, e_d, inv, deg_new): symmetric rows in
// Absolute Edge Order, oriented rows, hash tables. Used at load and after set_p.
int utri_build_rows(utri_graph* g, hipStream_t s) {
    const int64_t n = g->n, m = g->m, cnt = 2 * m;
    g->rows_gen++;
    if (cnt == 0) {
        UTRI_HIP_TRY(hipMemsetAsync(g->s_off, 0, sizeof(int64_t) * (n + 1), s));
        UTRI_HIP_TRY(hipMemsetAsync(g->o_off, 0, sizeof(int64_t) * (n + 1), s));
        UTRI_HIP_TRY(hipMemsetAsync(g->h_off, 0, sizeof(int64_t) * (n + 1), s));
        return UTRI_OK;
    }
    const unsigned nbits = n > 1 ? bitlen((uint64_t)(n - 1)) : 1;
    TmpBuf b1, b2, b3, b4, b5, b6, b7;
    uint32_t *ka, *kb, *oa, *ob;
    uint64_t *k64a, *k64b;
    UTRI_TRY(tmp_alloc(b1, cnt, &ka));
    UTRI_TRY(tmp_alloc(b2, cnt, &kb));
    UTRI_TRY(tmp_alloc(b3, cnt, &oa));
    UTRI_TRY(tmp_alloc(b4, cnt, &ob));
    UTRI_TRY(tmp_alloc(b5, cnt, &k64a));
    UTRI_TRY(tmp_alloc(b6, cnt, &k64b));
    const int nb = blocks_for(cnt);
    // pass 1: neighbour id ascending (least significant key)
    hipLaunchKernelGGL(k_key_nbr, dim3(nb), dim3(TPB), 0, s, g->e_lo, g->e_hi, g->inv, cnt, ka);
    hipLaunchKernelGGL(k_iota_u32, dim3(nb), dim3(TPB), 0, s, oa, cnt);
    UTRI_HIP_TRY(hipGetLastError());
    UTRI_TRY(sort_pairs(g, ka, kb, oa, ob, cnt, nbits, s));
    // pass 2: |d| descending (stable, keeps the neighbour order of ties)
    hipLaunchKernelGGL(k_key_absd, dim3(nb), dim3(TPB), 0, s, ob, g->e_d, cnt, k64a);
    UTRI_HIP_TRY(hipGetLastError());
    UTRI_TRY(sort_pairs(g, k64a, k64b, ob, oa, cnt, 62u, s));
    // pass 3: row ascending (most significant key)
    hipLaunchKernelGGL(k_key_row, dim3(nb), dim3(TPB), 0, s, oa, g->e_lo, g->e_hi, g->inv, cnt, ka);
    UTRI_HIP_TRY(hipGetLastError());
    UTRI_TRY(sort_pairs(g, ka, kb, oa, ob, cnt, nbits, s));
    // gather the symmetric rows
    int32_t* oflag = (int32_t*)ka;  // reuse
    hipLaunchKernelGGL(k_gather_sym, dim3(nb), dim3(TPB), 0, s, ob, g->e_lo, g->e_hi, g->inv,
                       g->e_d, cnt, g->s_adj, g->s_d, g->s_eid, g->s_row, oflag);
    UTRI_HIP_TRY(hipGetLastError());
    // row offsets from the (ascending) degrees of the new ids
    UTRI_TRY(utri_exclusive_scan_i32_to_i64(g, g->deg_new, g->s_off, n, s));
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, g->s_off + n, cnt);
    // oriented rows: entries with neighbour > row, order kept
    int64_t* opos = (int64_t*)k64a;
    UTRI_TRY(utri_exclusive_scan_i32_to_i64(g, oflag, opos, cnt, s));
    hipLaunchKernelGGL(k_scatter_oriented, dim3(nb), dim3(TPB), 0, s, oflag, opos, g->s_adj,
                       g->s_d, g->s_eid, cnt, g->o_adj, g->o_d, g->o_eid);
    hipLaunchKernelGGL(k_oriented_offsets, dim3(blocks_for(n + 1)), dim3(TPB), 0, s, g->s_off,
                       opos, oflag, n, cnt, g->o_off);
    UTRI_HIP_TRY(hipGetLastError());
    // code bits of the oriented rows: sign + up to 15 magnitude bits above the id
    g->idbits = (int)nbits;
    g->idmask = (nbits >= 32) ? 0xFFFFFFFFu : ((1u << nbits) - 1u);
    const int spare = 32 - (int)nbits;
    g->code_mb = (spare >= 3) ? std::min(spare - 1, 15) : 0;
    // UTRI_CODE_MB caps the magnitude bits (0 = no code): narrow codes on small graphs take
    // the decision path that large graphs take; results never depend on the width
    if (const char* e = getenv("UTRI_CODE_MB")) g->code_mb = std::max(0, std::min(g->code_mb, atoi(e)));
    if (g->code_mb > 0) {
        hipLaunchKernelGGL(k_pack_oriented, dim3(blocks_for(m)), dim3(TPB), 0, s, g->o_adj, g->o_d,
                           m, g->idbits, g->code_mb);
        UTRI_HIP_TRY(hipGetLastError());
    }
    // hash tables
    int64_t* hs;
    UTRI_TRY(tmp_alloc(b7, n, &hs));
    hipLaunchKernelGGL(k_hsize, dim3(blocks_for(n)), dim3(TPB), 0, s, g->deg_new, n, hs);
    UTRI_HIP_TRY(hipGetLastError());
    UTRI_TRY(utri_exclusive_scan_i64(g, hs, g->h_off, n, s));
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, g->h_off + n, g->h_total);
    UTRI_TRY(utri_fill_u64(g->h_tab, ~0ull, g->h_total * 2, s));  // 16 bytes per slot
    hipLaunchKernelGGL(k_hinsert, dim3(nb), dim3(TPB), 0, s, g->s_row, g->s_adj, g->s_d,
                       g->h_off, cnt, g->h_tab);
    UTRI_HIP_TRY(hipGetLastError());
    // temporaries are freed at scope exit; hipFree waits for the device
    UTRI_HIP_TRY(hipStreamSynchronize(s));
    return UTRI_OK;
}

static void free_graph(utri_graph* g) {
    if (!g) return;
    void* ptrs[] = {g->e_lo, g->e_hi, g->e_p, g->e_d, g->perm, g->inv, g->deg_new, g->s_off,
                    g->s_adj, g->s_d, g->s_eid, g->s_row, g->h_off, g->h_tab, g->o_off,
                    g->o_adj, g->o_d, g->o_eid, g->d_flags};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (int i = 0; i < SCR_COUNT; i++)
        if (g->scr[i]) (void)hipFree(g->scr[i]);
    if (g->batch.exec) (void)hipGraphExecDestroy(g->batch.exec);
    if (g->batch.graph) (void)hipGraphDestroy(g->batch.graph);
    if (g->batch.stream) (void)hipStreamDestroy(g->batch.stream);
    if (g->batch.ev) (void)hipEventDestroy(g->batch.ev);
    if (g->tev0) (void)hipEventDestroy(g->tev0);
    if (g->tev1) (void)hipEventDestroy(g->tev1);
    delete g;
}

void utri_free_graph_internal(utri_graph* g) { free_graph(g); }

static int load_impl(const int64_t* src, const int64_t* dst, const double* p, int64_t m_in,
                     int64_t n, int ptr_kind, hipStream_t s, utri_graph* g) {
    UTRI_HIP_TRY(hipGetDevice(&g->device));
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, g->device) == hipSuccess && prop.multiProcessorCount > 0)
            g->num_cu = prop.multiProcessorCount;
    }
    // d_flags: [0] error bits, [1] max degree, [2..3] self-loop count (u64), [4] max out-degree
    UTRI_TRY(dev_alloc(&g->d_flags, 8));
    UTRI_HIP_TRY(hipMemsetAsync(g->d_flags, 0, 8 * sizeof(uint32_t), s));
    // inputs on the device
    TmpBuf bs, bd, bp;
    const int64_t *dsrc = src, *ddst = dst;
    const double* dp = p;
    if (ptr_kind == UTRI_HOST_PTR && m_in > 0) {
        int64_t *a, *b;
        double* c;
        UTRI_TRY(tmp_alloc(bs, m_in, &a));
        UTRI_TRY(tmp_alloc(bd, m_in, &b));
        UTRI_TRY(tmp_alloc(bp, m_in, &c));
        UTRI_HIP_TRY(hipMemcpyAsync(a, src, sizeof(int64_t) * m_in, hipMemcpyHostToDevice, s));
        UTRI_HIP_TRY(hipMemcpyAsync(b, dst, sizeof(int64_t) * m_in, hipMemcpyHostToDevice, s));
        UTRI_HIP_TRY(hipMemcpyAsync(c, p, sizeof(double) * m_in, hipMemcpyHostToDevice, s));
        dsrc = a; ddst = b; dp = c;
    }
    // canonical keys, sorted
    TmpBuf bk0, bk1, bv0, bv1, bh, bpos;
    uint64_t *k0 = nullptr, *k1 = nullptr;
    double *v0 = nullptr, *v1 = nullptr;
    int32_t* head = nullptr;
    int64_t* pos = nullptr;
    unsigned long long* nself = (unsigned long long*)(g->d_flags + 2);
    int64_t m = 0;
    if (m_in > 0) {
        UTRI_TRY(tmp_alloc(bk0, m_in, &k0));
        UTRI_TRY(tmp_alloc(bk1, m_in, &k1));
        UTRI_TRY(tmp_alloc(bv0, m_in, &v0));
        UTRI_TRY(tmp_alloc(bv1, m_in, &v1));
        hipLaunchKernelGGL(k_canon, dim3(blocks_for(m_in)), dim3(TPB), 0, s, dsrc, ddst, dp, m_in,
                           n, k0, v0, g->d_flags, nself);
        UTRI_HIP_TRY(hipGetLastError());
        uint32_t flags = 0;
        UTRI_HIP_TRY(hipMemcpyAsync(&flags, g->d_flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        UTRI_HIP_TRY(hipStreamSynchronize(s));
        if (flags & (UTRI_FLAG_BAD_ID | UTRI_FLAG_BAD_P)) return UTRI_E_INVALID;
        unsigned end_bit = 32 + bitlen((uint64_t)n);
        UTRI_TRY(sort_pairs(g, k0, k1, v0, v1, m_in, end_bit, s));
        UTRI_TRY(tmp_alloc(bh, m_in, &head));
        UTRI_TRY(tmp_alloc(bpos, m_in, &pos));
        const uint64_t dropkey = ((uint64_t)n << 32) | (uint64_t)n;
        hipLaunchKernelGGL(k_heads, dim3(blocks_for(m_in)), dim3(TPB), 0, s, k1, v1, m_in, dropkey,
                           head, g->d_flags);
        UTRI_HIP_TRY(hipGetLastError());
        UTRI_TRY(utri_exclusive_scan_i32_to_i64(g, head, pos, m_in, s));
        int64_t lastpos = 0;
        int32_t lasthead = 0;
        uint64_t ns = 0;
        UTRI_HIP_TRY(hipMemcpyAsync(&lastpos, pos + m_in - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        UTRI_HIP_TRY(hipMemcpyAsync(&lasthead, head + m_in - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        UTRI_HIP_TRY(hipMemcpyAsync(&flags, g->d_flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        UTRI_HIP_TRY(hipMemcpyAsync(&ns, nself, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        UTRI_HIP_TRY(hipStreamSynchronize(s));
        if (flags & UTRI_FLAG_CONFLICT) return UTRI_E_CONFLICT;
        m = lastpos + lasthead;
        g->self_loops = (int64_t)ns;
        g->dups = m_in - (int64_t)ns - m;
    }
    if (m >= ((int64_t)1 << 31)) return UTRI_E_RANGE;
    g->n = n;
    g->m = m;
    UTRI_TRY(dev_alloc(&g->e_lo, m));
    UTRI_TRY(dev_alloc(&g->e_hi, m));
    UTRI_TRY(dev_alloc(&g->e_p, m));
    UTRI_TRY(dev_alloc(&g->e_d, m));
    if (m > 0) {
        hipLaunchKernelGGL(k_scatter_edges, dim3(blocks_for(m_in)), dim3(TPB), 0, s, k1, v1, head,
                           pos, m_in, g->e_lo, g->e_hi, g->e_p, g->e_d);
        UTRI_HIP_TRY(hipGetLastError());
    }
    // degrees and Node-Order relabelling (by degree, ties by the mixed id)
    UTRI_TRY(dev_alloc(&g->perm, n));
    UTRI_TRY(dev_alloc(&g->inv, n));
    UTRI_TRY(dev_alloc(&g->deg_new, n));
    if (n > 0) {
        TmpBuf bdeg, bdk, bdk2, bo1, bo2;
        int32_t* deg;
        uint64_t *dk, *dk2;
        uint32_t *o1, *o2;
        UTRI_TRY(tmp_alloc(bdeg, n, &deg));
        UTRI_TRY(tmp_alloc(bdk, n, &dk));
        UTRI_TRY(tmp_alloc(bdk2, n, &dk2));
        UTRI_TRY(tmp_alloc(bo1, n, &o1));
        UTRI_TRY(tmp_alloc(bo2, n, &o2));
        UTRI_HIP_TRY(hipMemsetAsync(deg, 0, sizeof(int32_t) * n, s));
        if (m > 0) {
            hipLaunchKernelGGL(k_degree, dim3(blocks_for(m)), dim3(TPB), 0, s, g->e_lo, g->e_hi, m, deg);
        }
        unsigned int* dmax = (unsigned int*)(g->d_flags + 1);
        hipLaunchKernelGGL(k_max_i32, dim3(blocks_for(n)), dim3(TPB), 0, s, deg, n, dmax);
        hipLaunchKernelGGL(k_rank_key, dim3(blocks_for(n)), dim3(TPB), 0, s, deg, dk, n);
        hipLaunchKernelGGL(k_iota_u32, dim3(blocks_for(n)), dim3(TPB), 0, s, o1, n);
        UTRI_HIP_TRY(hipGetLastError());
        uint32_t md = 0;
        UTRI_HIP_TRY(hipMemcpyAsync(&md, dmax, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        UTRI_HIP_TRY(hipStreamSynchronize(s));
        g->max_deg = md;
        unsigned dbits = bitlen(md) ? bitlen(md) : 1;
        UTRI_TRY(sort_pairs(g, dk, dk2, o1, o2, n, 32u + dbits, s));
        hipLaunchKernelGGL(k_relabel, dim3(blocks_for(n)), dim3(TPB), 0, s, o2, dk2, n, g->perm,
                           g->inv, g->deg_new);
        UTRI_HIP_TRY(hipGetLastError());
        UTRI_HIP_TRY(hipStreamSynchronize(s));
    }
    // row structures
    UTRI_TRY(dev_alloc(&g->s_off, n + 1));
    UTRI_TRY(dev_alloc(&g->s_adj, 2 * m));
    UTRI_TRY(dev_alloc(&g->s_d, 2 * m));
    UTRI_TRY(dev_alloc(&g->s_eid, 2 * m));
    UTRI_TRY(dev_alloc(&g->s_row, 2 * m));
    UTRI_TRY(dev_alloc(&g->o_off, n + 1));
    UTRI_TRY(dev_alloc(&g->o_adj, m + UTRI_ROW_PAD));
    UTRI_HIP_TRY(hipMemsetAsync(g->o_adj + m, 0, sizeof(int32_t) * UTRI_ROW_PAD, s));
    UTRI_TRY(dev_alloc(&g->o_d, m));
    UTRI_TRY(dev_alloc(&g->o_eid, m));
    UTRI_TRY(dev_alloc(&g->h_off, n + 1));
    // hash table total size: computed on the host from the degree histogram
    {
        std::vector<int32_t> hdeg((size_t)n);
        if (n > 0)
            UTRI_HIP_TRY(hipMemcpy(hdeg.data(), g->deg_new, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
        int64_t tot = 0;
        for (int64_t v = 0; v < n; v++) tot += utri_htable_slots(hdeg[v]);
        g->h_total = tot;
    }
    UTRI_TRY(dev_alloc(&g->h_tab, g->h_total / UTRI_HB * UTRI_HB_WORDS));
    UTRI_TRY(utri_build_rows(g, s));
    // maximum out-degree
    if (n > 0) {
        int32_t* od;
        TmpBuf bod;
        UTRI_TRY(tmp_alloc(bod, n, &od));
        hipLaunchKernelGGL(k_outdeg, dim3(blocks_for(n)), dim3(TPB), 0, s, g->o_off, n, od);
        unsigned int* omax = (unsigned int*)(g->d_flags + 4);
        UTRI_HIP_TRY(hipMemsetAsync(omax, 0, sizeof(uint32_t), s));
        hipLaunchKernelGGL(k_max_i32, dim3(blocks_for(n)), dim3(TPB), 0, s, od, n, omax);
        UTRI_HIP_TRY(hipGetLastError());
        uint32_t mo = 0;
        UTRI_HIP_TRY(hipMemcpyAsync(&mo, omax, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        UTRI_HIP_TRY(hipStreamSynchronize(s));
        g->max_out = mo;
    }
    return UTRI_OK;
}

int utri_load_internal(const int64_t* src, const int64_t* dst, const double* p, int64_t m_in,
                       int64_t n, int ptr_kind, hipStream_t s, utri_graph** out) {
    utri_graph* g = new (std::nothrow) utri_graph();
    if (!g) return UTRI_E_NOMEM;
    int rc = load_impl(src, dst, p, m_in, n, ptr_kind, s, g);
    if (rc != UTRI_OK) {
        (void)hipStreamSynchronize(s);
        free_graph(g);
        return rc;
    }
    *out = g;
    return UTRI_OK;
}

namespace {
__global__ void k_set_p(const double* __restrict__ p, int64_t m, double* __restrict__ ep,
                        double* __restrict__ ed) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    ep[e] = p[e];
    ed[e] = utri_d_of_p(p[e]);
}

__global__ void k_check_p(const double* __restrict__ p, int64_t m, uint32_t* __restrict__ flags) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m && !(p[e] >= 0.0 && p[e] <= 1.0)) atomicOr(flags, UTRI_FLAG_BAD_P);
}
}  // namespace

int utri_set_p_internal(utri_graph* g, const double* p, int ptr_kind, hipStream_t s) {
    const int64_t m = g->m;
    if (m == 0) return UTRI_OK;
    TmpBuf bp;
    const double* dp = p;
    if (ptr_kind == UTRI_HOST_PTR) {
        double* c;
        UTRI_TRY(tmp_alloc(bp, m, &c));
        UTRI_HIP_TRY(hipMemcpyAsync(c, p, sizeof(double) * m, hipMemcpyHostToDevice, s));
        dp = c;
    }
    UTRI_HIP_TRY(hipMemsetAsync(g->d_flags, 0, sizeof(uint32_t), s));
    hipLaunchKernelGGL(k_check_p, dim3(blocks_for(m)), dim3(TPB), 0, s, dp, m, g->d_flags);
    UTRI_HIP_TRY(hipGetLastError());
    uint32_t flags = 0;
    UTRI_HIP_TRY(hipMemcpyAsync(&flags, g->d_flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    UTRI_HIP_TRY(hipStreamSynchronize(s));
    if (flags) return UTRI_E_INVALID;
    hipLaunchKernelGGL(k_set_p, dim3(blocks_for(m)), dim3(TPB), 0, s, dp, m, g->e_p, g->e_d);
    UTRI_HIP_TRY(hipGetLastError());
    return utri_build_rows(g, s);
}
