// scan.hip -- exclusive prefix sums used by every query (row lengths -> work items,
// per-item counts -> output offsets). Three plain kernels (block sums, a one-block scan
// of the block sums, block-local scans plus offsets) and no memset, so the sequence can
// be recorded into a hipGraph and replayed.
#include "utri_internal.h"

namespace {

constexpr int STPB = 256;
constexpr int PER_THREAD = 4;
constexpr int PER_BLOCK = STPB * PER_THREAD;

template <class T>
__device__ inline int64_t load_as_i64(const T* p, int64_t i, int64_t n) {
    return i < n ? (int64_t)p[i] : 0;
}

// block-wide exclusive scan of one int64 per thread; returns the block total
__device__ inline int64_t block_excl_scan(int64_t v, int64_t* sh, int64_t& excl) {
    const int lane = threadIdx.x & (UTRI_WAVE - 1);
    const int wv = threadIdx.x / UTRI_WAVE;
    const int64_t incl = utri_wave_incl_scan(v);
    if (lane == UTRI_WAVE - 1) sh[wv] = incl;
    __syncthreads();
    int64_t wbase = 0, tot = 0;
    for (int q = 0; q < STPB / UTRI_WAVE; q++) {
        if (q < wv) wbase += sh[q];
        tot += sh[q];
    }
    __syncthreads();
    excl = wbase + incl - v;
    return tot;
}

template <class T>
__global__ void __launch_bounds__(STPB) k_block_sums(const T* __restrict__ in, int64_t n,
                                                     int64_t* __restrict__ bsum) {
    __shared__ int64_t sh[STPB / UTRI_WAVE];
    const int64_t base = (int64_t)blockIdx.x * PER_BLOCK + (int64_t)threadIdx.x * PER_THREAD;
    int64_t v = 0;
#pragma unroll
    for (int q = 0; q < PER_THREAD; q++) v += load_as_i64(in, base + q, n);
    int64_t excl;
    const int64_t tot = block_excl_scan(v, sh, excl);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(STPB) k_scan_sums(int64_t* __restrict__ bsum, int64_t nb,
                                                    int64_t* __restrict__ total) {
    __shared__ int64_t sh[STPB / UTRI_WAVE];
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += STPB) {
        const int64_t i = b0 + threadIdx.x;
        const int64_t v = i < nb ? bsum[i] : 0;
        int64_t excl;
        const int64_t tot = block_excl_scan(v, sh, excl);
        if (i < nb) bsum[i] = carry + excl;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

template <class T>
__global__ void __launch_bounds__(STPB) k_block_scan(const T* __restrict__ in, int64_t n,
                                                     const int64_t* __restrict__ boff,
                                                     int64_t* __restrict__ out) {
    __shared__ int64_t sh[STPB / UTRI_WAVE];
    const int64_t base = (int64_t)blockIdx.x * PER_BLOCK + (int64_t)threadIdx.x * PER_THREAD;
    int64_t vals[PER_THREAD];
    int64_t v = 0;
#pragma unroll
    for (int q = 0; q < PER_THREAD; q++) {
        vals[q] = load_as_i64(in, base + q, n);
        v += vals[q];
    }
    int64_t excl;
    (void)block_excl_scan(v, sh, excl);
    int64_t run = boff[blockIdx.x] + excl;
#pragma unroll
    for (int q = 0; q < PER_THREAD; q++) {
        if (base + q < n) out[base + q] = run;
        run += vals[q];
    }
}

template <class T>
int scan_impl(utri_graph* g, const T* in, int64_t* out, int64_t n, int64_t* total,
              hipStream_t s) {
    if (n <= 0) return UTRI_OK;
    const int64_t nb = (n + PER_BLOCK - 1) / PER_BLOCK;
    void* tmp;
    UTRI_TRY(utri_scratch(g, SCR_TEMP, sizeof(int64_t) * (size_t)(nb + 1), &tmp));
    int64_t* bsum = (int64_t*)tmp;
    hipLaunchKernelGGL(k_block_sums<T>, dim3((unsigned)nb), dim3(STPB), 0, s, in, n, bsum);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(STPB), 0, s, bsum, nb, total);
    hipLaunchKernelGGL(k_block_scan<T>, dim3((unsigned)nb), dim3(STPB), 0, s, in, n,
                       (const int64_t*)bsum, out);
    UTRI_HIP_TRY(hipGetLastError());
    return UTRI_OK;
}

}  // namespace

// out[i] = sum of in[0..i); *total (device, optional) = sum of all n values
int utri_scan_i32(utri_graph* g, const int32_t* in, int64_t* out, int64_t n, int64_t* total,
                  hipStream_t s) {
    return scan_impl<int32_t>(g, in, out, n, total, s);
}

int utri_scan_i64(utri_graph* g, const int64_t* in, int64_t* out, int64_t n, int64_t* total,
                  hipStream_t s) {
    return scan_impl<int64_t>(g, in, out, n, total, s);
}
