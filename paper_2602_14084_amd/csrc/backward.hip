// backward.hip -- per-edge gradient of the expected balanced count.
//
// E = sum over triangles of P_bal = (1 - d_e d_f d_g)/2 (Section 3 four-term sum in
// product form, d = 1 - 2 P+). With dd_e/dp_e = -2, dE/dp_e = sum over the triangles
// (e, f, g) through e of d_f * d_g. Edge-centric re-walk: every edge is owned by one
// lane of one wave; its triangles are found by streaming the shorter endpoint row and
// probing the longer row's hash table (cost sum_e min(deg), no merge of hub rows).
// Each product d_f * d_g is rounded to FP64 and added exactly in 2^-62 fixed point
// (LDS integer accumulators of the owning wave), then rounded once: the result does
// not depend on which lane found which triangle, and no global atomics are used.
#include <algorithm>

#include "walk_common.h"

using namespace utri_dev;

namespace {

struct GradLds {
    int32_t end[UTRI_WAVE];
    int64_t xoff[UTRI_WAVE];
    int64_t yoff[UTRI_WAVE];
    int64_t hoff[UTRI_WAVE];
    int32_t hlg[UTRI_WAVE];
    unsigned long long acc_lo[UTRI_WAVE];  // sum of the low 32 bits of each term
    unsigned long long acc_hi[UTRI_WAVE];  // sum of (term >> 32), two's complement
};

__global__ void __launch_bounds__(TPB) k_grad(SampleGraph G, double* __restrict__ grad) {
    __shared__ GradLds lds[WPB];
    const int wib = threadIdx.x / UTRI_WAVE;
    const int lane = utri_lane();
    GradLds& L = lds[wib];
    const int64_t gw = (int64_t)blockIdx.x * WPB + wib;
    const int64_t W = (int64_t)gridDim.x * WPB;
    const int64_t nbatch = (G.m + UTRI_WAVE - 1) / UTRI_WAVE;
    for (int64_t bt = gw; bt < nbatch; bt += W) {
        const int64_t e = bt * UTRI_WAVE + lane;
        int work = 0;
        int64_t xoff = 0, yoff = 0, hoff = 0;
        int lg = 0;
        if (e < G.m) {
            const int32_t a = G.inv[G.e_lo[e]], b = G.inv[G.e_hi[e]];
            const int64_t la = G.s_off[a + 1] - G.s_off[a], lb = G.s_off[b + 1] - G.s_off[b];
            const bool ax = (la < lb) || (la == lb && a < b);
            const int32_t x = ax ? a : b, y = ax ? b : a;
            work = (int)(ax ? la : lb);
            xoff = G.s_off[x];
            yoff = G.s_off[y];
            hoff = G.h_off[y];
            lg = log2_size(G.h_off[y + 1] - hoff);
        }
        const int incl = (int)utri_wave_incl_scan((int64_t)work);
        const int total = __shfl(incl, UTRI_WAVE - 1, UTRI_WAVE);
        L.end[lane] = incl;
        L.xoff[lane] = xoff;
        L.yoff[lane] = yoff;
        L.hoff[lane] = hoff;
        L.hlg[lane] = lg;
        L.acc_lo[lane] = 0;
        L.acc_hi[lane] = 0;
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
                    const double prod = __dmul_rn(G.s_d[px], G.s_d[L.yoff[sg] + py]);
                    const int64_t t = utri_fix62(prod);
                    atomicAdd(&L.acc_lo[sg], (unsigned long long)(uint32_t)(t & 0xFFFFFFFFll));
                    atomicAdd(&L.acc_hi[sg], (unsigned long long)(t >> 32));
                }
            }
        }
        utri_wave_sync();
        if (e < G.m) {
            // value = acc_hi * 2^32 + acc_lo as a 128-bit integer
            const int64_t h = (int64_t)L.acc_hi[lane];
            uint64_t lo = (uint64_t)h << 32;
            uint64_t hi = (uint64_t)(h >> 32);
            const uint64_t s2 = lo + (uint64_t)L.acc_lo[lane];
            hi += (s2 < lo) ? 1ull : 0ull;
            lo = s2;
            grad[e] = utri_i128_to_double((int64_t)hi, lo) * 0x1p-62;
        }
        utri_wave_sync();
    }
}

}  // namespace

int utri_grad_launch(utri_graph* g, double* grad, hipStream_t s) {
    if (g->m == 0) return UTRI_OK;
    SampleGraph G{g->m, g->e_lo, g->e_hi, g->e_d, g->inv, g->s_off, g->s_adj, g->s_d, g->h_off,
                  g->h_slot};
    const int64_t nbatch = (g->m + UTRI_WAVE - 1) / UTRI_WAVE;
    const int blocks = (int)std::min<int64_t>((int64_t)g->num_cu * 16, (nbatch + WPB - 1) / WPB);
    hipLaunchKernelGGL(k_grad, dim3(blocks), dim3(TPB), 0, s, G, grad);
    UTRI_HIP_TRY(hipGetLastError());
    return UTRI_OK;
}
