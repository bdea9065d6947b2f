// probe_kernels.hip -- HBM bandwidth probes for the measured roofline.
//
// Sec. V measures the bandwidth a CG iteration could reach by replacing its
// computation with device copies of every load and store.  The probes here do
// the same with one streaming kernel: dst[i] = sum over k < nread of
// src[k*n + i], i.e. nread coalesced read streams and one write stream of n
// doubles each.  nread = 1 is a copy; nread = 7 has the 7:1 read:write byte
// mix of the FP64 local operator (u and six geometric factors in, w out).
// With NT the loads and stores carry the non-temporal (streaming) hint, as the
// plain FP64 operator's do.
#include "nek_internal.h"

namespace nek {
namespace {

constexpr int PROBE_THREADS = 256;
constexpr int PROBE_PAIRS = 4;

typedef double dvec2 __attribute__((ext_vector_type(2)));

template <int R, bool NT>
__global__ void __launch_bounds__(PROBE_THREADS)
probe_kernel(int64_t n, const double *__restrict__ src, double *__restrict__ dst) {
    const int64_t npairs = n >> 1;
    const int64_t chunk = (int64_t)PROBE_THREADS * PROBE_PAIRS;
    for (int64_t base = blockIdx.x * chunk; base < npairs; base += (int64_t)gridDim.x * chunk) {
        dvec2 acc[PROBE_PAIRS];
#pragma unroll
        for (int m = 0; m < PROBE_PAIRS; ++m) acc[m] = dvec2{0.0, 0.0};
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const dvec2 *s2 = (const dvec2 *)(src + (int64_t)k * n);
#pragma unroll
            for (int m = 0; m < PROBE_PAIRS; ++m) {
                const int64_t q = base + threadIdx.x + (int64_t)m * PROBE_THREADS;
                if (q < npairs) acc[m] += NT ? __builtin_nontemporal_load(&s2[q]) : s2[q];
            }
        }
#pragma unroll
        for (int m = 0; m < PROBE_PAIRS; ++m) {
            const int64_t q = base + threadIdx.x + (int64_t)m * PROBE_THREADS;
            if (q < npairs) {
                if (NT) __builtin_nontemporal_store(acc[m], &((dvec2 *)dst)[q]);
                else ((dvec2 *)dst)[q] = acc[m];
            }
        }
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        double a = 0.0;
        for (int k = 0; k < R; ++k) a += src[(int64_t)k * n + n - 1];
        dst[n - 1] = a;
    }
}

}  // namespace

hipError_t launch_probe(int64_t n, int nread, const double *src, double *dst, int grid, bool streaming,
                        hipStream_t s) {
    const int64_t per = (int64_t)PROBE_THREADS * PROBE_PAIRS * 2;
    int64_t blocks = (n + per - 1) / per;
    if (grid > 0 && blocks > grid) blocks = grid;
    if (blocks < 1) blocks = 1;
    switch (nread) {
#define NEK_PROBE(R)                                                                                   \
    case R:                                                                                            \
        if (streaming)                                                                                 \
            hipLaunchKernelGGL((probe_kernel<R, true>), dim3((unsigned)blocks), dim3(PROBE_THREADS), 0, s, n, src, dst); \
        else                                                                                           \
            hipLaunchKernelGGL((probe_kernel<R, false>), dim3((unsigned)blocks), dim3(PROBE_THREADS), 0, s, n, src, dst); \
        break;
        NEK_PROBE(1) NEK_PROBE(2) NEK_PROBE(3) NEK_PROBE(4) NEK_PROBE(5) NEK_PROBE(6) NEK_PROBE(7)
        NEK_PROBE(8)
#undef NEK_PROBE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace nek
