// cg_kernels.hip -- direct-stiffness summation with masking, deterministic
// reductions and the vector steps of unpreconditioned CG (Sec. III, Sec. V,
// Sec. VI-B), all on the device.
//
// Reductions: every kernel reduces a fixed grid of RED_BLOCKS workgroups
// (wavefront shuffles, then LDS), writes one partial per workgroup, and the
// last workgroup to finish (ticket counter) sums the partials in index order
// and updates the CG scalars in device memory.  The order of every sum is
// fixed by the grid, so results are bitwise reproducible from run to run.
#include "nek_internal.h"

namespace nek {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// sum over the workgroup (RED_THREADS threads); result valid in thread 0
__device__ __forceinline__ double block_sum(double v, double *lds) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < RED_THREADS / 64; ++q) s += lds[q];
    }
    __syncthreads();
    return s;
}

__device__ __forceinline__ double load_coherent(const double *p) {
    unsigned long long bits =
        __hip_atomic_load((const unsigned long long *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double((long long)bits);
}

// Publish this workgroup's partial; returns true (in every thread) for the
// last workgroup, which then holds the ordered total in thread 0 via *total.
__device__ bool finish_partials(double s, double *partials, unsigned int *ticket,
                                double *total, double *lds) {
    __shared__ int last;
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = s;
        __threadfence();
        unsigned int t = atomicAdd(ticket, 1u);
        last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!last) return false;
    __threadfence();
    double v = 0.0;
    for (unsigned int q = threadIdx.x; q < gridDim.x; q += blockDim.x) v += load_coherent(&partials[q]);
    v = block_sum(v, lds);
    if (threadIdx.x == 0) {
        *total = v;
        *ticket = 0u;   // ready for the next launch
    }
    return true;
}

// ---------------------------------------------------------------- dssum + mask
__global__ void gs_kernel(int64_t n_rows, const int32_t *__restrict__ off,
                          const int32_t *__restrict__ idx, const uint8_t *__restrict__ keep,
                          double *__restrict__ w, const int *__restrict__ done) {
    if (done != nullptr && *done) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < n_rows; row += stride) {
        const int32_t o0 = off[row], o1 = off[row + 1];
        double s = 0.0;
        for (int32_t o = o0; o < o1; ++o) s += w[idx[o]];
        if (!keep[row]) s = 0.0;
        for (int32_t o = o0; o < o1; ++o) w[idx[o]] = s;
    }
}

// ---------------------------------------------------------------- CG steps
__global__ void cg_reset_kernel(CgScalars *sc, int max_iter, double rel_tol, double drop) {
    sc->bb = 0.0;
    sc->rho = 0.0;
    sc->pw = 0.0;
    sc->alpha = 0.0;
    sc->beta = 0.0;
    sc->rel_tol2 = rel_tol > 0.0 ? rel_tol * rel_tol : 0.0;   // scaled by bb in init
    sc->rho_last_true = 0.0;
    sc->drop2 = drop * drop;
    sc->it = 0;
    sc->max_iter = max_iter;
    sc->done = 0;
    sc->status = NEK_OK;
    sc->need_replace = 0;
    sc->n_replace = 0;
    for (int q = 0; q < 4; ++q) sc->ticket[q] = 0u;
}

// x = 0, r = b, p = b, rho = (b, b)
__global__ void __launch_bounds__(RED_THREADS)
cg_init_kernel(int64_t P, const double *__restrict__ b, double *__restrict__ x,
               double *__restrict__ r, double *__restrict__ p, const uint8_t *__restrict__ own,
               double *partials, CgScalars *sc) {
    __shared__ double lds[RED_THREADS / 64];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < P; t += stride) {
        const double bv = b[t];
        x[t] = 0.0;
        r[t] = bv;
        p[t] = bv;
        if (own[t]) acc += bv * bv;
    }
    double s = block_sum(acc, lds);
    double tot;
    if (finish_partials(s, partials, &sc->ticket[0], &tot, lds) && threadIdx.x == 0) {
        sc->bb = tot;
        sc->rho = tot;
        sc->rho_last_true = tot;
        sc->rel_tol2 = sc->rel_tol2 * tot;
        if (!(tot > 0.0)) {           // b = 0 (x = 0 is the solution) or non-finite
            sc->done = 1;
            if (!__builtin_isfinite(tot)) sc->status = NEK_ERR_BREAKDOWN;
        }
        if (sc->max_iter <= 0) sc->done = 1;
    }
}

// pw = (p, w); alpha = rho / pw
__global__ void __launch_bounds__(RED_THREADS)
cg_dot_pw_kernel(int64_t P, const double *__restrict__ p, const double *__restrict__ w,
                 const uint8_t *__restrict__ own, double *partials, CgScalars *sc) {
    if (sc->done) return;
    __shared__ double lds[RED_THREADS / 64];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < P; t += stride)
        if (own[t]) acc += p[t] * w[t];
    double s = block_sum(acc, lds);
    double tot;
    if (finish_partials(s, partials, &sc->ticket[1], &tot, lds) && threadIdx.x == 0) {
        sc->pw = tot;
        if (!(tot > 0.0) || !__builtin_isfinite(tot)) {
            sc->status = NEK_ERR_BREAKDOWN;
            sc->done = 1;
        } else {
            sc->alpha = sc->rho / tot;
        }
    }
}

// x += alpha p; r -= alpha w; rho' = (r, r); beta = rho'/rho
__global__ void __launch_bounds__(RED_THREADS)
cg_update_kernel(int64_t P, double *__restrict__ x, double *__restrict__ r,
                 const double *__restrict__ p, const double *__restrict__ w,
                 const uint8_t *__restrict__ own, double *partials, CgScalars *sc) {
    if (sc->done) return;
    __shared__ double lds[RED_THREADS / 64];
    const double alpha = sc->alpha;
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < P; t += stride) {
        x[t] = x[t] + alpha * p[t];
        const double rv = r[t] - alpha * w[t];
        r[t] = rv;
        if (own[t]) acc += rv * rv;
    }
    double s = block_sum(acc, lds);
    double tot;
    if (finish_partials(s, partials, &sc->ticket[2], &tot, lds) && threadIdx.x == 0) {
        sc->it += 1;
        if (!__builtin_isfinite(tot)) {
            sc->status = NEK_ERR_BREAKDOWN;
            sc->done = 1;
        } else {
            sc->beta = tot / sc->rho;
            sc->rho = tot;
            if (sc->rel_tol2 > 0.0 && tot <= sc->rel_tol2) {
                if (sc->drop2 > 0.0) sc->need_replace = 1;   // mixed: confirm with the true residual
                else sc->done = 1;
            }
            if (sc->drop2 > 0.0 && tot <= sc->drop2 * sc->rho_last_true) sc->need_replace = 1;
            if (tot == 0.0) sc->done = 1;
            if (sc->it >= sc->max_iter) sc->done = 1;
        }
    }
}

// reliable update: r = b - w (w = mask(dssum(A64 x))), rho = (r, r)
__global__ void __launch_bounds__(RED_THREADS)
cg_replace_kernel(int64_t P, const double *__restrict__ b, const double *__restrict__ w,
                  double *__restrict__ r, const uint8_t *__restrict__ own, double *partials,
                  CgScalars *sc) {
    __shared__ double lds[RED_THREADS / 64];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < P; t += stride) {
        const double rv = b[t] - w[t];
        r[t] = rv;
        if (own[t]) acc += rv * rv;
    }
    double s = block_sum(acc, lds);
    double tot;
    if (finish_partials(s, partials, &sc->ticket[3], &tot, lds) && threadIdx.x == 0) {
        sc->rho = tot;
        sc->rho_last_true = tot;
        sc->need_replace = 0;
        sc->n_replace += 1;
        if (!__builtin_isfinite(tot)) {
            sc->status = NEK_ERR_BREAKDOWN;
            sc->done = 1;
        } else if (sc->rel_tol2 > 0.0 && tot <= sc->rel_tol2) {
            sc->done = 1;
        }
    }
}

__global__ void __launch_bounds__(RED_THREADS)
gdot_kernel(int64_t P, const double *__restrict__ a, const double *__restrict__ b,
            const uint8_t *__restrict__ own, double *partials, unsigned int *ticket,
            double *result) {
    __shared__ double lds[RED_THREADS / 64];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < P; t += stride)
        if (own[t]) acc += a[t] * b[t];
    double s = block_sum(acc, lds);
    double tot;
    if (finish_partials(s, partials, ticket, &tot, lds) && threadIdx.x == 0) *result = tot;
}

__global__ void __launch_bounds__(RED_THREADS)
gdiff2_kernel(int64_t P, const double *__restrict__ a, const double *__restrict__ b,
              const uint8_t *__restrict__ own, double *partials, unsigned int *ticket,
              double *result) {
    __shared__ double lds[RED_THREADS / 64];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < P; t += stride)
        if (own[t]) {
            const double d = a[t] - b[t];
            acc += d * d;
        }
    double s = block_sum(acc, lds);
    double tot;
    if (finish_partials(s, partials, ticket, &tot, lds) && threadIdx.x == 0) *result = tot;
}

}  // namespace

hipError_t launch_gdiff2(int64_t P, const double *a, const double *b, const uint8_t *own,
                         double *partials, unsigned int *ticket, double *result, hipStream_t s) {
    hipLaunchKernelGGL(gdiff2_kernel, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, P, a, b, own,
                       partials, ticket, result);
    return hipGetLastError();
}

hipError_t launch_gs(const GsDevice &gs, double *w, const int *done, hipStream_t s) {
    if (gs.n_rows == 0) return hipSuccess;
    int64_t blocks = (gs.n_rows + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(gs_kernel, dim3((unsigned)blocks), dim3(256), 0, s, gs.n_rows, gs.row_off,
                       gs.row_idx, gs.row_keep, w, done);
    return hipGetLastError();
}

hipError_t launch_cg_reset(CgScalars *sc, int max_iter, double rel_tol, double drop, hipStream_t s) {
    hipLaunchKernelGGL(cg_reset_kernel, dim3(1), dim3(1), 0, s, sc, max_iter, rel_tol, drop);
    return hipGetLastError();
}

hipError_t launch_cg_init(int64_t P, const double *b, double *x, double *r, double *p,
                          const uint8_t *own, double *partials, CgScalars *sc, hipStream_t s) {
    hipLaunchKernelGGL(cg_init_kernel, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, P, b, x, r, p,
                       own, partials, sc);
    return hipGetLastError();
}

hipError_t launch_cg_dot_pw(int64_t P, const double *p, const double *w, const uint8_t *own,
                            double *partials, CgScalars *sc, hipStream_t s) {
    hipLaunchKernelGGL(cg_dot_pw_kernel, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, P, p, w, own,
                       partials, sc);
    return hipGetLastError();
}

hipError_t launch_cg_update(int64_t P, double *x, double *r, const double *p, const double *w,
                            const uint8_t *own, double *partials, CgScalars *sc, hipStream_t s) {
    hipLaunchKernelGGL(cg_update_kernel, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, P, x, r, p, w,
                       own, partials, sc);
    return hipGetLastError();
}

hipError_t launch_cg_replace(int64_t P, const double *b, const double *w, double *r,
                             const uint8_t *own, double *partials, CgScalars *sc, hipStream_t s) {
    hipLaunchKernelGGL(cg_replace_kernel, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, P, b, w, r,
                       own, partials, sc);
    return hipGetLastError();
}

hipError_t launch_gdot(int64_t P, const double *a, const double *b, const uint8_t *own,
                       double *partials, unsigned int *ticket, double *result, hipStream_t s) {
    hipLaunchKernelGGL(gdot_kernel, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, P, a, b, own,
                       partials, ticket, result);
    return hipGetLastError();
}

}  // namespace nek
