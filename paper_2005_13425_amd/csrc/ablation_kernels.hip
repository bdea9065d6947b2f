// ablation_kernels.hip -- the three earlier GPU designs of the local operator
// that Sec. IV of the paper describes, written for gfx950 to measure them next
// to the pencil kernel of ax_kernels.hip.  All compute Listing 1 in FP64 with
// the layouts of nek.h; none is used by the solver.
//
//   ORIGINAL (Sec. IV-A): one workgroup per element, threads striding over its
//     points, every operand in global memory.  The intermediate ur, us, ut go
//     to a global scratch of 3 n^3 doubles per element, as Listing 1's local
//     arrays did.
//   SHARED3D (Sec. IV-B): one thread per node (n^3 threads per workgroup), the
//     element's u, the three intermediates and D in LDS.  A workgroup holds at
//     most 1024 threads, so n <= 10 (the paper's limit on its GPU too).
//   LAYER2D (Sec. IV-C, the paper's own design): one thread per (i, j) column,
//     the workgroup marching through the k layers together; the thread keeps
//     its u and w columns in registers, the layer of u and the layers of ur and
//     us pass through LDS, two barriers per layer.
#include "nek_internal.h"

namespace nek {
namespace {

constexpr int ORIG_THREADS = 256;

template <int NX>
__global__ void __launch_bounds__(ORIG_THREADS)
ax_original_kernel(const double *__restrict__ D, const double *__restrict__ g,
                   const double *__restrict__ u, double *__restrict__ w, double *__restrict__ scratch) {
    constexpr int NN = NX * NX, N3 = NN * NX;
    const int64_t e = blockIdx.x;
    const gptr<const double> ue = (gptr<const double>)u + e * N3;
    const gptr<const double> ge = (gptr<const double>)g + e * 6 * N3;
    const gptr<double> we = (gptr<double>)w + e * N3;
    const gptr<double> ur = (gptr<double>)scratch + e * 3 * N3;
    const gptr<double> us = ur + N3, ut = us + N3;
    const gptr<const double> Dg = (gptr<const double>)D;
    for (int p = threadIdx.x; p < N3; p += ORIG_THREADS) {
        const int i = p % NX, j = (p / NX) % NX, k = p / NN;
        double wr = 0.0, ws = 0.0, wt = 0.0;
        for (int l = 0; l < NX; ++l) {
            wr += Dg[i + NX * l] * ue[l + NX * j + NN * k];
            ws += Dg[j + NX * l] * ue[i + NX * l + NN * k];
            wt += Dg[k + NX * l] * ue[i + NX * j + NN * l];
        }
        const double g1 = ge[p], g2 = ge[N3 + p], g3 = ge[2 * N3 + p];
        const double g4 = ge[3 * N3 + p], g5 = ge[4 * N3 + p], g6 = ge[5 * N3 + p];
        ur[p] = g1 * wr + g2 * ws + g3 * wt;
        us[p] = g2 * wr + g4 * ws + g5 * wt;
        ut[p] = g3 * wr + g5 * ws + g6 * wt;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < N3; p += ORIG_THREADS) {
        const int i = p % NX, j = (p / NX) % NX, k = p / NN;
        double s = 0.0;
        for (int l = 0; l < NX; ++l)
            s += Dg[l + NX * i] * ur[l + NX * j + NN * k] + Dg[l + NX * j] * us[i + NX * l + NN * k] +
                 Dg[l + NX * k] * ut[i + NX * j + NN * l];
        we[p] = s;
    }
}

template <int NX>
__global__ void __launch_bounds__(1024)
ax_shared3d_kernel(const double *__restrict__ D, const double *__restrict__ g,
                   const double *__restrict__ u, double *__restrict__ w) {
    constexpr int NN = NX * NX, N3 = NN * NX;
    __shared__ double su[N3], sr[N3], ss[N3], st[N3], sD[NN];
    const int64_t e = blockIdx.x;
    const int p = threadIdx.x;
    const bool on = p < N3;
    const int i = p % NX, j = (p / NX) % NX, k = p / NN;
    if (on) su[p] = ((gptr<const double>)u)[e * N3 + p];
    if (p < NN) sD[p] = ((gptr<const double>)D)[p];
    __syncthreads();
    if (on) {
        double wr = 0.0, ws = 0.0, wt = 0.0;
#pragma unroll
        for (int l = 0; l < NX; ++l) {
            wr += sD[i + NX * l] * su[l + NX * j + NN * k];
            ws += sD[j + NX * l] * su[i + NX * l + NN * k];
            wt += sD[k + NX * l] * su[i + NX * j + NN * l];
        }
        const gptr<const double> ge = (gptr<const double>)g + e * 6 * N3 + p;
        const double g1 = ge[0], g2 = ge[N3], g3 = ge[2 * N3], g4 = ge[3 * N3], g5 = ge[4 * N3], g6 = ge[5 * N3];
        sr[p] = g1 * wr + g2 * ws + g3 * wt;
        ss[p] = g2 * wr + g4 * ws + g5 * wt;
        st[p] = g3 * wr + g5 * ws + g6 * wt;
    }
    __syncthreads();
    if (on) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < NX; ++l)
            s += sD[l + NX * i] * sr[l + NX * j + NN * k] + sD[l + NX * j] * ss[i + NX * l + NN * k] +
                 sD[l + NX * k] * st[i + NX * j + NN * l];
        ((gptr<double>)w)[e * N3 + p] = s;
    }
}

constexpr int round64(int x) { return (x + 63) / 64 * 64; }

template <int NX>
__global__ void __launch_bounds__(round64(NX * NX))
ax_layer2d_kernel(const double *__restrict__ D, const double *__restrict__ g,
                  const double *__restrict__ u, double *__restrict__ w) {
    constexpr int NN = NX * NX, N3 = NN * NX;
    __shared__ double slab_u[NN], slab_r[NN], slab_s[NN], sD[NN];
    const int64_t e = blockIdx.x;
    const int t = threadIdx.x;
    const bool on = t < NN;
    const int i = t % NX, j = t / NX;
    const gptr<const double> ue = (gptr<const double>)u + e * N3;
    const gptr<const double> ge = (gptr<const double>)g + e * 6 * N3;
    double ucol[NX], wcol[NX];
#pragma unroll
    for (int k = 0; k < NX; ++k) {
        ucol[k] = on ? ue[t + NN * k] : 0.0;
        wcol[k] = 0.0;
    }
    if (on) sD[t] = ((gptr<const double>)D)[t];
#pragma unroll 1
    for (int k = 0; k < NX; ++k) {
        if (on) slab_u[t] = ucol[k];
        __syncthreads();   // layer k of u (and D) visible; last layer's ur, us read
        double ut = 0.0;
        if (on) {
            double wr = 0.0, ws = 0.0, wt = 0.0;
#pragma unroll
            for (int l = 0; l < NX; ++l) {
                wr += sD[i + NX * l] * slab_u[l + NX * j];
                ws += sD[j + NX * l] * slab_u[i + NX * l];
                wt += sD[k + NX * l] * ucol[l];
            }
            const int p = t + NN * k;
            const double g1 = ge[p], g2 = ge[N3 + p], g3 = ge[2 * N3 + p];
            const double g4 = ge[3 * N3 + p], g5 = ge[4 * N3 + p], g6 = ge[5 * N3 + p];
            slab_r[t] = g1 * wr + g2 * ws + g3 * wt;
            slab_s[t] = g2 * wr + g4 * ws + g5 * wt;
            ut = g3 * wr + g5 * ws + g6 * wt;
        }
        __syncthreads();   // layers of ur and us visible; layer k of u read
        if (on) {
            double s = 0.0;
#pragma unroll
            for (int l = 0; l < NX; ++l) s += sD[l + NX * i] * slab_r[l + NX * j] + sD[l + NX * j] * slab_s[i + NX * l];
            wcol[k] += s;
            // the t part of layer k reaches every layer m of the column
#pragma unroll
            for (int m = 0; m < NX; ++m) wcol[m] += sD[k + NX * m] * ut;
        }
    }
    if (on) {
        const gptr<double> we = (gptr<double>)w + e * N3;
#pragma unroll
        for (int k = 0; k < NX; ++k) we[t + NN * k] = wcol[k];
    }
}

template <int NX>
hipError_t launch_variant(int variant, int64_t E, const double *D, const double *g, const double *u, double *w,
                          double *scratch, hipStream_t s) {
    constexpr int NN = NX * NX;
    const dim3 grid((unsigned)E);
    switch (variant) {
    case NEK_AX_ORIGINAL:
        hipLaunchKernelGGL(ax_original_kernel<NX>, grid, dim3(ORIG_THREADS), 0, s, D, g, u, w, scratch);
        break;
    case NEK_AX_SHARED3D:
        if constexpr (NN * NX <= 1024)
            hipLaunchKernelGGL(ax_shared3d_kernel<NX>, grid, dim3(round64(NN * NX)), 0, s, D, g, u, w);
        else
            return hipErrorInvalidValue;
        break;
    case NEK_AX_LAYER2D:
        hipLaunchKernelGGL(ax_layer2d_kernel<NX>, grid, dim3(round64(NN)), 0, s, D, g, u, w);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_ax_variant(int variant, int64_t E, int N, const double *D, const double *g, const double *u,
                             double *w, double *scratch, hipStream_t s) {
    if (E < 1 || E > 0x7fffffff) return hipErrorInvalidValue;
    switch (N + 1) {
#define NEK_CASE(NX) \
    case NX: return launch_variant<NX>(variant, E, D, g, u, w, scratch, s);
        NEK_CASE(2) NEK_CASE(3) NEK_CASE(4) NEK_CASE(5) NEK_CASE(6) NEK_CASE(7) NEK_CASE(8)
        NEK_CASE(9) NEK_CASE(10) NEK_CASE(11) NEK_CASE(12) NEK_CASE(13) NEK_CASE(14)
        NEK_CASE(15) NEK_CASE(16)
#undef NEK_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace nek
