// jacobi_kernels.hip -- setup of the Jacobi preconditioner: the diagonal of
// the element operator of Listing 1 at every local point, and an in-place
// reciprocal.
//
// A_e u = D^T G D u with the reference gradient of basis function p = (i,j,k)
// nonzero only on the three grid lines through p, so
//   (A_e)_pp = sum_m [ D(m,i)^2 g_rr(m,j,k) + D(m,j)^2 g_ss(i,m,k) + D(m,k)^2 g_tt(i,j,m) ]
//            + 2 D(i,i) D(j,j) g_rs(p) + 2 D(i,i) D(k,k) g_rt(p) + 2 D(j,j) D(k,k) g_st(p),
// D(a,b) = dxm1(a,b) = D[a + n b].  One thread per local point; a setup
// kernel, run once per mesh, so it favours plainness over speed.
#include "nek_internal.h"

namespace nek {
namespace {

__global__ void __launch_bounds__(256)
ax_diag_kernel(int64_t E, int n, const double *__restrict__ D, const double *__restrict__ g,
               double *__restrict__ d) {
    const int64_t n3 = (int64_t)n * n * n;
    const int64_t P = E * n3;
    for (int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; L < P;
         L += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = L / n3;
        const int pt = (int)(L - e * n3);
        const int i = pt % n, j = (pt / n) % n, k = pt / (n * n);
        const double *grr = g + 6 * n3 * e;
        const double *grs = grr + n3, *grt = grr + 2 * n3, *gss = grr + 3 * n3;
        const double *gst = grr + 4 * n3, *gtt = grr + 5 * n3;
        double s = 0.0;
        for (int m = 0; m < n; ++m) {
            const double dri = D[m + n * i], dsj = D[m + n * j], dtk = D[m + n * k];
            s += dri * dri * grr[m + n * (j + n * k)];
            s += dsj * dsj * gss[i + n * (m + n * k)];
            s += dtk * dtk * gtt[i + n * (j + n * m)];
        }
        const double di = D[i + n * i], dj = D[j + n * j], dk = D[k + n * k];
        s += 2.0 * (di * dj * grs[pt] + di * dk * grt[pt] + dj * dk * gst[pt]);
        d[L] = s;
    }
}

__global__ void __launch_bounds__(256) reciprocal_kernel(int64_t P, double *__restrict__ v) {
    for (int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; L < P;
         L += (int64_t)gridDim.x * blockDim.x) {
        const double x = v[L];
        v[L] = x != 0.0 ? 1.0 / x : 0.0;
    }
}

int64_t setup_blocks(int64_t P) {
    const int64_t b = (P + 255) / 256;
    return b < 1 ? 1 : (b > 65536 ? 65536 : b);
}

}  // namespace

hipError_t launch_ax_diag(int64_t E, int N, const double *D, const double *g, double *d, hipStream_t s) {
    const int64_t P = E * n3_of(N);
    hipLaunchKernelGGL(ax_diag_kernel, dim3((unsigned)setup_blocks(P)), dim3(256), 0, s, E, N + 1, D, g, d);
    return hipGetLastError();
}

hipError_t launch_reciprocal(int64_t P, double *v, hipStream_t s) {
    hipLaunchKernelGGL(reciprocal_kernel, dim3((unsigned)setup_blocks(P)), dim3(256), 0, s, P, v);
    return hipGetLastError();
}

}  // namespace nek
