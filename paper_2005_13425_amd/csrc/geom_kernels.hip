// geom_kernels.hip -- synthetic box-mesh geometry on the device: nodal
// coordinates, geometric factors gxyz of Listing 1 and the diagonal mass.
//
// Mesh: Ex x Ey x Ez hexahedra on the unit cube, element e = ex + Ex(ey + Ey ez),
// nodes at the tensor GLL points, displaced by amp * a_d * sin(pi x) sin(pi y)
// sin(pi z) (zero on the boundary).  The Jacobian at a node is the derivative
// matrix applied to the nodal coordinates along r, s and t (isoparametric).
// The metric is formed from cross products of the Jacobian columns: with
// columns x_r, x_s, x_t, the rows of J^-1 are (x_s x x_t, x_t x x_r, x_r x x_s)/det,
// so W det J (J^-1 J^-T)_ab = W (c_a . c_b) / det with c the cross products.
#include "nek_internal.h"

namespace nek {
namespace {

struct Pt { double x, y, z; };

__device__ __forceinline__ Pt node_pos(int ex, int ey, int ez, int ii, int jj, int kk,
                                       const double *zg, double hx, double hy, double hz,
                                       double amp, double a0, double a1, double a2) {
    const double x0 = hx * (ex + 0.5 * (1.0 + zg[ii]));
    const double y0 = hy * (ey + 0.5 * (1.0 + zg[jj]));
    const double z0 = hz * (ez + 0.5 * (1.0 + zg[kk]));
    const double bump = amp * (sin(M_PI * x0) * sin(M_PI * y0) * sin(M_PI * z0));
    return Pt{x0 + a0 * bump, y0 + a1 * bump, z0 + a2 * bump};
}

__device__ __forceinline__ Pt cross(Pt u, Pt v) {
    return Pt{u.y * v.z - u.z * v.y, u.z * v.x - u.x * v.z, u.x * v.y - u.y * v.x};
}
__device__ __forceinline__ double dot(Pt u, Pt v) { return u.x * v.x + u.y * v.y + u.z * v.z; }

__global__ void box_geom_kernel(int Ex, int Ey, int Ez, int N, double amp, double a0, double a1,
                                double a2, GllTable tab, double *__restrict__ g,
                                double *__restrict__ bm, double *__restrict__ X) {
    const double *zg = tab.z, *wq = tab.w, *Dm = tab.D;
    const int n = N + 1;
    const int64_t n3 = (int64_t)n * n * n;
    const int64_t E = (int64_t)Ex * Ey * Ez;
    const int64_t P = E * n3;
    const double hx = 1.0 / Ex, hy = 1.0 / Ey, hz = 1.0 / Ez;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; L < P; L += stride) {
        const int64_t e = L / n3;
        const int q = (int)(L - e * n3);
        const int i = q % n, j = (q / n) % n, k = q / (n * n);
        const int ex = (int)(e % Ex), ey = (int)((e / Ex) % Ey), ez = (int)(e / ((int64_t)Ex * Ey));
        Pt xr{0, 0, 0}, xs{0, 0, 0}, xt{0, 0, 0};
        for (int l = 0; l < n; ++l) {
            const double dr = Dm[i + n * l], ds = Dm[j + n * l], dt = Dm[k + n * l];
            Pt pr = node_pos(ex, ey, ez, l, j, k, zg, hx, hy, hz, amp, a0, a1, a2);
            Pt ps = node_pos(ex, ey, ez, i, l, k, zg, hx, hy, hz, amp, a0, a1, a2);
            Pt pt = node_pos(ex, ey, ez, i, j, l, zg, hx, hy, hz, amp, a0, a1, a2);
            xr.x += dr * pr.x; xr.y += dr * pr.y; xr.z += dr * pr.z;
            xs.x += ds * ps.x; xs.y += ds * ps.y; xs.z += ds * ps.z;
            xt.x += dt * pt.x; xt.y += dt * pt.y; xt.z += dt * pt.z;
        }
        const Pt cr = cross(xs, xt), cs = cross(xt, xr), ct = cross(xr, xs);
        const double det = dot(xr, cr);
        const double Wd = wq[i] * wq[j] * wq[k] / det;
        double *ge = g + e * 6 * n3 + q;
        ge[0 * n3] = Wd * dot(cr, cr);
        ge[1 * n3] = Wd * dot(cr, cs);
        ge[2 * n3] = Wd * dot(cr, ct);
        ge[3 * n3] = Wd * dot(cs, cs);
        ge[4 * n3] = Wd * dot(cs, ct);
        ge[5 * n3] = Wd * dot(ct, ct);
        if (bm) bm[L] = wq[i] * wq[j] * wq[k] * det;
        if (X) {
            Pt pp = node_pos(ex, ey, ez, i, j, k, zg, hx, hy, hz, amp, a0, a1, a2);
            X[L] = pp.x;
            X[P + L] = pp.y;
            X[2 * P + L] = pp.z;
        }
    }
}

}  // namespace

hipError_t launch_box_geometry(int Ex, int Ey, int Ez, int N, double amp, double a0, double a1,
                               double a2, const GllTable &tab, double *g, double *bm, double *X,
                               hipStream_t s) {
    const int64_t P = (int64_t)Ex * Ey * Ez * n3_of(N);
    int64_t blocks = (P + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(box_geom_kernel, dim3((unsigned)blocks), dim3(256), 0, s, Ex, Ey, Ez, N, amp,
                       a0, a1, a2, tab, g, bm, X);
    return hipGetLastError();
}

}  // namespace nek
