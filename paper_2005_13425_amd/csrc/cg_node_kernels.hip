// cg_node_kernels.hip -- the CG's fused operator for small meshes: one thread
// per node, the element's p and the three intermediates ur, us, ut in LDS
// (the shared-memory design of Sec. IV-B).  With few elements the pencil
// kernel's n^2 threads per element leave most of the GPU idle and each
// element's n layers form one long latency chain; n^3 threads per element
// take every layer at once.
//
// Same contract as the CG-fused pencil operator: AxFuse with sc, r, x, dinv
// and partials; the vectors p, r, x, dinv and w in the CG layout, g in the
// layout of Listing 1.  FP64, n = 4..10 (n^3 <= 1024 threads), one workgroup
// per element, each leaving its element's partial of (p, A_L p): E partials,
// where the pencil kernel leaves one per workgroup of several elements at
// n < 8.
#include "nek_internal.h"
#include "reduce.h"

namespace nek {
namespace {

constexpr int node_threads(int nx) { return (nx * nx * nx + 63) / 64 * 64; }

// The operator on element e by the threads of one part of a workgroup: `t`
// the node of this thread (N3 or more: no node; such threads only take part
// in the barriers), `L` the part's LDS (4 n^3 + n^2 doubles), `rbase` its
// first thread for the sum of the partial (`red`: one double per wave of the
// workgroup).  A plain launch is one part per workgroup.
template <int NX>
__device__ __forceinline__ void node_body(int64_t e, bool real, int t, const AxFuse &fz, const double *D_,
                                          const double *g_, double *p_, double *w_, double *L, double *red,
                                          int rbase) {
    constexpr int NN = NX * NX, N3 = NN * NX, NT = node_threads(NX);
    // the CG scalars are written only by other launches
    const kptr<CgScalars> sc = (kptr<CgScalars>)fz.sc;
    // uniform: the CG has finished (tested once the loads are in flight,
    // before the first store)
    const int done = sc->done;
    double *su = L, *sr = L + N3, *ss = L + 2 * N3, *st = L + 3 * N3, *sD = L + 4 * N3;
    const gptr<const double> D = (gptr<const double>)D_;
    const gptr<double> p = (gptr<double>)p_, w = (gptr<double>)w_;
    const gptr<const double> fr = (gptr<const double>)fz.r;
    const gptr<double> fx = (gptr<double>)fz.x;
    const gptr<const float> fdinv = (gptr<const float>)fz.dinv;

    const bool on = real && t < N3;   // node (i, j, k) in the order of Listing 1
    const int i = t % NX, j = (t / NX) % NX, k = t / NN;
    const int64_t at = e * N3 + (int64_t)k * NN + cgl_col(i, j, NX);   // its entry of the CG vectors

    // geometric factors first: they do not depend on anything else
    double gv[6];
    {
        const gptr<const double> ge = (gptr<const double>)g_ + e * (6 * N3) + t;
#pragma unroll
        for (int q = 0; q < 6; ++q) gv[q] = on ? ge[q * N3] : 0.0;
    }
    // x += alpha p_old, p <- r + beta p_old (dinv r + beta p_old with Jacobi)
    const bool upd_x = fx != nullptr && sc->lag_applied == 0;
    double pv = 0.0, rv = 0.0, xv = 0.0;
    if (on) {
        pv = p[at];
        if (upd_x) xv = __builtin_nontemporal_load(&fx[at]);
        if (fr != nullptr) {
            rv = fr[at];
            if (fdinv != nullptr) rv = (double)fdinv[at] * rv;
        }
    }
    const double dv = t < NN ? D[t] : 0.0;
    if (done) return;
    if (on) {
        if (upd_x) __builtin_nontemporal_store(xv + sc->alpha * pv, &fx[at]);
        if (fr != nullptr) {
            pv = rv + sc->beta * pv;
            p[at] = pv;
        }
        su[t] = pv;
    }
    if (t < NN) sD[t] = dv;
    __syncthreads();

    // forward contractions with dxm1 (D[i + n l] = dxm1(i, l)), then the
    // geometric multiply
    if (on) {
        double wr = 0.0, ws = 0.0, wt = 0.0;
#pragma unroll
        for (int l = 0; l < NX; ++l) {
            wr += sD[i + NX * l] * su[l + NX * j + NN * k];
            ws += sD[j + NX * l] * su[i + NX * l + NN * k];
            wt += sD[k + NX * l] * su[i + NX * j + NN * l];
        }
        sr[t] = gv[0] * wr + gv[1] * ws + gv[2] * wt;
        ss[t] = gv[1] * wr + gv[3] * ws + gv[4] * wt;
        st[t] = gv[2] * wr + gv[4] * ws + gv[5] * wt;
    }
    __syncthreads();

    // transposed contractions summed (dxtm1(i, l) = dxm1(l, i))
    double pw = 0.0;
    if (on) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < NX; ++l)
            s += sD[l + NX * i] * sr[l + NX * j + NN * k] + sD[l + NX * j] * ss[i + NX * l + NN * k] +
                 sD[l + NX * k] * st[i + NX * j + NN * l];
        w[at] = s;
        pw = pv * s;
    }
    // this element's share of sum p (A_L p), as the pencil kernel leaves it
    if (fz.partials != nullptr) {
        const double bs = seg_sum<NT>(pw, red, rbase);
        if ((int)threadIdx.x == rbase && real) ((gptr<double>)fz.partials)[e] = bs;
    }
}

template <int NX>
constexpr int node_lds() { return 4 * NX * NX * NX + NX * NX; }

template <int NX>
__global__ void __launch_bounds__(node_threads(NX))
ax_node_fused_kernel(const double *__restrict__ D, const double *__restrict__ g, double *__restrict__ p,
                     double *__restrict__ w, AxFuse fz) {
    __shared__ double L[node_lds<NX>()];
    __shared__ double red[node_threads(NX) / 64];
    node_body<NX>(blockIdx.x, true, threadIdx.x, fz, D, g, p, w, L, red, 0);
}

// The served form's launch (see ServeNodeSlot): several elements per
// 1024-thread workgroup at n < 10.
template <int NX>
__device__ __forceinline__ void node_serve_part(const ServeNodeSlot &S, int64_t wg, double *lds, double *red) {
    constexpr int NT = node_threads(NX), PARTS = SERVE_NODE_THREADS / NT;
    const int q = (int)threadIdx.x / NT;
    const int qc = q < PARTS ? q : PARTS - 1;
    const int t = q < PARTS ? (int)threadIdx.x - q * NT : NT;
    const int64_t e = (wg - S.block0) * PARTS + qc;
    const bool real = e < S.E;
    node_body<NX>(real ? e : 0, real, t, S.fz, S.D, S.g, S.p, S.w, lds + (size_t)qc * node_lds<NX>(), red,
                  qc * NT);
}

// Two kernels: n = 9 needs more than 64 VGPRs (79 in its own kernel), the
// others fit 64, which lets two 1024-thread workgroups share a CU.
template <bool N9>
__device__ __forceinline__ void node_serve_body(const ServeNodeSlot *__restrict__ slots, int nslots, double *lds,
                                                double *red) {
    const ServeNodeSlot &S = slots[batch_slot(slots, nslots, (int64_t)blockIdx.x)];
    if constexpr (N9) {
        node_serve_part<9>(S, blockIdx.x, lds, red);
    } else {
        switch (S.nx) {
        case 4: node_serve_part<4>(S, blockIdx.x, lds, red); break;
        case 5: node_serve_part<5>(S, blockIdx.x, lds, red); break;
        case 6: node_serve_part<6>(S, blockIdx.x, lds, red); break;
        case 7: node_serve_part<7>(S, blockIdx.x, lds, red); break;
        case 8: node_serve_part<8>(S, blockIdx.x, lds, red); break;
        case 10: node_serve_part<10>(S, blockIdx.x, lds, red); break;
        default: break;
        }
    }
}

__global__ void __launch_bounds__(SERVE_NODE_THREADS, 8)
ax_node_serve_kernel(const ServeNodeSlot *__restrict__ slots, int nslots) {
    extern __shared__ __align__(16) double node_serve_lds[];
    __shared__ double red[SERVE_NODE_THREADS / 64];
    node_serve_body<false>(slots, nslots, node_serve_lds, red);
}

__global__ void __launch_bounds__(SERVE_NODE_THREADS)
ax_node_serve9_kernel(const ServeNodeSlot *__restrict__ slots, int nslots) {
    extern __shared__ __align__(16) double node_serve_lds[];
    __shared__ double red[SERVE_NODE_THREADS / 64];
    node_serve_body<true>(slots, nslots, node_serve_lds, red);
}

template <int NX>
hipError_t launch_node(int64_t E, const double *D, const double *g, double *p, double *w, const AxFuse &fz,
                       hipStream_t s) {
    hipLaunchKernelGGL(ax_node_fused_kernel<NX>, dim3((unsigned)E), dim3(node_threads(NX)), 0, s, D, g, p, w,
                       fz);
    return hipGetLastError();
}

}  // namespace

bool serve_node_shape(int N, int64_t E, ServeNodeShape &o) {
    if (N < AX_NODE_MIN_N || N > 9) return false;
    const int nx = N + 1;
    const int nt = (nx * nx * nx + 63) / 64 * 64;
    const int parts = SERVE_NODE_THREADS / nt;
    o.blocks = (E + parts - 1) / parts;
    o.lds_bytes = (size_t)parts * (4 * nx * nx * nx + nx * nx) * sizeof(double);
    o.n9 = N == 8;
    return true;
}

hipError_t launch_ax_node_serve(const ServeNodeSlot *slots, int nslots, int64_t blocks, size_t lds_bytes, bool n9,
                                hipStream_t s) {
    if (nslots < 1 || nslots > BATCH_MAX_SLOTS || blocks < 1 || blocks > 0x7fffffff) return hipErrorInvalidValue;
    if (n9)
        hipLaunchKernelGGL(ax_node_serve9_kernel, dim3((unsigned)blocks), dim3(SERVE_NODE_THREADS), lds_bytes, s,
                           slots, nslots);
    else
        hipLaunchKernelGGL(ax_node_serve_kernel, dim3((unsigned)blocks), dim3(SERVE_NODE_THREADS), lds_bytes, s,
                           slots, nslots);
    return hipGetLastError();
}

bool ax_node_fused_fits(int64_t E, int N) {
    return N >= AX_NODE_MIN_N && N <= 9 && E >= 1 && E <= AX_NODE_MAX_POINTS / n3_of(N);
}

hipError_t launch_ax_node_fused(int64_t E, int N, const double *D, const double *g, double *p, double *w,
                                const AxFuse &fz, hipStream_t s) {
    if (!ax_node_fused_fits(E, N) || fz.sc == nullptr || !fz.cg_layout) return hipErrorInvalidValue;
    switch (N) {
    case 3: return launch_node<4>(E, D, g, p, w, fz, s);
    case 4: return launch_node<5>(E, D, g, p, w, fz, s);
    case 5: return launch_node<6>(E, D, g, p, w, fz, s);
    case 6: return launch_node<7>(E, D, g, p, w, fz, s);
    case 7: return launch_node<8>(E, D, g, p, w, fz, s);
    case 8: return launch_node<9>(E, D, g, p, w, fz, s);
    case 9: return launch_node<10>(E, D, g, p, w, fz, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace nek
