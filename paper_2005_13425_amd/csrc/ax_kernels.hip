// ax_kernels.hip -- the local Poisson operator of Listing 1 (Sec. III) for
// gfx950, in FP64 and in FP32 (with g stored as FP32 or BF16).
//
// Per element: wr/ws/wt = contractions of u with dxm1 along r, s, t; the
// symmetric multiply by the six geometric factors gives ur/us/ut; w is the sum
// of the three contractions of ur/us/ut with dxtm1.
//
// Work layout (gfx950, wave64, 160 KB LDS per CU):
//   * a workgroup holds EPB whole elements (n^2 threads each, small degrees
//     packed so a workgroup has about 256 threads); the whole element is
//     staged in LDS (three padded n^3 buffers), which the large LDS of gfx950
//     allows, instead of one layer at a time as in the paper's 2D-thread
//     kernel (Sec. IV-C);
//   * the t-direction contractions run on a register column per thread
//     (thread (i,j) holds u(i,j,:) and accumulates w(i,j,:));
//   * the r- and s-direction contractions run as pencils: one thread applies
//     the whole n x n matrix to one line of n values, so the matrix entry is
//     the same for every lane and comes through the scalar cache, and each
//     LDS value is read once per direction (about 16 LDS accesses per point
//     instead of ~4n for a per-lane gather);
//   * the six geometric factors (75% of the HBM bytes) are loaded two layers
//     ahead of use;
//   * optionally the CG direction update p <- r + beta p is fused into the
//     load of u, writing p back once.
#include "nek_internal.h"
#include "reduce.h"

namespace nek {
namespace {

constexpr int round64(int x) { return (x + 63) / 64 * 64; }

// Work shape: EPB elements per workgroup, n^2 threads per element (rounded
// up to whole wavefronts).  LDS rows are padded to an odd number of words so
// that lanes walking pencils with stride RS hit distinct banks.
template <int NX, typename T>
struct AxShape {
    static constexpr int NN = NX * NX;
    static constexpr int N3 = NN * NX;
    static constexpr int EPB = NN >= 64 ? 1 : 256 / NN;
    static constexpr int THREADS = round64(EPB * NN);
    static constexpr int RS = NX | 1;                                  // row stride (elements)
    static constexpr int LS = NX * RS;                                 // layer stride
    static constexpr int BUF = NX * LS;                                // one n^3 buffer
    // waves per SIMD the register budget is held to: the LDS of one workgroup
    // (3 BUF values per element) allows about this many on a 160 KB CU
    static constexpr int MINW = (sizeof(T) == 8 && NX <= 10) ? 3 : 1;
};

template <typename GT>
__device__ __forceinline__ float g_to_f32(GT v);
template <>
__device__ __forceinline__ float g_to_f32<float>(float v) { return v; }
template <>
__device__ __forceinline__ float g_to_f32<uint16_t>(uint16_t v) {
    return __uint_as_float(((uint32_t)v) << 16);
}

template <typename T, typename GT>
__device__ __forceinline__ T load_g(const GT *p);
template <>
__device__ __forceinline__ double load_g<double, double>(const double *p) { return *p; }
template <>
__device__ __forceinline__ float load_g<float, float>(const float *p) { return *p; }
template <>
__device__ __forceinline__ float load_g<float, uint16_t>(const uint16_t *p) {
    return g_to_f32<uint16_t>(*p);
}

// T: compute type (double or float); GT: storage type of g; FUSE: p <- r + beta p.
//
// Per element, three LDS buffers B0, B1, B2 of n^3 (padded) values:
//   1. column threads (i,j) load u(i,j,:) into registers and store it in B0;
//   2. pencil threads: r-pencil (j,k) computes wr(:,j,k) = D u(:,j,k) -> B1,
//      s-pencil (i,k) computes ws(i,:,k) -> B2 (dxm1 uniform: scalar path);
//   3. column threads: wt from the register column, the symmetric g multiply,
//      ur -> B1, us -> B2 in place, and the transposed t contraction is
//      accumulated in a register column of w;
//   4. r-pencils: dxtm1 applied to ur(:,j,k) -> B0;
//   5. s-pencils: dxtm1 applied to us(i,:,k) -> B1;
//   6. column threads: w = t part + B0 + B1, stored to HBM.
// Five workgroup barriers per element; every LDS value is written once and
// read once or twice.
template <int NX, typename T, typename GT, bool FUSE>
__global__ void __launch_bounds__((AxShape<NX, T>::THREADS), (AxShape<NX, T>::MINW))
ax_kernel(int64_t E, const T *__restrict__ D, const GT *__restrict__ g, double *__restrict__ p,
          double *__restrict__ w, AxFuse fz)
{
    using S = AxShape<NX, T>;
    constexpr int NN = S::NN;
    constexpr int N3 = S::N3;
    constexpr int EPB = S::EPB;
    constexpr int RS = S::RS;
    constexpr int LS = S::LS;
    constexpr int BUF = S::BUF;

    if (FUSE && fz.sc->done) return;   // uniform: CG already finished

    __shared__ T lds[EPB * 3 * BUF];

    const int tid = threadIdx.x;
    const int eb = tid / NN;
    const int c = tid - eb * NN;
    const int a = c % NX;      // i for columns / r-pencils' j / s-pencils' i
    const int b = c / NX;      // j for columns / pencils' k
    const bool in_slab = tid < EPB * NN;
    const int64_t e = (int64_t)blockIdx.x * EPB + eb;
    const bool active = in_slab && e < E;

    T *B0 = lds + (in_slab ? eb : 0) * 3 * BUF;
    T *B1 = B0 + BUF;
    T *B2 = B1 + BUF;

    // ---- 1. u column (in the CG: x += alpha p_old and p <- r + beta p_old first)
    T ucol[NX];
    double pcol[NX];   // FP64 p of this column, kept for the interior (p, w) sum
    const int64_t base = e * N3 + c;
    if (active) {
#pragma unroll
        for (int k = 0; k < NX; ++k) pcol[k] = p[base + k * NN];
        if constexpr (FUSE) {
            if (fz.x != nullptr && fz.sc->lag_applied == 0) {
                const double al = fz.sc->alpha;
                double xx[NX];
#pragma unroll
                for (int k = 0; k < NX; ++k) xx[k] = fz.x[base + k * NN];
#pragma unroll
                for (int k = 0; k < NX; ++k) fz.x[base + k * NN] = xx[k] + al * pcol[k];
            }
            if (fz.r != nullptr) {
                const double bt = fz.sc->beta;
                double rr[NX];
#pragma unroll
                for (int k = 0; k < NX; ++k) rr[k] = fz.r[base + k * NN];
#pragma unroll
                for (int k = 0; k < NX; ++k) {
                    pcol[k] = rr[k] + bt * pcol[k];
                    p[base + k * NN] = pcol[k];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < NX; ++k) ucol[k] = (T)pcol[k];
    } else {
#pragma unroll
        for (int k = 0; k < NX; ++k) {
            ucol[k] = T(0);
            pcol[k] = 0.0;
        }
    }

    // geometric factors of the first two layers go out now, the rest one
    // layer ahead of use
    const GT *ge = g + e * (6 * N3) + c;
    T gq[2][6];
#pragma unroll
    for (int k = 0; k < 2 && k < NX; ++k)
#pragma unroll
        for (int q = 0; q < 6; ++q) gq[k][q] = active ? load_g<T, GT>(ge + q * N3 + k * NN) : T(0);

    const int col = b * RS + a;   // (i,j) of this column within a layer
    if (in_slab) {
#pragma unroll
        for (int k = 0; k < NX; ++k) B0[k * LS + col] = ucol[k];
    }
    __syncthreads();

    // ---- 2. forward pencils
    if (in_slab) {
        // r-pencil (j = a, k = b): wr(i) = sum_l dxm1(i,l) u(l,j,k)
        {
            T v[NX], o[NX];
            const T *src = B0 + b * LS + a * RS;
#pragma unroll
            for (int l = 0; l < NX; ++l) v[l] = src[l];
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                T acc = T(0);
#pragma unroll
                for (int l = 0; l < NX; ++l) acc += D[i + NX * l] * v[l];
                o[i] = acc;
            }
            T *dst = B1 + b * LS + a * RS;
#pragma unroll
            for (int i = 0; i < NX; ++i) dst[i] = o[i];
        }
        // s-pencil (i = a, k = b): ws(j) = sum_l dxm1(j,l) u(i,l,k)
        {
            T v[NX], o[NX];
            const T *src = B0 + b * LS + a;
#pragma unroll
            for (int l = 0; l < NX; ++l) v[l] = src[l * RS];
#pragma unroll
            for (int j = 0; j < NX; ++j) {
                T acc = T(0);
#pragma unroll
                for (int l = 0; l < NX; ++l) acc += D[j + NX * l] * v[l];
                o[j] = acc;
            }
            T *dst = B2 + b * LS + a;
#pragma unroll
            for (int j = 0; j < NX; ++j) dst[j * RS] = o[j];
        }
    }
    __syncthreads();

    // ---- 3. column: g multiply, ur/us back to LDS, transposed t contraction
    T wcol[NX];
#pragma unroll
    for (int k = 0; k < NX; ++k) wcol[k] = T(0);
    if (in_slab) {
#pragma unroll
        for (int k = 0; k < NX; ++k) {
            const T *gc = gq[k & 1];
            T wt = T(0);
#pragma unroll
            for (int l = 0; l < NX; ++l) wt += D[k + NX * l] * ucol[l];
            const T wr = B1[k * LS + col];
            const T ws = B2[k * LS + col];
            const T ur = gc[0] * wr + gc[1] * ws + gc[2] * wt;
            const T us = gc[1] * wr + gc[3] * ws + gc[4] * wt;
            const T ut = gc[2] * wr + gc[4] * ws + gc[5] * wt;
            B1[k * LS + col] = ur;
            B2[k * LS + col] = us;
            // w(i,j,m) += dxtm1(m,k) ut(i,j,k) = dxm1(k,m) ut
#pragma unroll
            for (int m = 0; m < NX; ++m) wcol[m] += D[k + NX * m] * ut;
            if (k + 2 < NX) {
#pragma unroll
                for (int q = 0; q < 6; ++q)
                    gq[k & 1][q] = active ? load_g<T, GT>(ge + q * N3 + (k + 2) * NN) : T(0);
            }
        }
    }
    __syncthreads();

    // ---- 4. r-pencils of dxtm1: sum_l dxtm1(i,l) ur(l,j,k), dxtm1(i,l) = D[l + n i]
    if (in_slab) {
        T v[NX], o[NX];
        const T *src = B1 + b * LS + a * RS;
#pragma unroll
        for (int l = 0; l < NX; ++l) v[l] = src[l];
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            T acc = T(0);
#pragma unroll
            for (int l = 0; l < NX; ++l) acc += D[l + NX * i] * v[l];
            o[i] = acc;
        }
        T *dst = B0 + b * LS + a * RS;
#pragma unroll
        for (int i = 0; i < NX; ++i) dst[i] = o[i];
    }
    __syncthreads();

    // ---- 5. s-pencils of dxtm1: sum_l dxtm1(j,l) us(i,l,k) -> B1
    if (in_slab) {
        T v[NX], o[NX];
        const T *src = B2 + b * LS + a;
#pragma unroll
        for (int l = 0; l < NX; ++l) v[l] = src[l * RS];
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            T acc = T(0);
#pragma unroll
            for (int l = 0; l < NX; ++l) acc += D[l + NX * j] * v[l];
            o[j] = acc;
        }
        T *dst = B1 + b * LS + a;
#pragma unroll
        for (int j = 0; j < NX; ++j) dst[j * RS] = o[j];
    }
    __syncthreads();

    // ---- 6. w = t part + r part + s part
    double pw = 0.0;
    if (active) {
        const bool inner_col = a > 0 && a < NX - 1 && b > 0 && b < NX - 1;
#pragma unroll
        for (int k = 0; k < NX; ++k) {
            const double wv = (double)(wcol[k] + B0[k * LS + col] + B1[k * LS + col]);
            w[base + k * NN] = wv;
            if (FUSE && inner_col && k > 0 && k < NX - 1) pw += pcol[k] * wv;
        }
    }
    // ---- 7. CG: per-workgroup sum of p w over element-interior points
    if constexpr (FUSE) {
        if (fz.partials != nullptr) {
            __shared__ double red[S::THREADS / 64];
            const double bs = block_sum<S::THREADS>(pw, red);
            if (threadIdx.x == 0) fz.partials[blockIdx.x] = bs;
        }
    }
}

template <int NX, typename T, typename GT>
hipError_t launch_one(int64_t E, const T *D, const GT *g, double *p, double *w, const AxFuse &fz,
                      hipStream_t s)
{
    using S = AxShape<NX, T>;
    const int64_t blocks = (E + S::EPB - 1) / S::EPB;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    if (fz.sc != nullptr)
        hipLaunchKernelGGL((ax_kernel<NX, T, GT, true>), dim3((unsigned)blocks), dim3(S::THREADS),
                           0, s, E, D, g, p, w, fz);
    else
        hipLaunchKernelGGL((ax_kernel<NX, T, GT, false>), dim3((unsigned)blocks), dim3(S::THREADS),
                           0, s, E, D, g, p, w, fz);
    return hipGetLastError();
}

template <typename T, typename GT>
hipError_t dispatch(int64_t E, int N, const T *D, const GT *g, double *p, double *w,
                    const AxFuse &fz, hipStream_t s)
{
    switch (N + 1) {
#define NEK_CASE(NX) \
    case NX: return launch_one<NX, T, GT>(E, D, g, p, w, fz, s);
        NEK_CASE(2) NEK_CASE(3) NEK_CASE(4) NEK_CASE(5) NEK_CASE(6) NEK_CASE(7) NEK_CASE(8)
        NEK_CASE(9) NEK_CASE(10) NEK_CASE(11) NEK_CASE(12) NEK_CASE(13) NEK_CASE(14)
        NEK_CASE(15) NEK_CASE(16)
#undef NEK_CASE
    default: return hipErrorInvalidValue;
    }
}

// round-to-nearest-even FP64 -> BF16 through FP32
__device__ __forceinline__ uint16_t f64_to_bf16(double v) {
    float f = (float)v;
    uint32_t b = __float_as_uint(f);
    if ((b & 0x7f800000u) == 0x7f800000u)                 // inf stays inf, nan stays nan
        return (uint16_t)((b >> 16) | ((b & 0x007fffffu) ? 0x0040u : 0u));
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

__global__ void convert_g_kernel(int64_t count, const double *__restrict__ g, int dtype,
                                 void *__restrict__ out)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += stride) {
        if (dtype == NEK_G_F32)
            ((float *)out)[t] = (float)g[t];
        else
            ((uint16_t *)out)[t] = f64_to_bf16(g[t]);
    }
}

}  // namespace

hipError_t launch_ax_f64(int64_t E, int N, const double *D, const double *g, double *p, double *w,
                         const AxFuse &fz, hipStream_t s)
{
    return dispatch<double, double>(E, N, D, g, p, w, fz, s);
}

hipError_t launch_ax_f32(int64_t E, int N, const float *D32, const void *g_lo, int g_dtype,
                         double *p, double *w, const AxFuse &fz, hipStream_t s)
{
    if (g_dtype == NEK_G_F32)
        return dispatch<float, float>(E, N, D32, (const float *)g_lo, p, w, fz, s);
    if (g_dtype == NEK_G_BF16)
        return dispatch<float, uint16_t>(E, N, D32, (const uint16_t *)g_lo, p, w, fz, s);
    return hipErrorInvalidValue;
}

int64_t ax_blocks(int64_t E, int N)
{
    const int nn = (N + 1) * (N + 1);
    const int64_t epb = nn >= 64 ? 1 : 256 / nn;   // AxShape<N+1, .>::EPB
    return (E + epb - 1) / epb;
}

hipError_t launch_convert_g(int64_t count, const double *g, int g_dtype, void *out, hipStream_t s)
{
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(convert_g_kernel, dim3((unsigned)blocks), dim3(256), 0, s, count, g,
                       g_dtype, out);
    return hipGetLastError();
}

}  // namespace nek
