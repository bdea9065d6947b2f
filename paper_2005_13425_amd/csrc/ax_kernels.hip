// ax_kernels.hip -- the local Poisson operator of Listing 1 (Sec. III) for
// gfx950, in FP64 and in FP32 (with g stored as FP32 or BF16).
//
// Per element: wr/ws/wt = contractions of u with dxm1 along r, s, t; the
// symmetric multiply by the six geometric factors gives ur/us/ut; w is the sum
// of the three contractions of ur/us/ut with dxtm1.
//
// Work layout (gfx950, wave64, 160 KB LDS per CU):
//   * a workgroup holds EPB whole elements (n^2 threads each, small degrees
//     packed so a workgroup has about 256 threads, two elements at n = 10 in
//     the plain FP64 form); the whole element is staged in LDS (two padded
//     n^3 buffers), which the large LDS of gfx950 allows, instead of one layer
//     at a time as in the paper's 2D-thread kernel (Sec. IV-C);
//   * the t-direction contractions run on a register column per thread
//     (thread (i,j) holds u(i,j,:) and forms w(i,j,:));
//   * the r- and s-direction contractions run as pencils: one thread applies
//     the whole n x n matrix to one line of n values, so the matrix entry is
//     the same for every lane and comes through the scalar cache, and each
//     LDS value is read once per direction (about 18 LDS accesses per point
//     instead of ~4n for a per-lane gather);
//   * the six geometric factors (75% of the HBM bytes) are loaded four layers
//     ahead of use;
//   * in the CG the updates x += alpha p and p <- r + beta p are fused into
//     the load of u, and the (p, A_L p) partial comes out of the same pass.
#include <type_traits>

#include "nek_internal.h"
#include "reduce.h"

namespace nek {
namespace {

constexpr int round64(int x) { return (x + 63) / 64 * 64; }

// Work shape: EPB elements per workgroup, n^2 threads per element (rounded
// up to whole wavefronts).  LDS rows are padded to an odd number of words so
// that lanes walking pencils with stride RS hit distinct banks.  WIDE: two
// elements per workgroup at n = 10 (see AxShapeFor).
#ifndef NEK_AX_WIDE_EPB
#define NEK_AX_WIDE_EPB 2
#endif
template <int NX, typename T, bool WIDE = false>
struct AxShape {
    static constexpr int NN = NX * NX;
    static constexpr int N3 = NN * NX;
    static constexpr int EPB = WIDE ? NEK_AX_WIDE_EPB : (NN >= 64 ? 1 : 256 / NN);
    static constexpr int THREADS = round64(EPB * NN);
    static constexpr int RS = NX | 1;                                  // row stride (elements)
    static constexpr int LS = NX * RS;                                 // layer stride
    static constexpr int BUF = NX * LS;                                // one n^3 buffer
    static constexpr int LDS_BYTES = EPB * 2 * BUF * (int)sizeof(T);   // two buffers per element
    // waves per SIMD the register budget is held to: as many as the LDS of
    // the workgroups that fit a 160 KB CU provides, capped so that the FP64
    // form of every degree compiles without register spills
    static constexpr int WPS = ((163840 / LDS_BYTES) * (THREADS / 64) + 3) / 4;
    static constexpr int REG_CAP = sizeof(T) == 8 ? ((NX <= 8 || NX == 10) ? 4 : (NX <= 14 ? 3 : 2)) : 4;
    static constexpr int MINW = WPS < 1 ? 1 : (WPS > REG_CAP ? REG_CAP : WPS);
    // the CG-fused form also carries the FP64 p column through the element
    static constexpr int MINW_FUSED = MINW < (NX <= 10 ? 3 : 2) ? MINW : (NX <= 10 ? 3 : 2);
    // layers of geometric factors held in registers ahead of their use
#ifdef NEK_AX_PF
    static constexpr int PF = NEK_AX_PF < NX ? NEK_AX_PF : NX;
#else
    static constexpr int PF = 4 < NX ? 4 : NX;
#endif
};

// The plain FP64 operator at n = 10 runs two elements per workgroup: the
// 2048 workgroups of E = 4096 fill exactly two rounds of 1024 (four per CU,
// as LDS allows), where one element per workgroup ran 4096 workgroups in 1.8
// rounds of 2304 (nine per CU) and the partial last round set the end (3.5%
// faster; the CG-fused form is 1% slower that way and keeps one element per
// workgroup).
template <int NX, typename T, bool FUSE, bool CGL>
using AxShapeFor = AxShape<NX, T, !FUSE && !CGL && sizeof(T) == 8 && NX == 10>;

// Loading the six geometric factors of one point of layer k.
//   FP64 g: the layout of Listing 1, six planes of n^3 per element (six loads).
//   FP32 / BF16 g (the mixed forms' own copy, written by nek_convert_g): the
//   six factors of a point side by side, point after point (24 or 12 bytes),
//   so a point is one or two loads per lane, coalesced across the lanes of a
//   layer.  BF16 pairs (g_2q, g_2q+1) share a 32-bit word, g_2q in the low
//   half.
// The factors are read through a buffer resource that spans exactly the
// elements of the workgroup (or of the part of a served workgroup).  A lane
// with no point of its own (padding, or an element past E) gets an offset
// past that range, which the hardware answers with zeros and no memory
// access, so every lane issues every load and no load sits in a branch.  The
// compiler then counts the loads in flight exactly and waits for a layer's
// factors only where they are used, PF layers after they were requested; with
// the loads inside `if (active)` it waited for all of them at the end of
// every such branch, which left the prefetch without effect (2-5% slower on
// the 32.8 M-point boxes at N = 9..15).
template <typename GT>
constexpr int gpoint_bytes() { return std::is_same<GT, double>::value ? (int)sizeof(double) : 6 * (int)sizeof(GT); }

struct GSrc {
    __amdgpu_buffer_rsrc_t rs;   // uniform over the part
    uint32_t vo;                 // the lane's byte offset at layer 0, or past the range
};

// elements [e0, e0 + EPB) of g, clipped to E; lane (eb, c) is point c of
// layer 0 of element e0 + eb
template <typename GT, int N3>
__device__ __forceinline__ GSrc g_source(gptr<const GT> g, int64_t e0, int64_t E, int EPB, int eb, int c,
                                         bool active) {
    constexpr int64_t EB = 6 * (int64_t)N3 * (int64_t)sizeof(GT);   // bytes per element
    int64_t ne = E - e0;
    ne = ne < 0 ? 0 : (ne > EPB ? EPB : ne);
    // e0 is the same for every lane of a wave (a part is whole waves); read
    // the values from the first lane so that the resource sits in scalar
    // registers whatever the compiler can prove
    const uint64_t a = (uint64_t)(g + (ne > 0 ? e0 : 0) * (6 * N3));
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    const uint32_t nb = __builtin_amdgcn_readfirstlane((uint32_t)(ne * EB));
    GSrc s;
    s.rs = __builtin_amdgcn_make_buffer_rsrc((void *)(((uint64_t)hi << 32) | lo), (short)0, (int)nb, 0x00020000);
    s.vo = active ? (uint32_t)(eb * EB + (int64_t)c * gpoint_bytes<GT>()) : 0x80000000u;
    return s;
}

typedef uint32_t gword3 __attribute__((ext_vector_type(3)));

template <typename T, typename GT, int N3, int NN>
struct GLoad;

template <int N3, int NN>
struct GLoad<double, double, N3, NN> {
    template <bool NT>
    __device__ static __forceinline__ void load(const GSrc &s, int k, double *o) {
#pragma unroll
        for (int q = 0; q < 6; ++q)
            o[q] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                                  s.rs, s.vo + (uint32_t)((q * N3 + k * NN) * 8), 0, NT ? 2 : 0));
    }
};

// six FP32 factors: two 12-byte loads
__device__ __forceinline__ void g6f(const GSrc &s, uint32_t off, float *o) {
    const gword3 x = __builtin_amdgcn_raw_buffer_load_b96(s.rs, s.vo + off, 0, 0);
    const gword3 y = __builtin_amdgcn_raw_buffer_load_b96(s.rs, s.vo + off + 12u, 0, 0);
    o[0] = __uint_as_float(x.x); o[1] = __uint_as_float(x.y); o[2] = __uint_as_float(x.z);
    o[3] = __uint_as_float(y.x); o[4] = __uint_as_float(y.y); o[5] = __uint_as_float(y.z);
}

// six BF16 factors: one 12-byte load
__device__ __forceinline__ void g6h(const GSrc &s, uint32_t off, float *o) {
    const gword3 x = __builtin_amdgcn_raw_buffer_load_b96(s.rs, s.vo + off, 0, 0);
    const uint32_t v[3] = {x.x, x.y, x.z};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        o[2 * q] = __uint_as_float(v[q] << 16);
        o[2 * q + 1] = __uint_as_float(v[q] & 0xffff0000u);
    }
}

template <int N3, int NN>
struct GLoad<float, float, N3, NN> {
    template <bool NT>
    __device__ static __forceinline__ void load(const GSrc &s, int k, float *o) { g6f(s, (uint32_t)(k * NN * 24), o); }
};

template <int N3, int NN>
struct GLoad<float, uint16_t, N3, NN> {
    template <bool NT>
    __device__ static __forceinline__ void load(const GSrc &s, int k, float *o) { g6h(s, (uint32_t)(k * NN * 12), o); }
};

// FP64 arithmetic on FP32 / BF16 factors (NEK_PREC_F64G*): the same loads,
// widened to FP64.
template <int N3, int NN>
struct GLoad<double, float, N3, NN> {
    template <bool NT>
    __device__ static __forceinline__ void load(const GSrc &s, int k, double *o) {
        float f[6];
        g6f(s, (uint32_t)(k * NN * 24), f);
#pragma unroll
        for (int q = 0; q < 6; ++q) o[q] = (double)f[q];
    }
};

template <int N3, int NN>
struct GLoad<double, uint16_t, N3, NN> {
    template <bool NT>
    __device__ static __forceinline__ void load(const GSrc &s, int k, double *o) {
        float f[6];
        g6h(s, (uint32_t)(k * NN * 12), f);
#pragma unroll
        for (int q = 0; q < 6; ++q) o[q] = (double)f[q];
    }
};

// The point (i, j) of a layer at within-layer offset c of the CG layout (the
// inverse of cgl_col).
template <int NX>
__device__ __forceinline__ void cgl_point(int c, int &i, int &j) {
    constexpr int M = NX - 2;   // interior points per row
    if (c >= NX * (NX - 1)) {
        i = NX - 1;
        j = c - NX * (NX - 1);
    } else if (c >= NX * M) {
        i = 0;
        j = c - NX * M;
    } else if constexpr (M > 0) {
        j = c / M;
        i = c - j * M + 1;
    }
}

// T: compute type (double or float); GT: storage type of g; FUSE: CG fusion;
// CGL: p, r, x, dinv and w in the CG layout (g always in that of Listing 1).
//
// Per element, two LDS buffers B0, B1 of n^3 (padded) values.  Thread (a, b)
// of an element plays three roles: the column (i,j) = (a,b), the r-pencil
// (j,k) = (a,b) and the s-pencil (i,k) = (a,b).
//   1. the column u(a,b,:) goes from HBM to B0;
//   2. forward contractions, one dxm1 column l at a time (outer products):
//      wr(:,a,b) += dxm1(:,l) u(l,a,b) -> B1 and wt(a,b,:) += dxm1(:,l)
//      u(a,b,l), kept in registers; then, once every thread has read u, each
//      s-pencil owner forms ws(a,:,b) += dxm1(:,l) u(a,l,b) and writes it over
//      its own pencil of B0;
//   3. column: the symmetric g multiply gives ur -> B1, us -> B0 (in place)
//      and ut in registers;
//   4. the ur pencil (:,a,b) and the us pencil (a,:,b) are read into registers;
//   5. transposed contractions, one dxtm1 row i at a time (inner products):
//      the r part at (i,a,b) -> B0 and the s part at (a,i,b) -> B1;
//   6. per layer i of the column, the t part (inner product of dxtm1 row i
//      with ut) is added to B0 + B1 and the sum stored to HBM as w(a,b,i).
// Only one column or row of the derivative matrix (n values, uniform across
// the workgroup) is live at a time, so it stays in scalar registers.  Two
// buffers instead of three keep more elements resident per CU (the high
// degrees were occupancy-bound).  Six workgroup barriers per element.
// In the CG layout thread (a, b) loads and stores the vector entries at
// offset c = a + n b of each layer, which belong to another column; they pass
// through LDS, with one more barrier before w is stored.
//
// A part of a workgroup runs the body: `tid` is the thread's index within the
// part (THREADS or more for threads of the workgroup that belong to no part:
// they only take part in the barriers), `lds` the part's EPB * 2 * BUF values
// and `rbase` the first thread of the part, for the sum of its partial (`red`
// holds one double per wave of the workgroup).  A plain launch is one part
// per workgroup (tid = threadIdx.x, rbase = 0).
template <int NX, typename T, typename GT, bool FUSE, bool CGL>
__device__ __forceinline__ void ax_body(int64_t blk, int64_t E, kptr<T> D, gptr<const GT> g,
                                        gptr<double> p, gptr<double> w, const AxFuse &fz,
                                        int tid, T *lds, double *red, int rbase)
{
    using S = AxShapeFor<NX, T, FUSE, CGL>;
    // The plain FP64 operator streams g and w with the non-temporal hint from
    // N = 7 up: 8-12% faster at E = 4096 and on the 32.8 M-point boxes
    // (N = 7..15), 9% slower at N = 5.  u keeps plain loads: a layer of n^2
    // columns splits over two waves inside a cache line, and with the hint
    // that line was fetched twice (2% slower at E = 4096).  The CG-fused form
    // re-reads p, r, x and w soon after and keeps the default caching.
    constexpr bool STREAM = !FUSE && !CGL && sizeof(T) == 8 && NX >= 8;
    constexpr int NN = S::NN;
    constexpr int N3 = S::N3;
    constexpr int EPB = S::EPB;
    constexpr int RS = S::RS;
    constexpr int LS = S::LS;
    constexpr int BUF = S::BUF;
    constexpr int PF = S::PF;

    // the CG scalars are written only by other launches
    const kptr<CgScalars> sc = (kptr<CgScalars>)fz.sc;
    const gptr<const double> fr = (gptr<const double>)fz.r;
    const gptr<double> fx = (gptr<double>)fz.x;
    const gptr<const float> fdinv = (gptr<const float>)fz.dinv;
    if (FUSE && sc->done) return;   // uniform: CG already finished

    const int eb = tid / NN;
    const int c = tid - eb * NN;
    const int a = c % NX;
    const int b = c / NX;
    const bool in_slab = tid < EPB * NN;
    const int64_t e = blk * EPB + eb;
    const bool active = in_slab && e < E;

    T *B0 = lds + (in_slab ? eb : 0) * 2 * BUF;
    T *B1 = B0 + BUF;
    const int col = b * RS + a;       // column (a,b) within a layer
    const int rpen = b * LS + a * RS; // start of r-pencil (:,a,b)
    const int spen = b * LS + a;      // start of s-pencil (a,:,b), stride RS
    // Vector entries (p, r, x, dinv, w) this thread moves between HBM and LDS:
    // offset c + k n^2 of the element, which is point (a, b, k) in the layout
    // of Listing 1 and point (av, bv, k) in the CG layout.  g is always read
    // for the thread's own column (a, b).
    int av = a, bv = b;
    if constexpr (CGL) cgl_point<NX>(c, av, bv);
    const int colv = bv * RS + av;

    // ---- 1. u column (in the CG: x += alpha p_old and p <- r + beta p_old first)
    const int64_t base = e * N3 + c;
    // (p, A_L p) in the CG: p^T D^T G D p = (D p)^T G (D p), summed in FP64
    // point by point at the geometric multiply from the gradient and the
    // multiplied gradient in registers.  Taking it from p and w instead meant
    // reading p again at the end, and p written at the start was no longer in
    // L2 by then: 32.8 MB more to read per launch at E = 4096, N = 9 (the FP32
    // operator's iterations were unchanged by the switch, 4-5% faster).
    {
        double pv[NX];
        if (active) {
#pragma unroll
            for (int k = 0; k < NX; ++k)
                pv[k] = p[base + k * NN];
            if constexpr (FUSE) {
                if (fx != nullptr && sc->lag_applied == 0) {
                    // x is not touched again before the next iteration's
                    // operator: in FP64 it streams past the caches, which keeps
                    // w and r there for the assembly (3 us per CG iteration at
                    // E = 4096, N = 9; the FP32 form lost 2% with it)
                    constexpr bool XNT = sizeof(T) == 8;
                    const double al = sc->alpha;
                    double xx[NX];
#pragma unroll
                    for (int k = 0; k < NX; ++k)
                        xx[k] = XNT ? __builtin_nontemporal_load(&fx[base + k * NN]) : fx[base + k * NN];
#pragma unroll
                    for (int k = 0; k < NX; ++k) {
                        if constexpr (XNT) __builtin_nontemporal_store(xx[k] + al * pv[k], &fx[base + k * NN]);
                        else fx[base + k * NN] = xx[k] + al * pv[k];
                    }
                }
                if (fr != nullptr) {
                    const double bt = sc->beta;
                    double rr[NX];
#pragma unroll
                    for (int k = 0; k < NX; ++k) rr[k] = fr[base + k * NN];
                    if (fdinv != nullptr) {   // z = M^-1 r, formed on the way in
#pragma unroll
                        for (int k = 0; k < NX; ++k) rr[k] = (double)fdinv[base + k * NN] * rr[k];
                    }
#pragma unroll
                    for (int k = 0; k < NX; ++k) {
                        pv[k] = rr[k] + bt * pv[k];
                        p[base + k * NN] = pv[k];
                    }
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < NX; ++k) pv[k] = 0.0;
        }
        if (in_slab) {
#pragma unroll
            for (int k = 0; k < NX; ++k) B0[k * LS + colv] = (T)pv[k];
        }
    }

    // geometric factors of the first PF layers go out now, each later layer
    // PF layers ahead of its use
    const GSrc gs = g_source<GT, N3>(g, blk * EPB, E, EPB, eb, c, active);
    T gq[PF][6];
#pragma unroll
    for (int k = 0; k < PF; ++k) GLoad<T, GT, N3, NN>::template load<STREAM>(gs, k, gq[k]);
    __syncthreads();

    // ---- 2. forward contractions: outer products with dxm1(:, l) = D[n l .. n l + n)
    T wt[NX];
    {
        T wr[NX];
#pragma unroll
        for (int q = 0; q < NX; ++q) {
            wr[q] = T(0);
            wt[q] = T(0);
        }
        if (in_slab) {
#pragma unroll 2
            for (int l = 0; l < NX; ++l) {
                const T vr = B0[rpen + l];          // u(l, a, b)
                const T vt = B0[l * LS + col];      // u(a, b, l)
                const kptr<T> Dl = D + NX * l;
#pragma unroll
                for (int q = 0; q < NX; ++q) {
                    const T d = Dl[q];
                    wr[q] += d * vr;
                    wt[q] += d * vt;
                }
            }
#pragma unroll
            for (int q = 0; q < NX; ++q) B1[rpen + q] = wr[q];   // wr(q, a, b)
        }
    }
    __syncthreads();
    // the s-pencil (a, :, b) of B0 is now read and rewritten by its owner only
    if (in_slab) {
        T ws[NX];
#pragma unroll
        for (int q = 0; q < NX; ++q) ws[q] = T(0);
#pragma unroll 2
        for (int l = 0; l < NX; ++l) {
            const T vs = B0[spen + l * RS];         // u(a, l, b)
            const kptr<T> Dl = D + NX * l;
#pragma unroll
            for (int q = 0; q < NX; ++q) ws[q] += Dl[q] * vs;
        }
#pragma unroll
        for (int q = 0; q < NX; ++q) B0[spen + q * RS] = ws[q];  // ws(a, q, b)
    }
    __syncthreads();

    // ---- 3. column: symmetric geometric multiply
    T ut[NX];
    double pw = 0.0;
#pragma unroll
    for (int k = 0; k < NX; ++k) {
        const T *gc = gq[k % PF];
        T urv = T(0), usv = T(0), utv = T(0);
        if (in_slab) {
            const T wrv = B1[k * LS + col];
            const T wsv = B0[k * LS + col];
            urv = gc[0] * wrv + gc[1] * wsv + gc[2] * wt[k];
            usv = gc[1] * wrv + gc[3] * wsv + gc[4] * wt[k];
            utv = gc[2] * wrv + gc[4] * wsv + gc[5] * wt[k];
            B1[k * LS + col] = urv;
            B0[k * LS + col] = usv;
            if constexpr (FUSE)
                pw += (double)wrv * (double)urv + (double)wsv * (double)usv + (double)wt[k] * (double)utv;
        }
        ut[k] = utv;
        if (k + PF < NX) GLoad<T, GT, N3, NN>::template load<STREAM>(gs, k + PF, gq[k % PF]);
    }
    __syncthreads();

    // ---- 4. ur and us pencils into registers
    T vr[NX], vs[NX];
#pragma unroll
    for (int l = 0; l < NX; ++l) {
        vr[l] = in_slab ? B1[rpen + l] : T(0);          // ur(l, a, b)
        vs[l] = in_slab ? B0[spen + l * RS] : T(0);     // us(a, l, b)
    }
    __syncthreads();

    // ---- 5. transposed contractions: inner products with dxtm1(i, :) = D[n i .. n i + n)
    if (in_slab) {
#pragma unroll 2
        for (int i = 0; i < NX; ++i) {
            const kptr<T> Di = D + NX * i;
            T pr = T(0), ps = T(0);
#pragma unroll
            for (int l = 0; l < NX; ++l) {
                const T d = Di[l];
                pr += d * vr[l];
                ps += d * vs[l];
            }
            B0[rpen + i] = pr;              // r part at (i, a, b)
            B1[spen + i * RS] = ps;         // s part at (a, i, b)
        }
    }
    __syncthreads();

    // ---- 6. w(a, b, i) = r part + s part + t part, the t part formed here
    if (active) {
#pragma unroll 2
        for (int i = 0; i < NX; ++i) {
            const kptr<T> Di = D + NX * i;
            T pt = T(0);
#pragma unroll
            for (int l = 0; l < NX; ++l) pt += Di[l] * ut[l];
            const T wv = (B0[i * LS + col] + B1[i * LS + col]) + pt;
            if constexpr (CGL) {
                B0[i * LS + col] = wv;                   // stored below, from another thread
            } else {
                if constexpr (STREAM) __builtin_nontemporal_store((double)wv, &w[base + i * NN]);
                else w[base + i * NN] = (double)wv;
                if constexpr (FUSE) B0[i * LS + col] = wv;   // the column's own slots
            }
        }
    }
    if constexpr (CGL) {
        // ---- 6b. w leaves LDS at the thread's CG-layout entries; the CG-fused
        // FP32 operator stores its FP32 result as it is (the assemble-update
        // widens it), 4 bytes per point less to write and to read back
        using WT = std::conditional_t<FUSE && sizeof(T) == 4, float, double>;
        __syncthreads();
        if (active) {
#pragma unroll
            for (int k = 0; k < NX; ++k) {
                const T wv = B0[k * LS + colv];
                ((gptr<WT>)w)[base + k * NN] = (WT)wv;
            }
        }
    }
    // ---- 7. CG: sum of p (A_L p) over all local points (formed in step 3).
    // For a continuous p that vanishes on masked nodes this is
    // (p, mask(dssum(A_L p))) over unique nodes, so the assembly needs no
    // product of its own.
    if constexpr (FUSE) {
        if (fz.partials != nullptr) {
            const double bs = seg_sum<S::THREADS>(pw, red, rbase);
            if ((int)threadIdx.x == rbase && blk * EPB < E) ((gptr<double>)fz.partials)[blk] = bs;
        }
    }
}

template <int NX, typename T, typename GT, bool FUSE, bool CGL>
__global__ void __launch_bounds__((AxShapeFor<NX, T, FUSE, CGL>::THREADS),
                                  (FUSE || CGL ? AxShapeFor<NX, T, FUSE, CGL>::MINW_FUSED
                                               : AxShapeFor<NX, T, FUSE, CGL>::MINW))
ax_kernel(int64_t E, const T *__restrict__ D, const GT *__restrict__ g, double *__restrict__ p,
          double *__restrict__ w, AxFuse fz)
{
    using S = AxShapeFor<NX, T, FUSE, CGL>;
    __shared__ T lds[S::EPB * 2 * S::BUF];
    __shared__ double red[S::THREADS / 64];
    ax_body<NX, T, GT, FUSE, CGL>(blockIdx.x, E, (kptr<T>)D, (gptr<const GT>)g, (gptr<double>)p,
                             (gptr<double>)w, fz, threadIdx.x, lds, red, 0);
}

// The served form: the CG-fused operator of every admitted solve of any
// degree and precision in one launch of 256-thread workgroups.  Solve s owns
// workgroups [block0, next block0); a workgroup holds 256 / THREADS parts of
// the solve's own shape (two pencil workgroups of 128 threads at n = 10, four
// of 64 at n = 8), and part q of workgroup b does exactly what workgroup
// (b - block0) * parts + q of the solve's own launch would do, with the same
// partial of (p, A_L p) summed in the same order: a solve's arithmetic does
// not depend on which others share the launch, or on sharing it at all.  The
// LDS is given at launch, sized for the largest shape in it.
template <int NX, typename T, typename GT>
struct ServeShape {
    using S = AxShapeFor<NX, T, true, true>;
    static constexpr int PARTS = SERVE_THREADS / S::THREADS;
    static constexpr int PART_LDS = S::EPB * 2 * S::BUF;   // values of T
    static constexpr size_t LDS_BYTES = (size_t)PARTS * PART_LDS * sizeof(T);
};

template <int NX, typename T, typename GT>
__device__ __forceinline__ void serve_part(const ServeAxSlot &S, int64_t wg, char *lds_raw, double *red) {
    using H = ServeShape<NX, T, GT>;
    constexpr int TH = H::S::THREADS;
    const int q = (int)threadIdx.x / TH;                  // H::PARTS: no part
    const int qc = q < H::PARTS ? q : H::PARTS - 1;
    const int tid = q < H::PARTS ? (int)threadIdx.x - q * TH : TH;
    const int64_t blk = (wg - S.block0) * H::PARTS + qc;
    ax_body<NX, T, GT, true, true>(blk, S.E, (kptr<T>)S.D, (gptr<const GT>)S.g, (gptr<double>)S.p,
                                   (gptr<double>)S.w, S.fz, tid, (T *)lds_raw + (size_t)qc * H::PART_LDS, red,
                                   qc * TH);
}

// The two merged kernels split the shapes by register need: B takes the FP64
// shapes whose own kernel holds fewer than four waves per SIMD (odd n from 9,
// and n >= 13), A everything else (at most 128 VGPRs, four waves per SIMD:
// the LDS of two n = 10 pencil workgroups, 35 KB, allows four workgroups per
// CU).  The served workload's degrees 5, 7, 9, 11 all run in A.
template <int NX, typename T>
constexpr bool serve_in_b() { return sizeof(T) == 8 && (NX >= 13 || NX == 9 || NX == 11); }

template <bool B, typename T, typename GT>
__device__ __forceinline__ void serve_dispatch(const ServeAxSlot &S, int64_t wg, char *lds, double *red) {
    switch (S.nx) {
#define NEK_SCASE(NX) \
    case NX:                                                        \
        if constexpr (serve_in_b<NX, T>() == B) serve_part<NX, T, GT>(S, wg, lds, red); \
        break;
        NEK_SCASE(2) NEK_SCASE(3) NEK_SCASE(4) NEK_SCASE(5) NEK_SCASE(6) NEK_SCASE(7) NEK_SCASE(8)
        NEK_SCASE(9) NEK_SCASE(10) NEK_SCASE(11) NEK_SCASE(12) NEK_SCASE(13) NEK_SCASE(14)
        NEK_SCASE(15) NEK_SCASE(16)
#undef NEK_SCASE
    default: break;
    }
}

template <bool B>
__device__ __forceinline__ void serve_body(const ServeAxSlot *__restrict__ slots, int nslots, char *lds,
                                           double *red)
{
    const ServeAxSlot &S = slots[batch_slot(slots, nslots, (int64_t)blockIdx.x)];
    switch (S.precision) {
    case NEK_PREC_F64: serve_dispatch<B, double, double>(S, blockIdx.x, lds, red); break;
    case NEK_PREC_F32G32: serve_dispatch<B, float, float>(S, blockIdx.x, lds, red); break;
    case NEK_PREC_F32GBF16: serve_dispatch<B, float, uint16_t>(S, blockIdx.x, lds, red); break;
    case NEK_PREC_F64G32: serve_dispatch<B, double, float>(S, blockIdx.x, lds, red); break;
    case NEK_PREC_F64GBF16: serve_dispatch<B, double, uint16_t>(S, blockIdx.x, lds, red); break;
    default: break;
    }
}

__global__ void __launch_bounds__(SERVE_THREADS, 4)
ax_serve_kernel(const ServeAxSlot *__restrict__ slots, int nslots)
{
    extern __shared__ __align__(16) char serve_lds[];
    __shared__ double red[SERVE_THREADS / 64];
    serve_body<false>(slots, nslots, serve_lds, red);
}

__global__ void __launch_bounds__(SERVE_THREADS, 2)
ax_serve_hi_kernel(const ServeAxSlot *__restrict__ slots, int nslots)
{
    extern __shared__ __align__(16) char serve_lds[];
    __shared__ double red[SERVE_THREADS / 64];
    serve_body<true>(slots, nslots, serve_lds, red);
}

template <int NX, typename T, typename GT>
void serve_shape_of(int64_t E, ServeAxShape &o) {
    using H = ServeShape<NX, T, GT>;
    const int64_t parts = (E + H::S::EPB - 1) / H::S::EPB;
    o.nparts = parts;
    o.blocks = (parts + H::PARTS - 1) / H::PARTS;
    o.lds_bytes = H::LDS_BYTES;
    o.hi = serve_in_b<NX, T>();
}

template <typename T, typename GT>
bool serve_shape_prec(int N, int64_t E, ServeAxShape &o) {
    switch (N + 1) {
#define NEK_HCASE(NX) \
    case NX: serve_shape_of<NX, T, GT>(E, o); return true;
        NEK_HCASE(2) NEK_HCASE(3) NEK_HCASE(4) NEK_HCASE(5) NEK_HCASE(6) NEK_HCASE(7) NEK_HCASE(8)
        NEK_HCASE(9) NEK_HCASE(10) NEK_HCASE(11) NEK_HCASE(12) NEK_HCASE(13) NEK_HCASE(14)
        NEK_HCASE(15) NEK_HCASE(16)
#undef NEK_HCASE
    default: return false;
    }
}

template <int NX, typename T, typename GT>
hipError_t launch_one(int64_t E, const T *D, const GT *g, double *p, double *w, const AxFuse &fz,
                      hipStream_t s)
{
    // the CG-fused form always works in the CG layout
    if (fz.sc != nullptr) {
        if (!fz.cg_layout) return hipErrorInvalidValue;
        using S = AxShapeFor<NX, T, true, true>;
        const int64_t blocks = (E + S::EPB - 1) / S::EPB;
        if (blocks > 0x7fffffff) return hipErrorInvalidValue;
        hipLaunchKernelGGL((ax_kernel<NX, T, GT, true, true>), dim3((unsigned)blocks), dim3(S::THREADS),
                           0, s, E, D, g, p, w, fz);
    } else if (fz.cg_layout) {
        if constexpr (sizeof(T) == 8) {
            using S = AxShapeFor<NX, T, false, true>;
            const int64_t blocks = (E + S::EPB - 1) / S::EPB;
            if (blocks > 0x7fffffff) return hipErrorInvalidValue;
            hipLaunchKernelGGL((ax_kernel<NX, T, GT, false, true>), dim3((unsigned)blocks),
                               dim3(S::THREADS), 0, s, E, D, g, p, w, fz);
        } else {
            return hipErrorInvalidValue;
        }
    } else {
        using S = AxShapeFor<NX, T, false, false>;
        const int64_t blocks = (E + S::EPB - 1) / S::EPB;
        if (blocks > 0x7fffffff) return hipErrorInvalidValue;
        hipLaunchKernelGGL((ax_kernel<NX, T, GT, false, false>), dim3((unsigned)blocks), dim3(S::THREADS),
                           0, s, E, D, g, p, w, fz);
    }
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

// g (six planes of n^3 per element) -> six values per point, point after point
__global__ void convert_g_kernel(int64_t E, int64_t n3, const double *__restrict__ g, int dtype,
                                 void *__restrict__ out) {
    const int64_t npts = E * n3;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npts; t += stride) {
        const int64_t e = t / n3, pt = t - e * n3;
        double v[6];
        for (int q = 0; q < 6; ++q) v[q] = g[(e * 6 + q) * n3 + pt];
        if (dtype == NEK_G_F32) {
            for (int q = 0; q < 6; ++q) ((float *)out)[t * 6 + q] = (float)v[q];
        } else {
            for (int q = 0; q < 3; ++q)
                ((uint32_t *)out)[t * 3 + q] = (uint32_t)f64_to_bf16(v[2 * q]) | ((uint32_t)f64_to_bf16(v[2 * q + 1]) << 16);
        }
    }
}

}  // namespace

bool serve_ax_shape(int N, int precision, int64_t E, ServeAxShape &out) {
    if (precision == NEK_PREC_F64) return serve_shape_prec<double, double>(N, E, out);
    if (precision == NEK_PREC_F32G32) return serve_shape_prec<float, float>(N, E, out);
    if (precision == NEK_PREC_F32GBF16) return serve_shape_prec<float, uint16_t>(N, E, out);
    if (precision == NEK_PREC_F64G32) return serve_shape_prec<double, float>(N, E, out);
    if (precision == NEK_PREC_F64GBF16) return serve_shape_prec<double, uint16_t>(N, E, out);
    return false;
}

hipError_t launch_ax_serve(const ServeAxSlot *slots, int nslots, int64_t blocks, size_t lds_bytes, bool hi,
                           hipStream_t s)
{
    if (nslots < 1 || nslots > BATCH_MAX_SLOTS || blocks < 1 || blocks > 0x7fffffff) return hipErrorInvalidValue;
    if (lds_bytes > 65536) {
        // n = 16 in FP64 takes 70 KB of the 160 KB of a CU: allowed once
        static const hipError_t attr = hipFuncSetAttribute((const void *)ax_serve_hi_kernel,
                                                           hipFuncAttributeMaxDynamicSharedMemorySize, 163840);
        if (attr != hipSuccess) return attr;
    }
    if (hi)
        hipLaunchKernelGGL(ax_serve_hi_kernel, dim3((unsigned)blocks), dim3(SERVE_THREADS), lds_bytes, s, slots,
                           nslots);
    else
        hipLaunchKernelGGL(ax_serve_kernel, dim3((unsigned)blocks), dim3(SERVE_THREADS), lds_bytes, s, slots,
                           nslots);
    return hipGetLastError();
}

hipError_t launch_ax_f64(int64_t E, int N, const double *D, const double *g, double *p, double *w,
                         const AxFuse &fz, hipStream_t s)
{
    return dispatch<double, double>(E, N, D, g, p, w, fz, s);
}

namespace {
template <int NX, typename GT>
hipError_t launch_fused_f64_glo(int64_t E, const double *D, const GT *g_lo, double *p, double *w, const AxFuse &fz,
                                hipStream_t s)
{
    using S = AxShapeFor<NX, double, true, true>;
    const int64_t blocks = (E + S::EPB - 1) / S::EPB;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((ax_kernel<NX, double, GT, true, true>), dim3((unsigned)blocks), dim3(S::THREADS), 0, s, E,
                       D, g_lo, p, w, fz);
    return hipGetLastError();
}

template <typename GT>
hipError_t dispatch_f64_glo(int64_t E, int N, const double *D, const GT *g_lo, double *p, double *w,
                            const AxFuse &fz, hipStream_t s)
{
    switch (N + 1) {
#define NEK_GCASE(NX) \
    case NX: return launch_fused_f64_glo<NX, GT>(E, D, g_lo, p, w, fz, s);
        NEK_GCASE(2) NEK_GCASE(3) NEK_GCASE(4) NEK_GCASE(5) NEK_GCASE(6) NEK_GCASE(7) NEK_GCASE(8)
        NEK_GCASE(9) NEK_GCASE(10) NEK_GCASE(11) NEK_GCASE(12) NEK_GCASE(13) NEK_GCASE(14)
        NEK_GCASE(15) NEK_GCASE(16)
#undef NEK_GCASE
    default: return hipErrorInvalidValue;
    }
}
}  // namespace

hipError_t launch_ax_f64_glo(int64_t E, int N, const double *D, const void *g_lo, int g_dtype, double *p,
                             double *w, const AxFuse &fz, hipStream_t s)
{
    if (fz.sc == nullptr || !fz.cg_layout) return hipErrorInvalidValue;   // the CG-fused form only
    if (g_dtype == NEK_G_F32) return dispatch_f64_glo<float>(E, N, D, (const float *)g_lo, p, w, fz, s);
    if (g_dtype == NEK_G_BF16) return dispatch_f64_glo<uint16_t>(E, N, D, (const uint16_t *)g_lo, p, w, fz, s);
    return hipErrorInvalidValue;
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

hipError_t launch_convert_g(int64_t E, int N, const double *g, int g_dtype, void *out, hipStream_t s)
{
    const int64_t n3 = n3_of(N);
    int64_t blocks = (E * n3 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(convert_g_kernel, dim3((unsigned)blocks), dim3(256), 0, s, E, n3, g, g_dtype, out);
    return hipGetLastError();
}

}  // namespace nek
