// cg_kernels.hip -- direct-stiffness summation with masking and the vector
// steps of unpreconditioned CG (Sec. III, Sec. V, Sec. VI-B), all on the device.
//
// Gather-scatter: nodes are grouped by copy count, each group stored as
// structure-of-arrays indices, so a thread handles one node with a fixed trip
// count and lanes load their indices coalesced.  Copies are summed in
// ascending local index (the oracle's order), masked nodes are written as 0.
// Inside the CG iteration the same rows feed the residual update directly
// (assemble-update): the assembled w is never written back.
//
// Vector steps: double2 loads, VEC_PAIRS pairs per thread issued together;
// the first-copy mask is one bit per point.
#include <algorithm>

#include "nek_internal.h"
#include "reduce.h"

namespace nek {
namespace {

typedef double dvec2 __attribute__((ext_vector_type(2)));

template <typename OwnPtr>
__device__ __forceinline__ unsigned own_pair(OwnPtr own, int64_t pt) {
    // bits of points pt, pt+1 (pt even)
    return (own[pt >> 5] >> (pt & 31)) & 3u;
}

// ---------------------------------------------------------------- dssum + mask
template <int C>
__device__ __forceinline__ void gs_row(gptr<const int32_t> idx, int32_t rows, int32_t row,
                                       gptr<double> w) {
    int32_t id[C];
#pragma unroll
    for (int m = 0; m < C; ++m) id[m] = idx[(int64_t)m * rows + row];
    double v[C];
#pragma unroll
    for (int m = 0; m < C; ++m) v[m] = w[id[m]];
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < C; ++m) s += v[m];
#pragma unroll
    for (int m = 0; m < C; ++m) w[id[m]] = s;
}

__device__ __forceinline__ void gs_vblock(const GsArgs &a, int vb, gptr<double> w) {
    int g = 0;
    while (g + 1 < a.ngroups && vb >= a.grp[g + 1].block0) ++g;
    const GsGroup &G = a.grp[g];
    const int32_t row = (vb - G.block0) * GS_THREADS + (int32_t)threadIdx.x;
    if (row >= G.rows) return;
    const gptr<const int32_t> idx = (gptr<const int32_t>)G.idx;
    switch (G.kind) {
    case 0: w[idx[row]] = 0.0; break;
    case 2: gs_row<2>(idx, G.rows, row, w); break;
    case 3: gs_row<3>(idx, G.rows, row, w); break;
    case 4: gs_row<4>(idx, G.rows, row, w); break;
    case 5: gs_row<5>(idx, G.rows, row, w); break;
    case 6: gs_row<6>(idx, G.rows, row, w); break;
    case 7: gs_row<7>(idx, G.rows, row, w); break;
    case 8: gs_row<8>(idx, G.rows, row, w); break;
    default: {   // CSR rows with many copies
        const gptr<const int32_t> off = (gptr<const int32_t>)G.off;
        const int32_t o0 = off[row], o1 = off[row + 1];
        double s = 0.0;
        for (int32_t o = o0; o < o1; ++o) s += w[idx[o]];
        for (int32_t o = o0; o < o1; ++o) w[idx[o]] = s;
    }
    }
}

constexpr int N_XCD = 8;   // gfx950: workgroups are dealt round-robin to 8 XCDs

// The standalone gather-scatter splits every group by XCD the same way (the
// groups are each ordered by element).
__global__ void __launch_bounds__(GS_THREADS) gs_kernel(GsArgs a, double *__restrict__ w) {
    const gptr<double> wg = (gptr<double>)w;
    const int lb = blockIdx.x, per = gridDim.x / N_XCD, xcd = lb % N_XCD, lq = lb / N_XCD;
    for (int g = 0; g < a.ngroups; ++g) {
        const GsGroup &G = a.grp[g];
        const int gb = (G.rows + GS_THREADS - 1) / GS_THREADS;
        const int u0 = G.block0 + (int)((long)gb * xcd / N_XCD);
        const int u1 = G.block0 + (int)((long)gb * (xcd + 1) / N_XCD);
        for (int vb = u0 + lq; vb < u1; vb += per) gs_vblock(a, vb, wg);
    }
}

// ---------------------------------------------------------------- CG steps
__global__ void cg_reset_kernel(CgScalars *sc, unsigned int *tickets, int nticket, int max_iter,
                                double rel_tol, double drop) {
    for (int q = threadIdx.x; q < nticket; q += blockDim.x) tickets[q] = 0u;
    if (threadIdx.x != 0) return;
    sc->bb = 0.0;
    sc->rho = 0.0;
    sc->rr = 0.0;
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
    sc->lag_applied = 1;
    sc->pad_[0] = sc->pad_[1] = sc->pad_[2] = 0;
}

// Pairs of a chunk: chunk c covers pairs [c * VEC_THREADS * VEC_PAIRS, ...);
// thread t takes pairs base + t + m * VEC_THREADS (m < VEC_PAIRS), pair q
// covering points 2q and 2q+1.  Workgroups stride over the chunks.
constexpr int64_t VEC_CHUNK = (int64_t)VEC_THREADS * VEC_PAIRS;

// the odd last point belongs to the last thread of the grid
__device__ __forceinline__ bool owns_tail(int64_t P) {
    return (P & 1) && blockIdx.x == gridDim.x - 1 && threadIdx.x == VEC_THREADS - 1;
}

template <typename OwnPtr>
__device__ __forceinline__ bool own_bit(OwnPtr own, int64_t t) {
    return (own[t >> 5] >> (t & 31)) & 1u;
}

#define NEK_CHUNKS                                                                       \
    for (int64_t base = blockIdx.x * VEC_CHUNK; base < npairs; base += (int64_t)gridDim.x * VEC_CHUNK)

// x = 0, r = b, p = z = M^-1 b (z = b without a preconditioner),
// bb = rr = (b, b), rho = (b, z)
template <bool PRE>
__global__ void __launch_bounds__(VEC_THREADS)
cg_init_kernel(int64_t P, const double *__restrict__ b, double *__restrict__ x,
               double *__restrict__ r, double *__restrict__ p, const uint32_t *__restrict__ own,
               const float *__restrict__ dinv, RedSite red, CgScalars *sc) {
    constexpr int K = PRE ? 2 : 1;
    __shared__ double lds[VEC_THREADS / 64];
    const int64_t npairs = P >> 1;
    double acc[K];
#pragma unroll
    for (int c = 0; c < K; ++c) acc[c] = 0.0;
    NEK_CHUNKS {
        double2 bv[VEC_PAIRS], zv[VEC_PAIRS];
#pragma unroll
        for (int m = 0; m < VEC_PAIRS; ++m) {
            const int64_t q = base + threadIdx.x + (int64_t)m * VEC_THREADS;
            if (q < npairs) {
                bv[m] = ((const double2 *)b)[q];
                if constexpr (PRE) {
                    const float2 df = ((const float2 *)dinv)[q];
                    const double2 dv = make_double2(df.x, df.y);
                    zv[m] = make_double2(dv.x * bv[m].x, dv.y * bv[m].y);
                } else {
                    zv[m] = bv[m];
                }
            }
        }
#pragma unroll
        for (int m = 0; m < VEC_PAIRS; ++m) {
            const int64_t q = base + threadIdx.x + (int64_t)m * VEC_THREADS;
            if (q < npairs) {
                ((double2 *)x)[q] = make_double2(0.0, 0.0);
                ((double2 *)r)[q] = bv[m];
                ((double2 *)p)[q] = zv[m];
                const unsigned o = own_pair(own, 2 * q);
                if (o & 1u) {
                    acc[0] += bv[m].x * bv[m].x;
                    if constexpr (PRE) acc[K - 1] += bv[m].x * zv[m].x;
                }
                if (o & 2u) {
                    acc[0] += bv[m].y * bv[m].y;
                    if constexpr (PRE) acc[K - 1] += bv[m].y * zv[m].y;
                }
            }
        }
    }
    if (owns_tail(P)) {
        const int64_t t = P - 1;
        const double bv = b[t];
        const double zv = PRE ? (double)dinv[t] * bv : bv;
        x[t] = 0.0;
        r[t] = bv;
        p[t] = zv;
        if (own_bit(own, t)) {
            acc[0] += bv * bv;
            if constexpr (PRE) acc[K - 1] += bv * zv;
        }
    }
    double s[K], tot[K];
#pragma unroll
    for (int c = 0; c < K; ++c) s[c] = block_sum<VEC_THREADS>(acc[c], lds);
    if (grid_finish_k<VEC_THREADS, K>(s, red, tot, lds, blockIdx.x, gridDim.x) && threadIdx.x == 0) {
        const double bb = tot[0];
        sc->bb = bb;
        sc->rr = bb;
        sc->rho = tot[K - 1];
        sc->rho_last_true = bb;
        sc->rel_tol2 = sc->rel_tol2 * bb;
        if (!(bb > 0.0)) {            // b = 0 (x = 0 is the solution) or non-finite
            sc->done = 1;
            if (!__builtin_isfinite(bb)) sc->status = NEK_ERR_BREAKDOWN;
        } else if (!__builtin_isfinite(tot[K - 1])) {
            sc->done = 1;
            sc->status = NEK_ERR_BREAKDOWN;
        }
        if (sc->max_iter <= 0) sc->done = 1;
    }
}

// ---------------------------------------------------------------- assemble-update
// One unmasked shared node with C copies: the assembled value of w is the sum
// of its copies (ascending local index), and r - alpha * sum goes to every
// copy of r (r is continuous, so its first copy stands for all).  The node's
// contribution to (r, r) and (r, M^-1 r) is taken once.
template <int C, bool PRE, typename WT>
__device__ __forceinline__ void asm_row(gptr<const int32_t> idx, int32_t rows, int32_t row,
                                        gptr<const WT> w, gptr<double> r, gptr<const float> dinv,
                                        double alpha, double *acc) {
    int32_t id[C];
#pragma unroll
    for (int m = 0; m < C; ++m) id[m] = idx[(int64_t)m * rows + row];
    double v[C];
#pragma unroll
    for (int m = 0; m < C; ++m) v[m] = (double)w[id[m]];
    const double rv = r[id[0]];
    double dv = 0.0;
    if constexpr (PRE) dv = dinv[id[0]];
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < C; ++m) s += v[m];
    const double nr = rv - alpha * s;
#pragma unroll
    for (int m = 0; m < C; ++m) r[id[m]] = nr;
    acc[0] += nr * nr;
    if constexpr (PRE) acc[1] += nr * (dv * nr);
}

template <bool PRE, typename WT>
__device__ __forceinline__ void asm_vblock(const GsArgs &a, int vb, gptr<const WT> w, gptr<double> r,
                                           gptr<const float> dinv, double alpha, double *acc) {
    int g = 0;
    while (g + 1 < a.ngroups && vb >= a.grp[g + 1].block0) ++g;
    const GsGroup &G = a.grp[g];
    const int32_t row = (vb - G.block0) * GS_THREADS + (int32_t)threadIdx.x;
    if (row >= G.rows) return;
    const gptr<const int32_t> idx = (gptr<const int32_t>)G.idx;
    switch (G.kind) {
    case 0: break;   // copies of masked nodes: r stays 0
    case 2: asm_row<2, PRE, WT>(idx, G.rows, row, w, r, dinv, alpha, acc); break;
    case 3: asm_row<3, PRE, WT>(idx, G.rows, row, w, r, dinv, alpha, acc); break;
    case 4: asm_row<4, PRE, WT>(idx, G.rows, row, w, r, dinv, alpha, acc); break;
    case 5: asm_row<5, PRE, WT>(idx, G.rows, row, w, r, dinv, alpha, acc); break;
    case 6: asm_row<6, PRE, WT>(idx, G.rows, row, w, r, dinv, alpha, acc); break;
    case 7: asm_row<7, PRE, WT>(idx, G.rows, row, w, r, dinv, alpha, acc); break;
    case 8: asm_row<8, PRE, WT>(idx, G.rows, row, w, r, dinv, alpha, acc); break;
    default: {   // CSR rows with many copies
        const gptr<const int32_t> off = (gptr<const int32_t>)G.off;
        const int32_t o0 = off[row], o1 = off[row + 1];
        double s = 0.0;
        for (int32_t o = o0; o < o1; ++o) s += (double)w[idx[o]];
        const int32_t first = idx[o0];
        const double nr = r[first] - alpha * s;
        for (int32_t o = o0; o < o1; ++o) r[idx[o]] = nr;
        acc[0] += nr * nr;
        if constexpr (PRE) acc[1] += nr * (dinv[first] * nr);
    }
    }
}

// A row of one of the common kinds (2 to 4 copies: faces and edges of a
// hexahedral mesh), split into its loads and its update so that the loads of
// several rows and of the other points are in flight together.
struct RowJob {
    int C = 0;                // copies; 0: no row
    int32_t id[4];
    double v[4];
    double rv = 0.0, dv = 0.0;
};

__device__ __forceinline__ bool fast_kind(int kind) { return kind >= 2 && kind <= 4; }

__device__ __forceinline__ void row_setup(const GsArgs &a, int vb, RowJob &J) {
    int g = 0;
    while (g + 1 < a.ngroups && vb >= a.grp[g + 1].block0) ++g;
    const GsGroup &G = a.grp[g];
    const int32_t row = (vb - G.block0) * GS_THREADS + (int32_t)threadIdx.x;
    J.C = (fast_kind(G.kind) && row < G.rows) ? G.kind : 0;
    const gptr<const int32_t> idx = (gptr<const int32_t>)G.idx;
#pragma unroll
    for (int m = 0; m < 4; ++m)
        if (m < J.C) J.id[m] = idx[(int64_t)m * G.rows + row];
}

template <bool PRE, typename WT>
__device__ __forceinline__ void row_load(RowJob &J, gptr<const WT> w, gptr<const double> r,
                                         gptr<const float> dinv) {
    if (J.C == 0) return;
#pragma unroll
    for (int m = 0; m < 4; ++m)
        if (m < J.C) J.v[m] = (double)w[J.id[m]];
    J.rv = r[J.id[0]];
    if constexpr (PRE) J.dv = dinv[J.id[0]];
}

template <bool PRE>
__device__ __forceinline__ void row_finish(const RowJob &J, gptr<double> r, double alpha, double *acc) {
    if (J.C == 0) return;
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m)
        if (m < J.C) s += J.v[m];
    const double nr = J.rv - alpha * s;
#pragma unroll
    for (int m = 0; m < 4; ++m)
        if (m < J.C) r[J.id[m]] = nr;
    acc[0] += nr * nr;
    if constexpr (PRE) acc[1] += nr * (J.dv * nr);
}

// The other points of one chunk of pairs: bits first, then values, then update.
template <bool PRE>
struct PairChunk {
    unsigned rb[VEC_PAIRS];
    double2 rv[VEC_PAIRS], wv[VEC_PAIRS], dv[VEC_PAIRS];
};

template <bool PRE>
__device__ __forceinline__ void chunk_bits(int64_t base, int64_t npairs, gptr<const uint32_t> rowed,
                                           PairChunk<PRE> &Q) {
#pragma unroll
    for (int m = 0; m < VEC_PAIRS; ++m) {
        const int64_t q = base + threadIdx.x + (int64_t)m * VEC_THREADS;
        Q.rb[m] = q < npairs ? own_pair(rowed, 2 * q) : 3u;
    }
}

template <bool PRE, typename WT>
__device__ __forceinline__ void chunk_load(int64_t base, gptr<const double> r, gptr<const WT> w,
                                           gptr<const float> dinv, PairChunk<PRE> &Q) {
#pragma unroll
    for (int m = 0; m < VEC_PAIRS; ++m) {
        const int64_t q = base + threadIdx.x + (int64_t)m * VEC_THREADS;
        if (Q.rb[m] != 3u) {
            Q.rv[m] = ((gptr<const double2>)r)[q];
            if constexpr (sizeof(WT) == 8) {
                Q.wv[m] = ((gptr<const double2>)w)[q];
            } else {
                const float2 wf = ((gptr<const float2>)w)[q];
                Q.wv[m] = make_double2(wf.x, wf.y);
            }
            if constexpr (PRE) {
                const float2 df = ((gptr<const float2>)dinv)[q];
                Q.dv[m] = make_double2(df.x, df.y);
            }
        }
    }
}

template <bool PRE>
__device__ __forceinline__ void chunk_finish(int64_t base, gptr<double> r, double alpha, const PairChunk<PRE> &Q,
                                             double *acc) {
    constexpr int K = PRE ? 2 : 1;
#pragma unroll
    for (int m = 0; m < VEC_PAIRS; ++m) {
        const int64_t q = base + threadIdx.x + (int64_t)m * VEC_THREADS;
        const unsigned rb = Q.rb[m];
        if (rb == 3u) continue;
        double2 nr;
        nr.x = Q.rv[m].x - alpha * Q.wv[m].x;
        nr.y = Q.rv[m].y - alpha * Q.wv[m].y;
        // a copy of a shared node belongs to its row (written there).  The
        // next read of r is the next operator launch, after the whole g
        // stream: the pairs bypass the caches (1% of a CG step).
        if (rb == 0u) {
            dvec2 t;
            t.x = nr.x;
            t.y = nr.y;
            __builtin_nontemporal_store(t, &((gptr<dvec2>)r)[q]);
        } else if (rb == 2u) {
            r[2 * q] = nr.x;
        } else {
            r[2 * q + 1] = nr.y;
        }
        if (!(rb & 1u)) {
            acc[0] += nr.x * nr.x;
            if constexpr (PRE) acc[K - 1] += nr.x * (Q.dv[m].x * nr.x);
        }
        if (!(rb & 2u)) {
            acc[0] += nr.y * nr.y;
            if constexpr (PRE) acc[K - 1] += nr.y * (Q.dv[m].y * nr.y);
        }
    }
}

// The CG step after the operator (see launch_cg_assemble_update).
//
// Work split: the workgroups on one XCD (index % 8) take one contiguous eighth
// of every row group and one contiguous eighth of the chunks of pairs, so an
// XCD works on about one eighth of the elements for all of them and the
// cache lines that rows and pairs share stay in its L2 (the row groups are
// each ordered by element; splitting their concatenation instead cost 25%).
//
// Every workgroup first puts in flight the loads that do not depend on
// anything: the operator's partials (for alpha), the indices of its first two
// row blocks of the common kinds and the bits of its first chunk of pairs;
// then the values those select; only then does it wait for alpha.  Further
// row blocks and chunks (large meshes), rows of rare kinds, then the
// reduction: rr = (r, r), rho' = (r, z), beta = rho' / rho, convergence on rr
// and the iteration cap.  lb / nb as in the gather-scatter.  WT: the type the
// operator stored w in (FP32 for the FP32 operator, which computes it in FP32:
// widening on the way in gives the same values as storing FP64).
template <bool PRE, typename WT>
__device__ __forceinline__ void assemble_update_body(int lb, int nb, int64_t P, const GsArgs &a,
                                                     gptr<const uint32_t> rowed, gptr<double> r,
                                                     gptr<const WT> w, gptr<const float> dinv,
                                                     gptr<const double> axparts, int64_t nparts,
                                                     const RedSite &red, gptr<CgScalars> sc) {
    constexpr int K = PRE ? 2 : 1;
    // partials loaded per thread at once (all of them up to E = 4096 at N = 9;
    // fewer with a preconditioner, whose chunk holds dinv too)
    constexpr int PPT = PRE ? 8 : 16;
    // A launch queued after the solve finished exits before its second round
    // of loads.  Thread 0 alone reads the flag, with the first loads in
    // flight, and passes it on through LDS: every wave of a workgroup takes
    // the same decision even when workgroup 0 of this launch flags a
    // breakdown meanwhile (every workgroup then finds the same breakdown
    // from the same partials).
    __shared__ int done_s;
    if (threadIdx.x == 0) done_s = sc->done;
    __shared__ double lds[VEC_THREADS / 64];
    __shared__ double alpha_s;
    __shared__ int breakdown;

    const int xcd = lb % N_XCD, per = nb / N_XCD, lq = lb / N_XCD;
    const int64_t npairs = P >> 1;
    // chunks: the workgroups of one XCD take one contiguous eighth
    const int64_t nch = (npairs + VEC_CHUNK - 1) / VEC_CHUNK;
    const int64_t c0 = nch * xcd / N_XCD, c1 = nch * (xcd + 1) / N_XCD;
    const int64_t base0 = (c0 + lq < c1) ? (c0 + lq) * VEC_CHUNK : npairs;
    // row blocks: of every group, the workgroups of one XCD take one contiguous eighth
    int vbl[2] = {-1, -1};
    {
        int found = 0;
        for (int g = 0; g < a.ngroups && found < 2; ++g) {
            const GsGroup &G = a.grp[g];
            if (!fast_kind(G.kind)) continue;
            const int gb = (G.rows + GS_THREADS - 1) / GS_THREADS;
            const int u0 = G.block0 + (int)((long)gb * xcd / N_XCD);
            const int u1 = G.block0 + (int)((long)gb * (xcd + 1) / N_XCD);
            for (int vb = u0 + lq; vb < u1 && found < 2; vb += per) vbl[found++] = vb;
        }
    }

    // ---- 1. independent loads
    double part[PPT];
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
        const int64_t q = threadIdx.x + (int64_t)m * VEC_THREADS;
        part[m] = q < nparts ? axparts[q] : 0.0;
    }
    RowJob J0, J1;
    if (vbl[0] >= 0) row_setup(a, vbl[0], J0);
    if (vbl[1] >= 0) row_setup(a, vbl[1], J1);
    PairChunk<PRE> Q;
    chunk_bits<PRE>(base0, npairs, rowed, Q);
    __syncthreads();
    if (done_s) return;

    // ---- 2. loads selected by the indices and bits
    row_load<PRE, WT>(J0, w, r, dinv);
    row_load<PRE, WT>(J1, w, r, dinv);
    chunk_load<PRE, WT>(base0, r, w, dinv, Q);

    // ---- 3. alpha = rho / (p, A p): every workgroup sums the partials in the
    // same order, so all of them hold the same alpha; workgroup 0 records it
    {
        double v = 0.0;
#pragma unroll
        for (int m = 0; m < PPT; ++m) v += part[m];
        for (int64_t q0 = (int64_t)PPT * VEC_THREADS; q0 < nparts; q0 += (int64_t)PPT * VEC_THREADS) {
            double more[PPT];
#pragma unroll
            for (int m = 0; m < PPT; ++m) {
                const int64_t q = q0 + threadIdx.x + (int64_t)m * VEC_THREADS;
                more[m] = q < nparts ? axparts[q] : 0.0;
            }
#pragma unroll
            for (int m = 0; m < PPT; ++m) v += more[m];
        }
        const double pw = block_sum<VEC_THREADS>(v, lds);
        if (threadIdx.x == 0) {
            const bool bad = !(pw > 0.0) || !__builtin_isfinite(pw);
            breakdown = bad ? 1 : 0;
            alpha_s = bad ? 0.0 : sc->rho / pw;
            if (lb == 0) {
                sc->pw = pw;
                sc->alpha = alpha_s;
                sc->lag_applied = bad ? 1 : 0;
                if (bad) {
                    sc->status = NEK_ERR_BREAKDOWN;
                    sc->done = 1;
                }
            }
        }
        __syncthreads();
    }
    if (breakdown) return;
    const double alpha = alpha_s;

    // ---- 4. updates of what is loaded, then the rest
    double acc[K];
#pragma unroll
    for (int c = 0; c < K; ++c) acc[c] = 0.0;
    row_finish<PRE>(J0, r, alpha, acc);
    row_finish<PRE>(J1, r, alpha, acc);
    chunk_finish<PRE>(base0, r, alpha, Q, acc);
    // Large meshes: the further row blocks and chunks, two at a time in
    // flight (the indices or bits of the next are loaded before the current
    // one is updated); the updates keep the order of a plain loop.
    {
        int seen = 0;   // row blocks of the common kinds past the first two
        RowJob cur;
        bool have = false;
        for (int g = 0; g < a.ngroups; ++g) {
            const GsGroup &G = a.grp[g];
            if (G.kind == 0) continue;
            const int gb = (G.rows + GS_THREADS - 1) / GS_THREADS;
            const int u0 = G.block0 + (int)((long)gb * xcd / N_XCD);
            const int u1 = G.block0 + (int)((long)gb * (xcd + 1) / N_XCD);
            for (int vb = u0 + lq; vb < u1; vb += per) {
                if (fast_kind(G.kind)) {
                    if (seen++ < 2) continue;
                    RowJob nx;
                    row_setup(a, vb, nx);
                    if (have) row_finish<PRE>(cur, r, alpha, acc);
                    row_load<PRE, WT>(nx, w, r, dinv);
                    cur = nx;
                    have = true;
                } else {   // rare kinds: corners of 8 elements, many-copy CSR rows
                    if (have) row_finish<PRE>(cur, r, alpha, acc);
                    have = false;
                    asm_vblock<PRE, WT>(a, vb, w, r, dinv, alpha, acc);
                }
            }
        }
        if (have) row_finish<PRE>(cur, r, alpha, acc);
    }
    {
        PairChunk<PRE> cur;
        int64_t cbase = -1;
        for (int64_t c = c0 + lq + per; c < c1; c += per) {
            const int64_t base = c * VEC_CHUNK;
            PairChunk<PRE> nx;
            chunk_bits<PRE>(base, npairs, rowed, nx);
            if (cbase >= 0) chunk_finish<PRE>(cbase, r, alpha, cur, acc);
            chunk_load<PRE, WT>(base, r, w, dinv, nx);
            cur = nx;
            cbase = base;
        }
        if (cbase >= 0) chunk_finish<PRE>(cbase, r, alpha, cur, acc);
    }
    if ((P & 1) && lb == nb - 1 && threadIdx.x == VEC_THREADS - 1) {
        const int64_t t = P - 1;
        if (!own_bit(rowed, t)) {
            const double nr = r[t] - alpha * (double)w[t];
            r[t] = nr;
            acc[0] += nr * nr;
            if constexpr (PRE) acc[K - 1] += nr * (dinv[t] * nr);
        }
    }
    double s[K], tot[K];
#pragma unroll
    for (int c = 0; c < K; ++c) s[c] = block_sum<VEC_THREADS>(acc[c], lds);
    if (grid_finish_k<VEC_THREADS, K>(s, red, tot, lds, lb, nb) && threadIdx.x == 0) {
        const double rr = tot[0], rz = tot[K - 1];
        sc->it += 1;
        if (!__builtin_isfinite(rr) || !__builtin_isfinite(rz)) {
            sc->status = NEK_ERR_BREAKDOWN;
            sc->done = 1;
        } else {
            sc->beta = rz / sc->rho;
            sc->rho = rz;
            sc->rr = rr;
            if (sc->rel_tol2 > 0.0 && rr <= sc->rel_tol2) {
                if (sc->drop2 > 0.0) sc->need_replace = 1;   // mixed: confirm with the true residual
                else sc->done = 1;
            }
            if (sc->drop2 > 0.0 && rr <= sc->drop2 * sc->rho_last_true) sc->need_replace = 1;
            if (rr == 0.0) sc->done = 1;
            if (sc->it >= sc->max_iter) sc->done = 1;
        }
    }
}

template <bool PRE, typename WT>
__global__ void __launch_bounds__(VEC_THREADS)
assemble_update_kernel(int64_t P, GsArgs a, const uint32_t *__restrict__ rowed, double *__restrict__ r,
                       const WT *__restrict__ w, const float *__restrict__ dinv,
                       const double *__restrict__ axparts, int64_t nparts, RedSite red, CgScalars *sc) {
    assemble_update_body<PRE, WT>(blockIdx.x, gridDim.x, P, a, (gptr<const uint32_t>)rowed, (gptr<double>)r,
                              (gptr<const WT>)w, (gptr<const float>)dinv,
                              (gptr<const double>)axparts, nparts, red, (gptr<CgScalars>)sc);
}

__global__ void __launch_bounds__(VEC_THREADS)
assemble_update_batch_kernel(const AsmSlot *__restrict__ slots, int nslots) {
    const AsmSlot &S = slots[batch_slot(slots, nslots, (int64_t)blockIdx.x)];
    const int lb = (int)((int64_t)blockIdx.x - S.block0);
    if (lb >= S.nblocks) return;
    if (S.w_f32)
        assemble_update_body<false, float>(lb, (int)S.nblocks, S.P, S.args, (gptr<const uint32_t>)S.rowed,
                                           (gptr<double>)S.r, (gptr<const float>)S.w, nullptr,
                                           (gptr<const double>)S.axparts, S.nparts, S.red, (gptr<CgScalars>)S.sc);
    else
        assemble_update_body<false, double>(lb, (int)S.nblocks, S.P, S.args, (gptr<const uint32_t>)S.rowed,
                                            (gptr<double>)S.r, (gptr<const double>)S.w, nullptr,
                                            (gptr<const double>)S.axparts, S.nparts, S.red, (gptr<CgScalars>)S.sc);
}

__global__ void __launch_bounds__(VEC_THREADS)
assemble_update_batch_karg_kernel(AsmKargTable t) {
    const int64_t blk = (int64_t)blockIdx.x;
    int i = 0;
#pragma unroll
    for (int k = 1; k < ASM_KARG_SLOTS; ++k) i += t.block0[k] <= blk ? 1 : 0;
    const AsmSlot &S = t.slot[i];
    // the slots tile the grid (checked by the launcher), so lb < S.nblocks
    // and every field of S is requested at once
    const int lb = (int)(blk - S.block0);
    if (S.w_f32)
        assemble_update_body<false, float>(lb, (int)S.nblocks, S.P, S.args, (gptr<const uint32_t>)S.rowed,
                                           (gptr<double>)S.r, (gptr<const float>)S.w, nullptr,
                                           (gptr<const double>)S.axparts, S.nparts, S.red, (gptr<CgScalars>)S.sc);
    else
        assemble_update_body<false, double>(lb, (int)S.nblocks, S.P, S.args, (gptr<const uint32_t>)S.rowed,
                                            (gptr<double>)S.r, (gptr<const double>)S.w, nullptr,
                                            (gptr<const double>)S.axparts, S.nparts, S.red, (gptr<CgScalars>)S.sc);
}

__global__ void gather_scalars_kernel(CgScalars *const *src, int n, CgScalars *dst) {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    static_assert(sizeof(CgScalars) % sizeof(u32x4) == 0, "CgScalars is copied in 16-byte pieces");
    constexpr int PIECES = sizeof(CgScalars) / sizeof(u32x4);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const gptr<const u32x4> from = (gptr<const u32x4>)src[i];
    const gptr<u32x4> to = (gptr<u32x4>)(dst + i);
#pragma unroll
    for (int q = 0; q < PIECES; ++q) to[q] = from[q];
}

// x += alpha p when the last alpha has not reached x yet (end of a solve,
// or before a true-residual evaluation)
__global__ void __launch_bounds__(VEC_THREADS)
cg_finish_kernel(int64_t P, double *__restrict__ x, const double *__restrict__ p,
                 const CgScalars *sc) {
    if (sc->lag_applied) return;
    const double alpha = sc->alpha;
    const int64_t npairs = P >> 1;
    NEK_CHUNKS {
#pragma unroll
        for (int m = 0; m < VEC_PAIRS; ++m) {
            const int64_t q = base + threadIdx.x + (int64_t)m * VEC_THREADS;
            if (q < npairs) {
                double2 xv = ((double2 *)x)[q];
                const double2 pv = ((const double2 *)p)[q];
                xv.x += alpha * pv.x;
                xv.y += alpha * pv.y;
                ((double2 *)x)[q] = xv;
            }
        }
    }
    if (owns_tail(P)) x[P - 1] += alpha * p[P - 1];
}

// reliable update: r = b - w (w = mask(dssum(A64 x)) with x current), rho = (r, r)
__global__ void __launch_bounds__(VEC_THREADS)
cg_replace_kernel(int64_t P, const double *__restrict__ b, const double *__restrict__ w,
                  double *__restrict__ r, const uint32_t *__restrict__ own, RedSite red,
                  CgScalars *sc) {
    __shared__ double lds[VEC_THREADS / 64];
    const int64_t npairs = P >> 1;
    double acc = 0.0;
    NEK_CHUNKS {
#pragma unroll
        for (int m = 0; m < VEC_PAIRS; ++m) {
            const int64_t q = base + threadIdx.x + (int64_t)m * VEC_THREADS;
            if (q < npairs) {
                const double2 bv = ((const double2 *)b)[q];
                const double2 wv = ((const double2 *)w)[q];
                const double2 nr = make_double2(bv.x - wv.x, bv.y - wv.y);
                ((double2 *)r)[q] = nr;
                const unsigned o = own_pair(own, 2 * q);
                if (o & 1u) acc += nr.x * nr.x;
                if (o & 2u) acc += nr.y * nr.y;
            }
        }
    }
    if (owns_tail(P)) {
        const int64_t t = P - 1;
        const double nr = b[t] - w[t];
        r[t] = nr;
        if (own_bit(own, t)) acc += nr * nr;
    }
    const double s = block_sum<VEC_THREADS>(acc, lds);
    double tot;
    if (grid_finish<VEC_THREADS>(s, red, &tot, lds) && threadIdx.x == 0) {
        // the next direction p <- r + beta p takes the replaced r, so beta takes
        // its (r, r) too: beta = (r, r)_true / rho_old, where the last update
        // left beta = (r, r)_recurrence / rho_old and rr = (r, r)_recurrence.
        // (With beta from the recurrence, BF16 g needed 9% more iterations in a
        // model of this solve at 8^3 elements, N = 9.)
        const double rr_rec = sc->rr;
        if (rr_rec > 0.0 && __builtin_isfinite(tot)) sc->beta = sc->beta * (tot / rr_rec);
        sc->rho = tot;
        sc->rr = tot;
        sc->rho_last_true = tot;
        sc->need_replace = 0;
        sc->n_replace += 1;
        sc->lag_applied = 1;          // the caller brought x up to date before this
        if (!__builtin_isfinite(tot)) {
            sc->status = NEK_ERR_BREAKDOWN;
            sc->done = 1;
        } else if (sc->rel_tol2 > 0.0 && tot <= sc->rel_tol2) {
            sc->done = 1;
        }
    }
}

template <bool DIFF>
__global__ void __launch_bounds__(VEC_THREADS)
gdot_kernel(int64_t P, const double *__restrict__ a, const double *__restrict__ b,
            const uint32_t *__restrict__ own, RedSite red, double *result) {
    __shared__ double lds[VEC_THREADS / 64];
    const int64_t npairs = P >> 1;
    double acc = 0.0;
    NEK_CHUNKS {
#pragma unroll
        for (int m = 0; m < VEC_PAIRS; ++m) {
            const int64_t q = base + threadIdx.x + (int64_t)m * VEC_THREADS;
            if (q < npairs) {
                const double2 av = ((const double2 *)a)[q];
                const double2 bv = ((const double2 *)b)[q];
                const unsigned o = own_pair(own, 2 * q);
                const double t0 = DIFF ? (av.x - bv.x) * (av.x - bv.x) : av.x * bv.x;
                const double t1 = DIFF ? (av.y - bv.y) * (av.y - bv.y) : av.y * bv.y;
                if (o & 1u) acc += t0;
                if (o & 2u) acc += t1;
            }
        }
    }
    if (owns_tail(P)) {
        const int64_t t = P - 1;
        const double t0 = DIFF ? (a[t] - b[t]) * (a[t] - b[t]) : a[t] * b[t];
        if (own_bit(own, t)) acc += t0;
    }
    const double s = block_sum<VEC_THREADS>(acc, lds);
    double tot;
    if (grid_finish<VEC_THREADS>(s, red, &tot, lds) && threadIdx.x == 0) *result = tot;
}

// ---------------------------------------------------------------- layout conversion
constexpr int PERM_THREADS = 256;
constexpr int64_t PERM_MAX_BLOCKS = 65536;

// Workgroups stride over elements; threads over an element's points in the
// order of Listing 1 (coalesced on that side).
template <typename DT>
__global__ void __launch_bounds__(PERM_THREADS)
permute_kernel(int64_t E, int n, const double *__restrict__ src, DT *__restrict__ dst, bool to_cg) {
    const int n3 = n * n * n;
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        const int64_t base = e * n3;
        for (int l = threadIdx.x; l < n3; l += PERM_THREADS) {
            const int nn = n * n, k = l / nn, ij = l - k * nn;
            const int64_t c = base + k * nn + cgl_col(ij % n, ij / n, n);
            if (to_cg) dst[c] = (DT)src[base + l];
            else dst[base + l] = (DT)src[c];
        }
    }
}

}  // namespace

hipError_t launch_permute(int64_t E, int N, const double *src, double *dst, bool to_cg, hipStream_t s) {
    if (E < 1) return hipSuccess;
    const int64_t blocks = E < PERM_MAX_BLOCKS ? E : PERM_MAX_BLOCKS;
    hipLaunchKernelGGL(permute_kernel<double>, dim3((unsigned)blocks), dim3(PERM_THREADS), 0, s, E, N + 1, src,
                       dst, to_cg);
    return hipGetLastError();
}

hipError_t launch_permute_to_cg_f32(int64_t E, int N, const double *src, float *dst, hipStream_t s) {
    if (E < 1) return hipSuccess;
    const int64_t blocks = E < PERM_MAX_BLOCKS ? E : PERM_MAX_BLOCKS;
    hipLaunchKernelGGL(permute_kernel<float>, dim3((unsigned)blocks), dim3(PERM_THREADS), 0, s, E, N + 1, src,
                       dst, true);
    return hipGetLastError();
}

int64_t vec_blocks(int64_t P) {
    const int64_t per = (int64_t)VEC_THREADS * VEC_PAIRS * 2;
    int64_t nb = (P + per - 1) / per;
    if (nb > RED_MAX_BLOCKS) nb = RED_MAX_BLOCKS;
    return nb < 1 ? 1 : nb;
}

int64_t gs_grid(const GsDevice &gs) {
    int64_t g = gs.args.nblocks < RED_MAX_BLOCKS ? gs.args.nblocks : RED_MAX_BLOCKS;
    g = (g + N_XCD - 1) / N_XCD * N_XCD;
    return g < N_XCD ? N_XCD : g;
}

hipError_t launch_gs(const GsDevice &gs, double *w, hipStream_t s) {
    if (gs.args.nblocks == 0) return hipSuccess;
    hipLaunchKernelGGL(gs_kernel, dim3((unsigned)gs_grid(gs)), dim3(GS_THREADS), 0, s, gs.args, w);
    return hipGetLastError();
}

static_assert(GS_THREADS == VEC_THREADS, "assemble-update takes one row per thread of a virtual block");

int64_t asm_blocks(const GsDevice &gs) {
    int64_t g = std::max(vec_blocks(gs.P), gs_grid(gs));
    g = (g + N_XCD - 1) / N_XCD * N_XCD;
    return g > RED_MAX_BLOCKS ? RED_MAX_BLOCKS : g;
}

hipError_t launch_cg_assemble_update(const GsDevice &gs, double *r, const double *w, bool w_f32, const float *dinv,
                                     const double *axparts, int64_t nparts, const RedSite &red,
                                     CgScalars *sc, hipStream_t s) {
    const dim3 grid((unsigned)asm_blocks(gs));
    if (w_f32 && dinv != nullptr) return hipErrorInvalidValue;   // the preconditioned CG is FP64 only
    if (dinv != nullptr)
        hipLaunchKernelGGL((assemble_update_kernel<true, double>), grid, dim3(VEC_THREADS), 0, s, gs.P, gs.args,
                           gs.rowed_bits, r, w, dinv, axparts, nparts, red, sc);
    else if (w_f32)
        hipLaunchKernelGGL((assemble_update_kernel<false, float>), grid, dim3(VEC_THREADS), 0, s, gs.P, gs.args,
                           gs.rowed_bits, r, (const float *)w, dinv, axparts, nparts, red, sc);
    else
        hipLaunchKernelGGL((assemble_update_kernel<false, double>), grid, dim3(VEC_THREADS), 0, s, gs.P, gs.args,
                           gs.rowed_bits, r, w, dinv, axparts, nparts, red, sc);
    return hipGetLastError();
}

hipError_t launch_assemble_update_batch(const AsmSlot *slots, int nslots, int64_t blocks, hipStream_t s) {
    if (nslots < 1 || nslots > BATCH_MAX_SLOTS || blocks < 1 || blocks > 0x7fffffff)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(assemble_update_batch_kernel, dim3((unsigned)blocks), dim3(VEC_THREADS), 0, s, slots,
                       nslots);
    return hipGetLastError();
}

hipError_t launch_assemble_update_batch_karg(const AsmSlot *slots, int nslots, int64_t blocks, hipStream_t s) {
    if (nslots < 1 || nslots > ASM_KARG_SLOTS || blocks < 1 || blocks > 0x7fffffff || slots[0].block0 != 0)
        return hipErrorInvalidValue;
    for (int k = 0; k < nslots; ++k) {
        const int64_t end = k + 1 < nslots ? slots[k + 1].block0 : blocks;
        if (slots[k].nblocks < 1 || slots[k].block0 + slots[k].nblocks != end) return hipErrorInvalidValue;
    }
    AsmKargTable t;
    for (int k = 0; k < ASM_KARG_SLOTS; ++k) {
        t.block0[k] = k < nslots ? slots[k].block0 : INT64_MAX;
        t.slot[k] = slots[k < nslots ? k : nslots - 1];
    }
    hipLaunchKernelGGL(assemble_update_batch_karg_kernel, dim3((unsigned)blocks), dim3(VEC_THREADS), 0, s, t);
    return hipGetLastError();
}

hipError_t launch_gather_scalars(CgScalars *const *src, int n, CgScalars *dst, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_scalars_kernel, dim3((n + 63) / 64), dim3(64), 0, s, src, n, dst);
    return hipGetLastError();
}

hipError_t launch_cg_reset(CgScalars *sc, unsigned int *tickets, int nticket, int max_iter,
                           double rel_tol, double drop, hipStream_t s) {
    hipLaunchKernelGGL(cg_reset_kernel, dim3(1), dim3(256), 0, s, sc, tickets, nticket, max_iter,
                       rel_tol, drop);
    return hipGetLastError();
}

hipError_t launch_cg_init(int64_t P, const double *b, double *x, double *r, double *p,
                          const uint32_t *own, const float *dinv, const RedSite &red, CgScalars *sc,
                          hipStream_t s) {
    if (dinv != nullptr)
        hipLaunchKernelGGL(cg_init_kernel<true>, dim3((unsigned)vec_blocks(P)), dim3(VEC_THREADS), 0, s,
                           P, b, x, r, p, own, dinv, red, sc);
    else
        hipLaunchKernelGGL(cg_init_kernel<false>, dim3((unsigned)vec_blocks(P)), dim3(VEC_THREADS), 0, s,
                           P, b, x, r, p, own, dinv, red, sc);
    return hipGetLastError();
}

hipError_t launch_cg_finish(int64_t P, double *x, const double *p, const CgScalars *sc, hipStream_t s) {
    hipLaunchKernelGGL(cg_finish_kernel, dim3((unsigned)vec_blocks(P)), dim3(VEC_THREADS), 0, s, P, x,
                       p, sc);
    return hipGetLastError();
}

hipError_t launch_cg_replace(int64_t P, const double *b, const double *w, double *r,
                             const uint32_t *own, const RedSite &red, CgScalars *sc, hipStream_t s) {
    hipLaunchKernelGGL(cg_replace_kernel, dim3((unsigned)vec_blocks(P)), dim3(VEC_THREADS), 0, s, P, b,
                       w, r, own, red, sc);
    return hipGetLastError();
}

hipError_t launch_gdot(int64_t P, const double *a, const double *b, const uint32_t *own,
                       const RedSite &red, double *result, hipStream_t s) {
    hipLaunchKernelGGL(gdot_kernel<false>, dim3((unsigned)vec_blocks(P)), dim3(VEC_THREADS), 0, s, P, a,
                       b, own, red, result);
    return hipGetLastError();
}

hipError_t launch_gdiff2(int64_t P, const double *a, const double *b, const uint32_t *own,
                         const RedSite &red, double *result, hipStream_t s) {
    hipLaunchKernelGGL(gdot_kernel<true>, dim3((unsigned)vec_blocks(P)), dim3(VEC_THREADS), 0, s, P, a,
                       b, own, red, result);
    return hipGetLastError();
}

}  // namespace nek
