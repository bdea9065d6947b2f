// Internal declarations shared by the libnek translation units (not part of
// the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "nek.h"
#include "reduce.h"

namespace nek {

// thread-local error text; returns code for convenient `return fail(...)`
int fail(int code, const std::string &msg);
void clear_error();
int check_hip(hipError_t e, const char *what);

#define NEK_HIP(call)                                                   \
    do {                                                                \
        hipError_t _e = (call);                                         \
        if (_e != hipSuccess) return ::nek::check_hip(_e, #call);       \
    } while (0)

inline bool aligned8(const void *p) { return ((uintptr_t)p & 7u) == 0; }

inline int64_t n3_of(int N) { return (int64_t)(N + 1) * (N + 1) * (N + 1); }

// ---------------------------------------------------------------- CG layout
// Inside the CG every local vector (x, r, p, w, b, M^-1) is stored in the "CG
// layout": element by element and layer k by layer k as in Listing 1, but
// within a layer first the points with 0 < i < n-1 (i fastest, then j), then
// the n points with i = 0, then the n points with i = n-1 (each in j order).
// The faces at fixed i, which the gather-scatter reads and writes most, become
// n runs of n contiguous values instead of n^2 values at stride n; the faces
// at fixed j and k stay runs of at least n-2.  A column (i, j) keeps the
// stride n^2 in k.  The user's b and x keep the layout of Listing 1; the
// solver converts on the way in and out.
// Offset of (i, j, k) within an element: k n^2 + cgl_col(i, j, n).
__host__ __device__ inline int cgl_col(int i, int j, int n) {
    return i == 0 ? n * (n - 2) + j : (i == n - 1 ? n * (n - 1) + j : j * (n - 2) + i - 1);
}

// ---------------------------------------------------------------- CG scalars
// Device-side CG state (one struct in device memory, written only by the
// last workgroup of a reduction kernel or by single-thread kernels).
struct CgScalars {
    double bb;            // (b, b)
    double rho;           // (r, r) of the current residual; (r, M^-1 r) with a preconditioner
    double rr;            // (r, r) of the current residual (the stopping test)
    double pw;            // (p, w)
    double alpha;
    double beta;
    double rel_tol2;      // rel_tol^2 * bb, 0 for fixed iterations
    double rho_last_true; // rho at the last reliable replacement
    double drop2;         // reliable_drop^2 (0: FP64 mode)
    int it;               // iterations completed
    int max_iter;
    int done;             // 1: converged, breakdown or max_iter reached
    int status;           // NEK_OK / NEK_ERR_BREAKDOWN
    int need_replace;     // mixed precision: r should be replaced by b - A64 x
    int n_replace;
    int lag_applied;      // 0: x still lacks alpha * p of the last (p, w)
    int pad_[3];          // size a multiple of 16 bytes
};

// Mixed precision: r is replaced by the FP64 true residual once ||r|| has
// fallen by this factor since the last replacement.  Measured at E = 4096,
// N = 9 (manufactured solution, to 1e-10): with BF16 g, 0.3 takes 1324
// iterations and 0.1 1412; with FP32 g both take 1148, and 0.1 needs 11
// replacements instead of 19 (0.8% less time).
// With FP64 arithmetic on FP32 g the operator is within FP32 rounding of g
// of the FP64 one, and the true residual follows the recurrence's until far
// below: 1e-3 needs 4 replacements to 1e-10 where 0.3 needs 19, for the same
// iterations.
inline double reliable_drop_default(int precision) {
    return precision == NEK_PREC_F32G32 ? 0.1 : (precision == NEK_PREC_F64G32 ? 1e-3 : 0.3);
}

// ---------------------------------------------------------------- ax_e
// Optional CG fusion of the local-operator launch (all device pointers):
//   r != null : p <- r + beta p on the way in (beta from sc);
//   dinv != null (with r) : p <- dinv r + beta p (Jacobi-preconditioned CG;
//                           dinv held in FP32);
//   x != null : x += alpha p_old first, if sc->lag_applied == 0;
//   partials != null : per-workgroup sum of p * (A_L p) over all local
//                      points, at partials[blockIdx] (the assemble-update
//                      launch that follows turns them into alpha);
//   sc != null : skip everything once sc->done is set.
struct AxFuse {
    const double *r = nullptr;
    double *x = nullptr;
    double *partials = nullptr;
    const CgScalars *sc = nullptr;
    const float *dinv = nullptr;
    // vectors p, r, x, dinv and w in the CG layout.  Always the case with
    // sc != null; without it, FP64 only (the true residual of a CG).
    bool cg_layout = false;
};

hipError_t launch_ax_f64(int64_t E, int N, const double *D, const double *g, double *p, double *w,
                         const AxFuse &fz, hipStream_t s);
hipError_t launch_ax_f32(int64_t E, int N, const float *D32, const void *g_lo, int g_dtype,
                         double *p, double *w, const AxFuse &fz, hipStream_t s);
// The CG-fused operator in FP64 arithmetic on factors stored in FP32 or BF16
// (g_lo from nek_convert_g; NEK_PREC_F64G*); AxFuse as for the CG (sc set,
// CG layout); w in FP64.
hipError_t launch_ax_f64_glo(int64_t E, int N, const double *D, const void *g_lo, int g_dtype, double *p,
                             double *w, const AxFuse &fz, hipStream_t s);
// The CG-fused operator with one thread per node, for small meshes
// (cg_node_kernels.hip): same arguments and results as launch_ax_f64 with a
// CG AxFuse, for N = 3..9 and at most AX_NODE_MAX_POINTS local points
// (ax_node_fused_fits); it leaves one partial of (p, A_L p) per element.
// Measured against the pencil operator (CG iteration time): 10-19% faster
// at E = 64..512 for N = 3..6, 5-13% up to E = 256 at N = 7, 8, 9 and at
// E = 512 for N = 7, 8 (262 144 and 373 248 points), even near the bound at
// lower degrees; 2% slower at E = 512, N = 9 (512 000 points).
#ifdef NEK_AX_NODE_MIN_N
constexpr int AX_NODE_MIN_N = NEK_AX_NODE_MIN_N;
#else
constexpr int AX_NODE_MIN_N = 3;
#endif
#ifdef NEK_AX_NODE_MAX_POINTS
constexpr int64_t AX_NODE_MAX_POINTS = NEK_AX_NODE_MAX_POINTS;
#else
constexpr int64_t AX_NODE_MAX_POINTS = 400000;
#endif
bool ax_node_fused_fits(int64_t E, int N);
hipError_t launch_ax_node_fused(int64_t E, int N, const double *D, const double *g, double *p, double *w,
                                const AxFuse &fz, hipStream_t s);
// the comparison designs of nek_ax_variant (ORIGINAL needs a scratch of 3P doubles)
hipError_t launch_ax_variant(int variant, int64_t E, int N, const double *D, const double *g, const double *u,
                             double *w, double *scratch, hipStream_t s);
// number of workgroups of an ax launch (one partial each)
int64_t ax_blocks(int64_t E, int N);

// ---------------------------------------------------------------- batched launches
// A launch that serves several solves gives each one a contiguous range of
// workgroups, described by a table of slots sorted by block0 (slots[0].block0
// is 0).  At most BATCH_MAX_SLOTS slots share a launch.
constexpr int BATCH_MAX_SLOTS = 64;

// Slot owning workgroup blk.  Every lane of the (full, 64-lane) wave loads one
// slot's block0 and a ballot counts the slots starting at or before blk: one
// load per workgroup instead of a chain of dependent ones.  The result is
// uniform across the wave.
template <typename Slot>
__device__ __forceinline__ int batch_slot(const Slot *__restrict__ slots, int nslots, int64_t blk) {
    const int lane = (int)(threadIdx.x & 63u);
    const bool before = lane < nslots && slots[lane].block0 <= blk;
    return __popcll(__ballot(before)) - 1;
}

// One solve in a merged operator launch of the served form (any degree and
// precision; see ax_serve_kernel).
constexpr int SERVE_THREADS = 256;
struct ServeAxSlot {
    int64_t block0;      // first workgroup of this solve in the launch
    int64_t E;
    int nx;              // N + 1
    int precision;       // NEK_PREC_*
    const void *D;       // double or float, by precision
    const void *g;       // FP64 g, or the paired FP32 / BF16 copy
    double *p;
    double *w;
    AxFuse fz;
};
// A solve's share of a merged operator launch: its workgroups, the partials
// it leaves (those of its own launch, ax_blocks), the LDS its workgroups use
// and which of the two merged kernels runs it (hi: the FP64 shapes that need
// more registers than four waves per SIMD allow; see ax_serve_kernel).
struct ServeAxShape {
    int64_t blocks = 0;
    int64_t nparts = 0;
    size_t lds_bytes = 0;
    bool hi = false;
};
bool serve_ax_shape(int N, int precision, int64_t E, ServeAxShape &out);
hipError_t launch_ax_serve(const ServeAxSlot *slots, int nslots, int64_t blocks, size_t lds_bytes, bool hi,
                           hipStream_t s);

// The one-thread-per-node operator of the served form: every small FP64
// solve (ax_node_fused_fits) in one launch of 1024-thread workgroups, each
// holding 1024 / node_threads parts (elements); part q of workgroup b is
// element (b - block0) * parts + q of the solve, with the partial of the
// solve's own launch.
constexpr int SERVE_NODE_THREADS = 1024;
struct ServeNodeSlot {
    int64_t block0;
    int64_t E;
    int nx;
    int pad_;
    const double *D;
    const double *g;
    double *p;
    double *w;
    AxFuse fz;
};
struct ServeNodeShape {
    int64_t blocks = 0;
    size_t lds_bytes = 0;
    bool n9 = false;     // n = 9 runs in a kernel of its own (more registers)
};
bool serve_node_shape(int N, int64_t E, ServeNodeShape &out);
hipError_t launch_ax_node_serve(const ServeNodeSlot *slots, int nslots, int64_t blocks, size_t lds_bytes, bool n9,
                                hipStream_t s);

hipError_t launch_convert_g(int64_t E, int N, const double *g, int g_dtype, void *out, hipStream_t s);

// ---------------------------------------------------------------- gather-scatter
// Nodes handled by the gather-scatter are grouped by their number of copies.
// A group of c copies stores its rows as structure-of-arrays indices:
// idx[m * rows + row] is the m-th copy (ascending local index) of the row.
// Group kind 0 lists the copies of masked nodes (written as 0).  Rows with
// more than GS_MAXC copies go to a CSR group.  Unmasked nodes with a single
// copy need no work and are not listed.
constexpr int GS_MAXC = 8;
constexpr int GS_THREADS = 256;

struct GsGroup {
    int kind;           // 0: zero list; 2..GS_MAXC: copies per row; -1: CSR
    int32_t rows;       // rows (or entries of the zero list)
    int32_t block0;     // first workgroup of this group
    const int32_t *idx; // SoA indices / zero list / CSR entries
    const int32_t *off; // CSR offsets (kind -1)
};

constexpr int GS_MAXG = GS_MAXC + 2;

struct GsArgs {
    int ngroups;
    int nblocks;
    GsGroup grp[GS_MAXG];
};

// Host image of a gather-scatter map (built on the host, uploaded into one
// device arena: the int32 index arrays, then the first-copy bits).
struct GsHostGroup {
    int kind;
    int32_t rows;
    size_t idx_at;   // offset of the group's indices in idx (int32 units)
    size_t off_at;   // CSR offsets (kind -1)
};
struct GsHost {
    int64_t E = 0;
    int N = 0;
    int64_t P = 0, U = 0, n_rows = 0, n_entries = 0, n_masked = 0, n_zero = 0;
    std::vector<int32_t> idx;
    std::vector<GsHostGroup> groups;
    std::vector<uint32_t> own;
    std::vector<uint32_t> rowed;   // P bits: copy of a shared node or of a masked node
    size_t idx_bytes() const { return ((idx.size() * sizeof(int32_t) + 4) + 255) & ~(size_t)255; }
    size_t own_bytes() const { return ((own.size() * sizeof(uint32_t)) + 255) & ~(size_t)255; }
    size_t arena_bytes() const { return idx_bytes() + own_bytes() + rowed.size() * sizeof(uint32_t); }
};

// Build the host image from glo[P] / dirichlet[P] (NULL = none); returns
// NEK_OK or an error code with msg set.
// cg_layout: index the copies by their position in the CG layout.
int gs_build_host(int64_t E, int N, const int64_t *glo, const uint8_t *dirichlet, bool cg_layout,
                  GsHost &out, std::string &msg);

struct GsDevice;
// Point a device handle at an arena that holds (or will hold) h's image: the
// index arrays at the start, then the first-copy bits, then the bits of the
// points that are copies of shared or masked nodes (h.idx_bytes() and
// h.own_bytes() give the offsets).
void gs_attach(const GsHost &h, void *arena, GsDevice &d);

struct GsDevice {
    int64_t E = 0;
    int N = 0;
    int64_t P = 0;
    int64_t n_unique = 0;
    int64_t n_rows = 0;      // unmasked shared nodes summed by the gather-scatter
    int64_t n_entries = 0;   // copies of those nodes
    int64_t n_masked = 0;    // masked unique nodes
    int64_t n_zero = 0;      // copies of masked nodes
    GsArgs args{};
    void *arena = nullptr;   // one allocation holding every index array
    uint32_t *own_bits = nullptr;    // P bits: first copy of every node
    uint32_t *rowed_bits = nullptr;  // P bits: copy of a shared or of a masked node
};

// dssum + mask in place
hipError_t launch_gs(const GsDevice &gs, double *w, hipStream_t s);
int64_t gs_grid(const GsDevice &gs);   // a multiple of 8

// ---------------------------------------------------------------- CG vector steps
constexpr int VEC_THREADS = 256;
constexpr int VEC_PAIRS = 4;            // double2 per thread per chunk
int64_t vec_blocks(int64_t P);          // workgroups of the vector kernels (<= RED_MAX_BLOCKS)

hipError_t launch_cg_reset(CgScalars *sc, unsigned int *tickets, int nticket, int max_iter,
                           double rel_tol, double drop, hipStream_t s);
// dinv (may be null): the Jacobi preconditioner M^-1 as a continuous local
// vector, in FP32 (a fixed SPD diagonal: its rounding changes the
// preconditioner, not the system solved)
hipError_t launch_cg_init(int64_t P, const double *b, double *x, double *r, double *p,
                          const uint32_t *own, const float *dinv, const RedSite &red, CgScalars *sc,
                          hipStream_t s);
// The CG step after the operator, with the dssum folded in: w holds the
// unassembled A_L p.  For every unmasked shared node the copies of w are
// summed (ascending local index, as nek_dssum does) and r <- r - alpha * sum
// is written to every copy of r; every unshared unmasked point gets
// r <- r - alpha w; copies of masked nodes are left alone (r is 0 there).
// Then rr = (r, r), rho' = (r, z) with z = M^-1 r, beta, convergence.  The
// assembled w itself is never stored.  alpha = rho / (p, A p), from the nparts
// per-workgroup partials of (p, A_L p) left by the ax launch, summed in index
// order by every workgroup (workgroup 0 records it, or flags a breakdown).
// w_f32: w holds FP32 values (the FP32 operator of the mixed form stores its
// FP32 result as it is; FP64 only without a preconditioner).
hipError_t launch_cg_assemble_update(const GsDevice &gs, double *r, const double *w, bool w_f32,
                                     const float *dinv, const double *axparts, int64_t nparts,
                                     const RedSite &red, CgScalars *sc, hipStream_t s);
int64_t asm_blocks(const GsDevice &gs);   // its grid: a multiple of 8, <= RED_MAX_BLOCKS

struct AsmSlot {
    int64_t block0;      // a multiple of 8, so a slot's workgroups keep their XCD order
    int64_t nblocks;     // asm_blocks of this solve
    int64_t P;
    GsArgs args;
    const uint32_t *rowed;
    double *r;
    const double *w;     // FP32 values when w_f32 (the FP32 operator's output)
    const double *axparts;
    int64_t nparts;
    RedSite red;
    CgScalars *sc;
    int w_f32;
};
hipError_t launch_assemble_update_batch(const AsmSlot *slots, int nslots, int64_t blocks, hipStream_t s);
// The same launch with the slots passed by value among the kernel arguments
// (at most ASM_KARG_SLOTS of them): a workgroup then finds its slot without
// first reading the device table, and takes every field of it in one round
// trip.  `slots` is a host array, read at the call; the slots must tile the
// grid (slot k's workgroups end where slot k+1's begin, the last at `blocks`).
constexpr int ASM_KARG_SLOTS = 8;
struct AsmKargTable {
    int64_t block0[ASM_KARG_SLOTS];   // slots[i].block0, unused entries INT64_MAX
    AsmSlot slot[ASM_KARG_SLOTS];
};
static_assert(sizeof(AsmKargTable) <= 4096, "kernel arguments are limited to 4 KiB");
hipError_t launch_assemble_update_batch_karg(const AsmSlot *slots, int nslots, int64_t blocks, hipStream_t s);

// copy the scalars of several solves into one contiguous array
hipError_t launch_gather_scalars(CgScalars *const *src, int n, CgScalars *dst, hipStream_t s);
hipError_t launch_cg_finish(int64_t P, double *x, const double *p, const CgScalars *sc, hipStream_t s);
// dst <- src converted between the layout of Listing 1 and the CG layout
// (to_cg: Listing 1 -> CG); dst and src must not overlap
hipError_t launch_permute(int64_t E, int N, const double *src, double *dst, bool to_cg, hipStream_t s);
// the same, Listing 1 -> CG layout, rounding to FP32
hipError_t launch_permute_to_cg_f32(int64_t E, int N, const double *src, float *dst, hipStream_t s);
hipError_t launch_cg_replace(int64_t P, const double *b, const double *w, double *r,
                             const uint32_t *own, const RedSite &red, CgScalars *sc, hipStream_t s);
// result <- sum own * a * b / sum own * (a - b)^2, deterministic, one device double
hipError_t launch_gdot(int64_t P, const double *a, const double *b, const uint32_t *own,
                       const RedSite &red, double *result, hipStream_t s);
hipError_t launch_gdiff2(int64_t P, const double *a, const double *b, const uint32_t *own,
                         const RedSite &red, double *result, hipStream_t s);

// storage of one reduction site inside a workspace
// one reduction site: RED_MAX_SUMS partials per workgroup, then per group
constexpr size_t RED_SITE_DOUBLES = (size_t)RED_MAX_SUMS * (RED_MAX_BLOCKS + RED_MAX_GROUPS);

inline RedSite red_site(double *mem, unsigned int *tickets, const double *extra = nullptr,
                        long nextra = 0) {
    return RedSite{mem, mem + (size_t)RED_MAX_SUMS * RED_MAX_BLOCKS, tickets, extra, nextra};
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// CG workspace: r, p, w | (p, A_L p) partials of ax | reduction sites |
// their counters | CG scalars | one scratch double | `extra` more vectors
// (nek_cg_solve: b and M^-1 in the CG layout; the server keeps b in its own
// arena and takes none).
enum { SITE_INIT, SITE_UPDATE, SITE_REPLACE, SITE_RESID, N_SITES };

struct CgLayout {
    size_t vec, axp, sites, tickets, scalars, scratch, extra, total;
};

inline CgLayout cg_layout(int64_t E, int N, int extra) {
    const size_t P = (size_t)(E * n3_of(N));
    const size_t vb = align256(P * sizeof(double));
    CgLayout L;
    L.vec = 0;
    L.axp = 3 * vb;
    // one partial per operator workgroup: ax_blocks, or one per element with
    // the one-thread-per-node operator
    const size_t nparts = (size_t)std::max<int64_t>(ax_blocks(E, N), E);
    L.sites = L.axp + align256(nparts * sizeof(double));
    L.tickets = L.sites + align256(N_SITES * RED_SITE_DOUBLES * sizeof(double));
    L.scalars = L.tickets + align256(N_SITES * RED_TICKETS * sizeof(unsigned int));
    L.scratch = L.scalars + align256(sizeof(CgScalars));
    L.extra = L.scratch + align256(sizeof(double));
    L.total = L.extra + (size_t)extra * vb;
    return L;
}

// Pointers into one CG workspace.
struct CgWs {
    double *r, *p, *w, *axp, *site_mem, *scratch;
    double *b = nullptr;                    // the extra vectors, if any
    float *dinv = nullptr;
    unsigned int *tickets;
    CgScalars *sc;
    RedSite site(int k, const double *extra = nullptr, long nextra = 0) const {
        return red_site(site_mem + (size_t)k * RED_SITE_DOUBLES, tickets + (size_t)k * RED_TICKETS,
                        extra, nextra);
    }
};

inline CgWs cg_ws(void *ws, int64_t E, int N, int extra) {
    const CgLayout L = cg_layout(E, N, extra);
    char *c = (char *)ws;
    const size_t vb = align256((size_t)(E * n3_of(N)) * sizeof(double));
    CgWs W;
    W.r = (double *)c;
    W.p = (double *)(c + vb);
    W.w = (double *)(c + 2 * vb);
    W.axp = (double *)(c + L.axp);
    W.site_mem = (double *)(c + L.sites);
    W.tickets = (unsigned int *)(c + L.tickets);
    W.sc = (CgScalars *)(c + L.scalars);
    W.scratch = (double *)(c + L.scratch);
    if (extra >= 1) W.b = (double *)(c + L.extra);
    if (extra >= 2) W.dinv = (float *)(c + L.extra + vb);
    return W;
}

// ---------------------------------------------------------------- geometry
// GLL nodes, weights and derivative matrix passed by value to kernels
struct GllTable {
    double z[NEK_MAX_DEGREE + 1];
    double w[NEK_MAX_DEGREE + 1];
    double D[(NEK_MAX_DEGREE + 1) * (NEK_MAX_DEGREE + 1)];
};

hipError_t launch_box_geometry(int Ex, int Ey, int Ez, int N, double amp, double a0, double a1,
                               double a2, const GllTable &tab, double *g, double *bm, double *X,
                               hipStream_t s);

hipError_t launch_probe(int64_t n, int nread, const double *src, int64_t stride, double *dst, int grid_cap,
                        bool streaming, bool read_only, bool blocked, hipStream_t s);
int64_t probe_blocks(int64_t n, int grid_cap);   // workgroups of a probe launch
// diagonal of the element operator at every local point, and the reciprocal
// of a continuous vector in place (0 stays 0)
hipError_t launch_ax_diag(int64_t E, int N, const double *D, const double *g, double *d, hipStream_t s);
hipError_t launch_reciprocal(int64_t P, double *v, hipStream_t s);

// host GLL routine shared by the setup entry points
int gll_host(int N, double *z, double *w, double *D);

}  // namespace nek
