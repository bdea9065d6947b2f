// Internal declarations shared by the libnek translation units (not part of
// the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

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

// ---------------------------------------------------------------- CG scalars
// Device-side CG state (one struct in device memory, written only by the
// last workgroup of a reduction kernel or by single-thread kernels).
struct CgScalars {
    double bb;            // (b, b)
    double rho;           // (r, r) of the current residual
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
    int pad_;
};

// ---------------------------------------------------------------- ax_e
// Optional CG fusion of the local-operator launch (all device pointers):
//   r != null : p <- r + beta p on the way in (beta from sc);
//   x != null : x += alpha p_old first, if sc->lag_applied == 0;
//   partials != null : per-workgroup sum of p * (A_L p) over all local
//                      points, at partials[blockIdx];
//   sc != null : skip everything once sc->done is set.
struct AxFuse {
    const double *r = nullptr;
    double *x = nullptr;
    double *partials = nullptr;
    const CgScalars *sc = nullptr;
};

hipError_t launch_ax_f64(int64_t E, int N, const double *D, const double *g, double *p, double *w,
                         const AxFuse &fz, hipStream_t s);
hipError_t launch_ax_f32(int64_t E, int N, const float *D32, const void *g_lo, int g_dtype,
                         double *p, double *w, const AxFuse &fz, hipStream_t s);
// number of workgroups of an ax launch (one partial each)
int64_t ax_blocks(int64_t E, int N);

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
    uint32_t *own_bits = nullptr;  // P bits: first copy of every node
};

// dssum + mask in place.  With sc != null, workgroup 0 also sums the nparts
// partials of (p, A_L p) left by the ax launch, in index order, into
// sc->pw and sc->alpha (or flags a breakdown).
hipError_t launch_gs(const GsDevice &gs, double *w, const double *axparts, int64_t nparts,
                     CgScalars *sc, hipStream_t s);
int64_t gs_grid(const GsDevice &gs);

// ---------------------------------------------------------------- CG vector steps
constexpr int VEC_THREADS = 256;
constexpr int VEC_PAIRS = 4;            // double2 per thread per chunk
int64_t vec_blocks(int64_t P);          // workgroups of the vector kernels (<= RED_MAX_BLOCKS)

hipError_t launch_cg_reset(CgScalars *sc, unsigned int *tickets, int nticket, int max_iter,
                           double rel_tol, double drop, hipStream_t s);
hipError_t launch_cg_init(int64_t P, const double *b, double *x, double *r, double *p,
                          const uint32_t *own, const RedSite &red, CgScalars *sc, hipStream_t s);
hipError_t launch_cg_update(int64_t P, double *r, const double *w, const uint32_t *own,
                            const RedSite &red, CgScalars *sc, hipStream_t s);
hipError_t launch_cg_finish(int64_t P, double *x, const double *p, const CgScalars *sc, hipStream_t s);
hipError_t launch_cg_replace(int64_t P, const double *b, const double *w, double *r,
                             const uint32_t *own, const RedSite &red, CgScalars *sc, hipStream_t s);
// result <- sum own * a * b / sum own * (a - b)^2, deterministic, one device double
hipError_t launch_gdot(int64_t P, const double *a, const double *b, const uint32_t *own,
                       const RedSite &red, double *result, hipStream_t s);
hipError_t launch_gdiff2(int64_t P, const double *a, const double *b, const uint32_t *own,
                         const RedSite &red, double *result, hipStream_t s);

// storage of one reduction site inside a workspace
constexpr size_t RED_SITE_DOUBLES = RED_MAX_BLOCKS + RED_MAX_GROUPS;

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

hipError_t launch_probe(int64_t n, int nread, const double *src, double *dst, int grid, hipStream_t s);

// host GLL routine shared by the setup entry points
int gll_host(int N, double *z, double *w, double *D);

}  // namespace nek
