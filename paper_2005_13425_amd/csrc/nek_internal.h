// Internal declarations shared by the libnek translation units (not part of
// the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "nek.h"

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

// ---------------------------------------------------------------- ax_e
// FP64 local operator, optionally fused with the CG direction update
// p <- r + beta * p (beta read on the device from *beta; r == nullptr means
// no fusion and p is only read).
hipError_t launch_ax_f64(int64_t E, int N, const double *D, const double *g,
                         const double *r, double *p, const double *beta,
                         double *w, const int *done, hipStream_t s);

// FP32 operator: p read in FP64, computed in FP32, w written FP64.
hipError_t launch_ax_f32(int64_t E, int N, const float *D32, const void *g_lo, int g_dtype,
                         const double *r, double *p, const double *beta,
                         double *w, const int *done, hipStream_t s);

hipError_t launch_convert_g(int64_t count, const double *g, int g_dtype, void *out, hipStream_t s);

// ---------------------------------------------------------------- gather-scatter
struct GsDevice {
    int64_t E = 0;
    int N = 0;
    int64_t P = 0;
    int64_t n_unique = 0;
    int64_t n_rows = 0;     // CSR rows: shared-or-masked nodes
    int64_t n_entries = 0;  // CSR entries
    int64_t n_masked = 0;   // masked unique nodes
    int32_t *row_off = nullptr;   // n_rows + 1
    int32_t *row_idx = nullptr;   // n_entries, ascending within a row
    uint8_t *row_keep = nullptr;  // n_rows: 0 = masked (write 0), 1 = keep sum
    uint8_t *own = nullptr;       // P: 1 on the first copy of every node
};

hipError_t launch_gs(const GsDevice &gs, double *w, const int *done, hipStream_t s);

// ---------------------------------------------------------------- reductions / CG
// Device-side CG scalars (one struct in device memory).
struct CgScalars {
    double bb;         // (b, b)
    double rho;        // (r, r) of the current residual
    double pw;         // (p, w)
    double alpha;
    double beta;
    double rel_tol2;   // rel_tol^2 * bb, 0 for fixed iterations
    double rho_last_true; // rho at the last reliable replacement
    double drop2;      // reliable_drop^2
    int it;            // iterations completed
    int max_iter;
    int done;          // 1: converged, breakdown or max_iter reached
    int status;        // NEK_OK / NEK_ERR_BREAKDOWN
    int need_replace;  // mixed precision: r must be replaced by b - A64 x
    int n_replace;
    unsigned int ticket[4];  // last-block tickets of the reduction kernels
};

constexpr int RED_BLOCKS = 1024;   // blocks of the grid-stride reduction kernels
constexpr int RED_THREADS = 256;

hipError_t launch_cg_reset(CgScalars *sc, int max_iter, double rel_tol, double drop, hipStream_t s);
hipError_t launch_cg_init(int64_t P, const double *b, double *x, double *r, double *p,
                          const uint8_t *own, double *partials, CgScalars *sc,
                          hipStream_t s);
hipError_t launch_cg_dot_pw(int64_t P, const double *p, const double *w, const uint8_t *own,
                            double *partials, CgScalars *sc, hipStream_t s);
hipError_t launch_cg_update(int64_t P, double *x, double *r, const double *p, const double *w,
                            const uint8_t *own, double *partials, CgScalars *sc,
                            hipStream_t s);
// r <- b - w (w = A64 x already gathered), rho <- (r, r); mixed-precision replacement.
hipError_t launch_cg_replace(int64_t P, const double *b, const double *w, double *r,
                             const uint8_t *own, double *partials, CgScalars *sc,
                             hipStream_t s);
// result <- sum own * (a - b)^2 (deterministic), one double in device memory
hipError_t launch_gdiff2(int64_t P, const double *a, const double *b, const uint8_t *own,
                         double *partials, unsigned int *ticket, double *result, hipStream_t s);
// result <- sum own * a * b (deterministic), one double in device memory
hipError_t launch_gdot(int64_t P, const double *a, const double *b, const uint8_t *own,
                       double *partials, unsigned int *ticket, double *result, hipStream_t s);

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

// host GLL routine shared by the setup entry points
int gll_host(int N, double *z, double *w, double *D);

}  // namespace nek
