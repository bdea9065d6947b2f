// api.hip -- the C ABI of libnek (declared in include/nek.h): argument
// checking, error reporting, setup routines, the gather-scatter handle and
// the device-resident CG driver.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "nek_internal.h"

struct nek_gs {
    nek::GsDevice d;
    double *partials = nullptr;      // RED_BLOCKS doubles for nek_gs_dot
    unsigned int *ticket = nullptr;  // one counter
};

namespace nek {

namespace {
thread_local std::string g_last_error;
}

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

void clear_error() { g_last_error.clear(); }

int check_hip(hipError_t e, const char *what) {
    return fail(NEK_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------- GLL (host)
// Nodes: end points -1, 1; interior points by the fixed-point Newton iteration
// x <- x - (x P_N - P_{N-1}) / ((N+1) P_N) started from Chebyshev-Gauss-Lobatto
// points, which converges to the zeros of (1 - x^2) P_N'.  Weights
// 2 / (N (N+1) P_N^2).  Derivative matrix from barycentric weights
// lambda_l = 1 / prod_{m != l} (z_l - z_m): D(i,l) = (lambda_l / lambda_i) / (z_i - z_l)
// off the diagonal, and the diagonal makes every row sum to zero.
int gll_host(int N, double *z, double *w, double *D) {
    if (N < 1 || N > NEK_MAX_DEGREE) return NEK_ERR_UNSUPPORTED;
    const int n = N + 1;
    double zz[NEK_MAX_DEGREE + 1], ww[NEK_MAX_DEGREE + 1];
    for (int q = 0; q < n; ++q) {
        double x = -cos(M_PI * q / N);
        for (int it = 0; it < 200; ++it) {
            double pm1 = 1.0, p = x;   // P_{k-1}, P_k
            for (int k = 1; k < N; ++k) {
                double pn = ((2 * k + 1) * x * p - k * pm1) / (k + 1);
                pm1 = p;
                p = pn;
            }
            double dx = (x * p - pm1) / ((N + 1) * p);
            x -= dx;
            if (fabs(dx) <= 1e-17) break;
        }
        zz[q] = x;
    }
    zz[0] = -1.0;
    zz[N] = 1.0;
    // enforce the exact symmetry of the node set
    for (int q = 0; q < n / 2; ++q) {
        double s = 0.5 * (zz[N - q] - zz[q]);
        zz[q] = -s;
        zz[N - q] = s;
    }
    if (n % 2) zz[N / 2] = 0.0;
    for (int q = 0; q < n; ++q) {
        double pm1 = 1.0, p = zz[q];
        for (int k = 1; k < N; ++k) {
            double pn = ((2 * k + 1) * zz[q] * p - k * pm1) / (k + 1);
            pm1 = p;
            p = pn;
        }
        ww[q] = 2.0 / (N * (N + 1.0) * p * p);
    }
    if (z) memcpy(z, zz, sizeof(double) * n);
    if (w) memcpy(w, ww, sizeof(double) * n);
    if (D) {
        double lam[NEK_MAX_DEGREE + 1];
        for (int l = 0; l < n; ++l) {
            double pr = 1.0;
            for (int m = 0; m < n; ++m)
                if (m != l) pr *= (zz[l] - zz[m]);
            lam[l] = 1.0 / pr;
        }
        for (int i = 0; i < n; ++i) {
            double diag = 0.0;
            for (int l = 0; l < n; ++l) {
                if (l == i) continue;
                double v = (lam[l] / lam[i]) / (zz[i] - zz[l]);
                D[i + n * l] = v;
                diag -= v;
            }
            D[i + n * i] = diag;
        }
    }
    return NEK_OK;
}

}  // namespace nek

using namespace nek;

// ====================================================================== ABI
extern "C" {

const char *nek_strerror(int code) {
    switch (code) {
    case NEK_OK: return "ok";
    case NEK_ERR_ARG: return "invalid argument";
    case NEK_ERR_UNSUPPORTED: return "unsupported degree or type";
    case NEK_ERR_DEVICE: return "device error";
    case NEK_ERR_NOMEM: return "out of memory";
    case NEK_ERR_BREAKDOWN: return "CG breakdown";
    case NEK_ERR_NOCONV: return "CG did not converge";
    case NEK_ERR_STATE: return "invalid state";
    default: return "unknown status";
    }
}

const char *nek_last_error(void) { return g_last_error.c_str(); }

int nek_version(void) { return 10000; }

int nek_gll(int N, double *z, double *w, double *D) {
    clear_error();
    int rc = gll_host(N, z, w, D);
    if (rc != NEK_OK) return fail(rc, "nek_gll: degree must be in 1..15");
    return NEK_OK;
}

int nek_box_numbering(int Ex, int Ey, int Ez, int N, int64_t *glo, uint8_t *dirichlet) {
    clear_error();
    if (Ex < 1 || Ey < 1 || Ez < 1) return fail(NEK_ERR_ARG, "nek_box_numbering: box sizes must be >= 1");
    if (N < 1 || N > NEK_MAX_DEGREE) return fail(NEK_ERR_UNSUPPORTED, "nek_box_numbering: degree must be in 1..15");
    const int n = N + 1;
    const int64_t LX = (int64_t)Ex * N + 1, LY = (int64_t)Ey * N + 1;
    const int64_t LXm = (int64_t)Ex * N, LYm = (int64_t)Ey * N, LZm = (int64_t)Ez * N;
    int64_t L = 0;
    for (int64_t e = 0; e < (int64_t)Ex * Ey * Ez; ++e) {
        const int64_t ex = e % Ex, ey = (e / Ex) % Ey, ez = e / ((int64_t)Ex * Ey);
        for (int k = 0; k < n; ++k) {
            const int64_t K = ez * N + k;
            for (int j = 0; j < n; ++j) {
                const int64_t J = ey * N + j;
                const int64_t rowbase = LX * (J + LY * K) + ex * N;
                const bool edgeJK = (J == 0 || J == LYm || K == 0 || K == LZm);
                for (int i = 0; i < n; ++i, ++L) {
                    if (glo) glo[L] = rowbase + i;
                    if (dirichlet) {
                        const int64_t I = ex * N + i;
                        dirichlet[L] = (edgeJK || I == 0 || I == LXm) ? 1 : 0;
                    }
                }
            }
        }
    }
    return NEK_OK;
}

int nek_box_geometry(int Ex, int Ey, int Ez, int N, double amp, const double *a, double *g,
                     double *bm, double *X, void *stream) {
    clear_error();
    if (Ex < 1 || Ey < 1 || Ez < 1) return fail(NEK_ERR_ARG, "nek_box_geometry: box sizes must be >= 1");
    if (N < 1 || N > NEK_MAX_DEGREE) return fail(NEK_ERR_UNSUPPORTED, "nek_box_geometry: degree must be in 1..15");
    if (!a || !g) return fail(NEK_ERR_ARG, "nek_box_geometry: a and g are required");
    if (!aligned8(g) || (bm && !aligned8(bm)) || (X && !aligned8(X)))
        return fail(NEK_ERR_ARG, "nek_box_geometry: outputs must be 8-byte aligned");
    GllTable tab;
    memset(&tab, 0, sizeof(tab));
    gll_host(N, tab.z, tab.w, tab.D);
    NEK_HIP(launch_box_geometry(Ex, Ey, Ez, N, amp, a[0], a[1], a[2], tab, g, bm, X,
                                (hipStream_t)stream));
    return NEK_OK;
}

// ---------------------------------------------------------------- ax
static int check_ax_args(const char *who, int64_t E, int N, const void *u, const void *D,
                         const void *g, const void *w, size_t usz) {
    if (E < 1) return fail(NEK_ERR_ARG, std::string(who) + ": E must be >= 1");
    if (N < 1 || N > NEK_MAX_DEGREE) return fail(NEK_ERR_UNSUPPORTED, std::string(who) + ": degree must be in 1..15");
    if (!u || !D || !g || !w) return fail(NEK_ERR_ARG, std::string(who) + ": null pointer");
    if (!aligned8(u) || !aligned8(w) || ((uintptr_t)D & 3u) || ((uintptr_t)g & 1u))
        return fail(NEK_ERR_ARG, std::string(who) + ": misaligned pointer");
    const uintptr_t ub = (uintptr_t)u, wb = (uintptr_t)w;
    const uintptr_t bytes = (uintptr_t)(E * n3_of(N)) * usz;
    if (ub < wb + bytes && wb < ub + bytes)
        return fail(NEK_ERR_ARG, std::string(who) + ": u and w overlap");
    return NEK_OK;
}

int nek_ax(int64_t E, int N, const double *u, const double *D, const double *g, double *w,
           void *stream) {
    clear_error();
    int rc = check_ax_args("nek_ax", E, N, u, D, g, w, sizeof(double));
    if (rc) return rc;
    if (!aligned8(D) || !aligned8(g)) return fail(NEK_ERR_ARG, "nek_ax: misaligned D or g");
    NEK_HIP(launch_ax_f64(E, N, D, g, nullptr, const_cast<double *>(u), nullptr, w, nullptr,
                          (hipStream_t)stream));
    return NEK_OK;
}

int nek_ax_f32(int64_t E, int N, const double *u, const float *D32, const void *g_lo, int g_dtype,
               double *w, void *stream) {
    clear_error();
    int rc = check_ax_args("nek_ax_f32", E, N, u, D32, g_lo, w, sizeof(double));
    if (rc) return rc;
    if (g_dtype != NEK_G_F32 && g_dtype != NEK_G_BF16)
        return fail(NEK_ERR_UNSUPPORTED, "nek_ax_f32: g_dtype must be NEK_G_F32 or NEK_G_BF16");
    if (g_dtype == NEK_G_F32 && ((uintptr_t)g_lo & 3u))
        return fail(NEK_ERR_ARG, "nek_ax_f32: misaligned g");
    NEK_HIP(launch_ax_f32(E, N, D32, g_lo, g_dtype, nullptr, const_cast<double *>(u), nullptr, w,
                          nullptr, (hipStream_t)stream));
    return NEK_OK;
}

int nek_convert_g(int64_t E, int N, const double *g, int g_dtype, void *g_lo, void *stream) {
    clear_error();
    if (E < 1) return fail(NEK_ERR_ARG, "nek_convert_g: E must be >= 1");
    if (N < 1 || N > NEK_MAX_DEGREE) return fail(NEK_ERR_UNSUPPORTED, "nek_convert_g: degree must be in 1..15");
    if (!g || !g_lo) return fail(NEK_ERR_ARG, "nek_convert_g: null pointer");
    if (g_dtype != NEK_G_F32 && g_dtype != NEK_G_BF16)
        return fail(NEK_ERR_UNSUPPORTED, "nek_convert_g: g_dtype must be NEK_G_F32 or NEK_G_BF16");
    if (!aligned8(g) || ((uintptr_t)g_lo & (g_dtype == NEK_G_F32 ? 3u : 1u)))
        return fail(NEK_ERR_ARG, "nek_convert_g: misaligned pointer");
    NEK_HIP(launch_convert_g(6 * E * n3_of(N), g, g_dtype, g_lo, (hipStream_t)stream));
    return NEK_OK;
}

// ---------------------------------------------------------------- gather-scatter
static void gs_free(nek_gs *h) {
    if (!h) return;
    (void)hipFree(h->d.row_off);
    (void)hipFree(h->d.row_idx);
    (void)hipFree(h->d.row_keep);
    (void)hipFree(h->d.own);
    (void)hipFree(h->partials);
    (void)hipFree(h->ticket);
    delete h;
}

int nek_gs_create(int64_t E, int N, const int64_t *glo, const uint8_t *dirichlet, nek_gs **out) {
    clear_error();
    if (!out) return fail(NEK_ERR_ARG, "nek_gs_create: out is null");
    *out = nullptr;
    if (E < 1) return fail(NEK_ERR_ARG, "nek_gs_create: E must be >= 1");
    if (N < 1 || N > NEK_MAX_DEGREE) return fail(NEK_ERR_UNSUPPORTED, "nek_gs_create: degree must be in 1..15");
    if (!glo) return fail(NEK_ERR_ARG, "nek_gs_create: glo is null");
    const int64_t P = E * n3_of(N);
    if (P >= ((int64_t)1 << 31)) return fail(NEK_ERR_ARG, "nek_gs_create: E*(N+1)^3 must be < 2^31");

    // dense renumbering of the ids: counting when the id range is compact
    int64_t gmin = glo[0], gmax = glo[0];
    for (int64_t L = 0; L < P; ++L) {
        gmin = std::min(gmin, glo[L]);
        gmax = std::max(gmax, glo[L]);
    }
    if (gmin < 0) return fail(NEK_ERR_ARG, "nek_gs_create: negative global id");
    std::vector<int32_t> dense((size_t)P);
    int64_t U = 0;
    if (gmax < 4 * P + 1024) {
        std::vector<int32_t> map((size_t)gmax + 1, -1);
        for (int64_t L = 0; L < P; ++L) {
            int32_t &m = map[(size_t)glo[L]];
            if (m < 0) m = (int32_t)U++;
            dense[(size_t)L] = m;
        }
    } else {
        std::vector<int64_t> ids(glo, glo + P);
        std::sort(ids.begin(), ids.end());
        ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
        U = (int64_t)ids.size();
        for (int64_t L = 0; L < P; ++L)
            dense[(size_t)L] = (int32_t)(std::lower_bound(ids.begin(), ids.end(), glo[L]) - ids.begin());
    }
    // copies of every node, in ascending local index (counting sort)
    std::vector<int32_t> cnt((size_t)U + 1, 0), first((size_t)U, -1);
    std::vector<uint8_t> masked((size_t)U, 0);
    for (int64_t L = 0; L < P; ++L) {
        const int32_t G = dense[(size_t)L];
        cnt[(size_t)G + 1]++;
        if (first[(size_t)G] < 0) first[(size_t)G] = (int32_t)L;
        if (dirichlet && dirichlet[L]) masked[(size_t)G] = 1;
    }
    for (int64_t G = 0; G < U; ++G) cnt[(size_t)G + 1] += cnt[(size_t)G];
    std::vector<int32_t> copies((size_t)P), fillpos(cnt.begin(), cnt.end() - 1);
    for (int64_t L = 0; L < P; ++L) copies[(size_t)fillpos[(size_t)dense[(size_t)L]]++] = (int32_t)L;

    std::vector<int32_t> row_off(1, 0), row_idx;
    std::vector<uint8_t> row_keep, own((size_t)P, 0);
    int64_t n_masked = 0;
    for (int64_t L = 0; L < P; ++L) {
        const int32_t G = dense[(size_t)L];
        if (first[(size_t)G] != (int32_t)L) continue;
        own[(size_t)L] = 1;
        const int32_t c0 = cnt[(size_t)G], c1 = cnt[(size_t)G + 1];
        if (masked[(size_t)G]) ++n_masked;
        if (c1 - c0 > 1 || masked[(size_t)G]) {
            for (int32_t q = c0; q < c1; ++q) row_idx.push_back(copies[(size_t)q]);
            row_off.push_back((int32_t)row_idx.size());
            row_keep.push_back(masked[(size_t)G] ? 0 : 1);
        }
    }

    nek_gs *h = new nek_gs();
    h->d.E = E;
    h->d.N = N;
    h->d.P = P;
    h->d.n_unique = U;
    h->d.n_rows = (int64_t)row_keep.size();
    h->d.n_entries = (int64_t)row_idx.size();
    h->d.n_masked = n_masked;
    hipError_t e = hipSuccess;
    auto up = [&](void **dst, const void *src, size_t bytes) {
        if (e != hipSuccess) return;
        e = hipMalloc(dst, bytes ? bytes : 8);
        if (e == hipSuccess && bytes) e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    };
    up((void **)&h->d.row_off, row_off.data(), row_off.size() * sizeof(int32_t));
    up((void **)&h->d.row_idx, row_idx.data(), row_idx.size() * sizeof(int32_t));
    up((void **)&h->d.row_keep, row_keep.data(), row_keep.size());
    up((void **)&h->d.own, own.data(), own.size());
    if (e == hipSuccess) e = hipMalloc((void **)&h->partials, RED_BLOCKS * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&h->ticket, sizeof(unsigned int));
    if (e == hipSuccess) e = hipMemset(h->ticket, 0, sizeof(unsigned int));
    if (e != hipSuccess) {
        gs_free(h);
        return fail(e == hipErrorOutOfMemory ? NEK_ERR_NOMEM : NEK_ERR_DEVICE,
                    std::string("nek_gs_create: ") + hipGetErrorString(e));
    }
    *out = h;
    return NEK_OK;
}

int nek_gs_destroy(nek_gs *gs) {
    clear_error();
    if (!gs) return NEK_OK;
    hipError_t e = hipDeviceSynchronize();
    gs_free(gs);
    if (e != hipSuccess) return check_hip(e, "nek_gs_destroy: hipDeviceSynchronize");
    return NEK_OK;
}

int nek_gs_info(const nek_gs *gs, int64_t *n_unique, int64_t *n_rows, int64_t *n_entries,
                int64_t *n_masked) {
    clear_error();
    if (!gs) return fail(NEK_ERR_ARG, "nek_gs_info: null handle");
    if (n_unique) *n_unique = gs->d.n_unique;
    if (n_rows) *n_rows = gs->d.n_rows;
    if (n_entries) *n_entries = gs->d.n_entries;
    if (n_masked) *n_masked = gs->d.n_masked;
    return NEK_OK;
}

int nek_dssum(const nek_gs *gs, double *w, void *stream) {
    clear_error();
    if (!gs || !w) return fail(NEK_ERR_ARG, "nek_dssum: null argument");
    if (!aligned8(w)) return fail(NEK_ERR_ARG, "nek_dssum: misaligned w");
    NEK_HIP(launch_gs(gs->d, w, nullptr, (hipStream_t)stream));
    return NEK_OK;
}

int nek_gs_dot(const nek_gs *gs, const double *a, const double *b, double *result, void *stream) {
    clear_error();
    if (!gs || !a || !b || !result) return fail(NEK_ERR_ARG, "nek_gs_dot: null argument");
    if (!aligned8(a) || !aligned8(b) || !aligned8(result)) return fail(NEK_ERR_ARG, "nek_gs_dot: misaligned pointer");
    NEK_HIP(launch_gdot(gs->d.P, a, b, gs->d.own, gs->partials, gs->ticket, result,
                        (hipStream_t)stream));
    return NEK_OK;
}

// ---------------------------------------------------------------- CG
void nek_cg_default_opts(nek_cg_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->max_iter = 100;
    o->rel_tol = 0.0;
    o->precision = NEK_PREC_F64;
    o->check_every = 0;
    o->true_residual = 0;
    o->reliable_drop = 0.0;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t nek_cg_workspace_bytes(int64_t E, int N) {
    if (E < 1 || N < 1 || N > NEK_MAX_DEGREE) return 0;
    const size_t P = (size_t)(E * n3_of(N));
    return 3 * align256(P * sizeof(double)) + align256(RED_BLOCKS * sizeof(double)) +
           align256(sizeof(CgScalars)) + align256(sizeof(double));
}

namespace {
struct HostSnap {
    CgScalars *buf = nullptr;
    ~HostSnap() {
        if (buf) (void)hipHostFree(buf);
    }
};
thread_local HostSnap g_snap;
}  // namespace

int nek_cg_solve(int64_t E, int N, const double *D, const double *g, const nek_gs *gs,
                 const double *b, double *x, const nek_cg_opts *opts_in, nek_cg_stats *st,
                 void *stream_v) {
    clear_error();
    nek_cg_opts opts;
    if (opts_in) opts = *opts_in;
    else nek_cg_default_opts(&opts);
    if (st) {
        st->iters = 0;
        st->status = NEK_OK;
        st->rel_res = -1.0;
        st->rel_res_true = -1.0;
        st->n_replacements = 0;
    }
    if (E < 1) return fail(NEK_ERR_ARG, "nek_cg_solve: E must be >= 1");
    if (N < 1 || N > NEK_MAX_DEGREE) return fail(NEK_ERR_UNSUPPORTED, "nek_cg_solve: degree must be in 1..15");
    if (!D || !g || !gs || !b || !x) return fail(NEK_ERR_ARG, "nek_cg_solve: null argument");
    if (!aligned8(D) || !aligned8(g) || !aligned8(b) || !aligned8(x))
        return fail(NEK_ERR_ARG, "nek_cg_solve: misaligned pointer");
    if (gs->d.E != E || gs->d.N != N) return fail(NEK_ERR_ARG, "nek_cg_solve: gather-scatter built for another mesh");
    if (b == x) return fail(NEK_ERR_ARG, "nek_cg_solve: b and x must differ");
    if (opts.max_iter < 0) return fail(NEK_ERR_ARG, "nek_cg_solve: max_iter must be >= 0");
    const bool mixed = opts.precision == NEK_PREC_F32G32 || opts.precision == NEK_PREC_F32GBF16;
    if (!mixed && opts.precision != NEK_PREC_F64)
        return fail(NEK_ERR_UNSUPPORTED, "nek_cg_solve: unknown precision");
    if (mixed && (!opts.D32 || !opts.g_lo))
        return fail(NEK_ERR_ARG, "nek_cg_solve: mixed precision needs D32 and g_lo");
    const int g_dtype = opts.precision == NEK_PREC_F32G32 ? NEK_G_F32 : NEK_G_BF16;
    const double drop = mixed ? (opts.reliable_drop > 0.0 ? opts.reliable_drop : 0.1) : 0.0;
    if (mixed && !(drop < 1.0)) return fail(NEK_ERR_ARG, "nek_cg_solve: reliable_drop must be < 1");
    int check_every = opts.check_every > 0 ? opts.check_every : (mixed ? 4 : 25);
    const bool poll = mixed || opts.rel_tol > 0.0;
    if (!poll) check_every = opts.max_iter > 0 ? opts.max_iter : 1;

    hipStream_t s = (hipStream_t)stream_v;
    const int64_t P = E * n3_of(N);
    const size_t need = nek_cg_workspace_bytes(E, N);
    char *ws = (char *)opts.workspace;
    bool own_ws = false;
    if (ws) {
        if (opts.workspace_bytes < need) return fail(NEK_ERR_ARG, "nek_cg_solve: workspace too small");
        if ((uintptr_t)ws & 255u) return fail(NEK_ERR_ARG, "nek_cg_solve: workspace must be 256-byte aligned");
    } else {
        hipError_t e = hipMallocAsync((void **)&ws, need, s);
        if (e != hipSuccess)
            return fail(e == hipErrorOutOfMemory ? NEK_ERR_NOMEM : NEK_ERR_DEVICE,
                        std::string("nek_cg_solve: workspace allocation: ") + hipGetErrorString(e));
        own_ws = true;
    }
    const size_t vb = align256((size_t)P * sizeof(double));
    double *r = (double *)ws;
    double *p = (double *)(ws + vb);
    double *w = (double *)(ws + 2 * vb);
    double *partials = (double *)(ws + 3 * vb);
    CgScalars *sc = (CgScalars *)(ws + 3 * vb + align256(RED_BLOCKS * sizeof(double)));
    double *scratch1 = (double *)((char *)sc + align256(sizeof(CgScalars)));   // one double

    if (!g_snap.buf) {
        hipError_t e = hipHostMalloc((void **)&g_snap.buf, 2 * sizeof(CgScalars), hipHostMallocDefault);
        if (e != hipSuccess) {
            if (own_ws) (void)hipFreeAsync(ws, s);
            return check_hip(e, "nek_cg_solve: hipHostMalloc");
        }
    }
    CgScalars *snap = g_snap.buf;

    int rc = NEK_OK;
    hipError_t he = hipSuccess;
    double true_rel = -1.0;
    CgScalars S;
    memset(&S, 0, sizeof(S));
#define CG_TRY(call)                                                     \
    do {                                                                 \
        he = (call);                                                     \
        if (he != hipSuccess) { rc = check_hip(he, #call); goto out; }   \
    } while (0)
    {
        CG_TRY(launch_cg_reset(sc, opts.max_iter, opts.rel_tol, drop, s));
        CG_TRY(launch_cg_init(P, b, x, r, p, gs->d.own, partials, sc, s));
        const int *done = &sc->done;
        int enq = 0;
        bool first = true;
        while (enq < opts.max_iter) {
            const int chunk = std::min(check_every, opts.max_iter - enq);
            for (int q = 0; q < chunk; ++q) {
                // first iteration: p = b as set by init; later ones fuse p <- r + beta p
                const double *rr = first ? nullptr : r;
                if (mixed)
                    CG_TRY(launch_ax_f32(E, N, opts.D32, opts.g_lo, g_dtype, rr, p, &sc->beta, w, done, s));
                else
                    CG_TRY(launch_ax_f64(E, N, D, g, rr, p, &sc->beta, w, done, s));
                CG_TRY(launch_gs(gs->d, w, done, s));
                CG_TRY(launch_cg_dot_pw(P, p, w, gs->d.own, partials, sc, s));
                CG_TRY(launch_cg_update(P, x, r, p, w, gs->d.own, partials, sc, s));
                first = false;
            }
            enq += chunk;
            if (!poll) continue;
            CG_TRY(hipMemcpyAsync(snap, sc, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
            CG_TRY(hipStreamSynchronize(s));
            if (snap->done) break;
            if (mixed && snap->need_replace) {
                // reliable update: r <- b - mask(dssum(A64 x)) in FP64
                CG_TRY(launch_ax_f64(E, N, D, g, nullptr, x, nullptr, w, nullptr, s));
                CG_TRY(launch_gs(gs->d, w, nullptr, s));
                CG_TRY(launch_cg_replace(P, b, w, r, gs->d.own, partials, sc, s));
            }
        }
        CG_TRY(hipMemcpyAsync(snap, sc, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
        CG_TRY(hipStreamSynchronize(s));
        S = *snap;
        if (opts.true_residual || mixed) {
            // ||b - mask(dssum(A64 x))|| over unique nodes, in FP64
            CG_TRY(launch_ax_f64(E, N, D, g, nullptr, x, nullptr, w, nullptr, s));
            CG_TRY(launch_gs(gs->d, w, nullptr, s));
            CG_TRY(launch_gdiff2(P, b, w, gs->d.own, partials, &sc->ticket[3], scratch1, s));
            double t2 = 0.0;
            CG_TRY(hipMemcpyAsync(&snap[1].bb, scratch1, sizeof(double), hipMemcpyDeviceToHost, s));
            CG_TRY(hipStreamSynchronize(s));
            t2 = snap[1].bb;
            true_rel = S.bb > 0.0 ? sqrt(t2 / S.bb) : 0.0;
        }
    }
out:
#undef CG_TRY
    if (own_ws) (void)hipFreeAsync(ws, s);
    if (rc != NEK_OK) {
        if (st) st->status = rc;
        return rc;
    }
    {
        int status = S.status;
        const double rel = S.bb > 0.0 ? sqrt(S.rho / S.bb) : 0.0;
        if (status == NEK_OK && opts.rel_tol > 0.0) {
            const double judged = mixed ? true_rel : rel;
            if (!(judged <= opts.rel_tol)) status = NEK_ERR_NOCONV;
        }
        if (st) {
            st->iters = S.it;
            st->status = status;
            st->rel_res = rel;
            st->rel_res_true = true_rel;
            st->n_replacements = S.n_replace;
        }
        if (status == NEK_ERR_BREAKDOWN) return fail(status, "nek_cg_solve: breakdown ((p,Ap) <= 0 or non-finite)");
        if (status == NEK_ERR_NOCONV) return fail(status, "nek_cg_solve: tolerance not reached");
    }
    return NEK_OK;
}

}  // extern "C"
