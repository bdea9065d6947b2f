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
    nek::GsDevice d;                 // the layout of Listing 1 (nek_dssum, nek_gs_dot, Jacobi setup)
    nek::GsDevice cg;                // the CG layout (nek_cg_solve)
    double *partials = nullptr;      // reduction site of nek_gs_dot
    unsigned int *ticket = nullptr;  // its counters
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
    NEK_HIP(launch_ax_f64(E, N, D, g, const_cast<double *>(u), w, AxFuse{}, (hipStream_t)stream));
    return NEK_OK;
}

int nek_ax_variant(int64_t E, int N, const double *u, const double *D, const double *g, double *w,
                   int variant, void *stream) {
    clear_error();
    int rc = check_ax_args("nek_ax_variant", E, N, u, D, g, w, sizeof(double));
    if (rc) return rc;
    if (!aligned8(D) || !aligned8(g)) return fail(NEK_ERR_ARG, "nek_ax_variant: misaligned D or g");
    const hipStream_t s = (hipStream_t)stream;
    if (variant == NEK_AX_PENCIL) {
        NEK_HIP(launch_ax_f64(E, N, D, g, const_cast<double *>(u), w, AxFuse{}, s));
        return NEK_OK;
    }
    if (variant != NEK_AX_ORIGINAL && variant != NEK_AX_SHARED3D && variant != NEK_AX_LAYER2D)
        return fail(NEK_ERR_UNSUPPORTED, "nek_ax_variant: unknown variant");
    if (variant == NEK_AX_SHARED3D && N > 9)
        return fail(NEK_ERR_UNSUPPORTED, "nek_ax_variant: SHARED3D takes n^3 <= 1024 threads, N <= 9");
    if (E > 0x7fffffff) return fail(NEK_ERR_ARG, "nek_ax_variant: E must be < 2^31");
    double *scratch = nullptr;
    if (variant == NEK_AX_ORIGINAL) {
        const hipError_t e = hipMallocAsync((void **)&scratch, (size_t)(3 * E * n3_of(N)) * sizeof(double), s);
        if (e != hipSuccess)
            return fail(e == hipErrorOutOfMemory ? NEK_ERR_NOMEM : NEK_ERR_DEVICE,
                        std::string("nek_ax_variant: scratch allocation: ") + hipGetErrorString(e));
    }
    const hipError_t e = launch_ax_variant(variant, E, N, D, g, u, w, scratch, s);
    if (scratch) (void)hipFreeAsync(scratch, s);
    NEK_HIP(e);
    return NEK_OK;
}

int nek_ax_f32(int64_t E, int N, const double *u, const float *D32, const void *g_lo, int g_dtype,
               double *w, void *stream) {
    clear_error();
    int rc = check_ax_args("nek_ax_f32", E, N, u, D32, g_lo, w, sizeof(double));
    if (rc) return rc;
    if (g_dtype != NEK_G_F32 && g_dtype != NEK_G_BF16)
        return fail(NEK_ERR_UNSUPPORTED, "nek_ax_f32: g_dtype must be NEK_G_F32 or NEK_G_BF16");
    if (((uintptr_t)g_lo & (g_dtype == NEK_G_F32 ? 7u : 3u)) || ((uintptr_t)D32 & 3u))
        return fail(NEK_ERR_ARG, "nek_ax_f32: misaligned g_lo (8 bytes for FP32, 4 for BF16) or D32");
    NEK_HIP(launch_ax_f32(E, N, D32, g_lo, g_dtype, const_cast<double *>(u), w, AxFuse{},
                          (hipStream_t)stream));
    return NEK_OK;
}

int nek_convert_g(int64_t E, int N, const double *g, int g_dtype, void *g_lo, void *stream) {
    clear_error();
    if (E < 1) return fail(NEK_ERR_ARG, "nek_convert_g: E must be >= 1");
    if (N < 1 || N > NEK_MAX_DEGREE) return fail(NEK_ERR_UNSUPPORTED, "nek_convert_g: degree must be in 1..15");
    if (!g || !g_lo) return fail(NEK_ERR_ARG, "nek_convert_g: null pointer");
    if (g_dtype != NEK_G_F32 && g_dtype != NEK_G_BF16)
        return fail(NEK_ERR_UNSUPPORTED, "nek_convert_g: g_dtype must be NEK_G_F32 or NEK_G_BF16");
    if (!aligned8(g) || ((uintptr_t)g_lo & (g_dtype == NEK_G_F32 ? 7u : 3u)))
        return fail(NEK_ERR_ARG, "nek_convert_g: misaligned pointer");
    NEK_HIP(launch_convert_g(E, N, g, g_dtype, g_lo, (hipStream_t)stream));
    return NEK_OK;
}

// ---------------------------------------------------------------- measurement
int nek_bw_probe(int64_t n, int nread, const double *src, int64_t src_stride, double *dst, int grid_cap,
                 int flags, void *stream) {
    clear_error();
    if (n < 2) return fail(NEK_ERR_ARG, "nek_bw_probe: n must be >= 2");
    if (nread < 1 || nread > 8) return fail(NEK_ERR_ARG, "nek_bw_probe: nread must be in 1..8");
    if (flags & ~(NEK_PROBE_NT | NEK_PROBE_READ_ONLY | NEK_PROBE_BLOCKED))
        return fail(NEK_ERR_ARG, "nek_bw_probe: unknown flag");
    const bool blk = (flags & NEK_PROBE_BLOCKED) != 0;
    if (!blk && (src_stride < n || (src_stride & 1)))
        return fail(NEK_ERR_ARG, "nek_bw_probe: src_stride must be even and >= n");
    if (grid_cap < 0) return fail(NEK_ERR_ARG, "nek_bw_probe: grid_cap must be >= 0");
    if (!src || !dst || ((uintptr_t)src & 15u) || ((uintptr_t)dst & 15u))
        return fail(NEK_ERR_ARG, "nek_bw_probe: null or misaligned pointer");
    const bool ro = (flags & NEK_PROBE_READ_ONLY) != 0;
    const int64_t ndst = ro ? probe_blocks(n, grid_cap) : n;
    const uintptr_t sb = (uintptr_t)src, db = (uintptr_t)dst;
    const int64_t nblk = (n + NEK_PROBE_BLOCK - 1) / NEK_PROBE_BLOCK;
    const uintptr_t src_end = sb + (uintptr_t)(blk ? nread * NEK_PROBE_BLOCK * nblk : (nread - 1) * src_stride + n) * 8;
    if (db < src_end && sb < db + (uintptr_t)ndst * 8)
        return fail(NEK_ERR_ARG, "nek_bw_probe: src and dst overlap");
    NEK_HIP(launch_probe(n, nread, src, src_stride, dst, grid_cap, (flags & NEK_PROBE_NT) != 0, ro, blk,
                         (hipStream_t)stream));
    return NEK_OK;
}

int64_t nek_bw_probe_groups(int64_t n, int grid_cap) {
    if (n < 2 || grid_cap < 0) return 0;
    return probe_blocks(n, grid_cap);
}

// ---------------------------------------------------------------- gather-scatter
static void gs_free(nek_gs *h) {
    if (!h) return;
    (void)hipFree(h->d.arena);
    (void)hipFree(h->cg.arena);
    (void)hipFree(h->partials);
    (void)hipFree(h->ticket);
    delete h;
}

}  // extern "C"

namespace nek {

namespace {
int gs_build_std(int64_t E, int N, const int64_t *glo, const uint8_t *dirichlet, GsHost &H,
                 std::string &msg) {
    const int64_t n3 = n3_of(N);
    const int64_t P = E * n3;
    if (P >= ((int64_t)1 << 31)) {
        msg = "E*(N+1)^3 must be < 2^31";
        return NEK_ERR_ARG;
    }
    // dense renumbering of the ids in order of first appearance
    int64_t gmin = glo[0], gmax = glo[0];
    for (int64_t L = 0; L < P; ++L) {
        gmin = std::min(gmin, glo[L]);
        gmax = std::max(gmax, glo[L]);
    }
    if (gmin < 0) {
        msg = "negative global id";
        return NEK_ERR_ARG;
    }
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
        std::vector<int32_t> first_seen((size_t)U, -1);
        int32_t next = 0;
        for (int64_t L = 0; L < P; ++L) {
            const size_t sid = (size_t)(std::lower_bound(ids.begin(), ids.end(), glo[L]) - ids.begin());
            if (first_seen[sid] < 0) first_seen[sid] = next++;
            dense[(size_t)L] = first_seen[sid];
        }
    }
    // copies of every node in ascending local index (counting sort); node
    // order is the order of first copies
    std::vector<int32_t> start((size_t)U + 1, 0);
    std::vector<uint8_t> masked((size_t)U, 0);
    for (int64_t L = 0; L < P; ++L) {
        const int32_t G = dense[(size_t)L];
        start[(size_t)G + 1]++;
        if (dirichlet && dirichlet[L]) masked[(size_t)G] = 1;
    }
    for (int64_t G = 0; G < U; ++G) start[(size_t)G + 1] += start[(size_t)G];
    std::vector<int32_t> copies((size_t)P), fillpos(start.begin(), start.end() - 1);
    for (int64_t L = 0; L < P; ++L) copies[(size_t)fillpos[(size_t)dense[(size_t)L]]++] = (int32_t)L;

    // groups: copies of masked nodes are zeroed; unmasked nodes with two or
    // more copies are summed; unmasked single-copy nodes need nothing
    std::vector<int32_t> zero;
    std::vector<std::vector<int32_t>> rows(GS_MAXC + 1);
    std::vector<int32_t> csr_nodes;
    int64_t n_masked = 0, n_rows = 0, n_entries = 0;
    for (int64_t G = 0; G < U; ++G) {
        const int32_t c0 = start[(size_t)G], c1 = start[(size_t)G + 1];
        const int c = c1 - c0;
        if (masked[(size_t)G]) {
            ++n_masked;
            for (int32_t q = c0; q < c1; ++q) zero.push_back(copies[(size_t)q]);
            continue;
        }
        if (c == 1) continue;
        ++n_rows;
        n_entries += c;
        if (c <= GS_MAXC) rows[(size_t)c].push_back((int32_t)G);
        else csr_nodes.push_back((int32_t)G);
    }
    std::sort(zero.begin(), zero.end());

    H = GsHost();
    H.E = E;
    H.N = N;
    H.P = P;
    H.U = U;
    H.n_rows = n_rows;
    H.n_entries = n_entries;
    H.n_masked = n_masked;
    H.n_zero = (int64_t)zero.size();
    std::vector<int32_t> &host = H.idx;
    if (!zero.empty()) {
        H.groups.push_back({0, (int32_t)zero.size(), host.size(), 0});
        host.insert(host.end(), zero.begin(), zero.end());
    }
    for (int c = 2; c <= GS_MAXC; ++c) {
        const auto &R = rows[(size_t)c];
        if (R.empty()) continue;
        const size_t at = host.size();
        host.resize(at + (size_t)c * R.size());
        for (size_t rr = 0; rr < R.size(); ++rr)
            for (int m = 0; m < c; ++m)
                host[at + (size_t)m * R.size() + rr] = copies[(size_t)start[(size_t)R[rr]] + m];
        H.groups.push_back({c, (int32_t)R.size(), at, 0});
    }
    if (!csr_nodes.empty()) {
        const size_t off_at = host.size();
        host.resize(off_at + csr_nodes.size() + 1);
        const size_t idx_at = host.size();
        int32_t o = 0;
        for (size_t rr = 0; rr < csr_nodes.size(); ++rr) {
            host[off_at + rr] = o;
            const int32_t G = csr_nodes[rr];
            for (int32_t q = start[(size_t)G]; q < start[(size_t)G + 1]; ++q) {
                host.push_back(copies[(size_t)q]);
                ++o;
            }
        }
        host[off_at + csr_nodes.size()] = o;
        H.groups.push_back({-1, (int32_t)csr_nodes.size(), idx_at, off_at});
    }
    const size_t words = (size_t)((P + 31) / 32);
    H.own.assign(words, 0u);
    H.rowed.assign(words, 0u);
    for (int64_t G = 0; G < U; ++G) {
        const int32_t c0 = start[(size_t)G], c1 = start[(size_t)G + 1];
        const int32_t L = copies[(size_t)c0];
        H.own[(size_t)L >> 5] |= 1u << (L & 31);
        if (c1 - c0 > 1 || masked[(size_t)G])
            for (int32_t q = c0; q < c1; ++q) {
                const int32_t Lq = copies[(size_t)q];
                H.rowed[(size_t)Lq >> 5] |= 1u << (Lq & 31);
            }
    }
    return NEK_OK;
}
}  // namespace

// In the CG layout the copies are the same, at other positions: the map is
// built from the numbering moved to those positions, so rows (ordered by their
// first copy) follow the CG layout too.  Copies of a node lie in distinct
// elements, so each row keeps its copies in the same (element) order and
// sums them in the same order as in the layout of Listing 1.
int gs_build_host(int64_t E, int N, const int64_t *glo, const uint8_t *dirichlet, bool cg_layout,
                  GsHost &H, std::string &msg) {
    if (!cg_layout) return gs_build_std(E, N, glo, dirichlet, H, msg);
    const int n = N + 1;
    const int64_t n3 = n3_of(N);
    if (E * n3 >= ((int64_t)1 << 31)) {
        msg = "E*(N+1)^3 must be < 2^31";
        return NEK_ERR_ARG;
    }
    std::vector<int32_t> pos((size_t)n3);
    for (int l = 0; l < (int)n3; ++l) {
        const int k = l / (n * n), ij = l - k * n * n;
        pos[(size_t)l] = k * n * n + cgl_col(ij % n, ij / n, n);
    }
    std::vector<int64_t> glo_c((size_t)(E * n3));
    std::vector<uint8_t> dir_c(dirichlet ? (size_t)(E * n3) : 0);
    for (int64_t e = 0; e < E; ++e)
        for (int l = 0; l < (int)n3; ++l) {
            const size_t from = (size_t)(e * n3 + l), to = (size_t)(e * n3 + pos[(size_t)l]);
            glo_c[to] = glo[from];
            if (dirichlet) dir_c[to] = dirichlet[from];
        }
    return gs_build_std(E, N, glo_c.data(), dirichlet ? dir_c.data() : nullptr, H, msg);
}

void gs_attach(const GsHost &H, void *arena, GsDevice &d) {
    d.E = H.E;
    d.N = H.N;
    d.P = H.P;
    d.n_unique = H.U;
    d.n_rows = H.n_rows;
    d.n_entries = H.n_entries;
    d.n_masked = H.n_masked;
    d.n_zero = H.n_zero;
    d.arena = arena;
    d.own_bits = (uint32_t *)((char *)arena + H.idx_bytes());
    d.rowed_bits = (uint32_t *)((char *)arena + H.idx_bytes() + H.own_bytes());
    const int32_t *base = (const int32_t *)arena;
    d.args.ngroups = 0;
    int32_t blocks = 0;
    for (const GsHostGroup &q : H.groups) {
        GsGroup &G = d.args.grp[d.args.ngroups++];
        G.kind = q.kind;
        G.rows = q.rows;
        G.block0 = blocks;
        G.idx = base + q.idx_at;
        G.off = q.kind == -1 ? base + q.off_at : nullptr;
        blocks += (q.rows + GS_THREADS - 1) / GS_THREADS;
    }
    d.args.nblocks = blocks;
}

}  // namespace nek

extern "C" {

int nek_gs_create(int64_t E, int N, const int64_t *glo, const uint8_t *dirichlet, nek_gs **out) {
    clear_error();
    if (!out) return fail(NEK_ERR_ARG, "nek_gs_create: out is null");
    *out = nullptr;
    if (E < 1) return fail(NEK_ERR_ARG, "nek_gs_create: E must be >= 1");
    if (N < 1 || N > NEK_MAX_DEGREE) return fail(NEK_ERR_UNSUPPORTED, "nek_gs_create: degree must be in 1..15");
    if (!glo) return fail(NEK_ERR_ARG, "nek_gs_create: glo is null");
    GsHost H, Hc;
    std::string msg;
    int rc = gs_build_host(E, N, glo, dirichlet, false, H, msg);
    if (rc == NEK_OK) rc = gs_build_host(E, N, glo, dirichlet, true, Hc, msg);
    if (rc != NEK_OK) return fail(rc, "nek_gs_create: " + msg);
    nek_gs *h = new nek_gs();
    // one arena per map: the index arrays, then the first-copy bits
    auto upload = [](const GsHost &M, GsDevice &d) -> hipError_t {
        void *arena = nullptr;
        hipError_t e = hipMalloc(&arena, M.arena_bytes());
        if (e != hipSuccess) return e;
        d.arena = arena;
        if (!M.idx.empty())
            e = hipMemcpy(arena, M.idx.data(), M.idx.size() * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy((char *)arena + M.idx_bytes(), M.own.data(), M.own.size() * sizeof(uint32_t),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy((char *)arena + M.idx_bytes() + M.own_bytes(), M.rowed.data(),
                          M.rowed.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) gs_attach(M, arena, d);
        return e;
    };
    hipError_t e = upload(H, h->d);
    if (e == hipSuccess) e = upload(Hc, h->cg);
    if (e == hipSuccess) e = hipMalloc((void **)&h->partials, RED_SITE_DOUBLES * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&h->ticket, RED_TICKETS * sizeof(unsigned int));
    if (e == hipSuccess) e = hipMemset(h->ticket, 0, RED_TICKETS * sizeof(unsigned int));
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
    NEK_HIP(launch_gs(gs->d, w, (hipStream_t)stream));
    return NEK_OK;
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

int nek_jacobi_inverse(int64_t E, int N, const double *D, const double *g, const nek_gs *gs,
                       double *dinv, void *stream) {
    clear_error();
    if (E < 1) return fail(NEK_ERR_ARG, "nek_jacobi_inverse: E must be >= 1");
    if (N < 1 || N > NEK_MAX_DEGREE) return fail(NEK_ERR_UNSUPPORTED, "nek_jacobi_inverse: degree must be in 1..15");
    if (!D || !g || !gs || !dinv) return fail(NEK_ERR_ARG, "nek_jacobi_inverse: null argument");
    if (!aligned8(D) || !aligned8(g) || !aligned16(dinv))
        return fail(NEK_ERR_ARG, "nek_jacobi_inverse: misaligned pointer (dinv needs 16 bytes)");
    if (gs->d.E != E || gs->d.N != N)
        return fail(NEK_ERR_ARG, "nek_jacobi_inverse: gather-scatter built for another mesh");
    const hipStream_t s = (hipStream_t)stream;
    NEK_HIP(launch_ax_diag(E, N, D, g, dinv, s));
    NEK_HIP(launch_gs(gs->d, dinv, s));   // assembled diagonal, 0 at masked nodes
    NEK_HIP(launch_reciprocal(E * n3_of(N), dinv, s));
    return NEK_OK;
}

int nek_gs_dot(const nek_gs *gs, const double *a, const double *b, double *result, void *stream) {
    clear_error();
    if (!gs || !a || !b || !result) return fail(NEK_ERR_ARG, "nek_gs_dot: null argument");
    if (!aligned16(a) || !aligned16(b) || !aligned8(result))
        return fail(NEK_ERR_ARG, "nek_gs_dot: a and b must be 16-byte aligned");
    const RedSite red = red_site(gs->partials, gs->ticket);
    NEK_HIP(launch_gdot(gs->d.P, a, b, gs->d.own_bits, red, result, (hipStream_t)stream));
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

size_t nek_cg_workspace_bytes(int64_t E, int N) {
    if (E < 1 || N < 1 || N > NEK_MAX_DEGREE) return 0;
    return cg_layout(E, N, 2).total;
}

namespace {
struct HostSnap {
    CgScalars *buf = nullptr;
    ~HostSnap() {
        if (buf) (void)hipHostFree(buf);
    }
};
thread_local HostSnap g_snap;

// What nek_cg_solve needs once its arguments have been checked.
struct CgPlan {
    bool mixed = false;   // any mixed precision: reliable updates, stop on the true residual
    bool f64_op = false;  // NEK_PREC_F64G*: FP64 operator arithmetic on g_lo
    int g_dtype = 0;
    double drop = 0.0;
    int check_every = 0;
    bool poll = false;
    int extra = 1;        // vectors kept in the CG layout beside r, p, w: b, and M^-1
    size_t need = 0;      // workspace bytes
};

int cg_check(const char *who, int64_t E, int N, const double *D, const double *g, const nek_gs *gs,
             const double *b, const double *x, const nek_cg_opts &opts, CgPlan &pl) {
    const std::string w(who);
    if (E < 1) return fail(NEK_ERR_ARG, w + ": E must be >= 1");
    if (N < 1 || N > NEK_MAX_DEGREE) return fail(NEK_ERR_UNSUPPORTED, w + ": degree must be in 1..15");
    if (!D || !g || !gs || !b || !x) return fail(NEK_ERR_ARG, w + ": null argument");
    if (!aligned8(D) || !aligned8(g) || !aligned16(b) || !aligned16(x))
        return fail(NEK_ERR_ARG, w + ": misaligned pointer (b and x need 16 bytes)");
    if (gs->d.E != E || gs->d.N != N) return fail(NEK_ERR_ARG, w + ": gather-scatter built for another mesh");
    if (b == x) return fail(NEK_ERR_ARG, w + ": b and x must differ");
    if (opts.max_iter < 0) return fail(NEK_ERR_ARG, w + ": max_iter must be >= 0");
    const int pr = opts.precision;
    pl.f64_op = pr == NEK_PREC_F64G32 || pr == NEK_PREC_F64GBF16;
    pl.mixed = pr == NEK_PREC_F32G32 || pr == NEK_PREC_F32GBF16 || pl.f64_op;
    if (!pl.mixed && pr != NEK_PREC_F64) return fail(NEK_ERR_UNSUPPORTED, w + ": unknown precision");
    if (pl.mixed && !opts.g_lo) return fail(NEK_ERR_ARG, w + ": mixed precision needs g_lo");
    if (pl.mixed && !pl.f64_op && !opts.D32) return fail(NEK_ERR_ARG, w + ": the FP32 operator needs D32");
    const bool g32 = pr == NEK_PREC_F32G32 || pr == NEK_PREC_F64G32;
    if (pl.mixed && (((uintptr_t)opts.g_lo & (g32 ? 7u : 3u)) || (!pl.f64_op && ((uintptr_t)opts.D32 & 3u))))
        return fail(NEK_ERR_ARG, w + ": misaligned g_lo or D32");
    if (opts.dinv && pl.mixed) return fail(NEK_ERR_UNSUPPORTED, w + ": the Jacobi preconditioner is FP64 only");
    if (opts.dinv && !aligned16(opts.dinv)) return fail(NEK_ERR_ARG, w + ": misaligned dinv");
    pl.g_dtype = g32 ? NEK_G_F32 : NEK_G_BF16;
    pl.drop = pl.mixed ? (opts.reliable_drop > 0.0 ? opts.reliable_drop : reliable_drop_default(opts.precision)) : 0.0;
    if (pl.mixed && !(pl.drop < 1.0)) return fail(NEK_ERR_ARG, w + ": reliable_drop must be < 1");
    pl.check_every = opts.check_every > 0 ? opts.check_every : (pl.mixed ? 4 : 25);
    pl.poll = pl.mixed || opts.rel_tol > 0.0;
    if (!pl.poll) pl.check_every = opts.max_iter > 0 ? opts.max_iter : 1;
    pl.extra = opts.dinv ? 2 : 1;
    pl.need = cg_layout(E, N, pl.extra).total;
    return NEK_OK;
}

// The CG driver behind both solve entry points.  ws: the workspace (pl.need
// bytes, 256-byte aligned).  snap: four host CgScalars the device scalars are
// copied into.  With events, the host reads the snapshot of a chunk while the
// next chunk already runs (pinned snap); without them it waits for the stream
// at every poll.
int cg_run(int64_t E, int N, const double *D, const double *g, const nek_gs *gs, const double *b, double *x,
           const nek_cg_opts &opts, const CgPlan &pl, char *ws, CgScalars *snap, bool with_events,
           hipStream_t s, CgScalars &S, double &true_rel) {
    const bool mixed = pl.mixed;
    const int64_t P = E * n3_of(N);
    const CgWs W = cg_ws(ws, E, N, pl.extra);
    double *r = W.r, *p = W.p, *w = W.w, *scratch1 = W.scratch;
    CgScalars *sc = W.sc;
    auto site = [&](int k) { return W.site(k, nullptr, 0); };
    const uint32_t *own = gs->cg.own_bits;
    const double *bc = W.b;        // b in the CG layout
    const float *dinvc = W.dinv;   // M^-1 in the CG layout, rounded to FP32

    // one CG iteration; `first` uses p = b as set by the init kernel.  Small
    // FP64 meshes take the one-thread-per-node operator, which leaves one
    // partial of (p, A_L p) per element
    const RedSite red_upd = site(SITE_UPDATE);
    const bool node_op = !mixed && ax_node_fused_fits(E, N);
    auto iterate = [&](bool first) -> hipError_t {
        AxFuse fz;
        fz.sc = sc;
        fz.partials = W.axp;
        fz.cg_layout = true;
        if (!first) {
            fz.r = r;
            fz.x = x;
            fz.dinv = dinvc;
        }
        hipError_t e = pl.f64_op ? launch_ax_f64_glo(E, N, D, opts.g_lo, pl.g_dtype, p, w, fz, s)
                     : mixed ? launch_ax_f32(E, N, opts.D32, opts.g_lo, pl.g_dtype, p, w, fz, s)
                             : (node_op ? launch_ax_node_fused(E, N, D, g, p, w, fz, s)
                                        : launch_ax_f64(E, N, D, g, p, w, fz, s));
        if (e != hipSuccess) return e;
        // the FP32 operator leaves w in FP32
        return launch_cg_assemble_update(gs->cg, r, w, mixed && !pl.f64_op, dinvc, W.axp,
                                         node_op ? E : ax_blocks(E, N), red_upd,
                                         sc, s);
    };
    AxFuse plain_cg;   // A x alone, on CG-layout vectors
    plain_cg.cg_layout = true;
    // w <- mask(dssum(A64 x)) with x brought up to date first
    auto true_ax = [&]() -> hipError_t {
        hipError_t e = launch_cg_finish(P, x, p, sc, s);
        if (e != hipSuccess) return e;
        e = launch_ax_f64(E, N, D, g, x, w, plain_cg, s);
        if (e != hipSuccess) return e;
        return launch_gs(gs->cg, w, s);
    };

    int rc = NEK_OK;
    hipError_t he = hipSuccess;
    true_rel = -1.0;
    memset(&S, 0, sizeof(S));
#define CG_TRY(call)                                                     \
    do {                                                                 \
        he = (call);                                                     \
        if (he != hipSuccess) { rc = check_hip(he, #call); goto out; }   \
    } while (0)
    hipEvent_t ev[2] = {nullptr, nullptr};
    {
        CG_TRY(launch_cg_reset(sc, W.tickets, N_SITES * RED_TICKETS, opts.max_iter, opts.rel_tol, pl.drop, s));
        CG_TRY(launch_permute(E, N, b, W.b, true, s));
        if (opts.dinv) CG_TRY(launch_permute_to_cg_f32(E, N, opts.dinv, W.dinv, s));
        CG_TRY(launch_cg_init(P, bc, x, r, p, own, dinvc, site(SITE_INIT), sc, s));
        if (pl.poll && with_events) {
            CG_TRY(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
            CG_TRY(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
        }
        // The host polls a snapshot of the device scalars after every chunk of
        // check_every iterations, one chunk behind when it has events: chunk
        // c+1 is already queued while the host waits for the snapshot of chunk
        // c, so the device never idles on the poll.  Kernels queued after the
        // solve has finished exit at once.
        int enq = 0, chunks = 0, prev = -1, replacements = 0;
        bool first = true;
        while (enq < opts.max_iter) {
            const int chunk = std::min(pl.check_every, opts.max_iter - enq);
            for (int q = 0; q < chunk; ++q) {
                CG_TRY(iterate(first));
                first = false;
            }
            enq += chunk;
            if (!pl.poll) continue;
            const int slot = chunks++ & 1;
            CG_TRY(hipMemcpyAsync(&snap[slot], sc, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
            int look = -1;
            if (with_events) {
                CG_TRY(hipEventRecord(ev[slot], s));
                if (prev >= 0) {
                    CG_TRY(hipEventSynchronize(ev[prev]));
                    look = prev;
                }
            } else {
                CG_TRY(hipStreamSynchronize(s));
                look = slot;
            }
            if (look >= 0) {
                const CgScalars &v = snap[look];
                if (v.done) break;
                // reliable update: r <- b - mask(dssum(A64 x)) in FP64, at most one
                // per snapshot that asked for it
                if (mixed && v.need_replace && v.n_replace >= replacements) {
                    CG_TRY(true_ax());
                    CG_TRY(launch_cg_replace(P, bc, w, r, own, site(SITE_REPLACE), sc, s));
                    ++replacements;
                }
            }
            prev = slot;
        }
        CG_TRY(launch_cg_finish(P, x, p, sc, s));
        CG_TRY(hipMemcpyAsync(&snap[2], sc, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
        if (opts.true_residual || mixed) {
            // ||b - mask(dssum(A64 x))|| over unique nodes, in FP64 (x is up to date:
            // the finish kernel above ran; running it again is a no-op only if the
            // lag flag says so, so evaluate A x directly)
            CG_TRY(launch_ax_f64(E, N, D, g, x, w, plain_cg, s));
            CG_TRY(launch_gs(gs->cg, w, s));
            CG_TRY(launch_gdiff2(P, bc, w, own, site(SITE_RESID), scratch1, s));
            CG_TRY(hipMemcpyAsync(&snap[3].bb, scratch1, sizeof(double), hipMemcpyDeviceToHost, s));
        }
        // x back to the layout of Listing 1 (through w, which is free now)
        CG_TRY(launch_permute(E, N, x, w, false, s));
        CG_TRY(hipMemcpyAsync(x, w, (size_t)P * sizeof(double), hipMemcpyDeviceToDevice, s));
        CG_TRY(hipStreamSynchronize(s));
        S = snap[2];
        if (opts.true_residual || mixed) true_rel = S.bb > 0.0 ? sqrt(snap[3].bb / S.bb) : 0.0;
    }
out:
#undef CG_TRY
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    return rc;
}

// Status and statistics of a finished solve.
int cg_report(const char *who, const nek_cg_opts &opts, const CgPlan &pl, const CgScalars &S, double true_rel,
              nek_cg_stats *st) {
    int status = S.status;
    const double rel = S.bb > 0.0 ? sqrt(S.rr / S.bb) : 0.0;
    if (status == NEK_OK && opts.rel_tol > 0.0) {
        const double judged = pl.mixed ? true_rel : rel;
        if (!(judged <= opts.rel_tol)) status = NEK_ERR_NOCONV;
    }
    if (st) {
        st->iters = S.it;
        st->status = status;
        st->rel_res = rel;
        st->rel_res_true = true_rel;
        st->n_replacements = S.n_replace;
    }
    if (status == NEK_ERR_BREAKDOWN) return fail(status, std::string(who) + ": breakdown ((p,Ap) <= 0 or non-finite)");
    if (status == NEK_ERR_NOCONV) return fail(status, std::string(who) + ": tolerance not reached");
    return NEK_OK;
}

void cg_stats_init(nek_cg_stats *st) {
    if (!st) return;
    st->iters = 0;
    st->status = NEK_OK;
    st->rel_res = -1.0;
    st->rel_res_true = -1.0;
    st->n_replacements = 0;
}
}  // namespace

int nek_cg_solve(int64_t E, int N, const double *D, const double *g, const nek_gs *gs,
                 const double *b, double *x, const nek_cg_opts *opts_in, nek_cg_stats *st,
                 void *stream_v) {
    clear_error();
    nek_cg_opts opts;
    if (opts_in) opts = *opts_in;
    else nek_cg_default_opts(&opts);
    cg_stats_init(st);
    CgPlan pl;
    int rc = cg_check("nek_cg_solve", E, N, D, g, gs, b, x, opts, pl);
    if (rc != NEK_OK) return rc;
    hipStream_t s = (hipStream_t)stream_v;
    char *ws = (char *)opts.workspace;
    bool own_ws = false;
    if (ws) {
        if (opts.workspace_bytes < pl.need) return fail(NEK_ERR_ARG, "nek_cg_solve: workspace too small");
        if ((uintptr_t)ws & 255u) return fail(NEK_ERR_ARG, "nek_cg_solve: workspace must be 256-byte aligned");
    } else {
        hipError_t e = hipMallocAsync((void **)&ws, pl.need, s);
        if (e != hipSuccess)
            return fail(e == hipErrorOutOfMemory ? NEK_ERR_NOMEM : NEK_ERR_DEVICE,
                        std::string("nek_cg_solve: workspace allocation: ") + hipGetErrorString(e));
        own_ws = true;
    }
    if (!g_snap.buf) {
        hipError_t e = hipHostMalloc((void **)&g_snap.buf, 4 * sizeof(CgScalars), hipHostMallocDefault);
        if (e != hipSuccess) {
            if (own_ws) (void)hipFreeAsync(ws, s);
            return check_hip(e, "nek_cg_solve: hipHostMalloc");
        }
    }
    CgScalars S;
    double true_rel = -1.0;
    rc = cg_run(E, N, D, g, gs, b, x, opts, pl, ws, g_snap.buf, true, s, S, true_rel);
    if (own_ws) {
        if (rc != NEK_OK) (void)hipStreamSynchronize(s);
        (void)hipFreeAsync(ws, s);
    }
    if (rc != NEK_OK) {
        if (st) st->status = rc;
        return rc;
    }
    return cg_report("nek_cg_solve", opts, pl, S, true_rel, st);
}

}  // extern "C"

// ---------------------------------------------------------------- CG without allocation
// The workspace of nek_cg_solve_noalloc.  In host code `scratch` names a
// host-side stand-in, not device memory: only the address that
// hipGetSymbolAddress returns for the current device is ever handed to a
// kernel or a copy.
static __device__ __align__(256) char scratch[NEK_CG_NOALLOC_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char *g_scratch_dev[MAX_DEVICES] = {};

// The device address of `scratch` on the current device, looked up once per
// device with that device current.
int scratch_address(char **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return check_hip(e, "nek_cg_solve_noalloc: hipGetDevice");
    if (dev < 0 || dev >= MAX_DEVICES) return fail(NEK_ERR_DEVICE, "nek_cg_solve_noalloc: device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return check_hip(e, "nek_cg_solve_noalloc: hipGetSymbolAddress");
        if (!p || ((uintptr_t)p & 255u)) return fail(NEK_ERR_DEVICE, "nek_cg_solve_noalloc: workspace symbol not 256-byte aligned");
        g_scratch_dev[dev] = (char *)p;
    }
    *out = g_scratch_dev[dev];
    return NEK_OK;
}
}  // namespace

extern "C" int nek_cg_solve_noalloc(int64_t E, int N, const double *D, const double *g, const nek_gs *gs,
                                    const double *b, double *x, const nek_cg_opts *opts_in, nek_cg_stats *st,
                                    void *stream_v) {
    clear_error();
    nek_cg_opts opts;
    if (opts_in) opts = *opts_in;
    else nek_cg_default_opts(&opts);
    cg_stats_init(st);
    if (opts.workspace) return fail(NEK_ERR_ARG, "nek_cg_solve_noalloc: takes no workspace (opts->workspace must be NULL)");
    CgPlan pl;
    int rc = cg_check("nek_cg_solve_noalloc", E, N, D, g, gs, b, x, opts, pl);
    if (rc != NEK_OK) return rc;
    if (pl.need > NEK_CG_NOALLOC_BYTES)
        return fail(NEK_ERR_ARG, "nek_cg_solve_noalloc: the solve needs " + std::to_string(pl.need) +
                                     " bytes of workspace, more than NEK_CG_NOALLOC_BYTES = " +
                                     std::to_string((size_t)NEK_CG_NOALLOC_BYTES));
    char *ws = nullptr;
    rc = scratch_address(&ws);
    if (rc != NEK_OK) return rc;
    CgScalars snap[4];   // polled with synchronous copies into pageable memory
    CgScalars S;
    double true_rel = -1.0;
    rc = cg_run(E, N, D, g, gs, b, x, opts, pl, ws, snap, false, (hipStream_t)stream_v, S, true_rel);
    if (rc != NEK_OK) {
        (void)hipStreamSynchronize((hipStream_t)stream_v);
        if (st) st->status = rc;
        return rc;
    }
    return cg_report("nek_cg_solve_noalloc", opts, pl, S, true_rel, st);
}
