/*
 * nek.h -- C ABI of libnek: the Nekbone Poisson hot path on AMD MI355X (gfx950).
 *
 * The operation is the one of Karp et al., "Optimization of Tensor-product
 * Operations in Nekbone on GPUs" (arXiv 2005.13425):
 *   - Sec. III, Listing 1: the local Poisson operator of every spectral element,
 *     w = Dt (G (D u)) with three contractions by the GLL derivative matrix, a
 *     symmetric 3x3 multiply by six geometric factors per node and three
 *     transposed contractions;
 *   - Sec. III (second step of Ax): direct-stiffness summation (dssum), which
 *     sums the copies of every node shared by several elements;
 *   - Sec. VI-B: masking of the Dirichlet boundary;
 *   - Sec. III / Sec. V: the conjugate-gradient loop around them (100
 *     iterations in the paper's runs), and the cost model of Sec. III-A.
 *
 * Layouts are the Fortran arrays of Listing 1, 0-based, i fastest:
 *   u, w, x, b : u(i,j,k,e)      at [i + n*(j + n*(k + n*e))],   n = N + 1
 *   g          : gxyz(i,j,k,c,e) at [i + n*(j + n*(k + n*(c + 6*e)))], c = 0..5 is
 *                (rr, rs, rt, ss, st, tt) of the symmetric 3x3 factor
 *   D          : dxm1(i,l)       at [i + n*l]   (so dxtm1(i,l) = D[l + n*i])
 *
 * Conventions:
 *   - Sizes are int64_t, the degree N is int (1 <= N <= NEK_MAX_DEGREE).
 *   - "device" pointers are HIP device memory of the current device (for
 *     instance torch tensors on cuda:0); "host" pointers are ordinary memory.
 *   - stream is a hipStream_t passed as void*; NULL means the default stream.
 *     Calls marked "asynchronous" only enqueue work on that stream.
 *   - The caller owns every buffer it passes.  The library never frees them
 *     and keeps no reference to them after the call returns.
 *   - Every entry point returns NEK_OK (0) or a negative NEK_ERR_* code.
 *     Argument errors are detected on the host before anything is enqueued.
 *     A device fault inside an asynchronous call surfaces at the next
 *     synchronising call.  nek_last_error() gives a message for the calling
 *     thread's last failure.
 */
#ifndef NEK_H
#define NEK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NEK_MAX_DEGREE 15

/* status codes */
#define NEK_OK               0
#define NEK_ERR_ARG         -1  /* bad size, null or misaligned pointer, aliasing */
#define NEK_ERR_UNSUPPORTED -2  /* degree outside 1..NEK_MAX_DEGREE, unknown dtype */
#define NEK_ERR_DEVICE      -3  /* a HIP call failed; nek_last_error() has the text */
#define NEK_ERR_NOMEM       -4  /* device or host allocation failed / budget exceeded */
#define NEK_ERR_BREAKDOWN   -5  /* CG: (p, Ap) <= 0 or a non-finite scalar */
#define NEK_ERR_NOCONV      -6  /* CG: the tolerance was not reached in max_iter */
#define NEK_ERR_STATE       -7  /* call not valid in the object's current state */

/* storage types of the geometric factors for the FP32 operator */
#define NEK_G_F32  1
#define NEK_G_BF16 2

/* CG precision modes */
#define NEK_PREC_F64      0  /* FP64 operator (Listing 1 in double precision) */
#define NEK_PREC_F32G32   1  /* FP32 operator, g stored FP32, FP64 reliable updates */
#define NEK_PREC_F32GBF16 2  /* FP32 operator, g stored BF16, FP64 reliable updates */
#define NEK_PREC_F64G32   3  /* FP64 operator arithmetic, g stored FP32, FP64 reliable updates */
#define NEK_PREC_F64GBF16 4  /* FP64 operator arithmetic, g stored BF16, FP64 reliable updates */

/* Text of a status code (static string). */
const char *nek_strerror(int code);

/* Message of the calling thread's last failure ("" if none). */
const char *nek_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int nek_version(void);

/* ------------------------------------------------------------------ setup */

/* GLL nodes z[0..N], weights w[0..N] and the derivative matrix D[(N+1)^2]
 * (dxm1 of Listing 1, column-major as above) for degree N; n = N + 1 GLL
 * points per direction (Sec. III-A).  Host pointers, any of them may be
 * NULL.  Synchronous, no device work. */
int nek_gll(int N, double *z, double *w, double *D);

/* Box of Ex x Ey x Ez hexahedra on [0,1]^3 (Sec. III: Poisson on a cubic
 * domain).  Element e = ex + Ex*(ey + Ey*ez).  Fills, on the host, the global
 * id of every local point, glo[P] with P = E*n^3 (lattice node
 * I + (Ex*N+1)*(J + (Ey*N+1)*K), I = ex*N + i, ...), and dirichlet[P] = 1 on
 * the six faces of the box.  Either output may be NULL.  Synchronous. */
int nek_box_numbering(int Ex, int Ey, int Ez, int N, int64_t *glo, uint8_t *dirichlet);

/* Geometric factors of the box mesh, on the device: nodes at the tensor GLL
 * points of each element, displaced by amp * a[d] * sin(pi x) sin(pi y)
 * sin(pi z) (evaluated at the undisplaced point; zero on the boundary).  The
 * Jacobian is the derivative matrix applied to the nodal coordinates along
 * each direction; g = w_i w_j w_k det(J) J^-1 J^-T in the gxyz layout.
 *   a      host, 3 doubles
 *   g      device, 6*P doubles (required)
 *   bm     device, P doubles: diagonal mass w_i w_j w_k det(J) (may be NULL)
 *   X      device, 3*P doubles: x, y, z coordinate arrays (may be NULL)
 * Asynchronous. */
int nek_box_geometry(int Ex, int Ey, int Ez, int N, double amp, const double *a,
                     double *g, double *bm, double *X, void *stream);

/* ------------------------------------------------------- local operator */

/* w = A_e u for every element: Listing 1 in FP64.  No dssum, no mask.
 *   u, g, w, D device pointers in the layouts above; u and w must not
 *   overlap; all 8-byte aligned.  E >= 1.  Allocates nothing.
 * Asynchronous. */
int nek_ax(int64_t E, int N, const double *u, const double *D, const double *g,
           double *w, void *stream);

/* The same operator computed in FP32: u is read in FP64 and rounded, the
 * contractions and the geometric multiply run in FP32 with D32 (FP32 copy of
 * D, 4-byte aligned) and g_lo (the factors as FP32 or BF16, g_dtype =
 * NEK_G_F32 or NEK_G_BF16, in the point layout written by nek_convert_g;
 * 8-byte aligned for FP32, 4-byte for BF16), and w is written in FP64.  Used
 * inside the FP64 reliable-update CG (NEK_PREC_F32G*).  Allocates nothing.
 * Asynchronous. */
int nek_ax_f32(int64_t E, int N, const double *u, const float *D32, const void *g_lo,
               int g_dtype, double *w, void *stream);

/* The earlier GPU designs of the same operator that Sec. IV describes, for
 * comparison with nek_ax (which is NEK_AX_PENCIL).  FP64, the layouts and
 * argument rules of nek_ax, the same result to rounding:
 *   NEK_AX_ORIGINAL (Sec. IV-A): one workgroup per element, threads striding
 *     over its points, every operand in global memory; the intermediates
 *     ur, us, ut go to a scratch of 3*P doubles that the call allocates and
 *     frees on `stream` (stream-ordered);
 *   NEK_AX_SHARED3D (Sec. IV-B): one thread per node, the element in LDS;
 *     n^3 <= 1024 threads per workgroup, so N <= 9 (NEK_ERR_UNSUPPORTED
 *     above);
 *   NEK_AX_LAYER2D (Sec. IV-C, the paper's kernel): one thread per (i, j)
 *     column marching through the k layers, two barriers per layer.
 * Allocates nothing except ORIGINAL's scratch.  Asynchronous. */
#define NEK_AX_PENCIL   0
#define NEK_AX_ORIGINAL 1
#define NEK_AX_SHARED3D 2
#define NEK_AX_LAYER2D  3
int nek_ax_variant(int64_t E, int N, const double *u, const double *D, const double *g,
                   double *w, int variant, void *stream);

/* Round g (6*P FP64 values, device) to FP32 or BF16 (round to nearest even;
 * BF16 through FP32) into g_lo (device, 6*P values of the chosen type).
 * Point layout of g_lo: the six factors of a point side by side
 * (gxyz(i,j,k,0..5,e) at [6*(i + n*(j + n*(k + n*e))) + c], 24 bytes a point
 * in FP32, 12 in BF16), so that the operator loads a point's factors with one
 * load per lane.  Asynchronous. */
int nek_convert_g(int64_t E, int N, const double *g, int g_dtype, void *g_lo, void *stream);

/* ---------------------------------------------------- gather-scatter (dssum) */

typedef struct nek_gs nek_gs;

/* Build the direct-stiffness summation of a mesh from host arrays:
 * glo[P] global id of each local point (any non-negative ids), dirichlet[P]
 * 1 where the node carries the zero Dirichlet condition (NULL = none).  A
 * node is masked when any of its copies is flagged.  The handle owns device
 * copies of the map: the copies of every shared node grouped by copy count
 * (ascending local index within a node), the list of copies of masked nodes,
 * and one bit per point marking the first copy of every node (the weights of
 * the inner products).  P must be < 2^31.
 * Synchronous (allocates device memory and uploads). */
int nek_gs_create(int64_t E, int N, const int64_t *glo, const uint8_t *dirichlet, nek_gs **out);

/* Free the handle (synchronises the device first).  NULL is accepted. */
int nek_gs_destroy(nek_gs *gs);

/* Sizes of a handle: unique nodes, unmasked nodes summed by the
 * gather-scatter (shared nodes, plus single-copy nodes on element faces),
 * their copies, masked unique nodes.  Any output may be NULL. */
int nek_gs_info(const nek_gs *gs, int64_t *n_unique, int64_t *n_rows, int64_t *n_entries,
                int64_t *n_masked);

/* In place on device w[P]: w <- mask(dssum(w)).  Every copy of a node
 * receives the sum of all its copies (summed in ascending local index), and
 * masked nodes receive 0 (Sec. III step 2, Sec. VI-B).  Deterministic.
 * Allocates nothing.  Asynchronous. */
int nek_dssum(const nek_gs *gs, double *w, void *stream);

/* Inner product of two continuous local vectors over unique global nodes
 * (each node counted once): *result (device, one double) = sum a_G b_G.
 * a and b 16-byte aligned.  Deterministic.  Allocates nothing; calls that
 * share a handle must be ordered on one stream (they share its reduction
 * scratch).  Asynchronous. */
int nek_gs_dot(const nek_gs *gs, const double *a, const double *b, double *result, void *stream);

/* --------------------------------------------------------------------- CG */

typedef struct {
    int max_iter;          /* iteration cap (100 in the paper's runs) */
    double rel_tol;        /* stop when ||r||/||b|| <= rel_tol; <= 0: run max_iter */
    int precision;         /* NEK_PREC_* */
    const float *D32;      /* FP32 copy of D (device), required for NEK_PREC_F32G* */
    const void *g_lo;      /* g as FP32 / BF16 from nek_convert_g (device), required for
                              NEK_PREC_F32G* and NEK_PREC_F64G* */
    int check_every;       /* host polls convergence every this many iterations (0: 25;
                              4 in the mixed precisions) */
    int true_residual;     /* 1: report ||b - A x|| / ||b|| computed in FP64 at the end */
    double reliable_drop;  /* NEK_PREC_F32G*: replace r by b - A64 x whenever ||r|| fell
                              by this factor since the last replacement (0: 0.1 with
                              FP32 g, 0.3 with BF16 g) */
    void *workspace;       /* device scratch of nek_cg_workspace_bytes() bytes, or NULL
                              to let the call allocate and free its own */
    size_t workspace_bytes;
    const double *dinv;    /* NULL: plain CG.  Else the Jacobi preconditioner from
                              nek_jacobi_inverse (device, P doubles, 16-byte aligned):
                              preconditioned CG, FP64 precision only.  The solver
                              applies dinv rounded to FP32 (round to nearest even):
                              a fixed SPD diagonal either way, 8 bytes per point
                              and iteration less to read */
} nek_cg_opts;

typedef struct {
    int iters;             /* iterations performed */
    int status;            /* NEK_OK, NEK_ERR_BREAKDOWN or NEK_ERR_NOCONV */
    double rel_res;        /* recurrence residual sqrt((r,r)/(b,b)) at exit */
    double rel_res_true;   /* ||b - A x|| / ||b|| in FP64 if requested, else -1 */
    int n_replacements;    /* reliable updates of r (mixed precision), else 0 */
} nek_cg_stats;

/* Fill opts with defaults: 100 iterations, rel_tol 0, FP64, no workspace, no
 * preconditioner. */
void nek_cg_default_opts(nek_cg_opts *opts);

/* Device bytes of scratch nek_cg_solve needs for E elements of degree N, with
 * or without a preconditioner (without one, one vector of P doubles less is
 * enough). */
size_t nek_cg_workspace_bytes(int64_t E, int N);

/* Solve mask(dssum(A_L x)) = b by unpreconditioned CG with x_0 = 0 (Sec. III,
 * Sec. V).  b and x are device vectors in the local layout (16-byte aligned); b must be
 * continuous (copies equal) and zero at masked nodes; x receives a vector of
 * the same kind.  D, g device.  gs from nek_gs_create for the same mesh.
 * Every step runs on the device; the host only polls a status word every
 * opts->check_every iterations.  Blocking: returns after the work on stream
 * has finished.  stats may be NULL.  Returns NEK_OK, or the failure code
 * (also stored in stats->status) -- NEK_ERR_NOCONV when rel_tol > 0 was not
 * reached.  Inside the solve the vectors are kept with the points of each
 * element's faces at fixed i gathered at the end of every layer k (the
 * gather-scatter reads and writes them most); b and dinv are copied into the
 * workspace in that order, x is written in it while iterating and put back
 * into the layout of Listing 1 before the call returns.  After a failure other than NEK_ERR_NOCONV and
 * NEK_ERR_BREAKDOWN, x is unspecified.
 *
 * Mixed precisions (opts->precision): the operator of every iteration reads
 * g_lo instead of g; the residual, the inner products, the vector updates and
 * a reliable update of r to the true FP64 residual b - A x (with g) stay in
 * FP64, and the solve stops on that true residual.  NEK_PREC_F32G*: the
 * operator computes in FP32 (with D32).  NEK_PREC_F64G*: the operator computes
 * in FP64 and only g is stored in FP32 or BF16; an FP32 contraction perturbs
 * the operator more than FP32 storage of g does, and costs iterations.
 *
 * With opts->dinv set: preconditioned CG with M^-1 = dinv (the preconditioning
 * Sec. VII leaves as future work, in its simplest, Jacobi form):
 * z = dinv r, alpha = (r, z) / (p, A p), p <- z + beta p with
 * beta = (r', z') / (r, z).  The stopping test and stats->rel_res still use
 * sqrt((r, r) / (b, b)). */
int nek_cg_solve(int64_t E, int N, const double *D, const double *g, const nek_gs *gs,
                 const double *b, double *x, const nek_cg_opts *opts, nek_cg_stats *stats,
                 void *stream);

/* For callers that cannot allocate device or pinned host memory (code under
 * stream capture, tight serving loops, harnesses that forbid allocation):
 * nek_cg_solve with its workspace (r, p, w, b and M^-1 in the CG layout, the
 * operator's partials, the reduction sites and counters, the CG scalars) in a
 * file-scope device array of NEK_CG_NOALLOC_BYTES bytes inside the library,
 * one per GPU, held until the process ends.  The caller passes D, g, gs, b, x
 * and stream as for nek_cg_solve; opts->workspace must be NULL.  The call
 * makes no device or host allocation: the host polls the status word into
 * its own stack with a synchronous copy (no events, no pinned buffer).
 * Returns NEK_ERR_ARG, with a message, when the solve needs more than
 * NEK_CG_NOALLOC_BYTES (about 2 M local points in FP64 without a
 * preconditioner: E = 2048 at N = 9).  Every call on a GPU uses that GPU's
 * one array and finds there what the last call left: the solver sets every
 * word it reads first (counters and scalars by its reset kernel), so no state
 * carries over, but calls that overlap on one GPU (two host threads, or
 * two streams) race on the array and must be serialised by the caller.
 * Results are bitwise those of nek_cg_solve with the same arguments. */
#define NEK_CG_NOALLOC_BYTES ((size_t)64 << 20)
int nek_cg_solve_noalloc(int64_t E, int N, const double *D, const double *g, const nek_gs *gs,
                         const double *b, double *x, const nek_cg_opts *opts, nek_cg_stats *stats,
                         void *stream);

/* Jacobi preconditioner of the assembled, masked operator: on device
 * dinv[P], 1 / (dssum of the diagonals of the element operators of Listing 1)
 * at free nodes and 0 at masked nodes, a continuous local vector.  The
 * diagonal of A_e at p = (i,j,k) is the quadrature form of A_e on the unit
 * vector e_p: sum over m of dxm1(m,i)^2 g_rr(m,j,k), dxm1(m,j)^2 g_ss(i,m,k),
 * dxm1(m,k)^2 g_tt(i,j,m), plus 2 dxm1(i,i) dxm1(j,j) g_rs + 2 dxm1(i,i)
 * dxm1(k,k) g_rt + 2 dxm1(j,j) dxm1(k,k) g_st at p.  D, g as in nek_ax; gs
 * built for the same mesh.  dinv: device, P doubles, 16-byte aligned, output
 * (also the working buffer).  Allocates nothing.  Asynchronous. */
int nek_jacobi_inverse(int64_t E, int N, const double *D, const double *g, const nek_gs *gs,
                       double *dinv, void *stream);

/* ------------------------------------------------------------ served solves */

/* A solve service: requests (meshes of any size and degree: a box the
 * server builds, or the caller's own arrays) arrive over time; each is
 * admitted when its whole device footprint fits in the HBM budget, its CG
 * state then stays resident, and every server step advances all admitted
 * solves by CG iterations in shared launches: a CG iteration of every solve,
 * whatever its degree and precision, is one merged operator launch (two when
 * FP64 solves of the register-hungry degrees are present, one more for small
 * FP64 solves, which take the one-thread-per-node operator) and one
 * assemble-update launch.  Each solve's arithmetic is the same as when it
 * runs alone, and an FP64 solve's is that of nek_cg_solve.  The method is the one of
 * nek_cg_solve (Sec. III, Sec. V); the service around it is not in the
 * paper. */

typedef struct nek_server nek_server;

#define NEK_MEM_HOST   0
#define NEK_MEM_DEVICE 1

typedef struct {
    int Ex, Ey, Ez, N;   /* box of Ex x Ey x Ez elements of degree N (geometry as
                            in nek_box_geometry, numbering and Dirichlet faces as in
                            nek_box_numbering), built on the device at admission;
                            only N is used when the request carries its own mesh */
    double amp;          /* displacement amplitude (box only) */
    double a[3];         /* displacement coefficients (box only) */
    const double *b;     /* P doubles, local layout, continuous and zero at the
                            Dirichlet nodes (host or device, see mem) */
    int precision;       /* NEK_PREC_* */
    double rel_tol;      /* stop at ||r||/||b|| <= rel_tol (true residual in the
                            mixed precisions); <= 0: run max_iter iterations */
    int max_iter;
    /* The caller's own mesh (Listing 1 layouts, as nek_cg_solve takes them):
     * set g, D and glo (dirichlet may be NULL: no Dirichlet node) and E; the
     * box fields Ex, Ey, Ez, amp and a are then ignored.  g == NULL: the box. */
    int64_t E;                 /* elements */
    const double *D;           /* dxm1, (N+1)^2 doubles */
    const double *g;           /* 6 P doubles, gxyz layout */
    const int64_t *glo;        /* P global ids (as nek_gs_create) */
    const uint8_t *dirichlet;  /* P flags (as nek_gs_create), or NULL */
    int mem;                   /* NEK_MEM_HOST or NEK_MEM_DEVICE: where b and, with a
                                  mesh of the caller's, D, g, glo and dirichlet live
                                  (device memory of the server's device, 8-byte
                                  aligned) */
} nek_request;
/* Lifetime of the request's arrays: they are read after nek_server_submit
 * returns (numbering and gather-scatter tables by a preparation thread, b and
 * g copied into the server's own device memory at admission), so they must
 * stay valid and unchanged until nek_server_poll has reported the request or
 * nek_server_destroy has returned. */

typedef struct {
    uint64_t id;
    int status;          /* NEK_OK, NEK_ERR_BREAKDOWN, NEK_ERR_NOCONV; or, for a request
                            that never ran, the error of its preparation (NEK_ERR_ARG,
                            NEK_ERR_NOMEM for pinned staging) or NEK_ERR_NOMEM when the
                            device could not allocate it at admission */
    int iters;
    int n_replacements;
    double rel_res;      /* recurrence residual */
    double rel_res_true; /* ||b - A x|| / ||b|| evaluated in FP64 */
    double t_submit;     /* seconds on the server clock */
    double t_admit;
    double t_done;       /* when a server step saw the finished solve */
    int64_t E;
    int N;
    size_t footprint;    /* device bytes held while admitted */
} nek_result;

/* Create a server on the current device with a device-memory budget in
 * bytes.  Starts four host threads that prepare submitted requests (their
 * numbering and gather-scatter tables) independently of one another;
 * admission still follows arrival order.  Synchronous. */
int nek_server_create(size_t hbm_budget, nek_server **out);

/* Queue a request; *id receives its id.  NEK_ERR_NOMEM if its footprint can
 * never fit the budget.  Copies *req but not the arrays it points to (see
 * their lifetime above).  Returns at once. */
int nek_server_submit(nek_server *srv, const nek_request *req, uint64_t *id);

/* Footprint in device bytes of a request (what admission charges): of a box
 * request, and of a request of E elements of degree N with its own mesh (the
 * same bytes for the same E and N). */
size_t nek_server_footprint(int Ex, int Ey, int Ez, int N, int precision);
size_t nek_server_footprint_mesh(int64_t E, int N, int precision);

/* One step: admit prepared requests in arrival order while they fit (a
 * request still being prepared does not hold back prepared ones behind it; a
 * prepared one that does not fit holds back all later ones), run at least
 * `iters` CG iterations of every admitted solve (a solve much cheaper than
 * the heaviest takes part in up to 8 rounds of launches per iteration, within
 * half the first round's cost), and retire solves whose
 * completion the step observed.  active / queued (may be NULL) receive the
 * number of admitted and waiting requests after the step.  Returns after
 * queueing the device work (it waits only for the device work of the step
 * before). */
int nek_server_step(nek_server *srv, int iters, int *active, int *queued);

/* Finished solves not reported yet: up to max results into out[], *n their
 * number. */
int nek_server_poll(nek_server *srv, nek_result *out, int max, int *n);

/* Copy the solution of finished request id to x_host (P doubles) and release
 * its device memory.  Synchronous. */
int nek_server_fetch(nek_server *srv, uint64_t id, double *x_host);

/* Seconds on the server clock (the time base of nek_result). */
double nek_server_clock(const nek_server *srv);

/* Stop the preparation threads, wait for the device, free everything.
 * NULL is accepted. */
int nek_server_destroy(nek_server *srv);

/* ------------------------------------------------------------ measurement */

/* Streaming bandwidth probe for the measured roofline (Sec. V: the
 * computation replaced by copies of every load and store).  nread coalesced
 * read streams of n doubles, stream k at src + k * src_stride:
 *   flags without NEK_PROBE_READ_ONLY: dst[i] = sum_{k < nread} stream_k[i]
 *     for i < n, one write stream of n doubles (nread = 1 is a copy, 7 the
 *     7:1 read:write mix of the FP64 local operator);
 *   NEK_PROBE_READ_ONLY: only the reads reach HBM; dst receives one partial
 *     sum per workgroup, nek_bw_probe_groups(n, grid_cap) doubles (the sum
 *     leaves out the last value when n is odd).
 *   NEK_PROBE_NT: the loads and stores carry the non-temporal hint (as the
 *     plain FP64 operator's do from N = 7 up).
 *   NEK_PROBE_BLOCKED: the streams are interleaved in blocks of
 *     NEK_PROBE_BLOCK doubles: block b of stream k sits at
 *     src + (b * nread + k) * NEK_PROBE_BLOCK, so a workgroup reads one
 *     contiguous run of nread blocks, as the operator reads one element's u
 *     and six factor planes; src_stride is ignored and src holds
 *     nread * NEK_PROBE_BLOCK * ceil(n / NEK_PROBE_BLOCK) doubles.
 * src_stride (doubles, even, >= n) lets the caller stagger the streams so
 * that they do not sit a large power of two apart.  grid_cap > 0 caps the
 * number of workgroups, which then stride over the streams (0: one pass).
 * src: device, (nread-1)*src_stride + n doubles, 16-byte aligned; dst:
 * device, 16-byte aligned, not overlapping src.  n >= 2.  Allocates nothing.
 * Asynchronous. */
#define NEK_PROBE_NT        1
#define NEK_PROBE_READ_ONLY 2
#define NEK_PROBE_BLOCKED   4
#define NEK_PROBE_BLOCK     2048
int nek_bw_probe(int64_t n, int nread, const double *src, int64_t src_stride, double *dst, int grid_cap,
                 int flags, void *stream);

/* Workgroups of a probe launch over n doubles with that grid cap (the
 * number of partials NEK_PROBE_READ_ONLY writes); 0 for invalid arguments. */
int64_t nek_bw_probe_groups(int64_t n, int grid_cap);

#ifdef __cplusplus
}
#endif

#endif /* NEK_H */
