/*
 * nek_oracle.c -- plain, slow, obviously correct FP64 CPU oracle for the
 * Nekbone Poisson hot path (Karp et al., "Optimization of Tensor-product
 * Operations in Nekbone on GPUs", arXiv 2005.13425).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table or
 * helper with the GPU path.
 *
 * What it computes, each routine citing the passage it follows:
 *   or_gll        Gauss-Lobatto-Legendre nodes and weights (Sec. III-A: n GLL
 *                 points per direction, n = degree + 1).
 *   or_dxm1       the GLL derivative matrix dxm1(i,l) of Listing 1.
 *   or_box_coords nodal coordinates of a box of hexahedra on [0,1]^3 (Sec. III:
 *                 Poisson on a cubic domain), optionally displaced by a smooth
 *                 sine bump that vanishes on the boundary.
 *   or_geom       the six geometric factors gxyz(i,j,k,1..6,e) of Listing 1:
 *                 quadrature weight * det J * (J^-1 J^-T), J the isoparametric
 *                 Jacobian; also the diagonal mass w * det J.
 *   or_box_glonum global node numbering of the box lattice and the Dirichlet
 *                 flags of the domain boundary.
 *   or_ax         the local operator of Sec. III (Listing 1) from its
 *                 definition D^T G D: the reference gradient by three
 *                 one-dimensional derivatives, the geometric factors applied
 *                 per point, the transposed derivatives accumulated; per
 *                 element, no summation across elements.
 *   or_dssum      direct-stiffness summation: the second step of Ax in
 *                 Sec. III (local results are communicated to the elements
 *                 that share the node): every copy of a global node receives
 *                 the sum of all copies.
 *   or_mask       zero the Dirichlet nodes (masking, Sec. VI-B).
 *   or_gdot       inner product of two continuous vectors over unique global
 *                 nodes.
 *   or_cg         unpreconditioned conjugate gradients on the assembled,
 *                 masked system (Sec. III; 100 iterations in Sec. V).
 *   or_ax_diag    the diagonal of the element operator of Listing 1, from
 *                 the quadrature form of A_e applied to unit vectors.
 *   or_pcg        conjugate gradients preconditioned by the inverse of the
 *                 assembled diagonal (Jacobi): the preconditioning that
 *                 Sec. VII names as future work, in its simplest form.
 *
 * Layouts follow the Fortran arrays of Listing 1, 0-based:
 *   u(i,j,k,e)        at u[i + n*(j + n*(k + n*e))]
 *   gxyz(i,j,k,c,e)   at g[i + n*(j + n*(k + n*(c + 6*e)))], c = 0..5
 *   dxm1(i,l)         at D[i + n*l]      (so dxtm1(i,l) = dxm1(l,i) = D[l + n*i])
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* Legendre polynomial P_N(x) and its first derivative, by the three-term
 * recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}, and the derivative
 * recurrence P'_{k+1} = P'_{k-1} + (2k+1) P_k. */
static void legendre(int N, double x, double *PN, double *dPN)
{
    double p0 = 1.0, p1 = x;      /* P_0, P_1 */
    double d0 = 0.0, d1 = 1.0;    /* P'_0, P'_1 */
    if (N == 0) { *PN = 1.0; *dPN = 0.0; return; }
    for (int k = 1; k < N; ++k) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        double d2 = d0 + (2.0 * k + 1.0) * p1;
        p0 = p1; p1 = p2;
        d0 = d1; d1 = d2;
    }
    *PN = p1;
    *dPN = d1;
}

/* GLL nodes z[0..N] and weights w[0..N] for degree N >= 1 (n = N+1 points).
 * The end points are -1 and +1; the interior points are the roots of P'_N,
 * found by Newton's method from Chebyshev-Gauss-Lobatto starting guesses,
 * using P''_N = (2x P'_N - N(N+1) P_N) / (1 - x^2) (Legendre's equation).
 * Weights: w_i = 2 / (N (N+1) P_N(z_i)^2).  Returns 0, or -1 for N < 1. */
int or_gll(int N, double *z, double *w)
{
    if (N < 1) return -1;
    z[0] = -1.0;
    z[N] = 1.0;
    for (int i = 1; i < N; ++i) {
        double x = -cos(OR_PI * (double)i / (double)N);
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(N, x, &P, &dP);
            double d2P = (2.0 * x * dP - N * (N + 1.0) * P) / (1.0 - x * x);
            double dx = dP / d2P;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        z[i] = x;
    }
    for (int i = 0; i <= N; ++i) {
        double P, dP;
        legendre(N, z[i], &P, &dP);
        w[i] = 2.0 / (N * (N + 1.0) * P * P);
    }
    return 0;
}

/* dxm1(i,l) = derivative of the l-th GLL Lagrange basis function at node i
 * (the differential matrix of Listing 1), stored at D[i + n*l].
 * Textbook closed form for GLL points:
 *   i != l : P_N(z_i) / (P_N(z_l) (z_i - z_l))
 *   i == l == 0 : -N(N+1)/4,   i == l == N : +N(N+1)/4,   otherwise 0. */
int or_dxm1(int N, const double *z, double *D)
{
    if (N < 1) return -1;
    int n = N + 1;
    for (int l = 0; l < n; ++l) {
        for (int i = 0; i < n; ++i) {
            double v;
            if (i != l) {
                double Pi, Pl, d;
                legendre(N, z[i], &Pi, &d);
                legendre(N, z[l], &Pl, &d);
                v = Pi / (Pl * (z[i] - z[l]));
            } else if (i == 0) {
                v = -0.25 * N * (N + 1.0);
            } else if (i == N) {
                v = 0.25 * N * (N + 1.0);
            } else {
                v = 0.0;
            }
            D[i + n * l] = v;
        }
    }
    return 0;
}

/* Nodal coordinates of an Ex x Ey x Ez box of hexahedra on [0,1]^3.
 * Element e = ex + Ex*(ey + Ey*ez); node (i,j,k) of element e sits at the
 * tensor GLL point: x0 = (ex + (z_i+1)/2)/Ex, y0 = (ey + (z_j+1)/2)/Ey,
 * z0 = (ez + (z_k+1)/2)/Ez.  The displaced mesh adds
 *   amp * a[d] * sin(pi x0) sin(pi y0) sin(pi z0)
 * to coordinate d, a smooth bump that vanishes on the boundary of the box.
 * X holds three arrays of P = E n^3 values: X[0..P) = x, X[P..2P) = y,
 * X[2P..3P) = z, each in the u(i,j,k,e) layout. */
void or_box_coords(int Ex, int Ey, int Ez, int N, const double *zg,
                   double amp, const double *a, double *X)
{
    int n = N + 1;
    int64_t E = (int64_t)Ex * Ey * Ez;
    int64_t P = E * n * n * n;
    for (int ez = 0; ez < Ez; ++ez)
    for (int ey = 0; ey < Ey; ++ey)
    for (int ex = 0; ex < Ex; ++ex) {
        int64_t e = ex + (int64_t)Ex * (ey + (int64_t)Ey * ez);
        for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            int64_t L = i + n * (j + n * (k + n * e));
            double x0 = (ex + 0.5 * (zg[i] + 1.0)) / Ex;
            double y0 = (ey + 0.5 * (zg[j] + 1.0)) / Ey;
            double z0 = (ez + 0.5 * (zg[k] + 1.0)) / Ez;
            double s = sin(OR_PI * x0) * sin(OR_PI * y0) * sin(OR_PI * z0);
            X[L] = x0 + amp * a[0] * s;
            X[P + L] = y0 + amp * a[1] * s;
            X[2 * P + L] = z0 + amp * a[2] * s;
        }
    }
}

/* Geometric factors of Listing 1 (gxyz) for E elements of degree N.
 * Per node, the Jacobian J_ab = d x_a / d r_b of the isoparametric map is the
 * derivative matrix applied to the nodal coordinates along r (i), s (j) and
 * t (k).  With W = w_i w_j w_k the tensor GLL weight and K = J^-1 J^-T,
 *   gxyz(.,c) = W det(J) K_c,  c = (rr, rs, rt, ss, st, tt).
 * bm (may be NULL) receives the diagonal mass W det(J).
 * Returns the minimum of det(J) over all nodes. */
double or_geom(int64_t E, int N, const double *wq, const double *D,
               const double *X, double *g, double *bm)
{
    int n = N + 1;
    int64_t n3 = (int64_t)n * n * n;
    int64_t P = E * n3;
    double detmin = INFINITY;
    for (int64_t e = 0; e < E; ++e) {
        for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            int64_t L = i + n * (j + n * (k + n * e));
            double J[3][3];
            for (int a = 0; a < 3; ++a) {
                const double *xa = X + a * P + e * n3;
                double dr = 0.0, ds = 0.0, dt = 0.0;
                for (int l = 0; l < n; ++l) {
                    dr += D[i + n * l] * xa[l + n * (j + n * k)];
                    ds += D[j + n * l] * xa[i + n * (l + n * k)];
                    dt += D[k + n * l] * xa[i + n * (j + n * l)];
                }
                J[a][0] = dr; J[a][1] = ds; J[a][2] = dt;
            }
            double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
                       - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
                       + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
            if (det < detmin) detmin = det;
            /* inverse via the adjugate: Ji[b][a] = cofactor(a,b) / det */
            double Ji[3][3];
            Ji[0][0] =  (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
            Ji[0][1] = -(J[0][1] * J[2][2] - J[0][2] * J[2][1]) / det;
            Ji[0][2] =  (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
            Ji[1][0] = -(J[1][0] * J[2][2] - J[1][2] * J[2][0]) / det;
            Ji[1][1] =  (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
            Ji[1][2] = -(J[0][0] * J[1][2] - J[0][2] * J[1][0]) / det;
            Ji[2][0] =  (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
            Ji[2][1] = -(J[0][0] * J[2][1] - J[0][1] * J[2][0]) / det;
            Ji[2][2] =  (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
            double K[3][3];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    K[a][b] = Ji[a][0] * Ji[b][0] + Ji[a][1] * Ji[b][1] + Ji[a][2] * Ji[b][2];
            double W = wq[i] * wq[j] * wq[k];
            double s = W * det;
            int64_t base = i + n * (j + n * k);
            double *ge = g + 6 * n3 * e;
            ge[0 * n3 + base] = s * K[0][0];
            ge[1 * n3 + base] = s * K[0][1];
            ge[2 * n3 + base] = s * K[0][2];
            ge[3 * n3 + base] = s * K[1][1];
            ge[4 * n3 + base] = s * K[1][2];
            ge[5 * n3 + base] = s * K[2][2];
            if (bm) bm[L] = s;
        }
    }
    return detmin;
}

/* Global numbering of the box lattice: node (i,j,k) of element
 * (ex,ey,ez) is lattice point I = ex*N+i, J = ey*N+j, K = ez*N+k with id
 * I + (Ex*N+1)*(J + (Ey*N+1)*K).  dirichlet (may be NULL) is 1 on the
 * six faces of the box (zero Dirichlet condition), else 0. */
void or_box_glonum(int Ex, int Ey, int Ez, int N, int64_t *glo, uint8_t *dirichlet)
{
    int n = N + 1;
    int64_t nx = (int64_t)Ex * N + 1, ny = (int64_t)Ey * N + 1;
    for (int ez = 0; ez < Ez; ++ez)
    for (int ey = 0; ey < Ey; ++ey)
    for (int ex = 0; ex < Ex; ++ex) {
        int64_t e = ex + (int64_t)Ex * (ey + (int64_t)Ey * ez);
        for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            int64_t L = i + n * (j + n * (k + n * e));
            int64_t I = (int64_t)ex * N + i, J = (int64_t)ey * N + j, K = (int64_t)ez * N + k;
            glo[L] = I + nx * (J + ny * K);
            if (dirichlet)
                dirichlet[L] = (I == 0 || I == (int64_t)Ex * N ||
                                J == 0 || J == (int64_t)Ey * N ||
                                K == 0 || K == (int64_t)Ez * N) ? 1 : 0;
        }
    }
}

/* One-dimensional derivative along direction dir (0: r, index i; 1: s,
 * index j; 2: t, index k) of an n^3 block f in the layout of Listing 1:
 *   out(p) = sum over m of M(p_dir, m) f(p with its dir index set to m)
 * with M = dxm1 (transpose = 0), or M = dxtm1 = dxm1^T (transpose = 1), the
 * transposed derivative of the weak form.  With accumulate the sum is added
 * to out(p), else it replaces it. */
static void derivative_1d(int n, const double *D, int transpose, int dir,
                          const double *f, double *out, int accumulate)
{
    const int64_t stride = dir == 0 ? 1 : (dir == 1 ? n : (int64_t)n * n);
    const int64_t n3 = (int64_t)n * n * n;
    for (int64_t p = 0; p < n3; ++p) {
        int q = (int)((p / stride) % n);            /* index of p along dir */
        int64_t line = p - (int64_t)q * stride;     /* the point of the line with index 0 */
        double sum = 0.0;
        for (int m = 0; m < n; ++m) {
            /* dxm1(q,m) = D[q + n m]; dxtm1(q,m) = dxm1(m,q) = D[m + n q] */
            double coef = transpose ? D[m + n * q] : D[q + n * m];
            sum = sum + coef * f[line + m * stride];
        }
        out[p] = accumulate ? out[p] + sum : sum;
    }
}

/* The local Poisson operator of Sec. III (Listing 1 is its reference form):
 * per element, w = sum over a, b of D_a^T G_ab D_b u, where D_a is the
 * derivative along reference direction a and G is the symmetric 3x3 field
 * of geometric factors.  Written out from that definition in three passes:
 *   1. the reference gradient (D_r u, D_s u, D_t u), one derivative at a
 *      time, into three whole arrays;
 *   2. the flux G grad u at every point;
 *   3. w = D_r^T flux_r, then + D_s^T flux_s, then + D_t^T flux_t.
 * Elements are independent, so the element loop may be shared among
 * threads; every element's arithmetic is the same whatever the thread
 * count. */
void or_ax(int64_t E, int N, const double *D, const double *g,
           const double *u, double *w, int nthreads)
{
    int n = N + 1;
    int64_t n3 = (int64_t)n * n * n;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads)
#endif
    {
        double *grad = (double *)malloc(sizeof(double) * 3 * n3);
        double *flux = (double *)malloc(sizeof(double) * 3 * n3);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (int64_t e = 0; e < E; ++e) {
            const double *ue = u + n3 * e;
            const double *ge = g + 6 * n3 * e;   /* rr, rs, rt, ss, st, tt */
            double *we = w + n3 * e;
            for (int a = 0; a < 3; ++a)
                derivative_1d(n, D, 0, a, ue, grad + a * n3, 0);
            for (int64_t p = 0; p < n3; ++p) {
                double G[3][3];
                G[0][0] = ge[0 * n3 + p];
                G[0][1] = G[1][0] = ge[1 * n3 + p];
                G[0][2] = G[2][0] = ge[2 * n3 + p];
                G[1][1] = ge[3 * n3 + p];
                G[1][2] = G[2][1] = ge[4 * n3 + p];
                G[2][2] = ge[5 * n3 + p];
                for (int a = 0; a < 3; ++a) {
                    double f = 0.0;
                    for (int b = 0; b < 3; ++b) f = f + G[a][b] * grad[b * n3 + p];
                    flux[a * n3 + p] = f;
                }
            }
            for (int a = 0; a < 3; ++a)
                derivative_1d(n, D, 1, a, flux + a * n3, we, a > 0);
        }
        free(grad); free(flux);
    }
}

/* Direct-stiffness summation (Sec. III, second step of Ax): every local copy
 * of a global node is replaced by the sum of all copies of that node.  The
 * sum over copies is taken in ascending local index.  U = number of global
 * ids (every glo value lies in [0, U)).  Returns 0, -1 on a bad id, -2 when
 * out of memory. */
int or_dssum(int64_t P, const int64_t *glo, int64_t U, double *w)
{
    double *S = (double *)calloc((size_t)U, sizeof(double));
    if (!S) return -2;
    for (int64_t L = 0; L < P; ++L) {
        if (glo[L] < 0 || glo[L] >= U) { free(S); return -1; }
        S[glo[L]] += w[L];
    }
    for (int64_t L = 0; L < P; ++L) w[L] = S[glo[L]];
    free(S);
    return 0;
}

/* Masking of the Dirichlet nodes (Sec. VI-B): w = 0 where dirichlet is set. */
void or_mask(int64_t P, const uint8_t *dirichlet, double *w)
{
    for (int64_t L = 0; L < P; ++L)
        if (dirichlet[L]) w[L] = 0.0;
}

/* Inner product of two continuous local vectors taken over unique global
 * nodes: each global id contributes once, through its first local copy in
 * ascending local order.  The terms are summed with Neumaier's compensated
 * summation, so the result is the exact sum of the rounded products to
 * within about one rounding: CG (Sec. III) amplifies the error of a plain
 * running sum over millions of terms into its iterates.  Returns NAN when
 * out of memory. */
double or_gdot(int64_t P, const int64_t *glo, int64_t U, const double *a, const double *b)
{
    uint8_t *seen = (uint8_t *)calloc((size_t)U, 1);
    if (!seen) return NAN;
    double s = 0.0, comp = 0.0;
    for (int64_t L = 0; L < P; ++L) {
        int64_t G = glo[L];
        if (!seen[G]) {
            seen[G] = 1;
            double term = a[L] * b[L];
            double t = s + term;
            if (fabs(s) >= fabs(term)) comp += (s - t) + term;
            else comp += (term - t) + s;
            s = t;
        }
    }
    free(seen);
    return s + comp;
}

/* Unpreconditioned conjugate gradients on the assembled, masked operator
 * (Sec. III: CG on Ax = f; Sec. V: 100 iterations; Sec. VII: no
 * preconditioner yet).  Vectors are continuous local vectors (all copies of
 * a node equal) that are zero at Dirichlet nodes; b must be such a vector.
 *   x_0 = 0, r_0 = b, p_0 = r_0, rho_0 = (r_0, r_0)
 *   per iteration:  w = mask(dssum(A_L p));  alpha = rho / (p, w)
 *                   x += alpha p;  r -= alpha w;  rho' = (r, r)
 *                   beta = rho' / rho;  p = r + beta p
 * With rel_tol > 0 the loop stops once sqrt(rho'/(b,b)) <= rel_tol; with
 * rel_tol <= 0 it runs exactly max_iter iterations (or stops when rho' = 0).
 * res_hist (may be NULL, length max_iter+1) receives sqrt(rho/(b,b)) at the
 * start and after each iteration.  *iters receives the iteration count.
 * Returns 0 on success, 1 when rel_tol was not reached, -5 on breakdown
 * ((p,w) <= 0 or a non-finite scalar), -2 when out of memory. */
int or_cg(int64_t E, int N, const double *D, const double *g,
          const int64_t *glo, int64_t U, const uint8_t *dirichlet,
          const double *b, double *x, int max_iter, double rel_tol,
          int *iters, double *res_hist, int nthreads)
{
    int n = N + 1;
    int64_t P = E * n * n * n;
    double *r = (double *)malloc(sizeof(double) * P);
    double *p = (double *)malloc(sizeof(double) * P);
    double *w = (double *)malloc(sizeof(double) * P);
    int status = 0, it = 0;
    if (!r || !p || !w) { free(r); free(p); free(w); return -2; }
    for (int64_t L = 0; L < P; ++L) { x[L] = 0.0; r[L] = b[L]; p[L] = b[L]; }
    double bb = or_gdot(P, glo, U, b, b);
    double rho = bb;
    if (res_hist) res_hist[0] = bb > 0.0 ? 1.0 : 0.0;
    for (it = 0; it < max_iter; ) {
        if (rho == 0.0) break;
        or_ax(E, N, D, g, p, w, nthreads);
        if (or_dssum(P, glo, U, w) != 0) { status = -2; break; }
        or_mask(P, dirichlet, w);
        double pw = or_gdot(P, glo, U, p, w);
        if (!(pw > 0.0) || !isfinite(pw)) { status = -5; break; }
        double alpha = rho / pw;
        for (int64_t L = 0; L < P; ++L) {
            x[L] = x[L] + alpha * p[L];
            r[L] = r[L] - alpha * w[L];
        }
        double rho_new = or_gdot(P, glo, U, r, r);
        ++it;
        if (!isfinite(rho_new)) { status = -5; break; }
        if (res_hist) res_hist[it] = sqrt(rho_new / bb);
        if (rel_tol > 0.0 && sqrt(rho_new / bb) <= rel_tol) { rho = rho_new; break; }
        double beta = rho_new / rho;
        rho = rho_new;
        for (int64_t L = 0; L < P; ++L) p[L] = r[L] + beta * p[L];
    }
    if (status == 0 && rel_tol > 0.0 && !(sqrt(rho / bb) <= rel_tol)) status = 1;
    *iters = it;
    free(r); free(p); free(w);
    return status;
}

/* Diagonal of the element operator of Listing 1, per local point.
 * A_e u = sum over quadrature points m of grad(phi)(m)^T G(m) grad(u)(m), with
 * the reference-space gradient of the basis function phi_p, p = (i,j,k), at
 * m = (i',j',k') equal to
 *   ( dxm1(i',i) [j'=j][k'=k],  [i'=i] dxm1(j',j) [k'=k],  [i'=i][j'=j] dxm1(k',k) ).
 * So (A_e)_pp = sum_m grad(phi_p)(m)^T G(m) grad(phi_p)(m).  Only the points m
 * on the three grid lines through p make a term non-zero: the rr term runs
 * over i', the ss term over j', the tt term over k', and each off-diagonal
 * term (rs, rt, st, each twice by symmetry) survives only at m = p.
 * Every element on its own; d has the layout of u. */
void or_ax_diag(int64_t E, int N, const double *D, const double *g, double *d)
{
    int n = N + 1;
    int64_t n3 = (int64_t)n * n * n;
    for (int64_t e = 0; e < E; ++e) {
        const double *ge = g + 6 * n3 * e;
        for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            int64_t p = i + n * (j + n * k);
            double s = 0.0;
            for (int m = 0; m < n; ++m) {     /* rr: points (m, j, k) */
                double dr = D[m + n * i];
                s = s + dr * ge[0 * n3 + (m + n * (j + n * k))] * dr;
            }
            for (int m = 0; m < n; ++m) {     /* ss: points (i, m, k) */
                double ds = D[m + n * j];
                s = s + ds * ge[3 * n3 + (i + n * (m + n * k))] * ds;
            }
            for (int m = 0; m < n; ++m) {     /* tt: points (i, j, m) */
                double dt = D[m + n * k];
                s = s + dt * ge[5 * n3 + (i + n * (j + n * m))] * dt;
            }
            double dii = D[i + n * i], djj = D[j + n * j], dkk = D[k + n * k];
            s = s + 2.0 * dii * ge[1 * n3 + p] * djj     /* rs at m = p */
                  + 2.0 * dii * ge[2 * n3 + p] * dkk     /* rt */
                  + 2.0 * djj * ge[4 * n3 + p] * dkk;    /* st */
            d[n3 * e + p] = s;
        }
    }
}

/* Conjugate gradients preconditioned with M^-1 = dinv, a continuous local
 * vector (for Jacobi: the mask divided by the assembled diagonal, zero at
 * Dirichlet nodes).  The textbook preconditioned recurrence:
 *   x_0 = 0, r_0 = b, z_0 = dinv r_0, p_0 = z_0, rz = (r_0, z_0)
 *   per iteration:  w = mask(dssum(A_L p));  alpha = rz / (p, w)
 *                   x += alpha p;  r -= alpha w;  z = dinv r
 *                   rz' = (r, z);  beta = rz' / rz;  p = z + beta p
 * The stopping test and res_hist use the unpreconditioned residual,
 * sqrt((r, r) / (b, b)), as or_cg does.  Return codes as or_cg. */
int or_pcg(int64_t E, int N, const double *D, const double *g,
           const int64_t *glo, int64_t U, const uint8_t *dirichlet, const double *dinv,
           const double *b, double *x, int max_iter, double rel_tol,
           int *iters, double *res_hist, int nthreads)
{
    int n = N + 1;
    int64_t P = E * n * n * n;
    double *r = (double *)malloc(sizeof(double) * P);
    double *z = (double *)malloc(sizeof(double) * P);
    double *p = (double *)malloc(sizeof(double) * P);
    double *w = (double *)malloc(sizeof(double) * P);
    int status = 0, it = 0;
    if (!r || !z || !p || !w) { free(r); free(z); free(p); free(w); return -2; }
    for (int64_t L = 0; L < P; ++L) {
        x[L] = 0.0;
        r[L] = b[L];
        z[L] = dinv[L] * r[L];
        p[L] = z[L];
    }
    double bb = or_gdot(P, glo, U, b, b);
    double rr = bb;
    double rz = or_gdot(P, glo, U, r, z);
    if (res_hist) res_hist[0] = bb > 0.0 ? 1.0 : 0.0;
    for (it = 0; it < max_iter; ) {
        if (rr == 0.0) break;
        or_ax(E, N, D, g, p, w, nthreads);
        if (or_dssum(P, glo, U, w) != 0) { status = -2; break; }
        or_mask(P, dirichlet, w);
        double pw = or_gdot(P, glo, U, p, w);
        if (!(pw > 0.0) || !isfinite(pw)) { status = -5; break; }
        double alpha = rz / pw;
        for (int64_t L = 0; L < P; ++L) {
            x[L] = x[L] + alpha * p[L];
            r[L] = r[L] - alpha * w[L];
            z[L] = dinv[L] * r[L];
        }
        rr = or_gdot(P, glo, U, r, r);
        double rz_new = or_gdot(P, glo, U, r, z);
        ++it;
        if (!isfinite(rr) || !isfinite(rz_new)) { status = -5; break; }
        if (res_hist) res_hist[it] = sqrt(rr / bb);
        if (rel_tol > 0.0 && sqrt(rr / bb) <= rel_tol) break;
        double beta = rz_new / rz;
        rz = rz_new;
        for (int64_t L = 0; L < P; ++L) p[L] = z[L] + beta * p[L];
    }
    if (status == 0 && rel_tol > 0.0 && !(sqrt(rr / bb) <= rel_tol)) status = 1;
    *iters = it;
    free(r); free(z); free(p); free(w);
    return status;
}

/* Number of threads the ax loop would use (1 without OpenMP). */
int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
