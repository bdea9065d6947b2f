"""Independent numpy constructions used to pin the oracle.

Nothing here calls the oracle's arithmetic; it rebuilds the same mathematical
objects a different way:

* GLL points from numpy's Legendre class (roots of P_N'), weights from the
  textbook formula with numpy's P_N;
* Lagrange basis derivatives from the product rule, not from the closed-form
  derivative matrix;
* the element stiffness matrix by brute-force quadrature over basis pairs;
* the affine element matrix as a sum of Kronecker products of 1D matrices.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gll_numpy(N: int):
    PN = npleg.Legendre.basis(N)
    inner = np.sort(PN.deriv().roots().real) if N >= 2 else np.array([])
    z = np.concatenate([[-1.0], inner, [1.0]])
    w = 2.0 / (N * (N + 1) * PN(z) ** 2)
    return z, w


def lagrange_deriv(z):
    """L[m, p] = l_p'(z_m) by the product rule:
    l_p'(x) = sum_{q != p} 1/(z_p - z_q) prod_{r != p, q} (x - z_r)/(z_p - z_r)."""
    n = len(z)
    L = np.zeros((n, n))
    for p in range(n):
        for m in range(n):
            s = 0.0
            for q in range(n):
                if q == p:
                    continue
                t = 1.0 / (z[p] - z[q])
                for r in range(n):
                    if r == p or r == q:
                        continue
                    t *= (z[m] - z[r]) / (z[p] - z[r])
                s += t
            L[m, p] = s
    return L


def element_stiffness_brute(X_e, z, wq):
    """Dense stiffness of one element by quadrature at the GLL nodes.

    X_e: (3, n, n, n) nodal coordinates indexed [d, k, j, i].
    Basis p = (pi, pj, pk) is l_pi(r) l_pj(s) l_pk(t); its reference gradient at
    node m = (a, b, c) is (l_pi'(z_a) d_{pj b} d_{pk c}, d_{pi a} l_pj'(z_b) d_{pk c},
    d_{pi a} d_{pj b} l_pk'(z_c)).  Returns K (n^3, n^3) in i-fastest ordering.
    """
    n = len(z)
    L = lagrange_deriv(z)
    n3 = n ** 3
    # reference gradients G[m, p, 3]
    G = np.zeros((n3, n3, 3))
    for c in range(n):
        for b in range(n):
            for a in range(n):
                m = a + n * (b + n * c)
                for pk in range(n):
                    for pj in range(n):
                        for pi in range(n):
                            p = pi + n * (pj + n * pk)
                            G[m, p, 0] = L[a, pi] * (pj == b) * (pk == c)
                            G[m, p, 1] = (pi == a) * L[b, pj] * (pk == c)
                            G[m, p, 2] = (pi == a) * (pj == b) * L[c, pk]
    Xf = X_e.reshape(3, n3)          # i-fastest flattening matches p, m ordering
    K = np.zeros((n3, n3))
    for m in range(n3):
        # Jacobian J[d, b] = sum_p x_d(p) dphi_p/dr_b at node m
        J = Xf @ G[m]                 # (3, 3)
        det = np.linalg.det(J)
        Jinv = np.linalg.inv(J)
        c_idx = np.unravel_index(m, (n, n, n))  # (c, b, a)
        W = wq[c_idx[2]] * wq[c_idx[1]] * wq[c_idx[0]]
        phys = G[m] @ Jinv            # (n3, 3): grad_x phi_p = J^-T grad_r phi_p
        K += W * det * (phys @ phys.T)
    return K


def affine_element_matrix(z, wq, hx, hy, hz):
    """Element matrix of an axis-aligned box element with sides hx, hy, hz:
    (hy hz / 2hx) W(x)W(x)K1 + (hx hz / 2hy) W(x)K1(x)W + (hx hy / 2hz) K1(x)W(x)W
    in (t, s, r) Kronecker order (r = i fastest), K1 = D^T W D."""
    L = lagrange_deriv(z)
    W = np.diag(wq)
    K1 = L.T @ W @ L
    t1 = (hy * hz / (2 * hx)) * np.kron(np.kron(W, W), K1)
    t2 = (hx * hz / (2 * hy)) * np.kron(np.kron(W, K1), W)
    t3 = (hx * hy / (2 * hz)) * np.kron(np.kron(K1, W), W)
    return t1 + t2 + t3


def cg_dense(A, b, iters):
    """Textbook CG on a dense SPD matrix; returns the residual-norm history."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rho = r @ r
    hist = [np.sqrt(rho / (b @ b))]
    for _ in range(iters):
        w = A @ p
        alpha = rho / (p @ w)
        x = x + alpha * p
        r = r - alpha * w
        rho_new = r @ r
        hist.append(np.sqrt(rho_new / (b @ b)))
        p = r + (rho_new / rho) * p
        rho = rho_new
    return x, np.array(hist)


def pcg_dense(A, b, Minv, iters):
    """Textbook preconditioned CG on a dense SPD matrix with a diagonal
    preconditioner Minv (a vector); returns x and ||r|| / ||b|| per step."""
    x = np.zeros_like(b)
    r = b.copy()
    z = Minv * r
    p = z.copy()
    rz = r @ z
    hist = [np.sqrt((r @ r) / (b @ b))]
    for _ in range(iters):
        w = A @ p
        alpha = rz / (p @ w)
        x = x + alpha * p
        r = r - alpha * w
        z = Minv * r
        rz_new = r @ z
        hist.append(np.sqrt((r @ r) / (b @ b)))
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, np.array(hist)
