"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these retypes the oracle's formulas: each pin is a closed form, a
textbook table, an independent construction (numpy Legendre roots, product-
rule Lagrange derivatives, brute-force quadrature, Kronecker products, dense
linear algebra) or an invariant of the operator.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from tests import _brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _val(s):
    return float(eval(s, {"sqrt": math.sqrt}))


# ---------------------------------------------------------------- GLL points
def test_gll_closed_forms():
    gold = _load("gll_closed_forms.json")["cases"]
    for N, case in gold.items():
        z, w = oracle.gll(int(N))
        np.testing.assert_allclose(z, [_val(s) for s in case["z"]], atol=1e-15)
        np.testing.assert_allclose(w, [_val(s) for s in case["w"]], rtol=1e-14)


@pytest.mark.parametrize("N", list(range(1, 17)))
def test_gll_against_numpy_legendre_and_quadrature(N):
    z, w = oracle.gll(N)
    zn, wn = _brute.gll_numpy(N)
    np.testing.assert_allclose(z, zn, atol=1e-13)
    np.testing.assert_allclose(w, wn, rtol=1e-12)
    np.testing.assert_allclose(z, -z[::-1], atol=1e-15)
    assert abs(w.sum() - 2.0) < 1e-14
    for m in range(2 * N):          # exact for degree <= 2N - 1
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(np.dot(w, z ** m) - exact) < 1e-13, (N, m)


# --------------------------------------------------------- derivative matrix
@pytest.mark.parametrize("N", list(range(1, 17)))
def test_dxm1_exact_on_polynomials(N):
    z, _ = oracle.gll(N)
    D = oracle.dxm1(N, z)            # D[i, l] = dxm1(i, l)
    for m in range(N + 1):
        dm = m * z ** (m - 1) if m > 0 else np.zeros_like(z)
        assert np.max(np.abs(D @ z ** m - dm)) < 1e-11 * max(1, m), (N, m)
    assert np.max(np.abs(D.sum(axis=1))) < 1e-11   # D . 1 = 0


@pytest.mark.parametrize("N", [1, 2, 3, 5, 9, 15])
def test_dxm1_matches_product_rule(N):
    z, _ = oracle.gll(N)
    np.testing.assert_allclose(oracle.dxm1(N, z), _brute.lagrange_deriv(z), atol=1e-10)


def test_dxm1_layout_is_column_major():
    N = 3
    n = N + 1
    D2 = oracle.dxm1(N)
    flat = oracle.dxm1_flat(N)
    for i in range(n):
        for l in range(n):
            assert flat[i + n * l] == D2[i, l]


def test_stiffness_1d_N2_closed_form():
    gold = _load("gll_closed_forms.json")["stiffness_1d_N2"]
    z, w = oracle.gll(2)
    D = oracle.dxm1(2, z)
    K1 = D.T @ np.diag(w) @ D
    np.testing.assert_allclose(K1, np.array(gold["matrix"]) / 6.0, atol=1e-14)


# ------------------------------------------------------------------ geometry
def test_affine_geometry_closed_form():
    Ex, Ey, Ez, N = 3, 2, 4, 4
    m = oracle.box_mesh(Ex, Ey, Ez, N)
    n = N + 1
    hx, hy, hz = 1 / Ex, 1 / Ey, 1 / Ez
    g = m.g.reshape(m.E, 6, n, n, n)       # [e, c, k, j, i]
    W = np.einsum("k,j,i->kji", m.wq, m.wq, m.wq)
    for e in range(m.E):
        np.testing.assert_allclose(g[e, 0], W * hy * hz / (2 * hx), rtol=1e-13)
        np.testing.assert_allclose(g[e, 3], W * hx * hz / (2 * hy), rtol=1e-13)
        np.testing.assert_allclose(g[e, 5], W * hx * hy / (2 * hz), rtol=1e-13)
        for c in (1, 2, 4):
            assert np.max(np.abs(g[e, c])) < 1e-14
    np.testing.assert_allclose(m.bm.reshape(m.E, n, n, n)[0], W * hx * hy * hz / 8, rtol=1e-13)
    assert abs(m.detmin - hx * hy * hz / 8) < 1e-15


def test_perturbed_geometry_valid_and_conforming():
    a = synth.geom_coeffs()
    m = oracle.box_mesh(2, 2, 2, 4, synth.AMP, a)
    assert m.detmin > 0
    assert abs(m.bm.sum() - 1.0) < 1e-6          # discrete volume of the unit cube
    # nodes sharing a global id coincide (conformity of numbering + geometry)
    for d in range(3):
        first = np.full(m.U, np.nan)
        first[m.glo[::-1]] = m.X[d][::-1]
        np.testing.assert_allclose(m.X[d], first[m.glo], atol=1e-15)
    # the displacement vanishes on the boundary: boundary nodes stay on the box faces
    bd = m.dirichlet.astype(bool)
    on_face = np.zeros(m.P, bool)
    for d in range(3):
        on_face |= (np.abs(m.X[d]) < 1e-15) | (np.abs(m.X[d] - 1) < 1e-15)
    assert np.all(on_face[bd])


def test_mask_and_multiplicity_counts():
    Ex, Ey, Ez, N = 2, 2, 2, 4
    m = oracle.box_mesh(Ex, Ey, Ez, N)
    mult = oracle.dssum(m.glo, np.ones(m.P), m.U)
    # unique nodes by multiplicity
    first = np.unique(m.glo, return_index=True)[1]
    counts = {k: int(np.sum(mult[first] == k)) for k in (1, 2, 4, 8)}
    assert counts == {1: 512, 2: 192, 4: 24, 8: 1}
    nd = int(m.dirichlet[first].sum())
    assert nd == m.U - (Ex * N - 1) * (Ey * N - 1) * (Ez * N - 1)


# ----------------------------------------------------------------- operator
def _rand_mesh(Ex=2, Ey=2, Ez=1, N=4, amp=synth.AMP):
    return oracle.box_mesh(Ex, Ey, Ez, N, amp, synth.geom_coeffs())


@pytest.mark.parametrize("N", [1, 2, 3, 5, 9])
def test_ax_constants_in_kernel_symmetric_psd(N):
    m = _rand_mesh(2, 1, 2, N)
    n3 = (N + 1) ** 3
    w1 = oracle.ax(m.E, N, m.D, m.g, np.ones(m.P))
    assert np.max(np.abs(w1)) < 1e-12 * max(1, N * N)
    rng = np.random.default_rng(5)
    u, v = rng.uniform(-1, 1, m.P), rng.uniform(-1, 1, m.P)
    Au, Av = oracle.ax(m.E, N, m.D, m.g, u), oracle.ax(m.E, N, m.D, m.g, v)
    for e in range(m.E):
        s = slice(e * n3, (e + 1) * n3)
        vAu, uAv = v[s] @ Au[s], u[s] @ Av[s]
        assert abs(vAu - uAv) < 1e-12 * (abs(vAu) + 1)
        assert u[s] @ Au[s] > -1e-12


@pytest.mark.parametrize("N", [1, 2, 3])
def test_ax_matches_bruteforce_element_stiffness(N):
    m = _rand_mesh(2, 1, 1, N)
    n = N + 1
    n3 = n ** 3
    zb, wb = _brute.gll_numpy(N)
    rng = np.random.default_rng(11)
    u = rng.uniform(-1, 1, m.P)
    w = oracle.ax(m.E, N, m.D, m.g, u)
    for e in range(m.E):
        Xe = m.X[:, e * n3:(e + 1) * n3].reshape(3, n, n, n)
        K = _brute.element_stiffness_brute(Xe, zb, wb)
        np.testing.assert_allclose(K, K.T, atol=1e-13)
        ev = np.linalg.eigvalsh(K)
        assert abs(ev[0]) < 1e-12 and ev[1] > 1e-6    # one zero mode (constants)
        Ku = K @ u[e * n3:(e + 1) * n3]
        err = np.linalg.norm(Ku - w[e * n3:(e + 1) * n3]) / np.linalg.norm(Ku)
        assert err < 1e-13, err


@pytest.mark.parametrize("N,box", [(3, (1, 1, 1)), (4, (2, 1, 1)), (2, (1, 3, 2))])
def test_ax_affine_kronecker_closed_form(N, box):
    Ex, Ey, Ez = box
    m = oracle.box_mesh(Ex, Ey, Ez, N)
    n3 = (N + 1) ** 3
    zb, wb = _brute.gll_numpy(N)
    A = _brute.affine_element_matrix(zb, wb, 1 / Ex, 1 / Ey, 1 / Ez)
    rng = np.random.default_rng(3)
    u = rng.uniform(-1, 1, m.P)
    w = oracle.ax(m.E, N, m.D, m.g, u)
    for e in range(m.E):
        s = slice(e * n3, (e + 1) * n3)
        ref = A @ u[s]
        assert np.linalg.norm(ref - w[s]) / np.linalg.norm(ref) < 1e-13


@pytest.mark.parametrize("mpow", [1, 2, 3, 4])
def test_energy_of_monomials(mpow):
    # u = x^m on the unit cube: sum_e u^T A_e u = int |grad u|^2 = m^2/(2m-1)
    N = 4
    m = oracle.box_mesh(2, 3, 2, N)
    u = m.X[0] ** mpow
    e = float(u @ oracle.ax(m.E, N, m.D, m.g, u))
    assert abs(e - mpow ** 2 / (2 * mpow - 1)) < 1e-13


def test_energy_of_coordinate_field_is_discrete_volume():
    # isoparametric: u = x has grad u = e1 exactly, so the energy is sum W detJ
    N = 5
    m = _rand_mesh(2, 2, 2, N)
    u = m.X[0].copy()
    e = float(u @ oracle.ax(m.E, N, m.D, m.g, u))
    assert abs(e - m.bm.sum()) < 1e-12


# ---------------------------------------------------------------- dssum/mask
def test_dssum_conservation_and_projection():
    m = _rand_mesh(3, 2, 2, 3)
    rng = np.random.default_rng(1)
    w = rng.uniform(-1, 1, m.P)
    mult = oracle.dssum(m.glo, np.ones(m.P), m.U)
    assert set(np.unique(mult)) <= {1.0, 2.0, 4.0, 8.0}
    s = oracle.dssum(m.glo, w, m.U)
    assert abs(np.sum(s / mult) - np.sum(w)) < 1e-12
    np.testing.assert_allclose(oracle.dssum(m.glo, s / mult, m.U), s, atol=1e-14)
    # the result is continuous: copies of a node agree
    first = np.zeros(m.U)
    first[m.glo] = s
    np.testing.assert_array_equal(s, first[m.glo])


def test_patch_test_linear_function():
    # affine elements, u a global linear function: interior rows of the assembled
    # operator vanish (GLL integrates the affine case exactly)
    N = 4
    m = oracle.box_mesh(3, 2, 2, N)
    x, y, z = m.X
    u = 0.3 + 1.5 * x - 0.7 * y + 2.0 * z
    r = oracle.masked_ax(m, u)
    assert np.max(np.abs(r)) < 1e-12


def test_mask_zeroes_boundary_only():
    m = _rand_mesh(2, 2, 2, 3)
    v = oracle.mask(m.dirichlet, np.ones(m.P))
    assert np.all(v[m.dirichlet == 1] == 0) and np.all(v[m.dirichlet == 0] == 1)


def test_gdot_counts_each_node_once():
    m = _rand_mesh(2, 2, 1, 3)
    rng = np.random.default_rng(4)
    vals = rng.uniform(-1, 1, m.U)
    a = vals[m.glo]
    assert abs(oracle.gdot(m.glo, a, a, m.U) - vals @ vals) < 1e-12


# ------------------------------------------------------------------------ CG
def _assembled(m):
    """Dense assembled masked operator on the interior (unmasked) global nodes,
    built column by column from the oracle operator."""
    first = np.unique(m.glo, return_index=True)[1]
    interior = [G for G in range(m.U) if m.dirichlet[first[G]] == 0]
    A = np.zeros((len(interior), len(interior)))
    for c, G in enumerate(interior):
        u = (m.glo == G).astype(float)
        Au = oracle.masked_ax(m, u)
        A[:, c] = Au[first[interior]]
    return A, np.array(interior), first


@pytest.mark.parametrize("N", [1, 2, 3])
def test_cg_matches_dense_solve(N):
    m = _rand_mesh(2, 2, 2, N)
    A, interior, first = _assembled(m)
    np.testing.assert_allclose(A, A.T, atol=1e-13)
    np.linalg.cholesky(A)                                 # SPD on the interior
    vals = synth.lattice_uniform(2, 2, 2, N)
    b = oracle.lattice_to_local(m, vals)
    res = oracle.cg(m, b, max_iter=400, rel_tol=1e-13)
    assert res.status == 0
    assert res.iters <= len(interior) + 5
    xd = np.linalg.solve(A, b[first[interior]])
    np.testing.assert_allclose(res.x[first[interior]], xd, rtol=1e-11, atol=1e-12)
    # recurrence history equals textbook CG on the dense matrix
    _, hist = _brute.cg_dense(A, b[first[interior]], min(10, res.iters))
    np.testing.assert_allclose(res.res_hist[: len(hist)], hist, rtol=1e-9)
    # x is continuous and zero on the boundary
    assert np.all(res.x[m.dirichlet == 1] == 0)


def test_cg_manufactured_solution_converges_spectrally():
    errs = []
    for N in (2, 3, 4, 5, 6):
        m = _rand_mesh(2, 2, 2, N)
        b = oracle.manufactured_rhs(m)
        res = oracle.cg(m, b, max_iter=2000, rel_tol=1e-13)
        assert res.status == 0
        x, y, z = m.X
        ustar = np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)
        errs.append(np.max(np.abs(res.x - ustar)))
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1)), errs
    assert errs[-1] < 1e-4


def test_cg_fixed_iterations_and_breakdown():
    m = _rand_mesh(2, 2, 2, 3)
    b = oracle.lattice_to_local(m, synth.lattice_uniform(2, 2, 2, 3))
    res = oracle.cg(m, b, max_iter=7, rel_tol=0.0)
    assert res.iters == 7 and res.status == 0
    assert np.all(np.diff(res.res_hist) != 0)
    bad = b.copy()
    bad[np.argmax(m.dirichlet == 0)] = np.nan
    assert oracle.cg(m, bad, max_iter=5).status == -5


# ---------------------------------------------------------------- Jacobi PCG
@pytest.mark.parametrize("N", [1, 2, 3])
def test_ax_diag_matches_bruteforce_element_stiffness(N):
    # the diagonal of the dense quadrature stiffness (Lagrange derivatives by
    # the product rule, not dxm1) of each perturbed element
    m = _rand_mesh(2, 1, 1, N)
    n3 = (N + 1) ** 3
    zb, wb = _brute.gll_numpy(N)
    d = oracle.ax_diag(m.E, N, m.D, m.g)
    for e in range(m.E):
        Xe = m.X[:, e * n3:(e + 1) * n3].reshape(3, N + 1, N + 1, N + 1)
        K = _brute.element_stiffness_brute(Xe, zb, wb)
        np.testing.assert_allclose(d[e * n3:(e + 1) * n3], np.diag(K), rtol=1e-13, atol=0)


@pytest.mark.parametrize("N,box", [(4, (2, 1, 1)), (6, (1, 1, 2))])
def test_ax_diag_is_listing1_on_unit_vectors(N, box):
    m = _rand_mesh(*box, N)
    d = oracle.ax_diag(m.E, N, m.D, m.g)
    rng = np.random.default_rng(5)
    for L in rng.choice(m.P, size=40, replace=False):
        e = np.zeros(m.P)
        e[L] = 1.0
        assert abs(oracle.ax(m.E, N, m.D, m.g, e)[L] - d[L]) <= 1e-14 * abs(d[L])


def test_ax_diag_affine_closed_form():
    N, box = 3, (2, 1, 1)
    m = oracle.box_mesh(*box, N)
    zb, wb = _brute.gll_numpy(N)
    A = _brute.affine_element_matrix(zb, wb, 1 / box[0], 1 / box[1], 1 / box[2])
    d = oracle.ax_diag(m.E, N, m.D, m.g)
    n3 = (N + 1) ** 3
    for e in range(m.E):
        np.testing.assert_allclose(d[e * n3:(e + 1) * n3], np.diag(A), rtol=1e-13)


@pytest.mark.parametrize("N", [1, 2, 3])
def test_jacobi_inverse_is_inverse_of_assembled_diagonal(N):
    m = _rand_mesh(2, 2, 2, N)
    A, interior, first = _assembled(m)
    inv = oracle.jacobi_inverse(m)
    np.testing.assert_allclose(inv[first[interior]], 1.0 / np.diag(A), rtol=1e-13)
    assert np.all(inv[m.dirichlet == 1] == 0.0)
    # continuous: every copy of a node holds the same value
    for G in interior:
        assert np.ptp(inv[m.glo == G]) == 0.0


@pytest.mark.parametrize("N", [1, 2, 3])
def test_pcg_matches_dense_solve_and_textbook_recurrence(N):
    m = _rand_mesh(2, 2, 2, N)
    A, interior, first = _assembled(m)
    inv = oracle.jacobi_inverse(m)
    b = oracle.lattice_to_local(m, synth.lattice_uniform(2, 2, 2, N))
    res = oracle.pcg(m, b, inv, max_iter=400, rel_tol=1e-13)
    assert res.status == 0
    assert res.iters <= len(interior) + 5
    xd = np.linalg.solve(A, b[first[interior]])
    np.testing.assert_allclose(res.x[first[interior]], xd, rtol=1e-11, atol=1e-12)
    _, hist = _brute.pcg_dense(A, b[first[interior]], 1.0 / np.diag(A), min(10, res.iters))
    np.testing.assert_allclose(res.res_hist[: len(hist)], hist, rtol=1e-9, atol=1e-14)
    assert np.all(res.x[m.dirichlet == 1] == 0)


def test_pcg_with_identity_preconditioner_is_cg_bitwise():
    m = _rand_mesh(2, 2, 2, 4)
    b = oracle.lattice_to_local(m, synth.lattice_uniform(2, 2, 2, 4))
    ident = (m.dirichlet == 0).astype(np.float64)
    a = oracle.pcg(m, b, ident, max_iter=25)
    c = oracle.cg(m, b, max_iter=25)
    np.testing.assert_array_equal(a.x, c.x)
    np.testing.assert_array_equal(a.res_hist, c.res_hist)


def test_pcg_fewer_iterations_on_stretched_elements():
    # elements of aspect 2:1:1 make the diagonal vary; Jacobi pays off there
    m = oracle.box_mesh(4, 2, 2, 5, synth.AMP, synth.geom_coeffs())
    b = oracle.lattice_to_local(m, synth.lattice_uniform(4, 2, 2, 5))
    plain = oracle.cg(m, b, max_iter=3000, rel_tol=1e-10)
    jac = oracle.pcg(m, b, oracle.jacobi_inverse(m), max_iter=3000, rel_tol=1e-10)
    assert plain.status == 0 and jac.status == 0
    assert jac.iters < plain.iters
    assert np.linalg.norm(jac.x - plain.x) / np.linalg.norm(plain.x) < 1e-8


def test_paper_accounting_numbers():
    acc = _load("paper_accounting.json")
    n = acc["n"]
    assert 12 * n + 34 == acc["flops_per_dof_per_iter"]
    assert 8 * 30 == acc["bytes_per_dof_per_iter"]
    assert abs((12 * n + 34) / 240 - acc["intensity"]) < 1e-15
    for hw in acc["rooflines_gflops"].values():
        # the paper prints the product truncated to whole GFlop/s (900 * 0.6417 = 577.5 -> 577)
        assert int(hw["bw_gbs"] * (12 * n + 34) / 240) == hw["gflops"]
