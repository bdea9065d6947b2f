"""The CG's internal layout and its assemble-update step, against the FP64 oracle.

Inside nek_cg_solve every vector is kept in the CG layout (the faces at fixed
i gathered at the end of each layer) and the dssum is folded into the residual
update, with rows of 2 to 4 copies on a fast path and every other row kind on
a general one.  These cases reach what the box tests of the paper's shapes do
not:

* every degree N = 1..15 (N = 1 has no points with 0 < i < n-1, N = 2 one per
  row), 40 iterations (12 at N = 1): the solution within rel-L2 1e-12 of the
  oracle's and the same recurrence residual to 1e-9 relative;
* a numbering in which groups of nodes are glued into one: nodes with 3, 5, 6
  and 12 copies (the general rows, including the CSR rows of more than 8
  copies) and nodes with two copies in one element; the operator stays SPD,
  so CG to 1e-11 must reach the oracle's solution;
* an odd number of local points with a glued numbering (the last point is
  handled apart from the pairs), solved to 1e-11; and the box numbering of
  that shape compared iterate by iterate (25 iterations, within rel-L2
  1e-12).  On the glued numberings CG is far
  too sensitive for that (a 1e-15 relative change of b moves the 25th iterate
  by 3e-6 in the oracle itself), so only converged solutions are compared;
* the solution comes back in the layout of Listing 1: x after 0 iterations is
  0, and after one iteration it equals alpha * b exactly as the oracle
  computes it (to rounding);
* at N = 5 on E = 2048 and N = 7, 8 on E = 1024, above the range of the
  one-thread-per-node operator that the small meshes here use at N = 3..9,
  the pencil operator: 30 iterations within 1e-12 of the oracle.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nek():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_13425_amd as nek
    return nek


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rel(a, b):
    a = a.detach().cpu().numpy() if hasattr(a, "detach") else np.asarray(a)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _mesh(box, N):
    return oracle.box_mesh(*box, N, synth.AMP, synth.geom_coeffs())


def _solve(nek, m, b, iters, rel_tol=0.0):
    gs = nek.GatherScatter(m.E, m.N, m.glo, m.dirichlet)
    x, res = nek.cg_solve(_dev(m.D), _dev(m.g), gs, _dev(b), max_iter=iters, rel_tol=rel_tol,
                          true_residual=True)
    torch.cuda.synchronize()
    gs.close()
    return x, res


BOX = {1: (5, 4, 4), 2: (4, 3, 3), 3: (3, 3, 3), 4: (3, 3, 2), 5: (3, 2, 2), 6: (3, 2, 2)}


@pytest.mark.parametrize("N", list(range(1, 16)))
def test_cg_every_degree(nek, N):
    box = BOX.get(N, (2, 2, 2))
    m = _mesh(box, N)
    b = oracle.lattice_to_local(m, synth.lattice_uniform(*box, N))
    iters = 12 if N == 1 else 40     # N = 1 converges to rounding noise by 30
    x, res = _solve(nek, m, b, iters)
    ref = oracle.cg(m, b, max_iter=iters)
    err = _rel(x, ref.x)
    print(f"CG N={N} box={box}: iters {res.iters}/{ref.iters} rel-L2 {err:.2e}", flush=True)
    assert res.status == 0 and res.iters == ref.iters
    assert err <= 1e-12
    assert abs(res.rel_res - ref.res_hist[-1]) <= 1e-9 * ref.res_hist[-1] + 1e-14


@pytest.mark.parametrize("N,box", [(5, (16, 16, 8)), (7, (16, 8, 8)), (8, (16, 8, 8))])
def test_cg_pencil_operator_above_the_node_range(nek, N, box):
    # Up to 400 000 local points the solver runs the operator with one thread
    # per node at N = 3..9 (the small meshes above); above that (442 368,
    # 524 288 and 746 496 points here) it takes the pencil operator
    m = _mesh(box, N)
    b = oracle.lattice_to_local(m, synth.lattice_uniform(*box, N))
    x, res = _solve(nek, m, b, 30)
    ref = oracle.cg(m, b, max_iter=30)
    err = _rel(x, ref.x)
    print(f"CG box={box} N={N}: rel-L2 {err:.2e}", flush=True)
    assert res.iters == ref.iters == 30
    assert err <= 1e-12


def _glued(box, N, seed=5):
    """A box numbering with groups of unmasked nodes merged into single nodes."""
    m = _mesh(box, N)
    glo = m.glo.copy()
    rng = np.random.default_rng(seed)
    copies = np.bincount(glo, minlength=m.U)
    masked = np.zeros(m.U, dtype=bool)
    masked[glo[m.dirichlet == 1]] = True
    free = np.flatnonzero(~masked)
    rng.shuffle(free)
    by_count = {c: [int(v) for v in free if copies[v] == c] for c in (1, 2, 4, 8)}
    groups = [
        by_count[1][0:3],                       # 3 copies in 3 elements or fewer
        by_count[2][0:1] + by_count[1][3:6],    # 5 copies
        by_count[2][1:4],                       # 6 copies
        by_count[8][0:1] + by_count[4][0:1],    # 12 copies: a CSR row
    ]
    # two element-interior nodes of one element: one node, two copies in one element
    n3 = (N + 1) ** 3
    e0 = m.E // 2
    inner = [int(glo[e0 * n3 + l]) for l in range(n3) if copies[glo[e0 * n3 + l]] == 1]
    groups.append(inner[:2])
    for grp in groups:
        assert len(grp) >= 2
        for v in grp[1:]:
            glo[glo == v] = grp[0]
    return dataclasses.replace(m, glo=glo), groups


def test_cg_glued_numbering_general_rows(nek):
    box, N = (4, 3, 3), 3
    m, groups = _glued(box, N)
    counts = np.bincount(m.glo)
    sizes = sorted(int(counts[g[0]]) for g in groups)
    assert sizes == [2, 3, 5, 6, 12]
    b = oracle.lattice_to_local(m, synth.lattice_uniform(*box, N))
    x, res = _solve(nek, m, b, 3000, rel_tol=1e-11)
    ref = oracle.cg(m, b, max_iter=3000, rel_tol=1e-11)
    err = _rel(x, ref.x)
    print(f"glued CG: iters {res.iters}/{ref.iters} rel-L2 {err:.2e} true {res.rel_res_true:.2e}", flush=True)
    assert res.status == 0 and ref.status == 0
    assert abs(res.iters - ref.iters) <= 3
    assert res.rel_res_true <= 1e-10
    assert err <= 1e-9
    # x is continuous under the glued numbering: copies of every node agree
    xh = x.cpu().numpy()
    for grp in groups:
        vals = xh[m.glo == grp[0]]
        assert np.all(vals == vals[0])


def test_cg_glued_numbering_odd_point_count(nek):
    box, N = (3, 3, 3), 4      # 27 * 125 local points: odd
    m, _ = _glued(box, N, seed=9)
    assert m.P % 2 == 1
    b = oracle.lattice_to_local(m, synth.lattice_uniform(*box, N))
    x, res = _solve(nek, m, b, 3000, rel_tol=1e-11)
    ref = oracle.cg(m, b, max_iter=3000, rel_tol=1e-11)
    err = _rel(x, ref.x)
    print(f"glued odd CG: iters {res.iters}/{ref.iters} rel-L2 {err:.2e}", flush=True)
    assert res.status == 0 and ref.status == 0
    assert res.rel_res_true <= 1e-10
    assert err <= 1e-9


def test_cg_box_odd_point_count_every_iteration(nek):
    # the box numbering of the same shape: here CG is well conditioned enough
    # to compare the iterate itself after 25 steps
    box, N = (3, 3, 3), 4
    m = _mesh(box, N)
    b = oracle.lattice_to_local(m, synth.lattice_uniform(*box, N))
    x, res = _solve(nek, m, b, 25)
    ref = oracle.cg(m, b, max_iter=25)
    err = _rel(x, ref.x)
    print(f"CG box={box} N={N} (odd point count), 25 iterations: rel-L2 {err:.2e}", flush=True)
    assert res.iters == ref.iters == 25
    assert err <= 1e-12


def test_cg_returns_listing_layout(nek):
    box, N = (3, 2, 2), 4
    m = _mesh(box, N)
    b = oracle.lattice_to_local(m, synth.lattice_uniform(*box, N))
    x0, r0 = _solve(nek, m, b, 0)
    assert r0.iters == 0
    assert not torch.any(x0 != 0)
    x1, r1 = _solve(nek, m, b, 1)
    ref = oracle.cg(m, b, max_iter=1)
    # one step from x0 = 0: x1 = alpha b, a multiple of b in the local layout
    alpha = float(np.dot(ref.x, b) / np.dot(b, b))
    assert _rel(x1, alpha * b) <= 1e-13
    assert _rel(x1, ref.x) <= 1e-13
