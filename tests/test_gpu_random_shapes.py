"""Seeded random box shapes and degrees through the whole solver, against the
FP64 oracle: the CG layout, the gather-scatter maps and the assemble-update
on shapes no other test picks (thin boxes, one element across, odd and even
point counts).  30 iterations of CG and of Jacobi PCG each; the same bars as
the fixed-shape tests (solution rel-L2 <= 1e-12 after 30 iterations, same
recurrence residual to 1e-9 relative).
"""
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


def _cases(count=10, seed=2024):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        box = tuple(int(v) for v in rng.integers(1, 6, size=3))
        N = int(rng.integers(2, 13))
        if box[0] * box[1] * box[2] * (N + 1) ** 3 > 60000:
            continue
        out.append((box, N))
    return out


@pytest.mark.parametrize("box,N", _cases())
def test_random_shape_cg_and_pcg(nek, box, N):
    m = oracle.box_mesh(*box, N, synth.AMP, synth.geom_coeffs(seed=box[0] + 7 * N))
    b = oracle.lattice_to_local(m, synth.lattice_uniform(*box, N, seed=11 + N))
    assert np.any(b != 0.0)
    gs = nek.GatherScatter(m.E, N, m.glo, m.dirichlet)
    Dt, gt = _dev(m.D), _dev(m.g)
    iters = 30
    x, res = nek.cg_solve(Dt, gt, gs, _dev(b), max_iter=iters)
    ref = oracle.cg(m, b, max_iter=iters)
    dinv = oracle.jacobi_inverse(m)
    xp, resp = nek.cg_solve(Dt, gt, gs, _dev(b), max_iter=iters, dinv=_dev(dinv))
    refp = oracle.pcg(m, b, dinv.astype(np.float32).astype(np.float64), max_iter=iters)
    torch.cuda.synchronize()
    gs.close()
    e1, e2 = _rel(x, ref.x), _rel(xp, refp.x)
    print(f"box={box} N={N} P={m.P}: CG {res.iters}/{ref.iters} rel-L2 {e1:.2e}; "
          f"PCG {resp.iters}/{refp.iters} rel-L2 {e2:.2e}", flush=True)
    for r_, f_, e_ in ((res, ref, e1), (resp, refp, e2)):
        assert r_.status == 0 and r_.iters == f_.iters
        assert e_ <= 1e-12
        assert abs(r_.rel_res - f_.res_hist[-1]) <= 1e-9 * f_.res_hist[-1] + 1e-14
