"""Jacobi-preconditioned CG on the GPU against the FP64 oracle.

* nek_jacobi_inverse against the oracle's inverse assembled diagonal (same D,
  g and numbering on both sides): elementwise relative difference <= 1e-14
  (each entry is a short sum of O(n) positive terms and a reciprocal),
  exact zeros at masked nodes;
* preconditioned CG after 100 iterations: rel-L2 <= 1e-12 against the oracle
  (the FP64 bar of the plain solver).  The solver holds M^-1 in FP32, so both
  sides get the oracle's inverse and the oracle applies it rounded to FP32
  (round to nearest even, as the solver's conversion does);
* to a tolerance: the same iteration count (+-3) and the converged solution;
* the identity preconditioner (the mask) reproduces plain CG bitwise: same
  kernels, the second sum of the paired reduction equals the first;
* argument errors.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


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


@pytest.mark.parametrize("N,box", [(1, (5, 4, 3)), (2, (4, 4, 4)), (3, (3, 3, 5)), (5, (3, 3, 3)),
                                   (7, (3, 2, 4)), (9, (2, 3, 3)), (12, (2, 2, 1))])
def test_jacobi_inverse_parity(nek, N, box):
    m = _mesh(box, N)
    gs = nek.GatherScatter(m.E, N, m.glo, m.dirichlet)
    d = nek.jacobi_inverse(_dev(m.D), _dev(m.g), gs).cpu().numpy()
    ref = oracle.jacobi_inverse(m)
    gs.close()
    masked = m.dirichlet == 1
    assert np.all(d[masked] == 0.0)
    free = ~masked
    assert np.all(ref[free] > 0.0)
    err = np.max(np.abs(d[free] - ref[free]) / ref[free])
    print(f"jacobi N={N} box={box}: max rel {err:.2e}", flush=True)
    assert err <= 1e-14


def _pcg_case(nek, box, N, iters, rel_tol=0.0):
    m = _mesh(box, N)
    b = oracle.lattice_to_local(m, synth.lattice_uniform(*box, N))
    gs = nek.GatherScatter(m.E, N, m.glo, m.dirichlet)
    Dt, gt = _dev(m.D), _dev(m.g)
    dinv = oracle.jacobi_inverse(m)
    x, res = nek.cg_solve(Dt, gt, gs, _dev(b), max_iter=iters, rel_tol=rel_tol, dinv=_dev(dinv),
                          true_residual=True)
    torch.cuda.synchronize()
    dinv32 = dinv.astype(np.float32).astype(np.float64)
    ref = oracle.pcg(m, b, dinv32, max_iter=iters, rel_tol=rel_tol)
    gs.close()
    return m, x, res, ref


def test_pcg_100_iterations_small_config(nek):
    m, x, res, ref = _pcg_case(nek, (4, 4, 4), 7, 100)
    print(f"PCG E=64 N=7: rel-L2 {_rel(x, ref.x):.2e} rel_res {res.rel_res:.3e} "
          f"oracle {ref.res_hist[-1]:.3e}", flush=True)
    assert res.iters == 100 and res.status == 0
    assert _rel(x, ref.x) <= TOL
    assert abs(res.rel_res - ref.res_hist[-1]) <= 1e-9 * ref.res_hist[-1]


def test_pcg_100_iterations_paper_shape(nek):
    m, x, res, ref = _pcg_case(nek, (16, 8, 8), 9, 100)
    print(f"PCG E=1024 N=9: rel-L2 {_rel(x, ref.x):.2e}", flush=True)
    assert res.iters == 100
    assert _rel(x, ref.x) <= TOL


def test_pcg_100_iterations_full_shape(nek):
    m, x, res, ref = _pcg_case(nek, (16, 16, 16), 9, 100)
    print(f"PCG E=4096 N=9: rel-L2 {_rel(x, ref.x):.2e}", flush=True)
    assert res.iters == 100
    assert _rel(x, ref.x) <= TOL


def test_pcg_to_tolerance(nek):
    m, x, res, ref = _pcg_case(nek, (4, 4, 4), 7, 2000, rel_tol=1e-13)
    print(f"PCG to 1e-13: iters {res.iters} oracle {ref.iters}", flush=True)
    assert res.status == 0 and ref.status == 0
    assert abs(res.iters - ref.iters) <= 3
    assert res.rel_res <= 1e-13 and res.rel_res_true <= 1e-12
    assert _rel(x, ref.x) <= 1e-10


def test_identity_preconditioner_is_plain_cg_bitwise(nek):
    m = _mesh((3, 4, 2), 6)
    b = _dev(oracle.lattice_to_local(m, synth.lattice_uniform(3, 4, 2, 6)))
    gs = nek.GatherScatter(m.E, 6, m.glo, m.dirichlet)
    Dt, gt = _dev(m.D), _dev(m.g)
    ident = _dev((m.dirichlet == 0).astype(np.float64))
    x1, r1 = nek.cg_solve(Dt, gt, gs, b, max_iter=2000, rel_tol=1e-11, dinv=ident)
    x2, r2 = nek.cg_solve(Dt, gt, gs, b, max_iter=2000, rel_tol=1e-11)
    torch.cuda.synchronize()
    gs.close()
    assert r1.iters == r2.iters and r1.status == 0
    assert torch.equal(x1, x2)


def test_jacobi_cuts_iterations_on_stretched_elements(nek):
    # 16 x 8 x 8 elements on the unit cube: aspect 2:1 in x
    box, N = (16, 8, 8), 5
    m = _mesh(box, N)
    b = _dev(oracle.lattice_to_local(m, synth.lattice_uniform(*box, N)))
    gs = nek.GatherScatter(m.E, N, m.glo, m.dirichlet)
    Dt, gt = _dev(m.D), _dev(m.g)
    dinv = nek.jacobi_inverse(Dt, gt, gs)
    xp, rp = nek.cg_solve(Dt, gt, gs, b, max_iter=5000, rel_tol=1e-10, dinv=dinv, true_residual=True)
    xc, rc = nek.cg_solve(Dt, gt, gs, b, max_iter=5000, rel_tol=1e-10, true_residual=True)
    torch.cuda.synchronize()
    gs.close()
    print(f"E=1024 N=5 to 1e-10: CG {rc.iters} iterations, Jacobi PCG {rp.iters}", flush=True)
    assert rp.status == 0 and rc.status == 0
    assert rp.iters < rc.iters
    assert rp.rel_res_true <= 1e-9 and _rel(xp, xc.cpu().numpy()) <= 1e-8


def test_jacobi_argument_errors(nek):
    m = _mesh((2, 2, 2), 4)
    gs = nek.GatherScatter(m.E, 4, m.glo, m.dirichlet)
    other = nek.GatherScatter(27, 4, *nek.box_numbering(3, 3, 3, 4))
    Dt, gt = _dev(m.D), _dev(m.g)
    dinv = nek.jacobi_inverse(Dt, gt, gs)
    b = _dev(oracle.lattice_to_local(m, synth.lattice_uniform(2, 2, 2, 4)))
    with pytest.raises(nek.NekError) as ei:        # gather-scatter built for another mesh
        nek._check(nek._lib.nek_jacobi_inverse(m.E, 4, Dt.data_ptr(), gt.data_ptr(), other.handle,
                                               dinv.data_ptr(), None), "nek_jacobi_inverse")
    assert ei.value.code == nek.NEK_ERR_ARG
    buf = torch.empty(m.P + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(nek.NekError) as ei:        # misaligned output
        nek._check(nek._lib.nek_jacobi_inverse(m.E, 4, Dt.data_ptr(), gt.data_ptr(), gs.handle,
                                               buf.data_ptr() + 8, None), "nek_jacobi_inverse")
    assert ei.value.code == nek.NEK_ERR_ARG
    glo32 = nek.convert_g(gt, 4, nek.NEK_G_F32)
    with pytest.raises(nek.NekError) as ei:        # mixed precision with a preconditioner
        nek.cg_solve(Dt, gt, gs, b, max_iter=10, precision=nek.NEK_PREC_F32G32,
                     D32=_dev(m.D.astype(np.float32)), g_lo=glo32, dinv=dinv)
    assert ei.value.code == nek.NEK_ERR_UNSUPPORTED
    gs.close()
    other.close()
