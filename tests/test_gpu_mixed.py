"""Mixed-precision forms inside FP64 reliable-update CG, against the FP64
oracle: the FP32 operator with g in FP32 or BF16 (NEK_PREC_F32G*), and the
FP64 operator reading g stored in FP32 or BF16 (NEK_PREC_F64G*).

* nek_convert_g: bit-exact against numpy's round-to-nearest-even (FP32 via
  astype, BF16 from the FP32 bits).
* nek_ax_f32: compared with the oracle applied to the same rounded inputs
  (u, D, g rounded to FP32 / BF16 and widened back), so the only difference
  left is FP32 arithmetic.  Bar: rel-L2 <= 2e-6, from ~(3n+4) FP32 roundings
  of terms of the size of |D||g||D||u| per output (n = 10: ~34 * 6e-8 = 2e-6
  worst case; the sums of signed terms cancel, so the norm-wise error is far
  below that).
* mixed CG to a true relative residual of 1e-10 on the manufactured solution:
  status OK, ||b - A64 x|| / ||b|| <= 1e-10 evaluated in FP64 by the library,
  and the solution within 1e-8 of the oracle's FP64 solve to 1e-13; with the
  FP64 operator on FP32 g the iteration count stays within 5% of the FP64
  solve's (FP32 contractions, not FP32 storage of g, cost the FP32 operator
  its extra iterations).
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


def _bf16_rne(x64):
    """FP64 -> FP32 (RNE) -> BF16 (RNE on the FP32 bits); returns uint16 bits."""
    f = np.asarray(x64, dtype=np.float64).astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return b.astype(np.uint16)


def _bf16_to_f64(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _point_major(a, E, n3):
    """[e][c][pt] -> [e][pt][c]: the six factors of a point side by side."""
    return a.reshape(E, 6, n3).transpose(0, 2, 1).reshape(-1)


def test_convert_g_bit_exact(nek):
    m = oracle.box_mesh(3, 2, 2, 5, synth.AMP, synth.geom_coeffs())
    g = _dev(m.g)
    n3 = 6 ** 3
    g32 = nek.convert_g(g, 5, nek.NEK_G_F32)
    np.testing.assert_array_equal(g32.cpu().numpy(), _point_major(m.g.astype(np.float32), m.E, n3))
    g16 = nek.convert_g(g, 5, nek.NEK_G_BF16)
    np.testing.assert_array_equal(g16.cpu().numpy().view(np.uint16), _point_major(_bf16_rne(m.g), m.E, n3))


@pytest.mark.parametrize("N", [1, 3, 5, 7, 9, 11, 15])
@pytest.mark.parametrize("gdt", ["f32", "bf16"])
def test_ax_f32_against_oracle_on_rounded_inputs(nek, N, gdt):
    box = (3, 2, 2) if N > 4 else (4, 4, 3)
    m = oracle.box_mesh(*box, N, synth.AMP, synth.geom_coeffs())
    u = synth.local_uniform(m.P, seed=40 + N)
    u32 = u.astype(np.float32).astype(np.float64)
    D32 = m.D.astype(np.float32)
    if gdt == "f32":
        glo = nek.convert_g(_dev(m.g), N, nek.NEK_G_F32)
        gr = m.g.astype(np.float32).astype(np.float64)
        code = nek.NEK_G_F32
    else:
        glo = nek.convert_g(_dev(m.g), N, nek.NEK_G_BF16)
        gr = _bf16_to_f64(_bf16_rne(m.g))
        code = nek.NEK_G_BF16
    w = nek.ax_f32(_dev(u), _dev(D32), glo, code, N)
    ref = oracle.ax(m.E, N, D32.astype(np.float64), gr, u32)
    assert _rel(w, ref) <= 2e-6
    # and the distance to the FP64 operator is the size the rounding of g implies
    full = oracle.ax(m.E, N, m.D, m.g, u)
    assert _rel(w, full) <= (2e-6 if gdt == "f32" else 2e-2)


def _prec(nek, prec):
    """(precision mode, storage type of g) of a test label"""
    return {"f32": (nek.NEK_PREC_F32G32, nek.NEK_G_F32), "bf16": (nek.NEK_PREC_F32GBF16, nek.NEK_G_BF16),
            "f64g32": (nek.NEK_PREC_F64G32, nek.NEK_G_F32),
            "f64gbf16": (nek.NEK_PREC_F64GBF16, nek.NEK_G_BF16)}[prec]


PRECS = ["f32", "bf16", "f64g32", "f64gbf16"]


@pytest.mark.parametrize("prec", PRECS)
def test_mixed_cg_reaches_1e10_true_residual(nek, prec):
    box, N = (4, 4, 4), 7
    m = oracle.box_mesh(*box, N, synth.AMP, synth.geom_coeffs())
    b = oracle.manufactured_rhs(m)
    gs = nek.GatherScatter(m.E, N, m.glo, m.dirichlet)
    Dt, gt = _dev(m.D), _dev(m.g)
    D32 = _dev(m.D.astype(np.float32))
    precision, code = _prec(nek, prec)
    glo = nek.convert_g(gt, N, code)
    x, res = nek.cg_solve(Dt, gt, gs, _dev(b), max_iter=3000, rel_tol=1e-10, precision=precision,
                          D32=D32, g_lo=glo)
    torch.cuda.synchronize()
    print(f"mixed {prec}: iters {res.iters} replacements {res.n_replacements} "
          f"true rel res {res.rel_res_true:.2e}", flush=True)
    assert res.status == 0
    assert 0 < res.rel_res_true <= 1e-10
    assert res.n_replacements >= 1
    ref = oracle.cg(m, b, max_iter=3000, rel_tol=1e-13)
    assert ref.status == 0
    assert _rel(x, ref.x) <= 1e-8
    # the FP64 solve of the same system takes a comparable number of iterations
    _, r64 = nek.cg_solve(Dt, gt, gs, _dev(b), max_iter=3000, rel_tol=1e-10)
    assert res.iters <= 1.5 * r64.iters + 20
    if prec == "f64g32":
        assert res.iters <= 1.05 * r64.iters + 5, (res.iters, r64.iters)
    gs.close()


@pytest.mark.parametrize("prec", PRECS)
def test_mixed_full_size_true_residual_by_the_oracle(nek, prec):
    # the mixed-precision workload at its full size (E = 4096, N = 9, manufactured
    # rhs, 1e-10): the oracle evaluates b - A x of the GPU's solution itself
    box, N = (16, 16, 16), 9
    m = oracle.box_mesh(*box, N, synth.AMP, synth.geom_coeffs())
    b = oracle.manufactured_rhs(m)
    gs = nek.GatherScatter(m.E, N, m.glo, m.dirichlet)
    Dt, gt = _dev(m.D), _dev(m.g)
    precision, code = _prec(nek, prec)
    x, res = nek.cg_solve(Dt, gt, gs, _dev(b), max_iter=5000, rel_tol=1e-10, precision=precision,
                          D32=_dev(m.D.astype(np.float32)), g_lo=nek.convert_g(gt, N, code))
    torch.cuda.synchronize()
    gs.close()
    xh = x.cpu().numpy()
    r = b - oracle.masked_ax(m, xh)
    # the residual over unique nodes, as the solver measures it
    true_rel = np.sqrt(oracle.gdot(m.glo, r, r, m.U) / oracle.gdot(m.glo, b, b, m.U))
    xs, ys, zs = m.X
    ustar = np.sin(np.pi * xs) * np.sin(np.pi * ys) * np.sin(np.pi * zs)
    print(f"mixed {prec} E=4096: iters {res.iters}, oracle true residual {true_rel:.3e}, "
          f"library {res.rel_res_true:.3e}, error vs sin {np.max(np.abs(xh - ustar)):.2e}", flush=True)
    assert res.status == 0
    assert true_rel <= 1.01e-10
    assert abs(true_rel - res.rel_res_true) <= 1e-3 * true_rel
    assert np.max(np.abs(xh - ustar)) <= 1e-6


def test_mixed_cg_fixed_iterations_and_errors(nek):
    m = oracle.box_mesh(2, 2, 2, 4, synth.AMP, synth.geom_coeffs())
    b = oracle.lattice_to_local(m, synth.lattice_uniform(2, 2, 2, 4))
    gs = nek.GatherScatter(m.E, 4, m.glo, m.dirichlet)
    Dt, gt = _dev(m.D), _dev(m.g)
    glo = nek.convert_g(gt, 4, nek.NEK_G_F32)
    x, res = nek.cg_solve(Dt, gt, gs, _dev(b), max_iter=20, precision=nek.NEK_PREC_F32G32,
                          D32=_dev(m.D.astype(np.float32)), g_lo=glo)
    assert res.iters == 20 and res.status == 0 and res.rel_res_true > 0
    # the FP64 operator on FP32 g needs no D32
    x2, res2 = nek.cg_solve(Dt, gt, gs, _dev(b), max_iter=20, precision=nek.NEK_PREC_F64G32, g_lo=glo)
    assert res2.iters == 20 and res2.status == 0 and res2.rel_res_true > 0
    # mixed precision without the FP32 inputs is an argument error
    with pytest.raises(nek.NekError) as ei:
        nek._check(nek._lib.nek_cg_solve(m.E, 4, Dt.data_ptr(), gt.data_ptr(), gs.handle,
                                         _dev(b).data_ptr(), x.data_ptr(),
                                         nek.ctypes.byref(_opts(nek, nek.NEK_PREC_F32G32)), None, None),
                   "nek_cg_solve")
    assert ei.value.code == nek.NEK_ERR_ARG
    gs.close()


def _opts(nek, prec):
    o = nek.CgOpts()
    nek._lib.nek_cg_default_opts(nek.ctypes.byref(o))
    o.precision = prec
    return o
