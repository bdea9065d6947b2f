"""nek_cg_solve_noalloc: the CG solve whose workspace is the library's own
fixed device array, against nek_cg_solve on the same arrays.

Both entry points run the same kernels in the same order, so the solutions,
iteration counts and residuals must be bitwise equal.  Two calls in a row,
the second on a smaller mesh (the array keeps the first call's contents), a
third repeating the first, and the two refusals that happen on the host: a
solve larger than the array and a caller workspace.
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


def _case(nek, box, N):
    m = oracle.box_mesh(*box, N, synth.AMP, synth.geom_coeffs())
    b = oracle.lattice_to_local(m, synth.lattice_uniform(*box, N))
    gs = nek.GatherScatter(m.E, N, m.glo, m.dirichlet)
    return m, gs, _dev(m.D), _dev(m.g), _dev(b)


def _both(nek, box, N, **kw):
    print(f"no-alloc CG box={box} N={N} {kw}", flush=True)
    m, gs, D, g, b = _case(nek, box, N)
    x_ref, r_ref = nek.cg_solve(D, g, gs, b, **kw)
    x = torch.full_like(b, float("nan"))
    x, r = nek.cg_solve_noalloc(D, g, gs, b, x, **kw)
    torch.cuda.synchronize()
    gs.close()
    return x_ref, r_ref, x, r


def _same(x_ref, r_ref, x, r):
    assert torch.equal(x, x_ref)
    assert r.iters == r_ref.iters and r.status == r_ref.status
    assert r.rel_res == r_ref.rel_res and r.rel_res_true == r_ref.rel_res_true


def test_noalloc_matches_cg_solve_twice(nek):
    # 1: E = 1024, N = 9 (pencil operator), 100 fixed iterations, 33 MB of workspace
    first = _both(nek, (16, 8, 8), 9, max_iter=100)
    _same(*first)
    assert first[3].iters == 100
    # 2: a smaller mesh next (E = 64, N = 7: the one-thread-per-node operator),
    # to a tolerance, so the host polls the status word
    second = _both(nek, (4, 4, 4), 7, max_iter=2000, rel_tol=1e-10, true_residual=True)
    _same(*second)
    assert second[3].rel_res <= 1e-10 and 0 < second[3].iters < 2000
    # 3: the first case again finds the second one's leftovers in the array
    third = _both(nek, (16, 8, 8), 9, max_iter=100)
    _same(*third)
    assert torch.equal(third[2], first[2])


def test_noalloc_against_oracle(nek):
    m, gs, D, g, b = _case(nek, (3, 3, 2), 5)
    x = torch.empty_like(b)
    x, r = nek.cg_solve_noalloc(D, g, gs, b, x, max_iter=40)
    torch.cuda.synchronize()
    gs.close()
    ref = oracle.cg(m, b.cpu().numpy(), max_iter=40).x
    err = np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert r.iters == 40 and err <= 1e-12, err


def test_noalloc_refusals(nek):
    # E = 4096, N = 9 needs about 131 MB, more than the 64 MiB array: refused
    # before anything is queued
    m, gs, D, g, b = _case(nek, (16, 16, 16), 9)
    assert nek.cg_workspace_bytes(m.E, 9) > nek.CG_NOALLOC_BYTES
    x = torch.zeros_like(b)
    with pytest.raises(nek.NekError, match="NEK_CG_NOALLOC_BYTES"):
        nek.cg_solve_noalloc(D, g, gs, b, x, max_iter=10)
    assert torch.count_nonzero(x).item() == 0
    gs.close()
    # a caller workspace is refused (the entry point uses its own)
    m, gs, D, g, b = _case(nek, (2, 2, 2), 4)
    opts = nek.CgOpts()
    nek._lib.nek_cg_default_opts(nek.ctypes.byref(opts))
    ws = nek.cg_workspace(m.E, 4)
    opts.workspace = nek.ctypes.c_void_p(ws.data_ptr())
    opts.workspace_bytes = ws.numel()
    st = nek.CgStats()
    x = torch.empty_like(b)
    rc = nek._lib.nek_cg_solve_noalloc(m.E, 4, D.data_ptr(), g.data_ptr(), gs.handle, b.data_ptr(), x.data_ptr(),
                                       nek.ctypes.byref(opts), nek.ctypes.byref(st), None)
    assert rc == nek.NEK_ERR_ARG
    assert b"workspace" in nek._lib.nek_last_error()
    torch.cuda.synchronize()
    gs.close()
