"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Inputs are seeded (synth) and the geometry, numbering and derivative matrix
come from the oracle, so both sides see the same arrays.  Bars: rel-L2 <= 1e-12
for FP64 floating point (the bar the method's target sets), bit-exact for the
integer numbering and for dssum (same summation order on both sides).
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


def _mesh(box, N, amp=synth.AMP):
    return oracle.box_mesh(*box, N, amp, synth.geom_coeffs())


# boxes span several workgroups and leave a ragged last workgroup for every
# degree (N = 9 runs two elements per workgroup: 27 elements leave one alone)
BOX_FOR_N = {1: (6, 5, 5), 2: (4, 4, 4), 3: (3, 3, 7), 4: (3, 3, 3), 5: (3, 3, 3), 6: (3, 3, 3), 9: (3, 3, 3)}


@pytest.mark.parametrize("N", list(range(1, 16)))
def test_ax_parity_every_degree(nek, N):
    box = BOX_FOR_N.get(N, (3, 2, 2))
    m = _mesh(box, N)
    print(f"ax parity N={N} E={m.E}", flush=True)
    u = synth.local_uniform(m.P, seed=100 + N)
    w = nek.ax(_dev(u), _dev(m.D), _dev(m.g), N)
    ref = oracle.ax(m.E, N, m.D, m.g, u)
    assert _rel(w, ref) <= TOL
    # invariant on the GPU output itself: constants are in the kernel
    w1 = nek.ax(torch.ones(m.P, dtype=torch.float64, device="cuda"), _dev(m.D), _dev(m.g), N)
    assert torch.max(torch.abs(w1)).item() < 1e-11 * max(1, N * N)


def test_ax_single_element_and_affine(nek):
    m = oracle.box_mesh(1, 1, 1, 9)
    u = synth.local_uniform(m.P, seed=3)
    w = nek.ax(_dev(u), _dev(m.D), _dev(m.g), 9)
    assert _rel(w, oracle.ax(1, 9, m.D, m.g, u)) <= TOL


@pytest.mark.parametrize("E_box", [(16, 8, 8), (16, 16, 16)])
def test_ax_parity_paper_shapes(nek, E_box):
    m = _mesh(E_box, 9)
    print(f"ax parity paper shape E={m.E}", flush=True)
    u = synth.local_uniform(m.P)
    w = nek.ax(_dev(u), _dev(m.D), _dev(m.g), 9)
    ref = oracle.ax(m.E, 9, m.D, m.g, u)
    assert _rel(w, ref) <= TOL


@pytest.mark.parametrize("N", sorted(synth.SWEEP_BOXES))
def test_ax_sampled_sweep_shape(nek, N):
    # the degree-sweep boxes (about 32.8 M local points each, the launch the
    # sweep times): compare sampled elements, including the first and the last
    Ex, Ey, Ez = synth.SWEEP_BOXES[N]
    print(f"sweep N={N} box {Ex}x{Ey}x{Ez}", flush=True)
    E = Ex * Ey * Ez
    n3 = (N + 1) ** 3
    z, wq = oracle.gll(N)
    # product geometry on the device, oracle operator on sampled elements
    g, _, X = nek.box_geometry(Ex, Ey, Ez, N, synth.AMP, synth.geom_coeffs(), want_coords=True)
    _, _, D = nek.gll(N)
    Dt = _dev(D)
    u = torch.rand(E * n3, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(7)) * 2 - 1
    w = nek.ax(u, Dt, g, N)
    torch.cuda.synchronize()
    rng = np.random.default_rng(9)
    sample = np.unique(np.concatenate([[0, E - 1], rng.integers(0, E, 64)]))
    gh = g.view(E, 6 * n3)[torch.from_numpy(sample).cuda()].cpu().numpy().reshape(-1)
    uh = u.view(E, n3)[torch.from_numpy(sample).cuda()].cpu().numpy().reshape(-1)
    wh = w.view(E, n3)[torch.from_numpy(sample).cuda()].cpu().numpy().reshape(-1)
    ref = oracle.ax(len(sample), N, D, gh, uh)
    assert _rel(wh, ref) <= TOL
    del g, X, u, w
    torch.cuda.empty_cache()


def test_geometry_parity(nek):
    for box, N in [((3, 2, 2), 4), ((4, 4, 4), 7), ((2, 2, 2), 9)]:
        m = _mesh(box, N)
        g, bm, X = nek.box_geometry(*box, N, synth.AMP, synth.geom_coeffs(), want_mass=True, want_coords=True)
        torch.cuda.synchronize()
        assert _rel(X, m.X.reshape(-1)) <= 1e-14
        assert _rel(bm, m.bm) <= 1e-12
        assert _rel(g, m.g) <= 1e-12


def test_dssum_bit_exact(nek):
    for box, N in [((4, 4, 4), 7), ((3, 2, 5), 3), ((16, 8, 8), 9)]:
        m = _mesh(box, N)
        gs = nek.GatherScatter(m.E, N, m.glo, m.dirichlet)
        info = gs.info()
        assert info["n_unique"] == m.U
        w = synth.local_uniform(m.P, seed=5)
        wt = _dev(w.copy())
        gs.dssum(wt)
        ref = oracle.mask(m.dirichlet, oracle.dssum(m.glo, w, m.U))
        np.testing.assert_array_equal(wt.cpu().numpy(), ref)
        gs.close()


def test_dssum_without_mask_and_general_ids(nek):
    m = _mesh((3, 3, 2), 4)
    # renumber ids with gaps and a permutation: the handle must not depend on compact ids
    perm = np.random.default_rng(2).permutation(m.U).astype(np.int64) * 7 + 11
    glo = perm[m.glo]
    gs = nek.GatherScatter(m.E, 4, glo, None)
    w = synth.local_uniform(m.P, seed=6)
    wt = _dev(w.copy())
    gs.dssum(wt)
    np.testing.assert_array_equal(wt.cpu().numpy(), oracle.dssum(m.glo, w, m.U))
    a, b = synth.local_uniform(m.P, 1), synth.local_uniform(m.P, 2)
    a = oracle.dssum(m.glo, a, m.U) / oracle.dssum(m.glo, np.ones(m.P), m.U)
    b = oracle.dssum(m.glo, b, m.U) / oracle.dssum(m.glo, np.ones(m.P), m.U)
    d = gs.dot(_dev(a), _dev(b)).item()
    ref = oracle.gdot(m.glo, a, b, m.U)
    assert abs(d - ref) <= 1e-13 * abs(ref)
    gs.close()


def _cg_case(nek, box, N, iters, rel_tol=0.0):
    m = _mesh(box, N)
    b = oracle.lattice_to_local(m, synth.lattice_uniform(*box, N))
    gs = nek.GatherScatter(m.E, N, m.glo, m.dirichlet)
    x, res = nek.cg_solve(_dev(m.D), _dev(m.g), gs, _dev(b), max_iter=iters, rel_tol=rel_tol,
                          true_residual=True)
    torch.cuda.synchronize()
    ref = oracle.cg(m, b, max_iter=iters, rel_tol=rel_tol)
    gs.close()
    return m, x, res, ref


def test_cg_100_iterations_small_config(nek):
    m, x, res, ref = _cg_case(nek, (4, 4, 4), 7, 100)
    print(f"CG E=64 N=7: iters {res.iters} rel_res {res.rel_res:.3e} oracle {ref.res_hist[-1]:.3e}", flush=True)
    assert res.iters == 100 and res.status == 0
    assert _rel(x, ref.x) <= TOL
    assert abs(res.rel_res - ref.res_hist[-1]) <= 1e-9 * ref.res_hist[-1]


def test_cg_100_iterations_paper_shape(nek):
    m, x, res, ref = _cg_case(nek, (16, 8, 8), 9, 100)
    print(f"CG E=1024 N=9: rel-L2 {_rel(x, ref.x):.2e}", flush=True)
    assert res.iters == 100
    assert _rel(x, ref.x) <= TOL


@pytest.mark.parametrize("box", [(16, 16, 8), (16, 16, 16)])
def test_cg_100_iterations_full_shapes(nek, box):
    # the benchmark's shapes (E = 2048, 4096 at N = 9), with a caller workspace
    # as the timed step uses
    N = 9
    m = _mesh(box, N)
    b = oracle.lattice_to_local(m, synth.lattice_uniform(*box, N))
    gs = nek.GatherScatter(m.E, N, m.glo, m.dirichlet)
    ws = nek.cg_workspace(m.E, N)
    x, res = nek.cg_solve(_dev(m.D), _dev(m.g), gs, _dev(b), max_iter=100, workspace=ws)
    torch.cuda.synchronize()
    gs.close()
    ref = oracle.cg(m, b, max_iter=100)
    err = _rel(x, ref.x)
    print(f"CG E={m.E} N=9, 100 iterations: rel-L2 {err:.2e}", flush=True)
    assert res.iters == 100 and err <= TOL


def test_cg_30_iterations_large_mesh(nek):
    # E = 8192 at N = 9: the assemble-update's workgroups take several row
    # blocks and chunks of pairs each, two at a time in flight
    box, N = (32, 16, 16), 9
    m = _mesh(box, N)
    b = oracle.lattice_to_local(m, synth.lattice_uniform(*box, N))
    gs = nek.GatherScatter(m.E, N, m.glo, m.dirichlet)
    x, res = nek.cg_solve(_dev(m.D), _dev(m.g), gs, _dev(b), max_iter=30)
    torch.cuda.synchronize()
    gs.close()
    ref = oracle.cg(m, b, max_iter=30)
    err = _rel(x, ref.x)
    print(f"CG E={m.E} N=9, 30 iterations: rel-L2 {err:.2e}", flush=True)
    assert res.iters == 30 and err <= TOL
    assert abs(res.rel_res - ref.res_hist[-1]) <= 1e-9 * ref.res_hist[-1]


def test_cg_to_tolerance(nek):
    m, x, res, ref = _cg_case(nek, (4, 4, 4), 7, 2000, rel_tol=1e-13)
    assert res.status == 0 and ref.status == 0
    assert abs(res.iters - ref.iters) <= 3
    assert res.rel_res <= 1e-13 and res.rel_res_true <= 1e-12
    assert _rel(x, ref.x) <= 1e-10


@pytest.mark.parametrize("N", [2, 4])
def test_cg_single_element(nek, N):
    # one element: every boundary node masked, no shared node, (N-1)^3 unknowns;
    # N = 2 leaves one unknown, so CG ends after one iteration
    m = _mesh((1, 1, 1), N)
    b = oracle.lattice_to_local(m, synth.lattice_uniform(1, 1, 1, N))
    gs = nek.GatherScatter(1, N, m.glo, m.dirichlet)
    x, res = nek.cg_solve(_dev(m.D), _dev(m.g), gs, _dev(b), max_iter=200, rel_tol=1e-13,
                          true_residual=True)
    torch.cuda.synchronize()
    gs.close()
    ref = oracle.cg(m, b, max_iter=200, rel_tol=1e-13)
    assert res.status == 0 and ref.status == 0
    assert res.iters <= (N - 1) ** 3 + 2 and abs(res.iters - ref.iters) <= 1
    assert _rel(x, ref.x) <= 1e-12
    assert np.all(x.cpu().numpy()[m.dirichlet == 1] == 0.0)


def test_cg_deterministic(nek):
    m = _mesh((4, 4, 4), 7)
    b = _dev(oracle.lattice_to_local(m, synth.lattice_uniform(4, 4, 4, 7)))
    gs = nek.GatherScatter(m.E, 7, m.glo, m.dirichlet)
    x1, _ = nek.cg_solve(_dev(m.D), _dev(m.g), gs, b, max_iter=60)
    x2, _ = nek.cg_solve(_dev(m.D), _dev(m.g), gs, b, max_iter=60)
    torch.cuda.synchronize()
    assert torch.equal(x1, x2)
    gs.close()


def test_cg_breakdown_and_noconv(nek):
    m = _mesh((2, 2, 2), 5)
    b = oracle.lattice_to_local(m, synth.lattice_uniform(2, 2, 2, 5))
    gs = nek.GatherScatter(m.E, 5, m.glo, m.dirichlet)
    bad = b.copy()
    bad[np.argmax(m.dirichlet == 0)] = np.nan
    _, res = nek.cg_solve(_dev(m.D), _dev(m.g), gs, _dev(bad), max_iter=5, raise_on_error=False)
    assert res.status == nek.NEK_ERR_BREAKDOWN
    _, res = nek.cg_solve(_dev(m.D), _dev(m.g), gs, _dev(b), max_iter=3, rel_tol=1e-12,
                          raise_on_error=False)
    assert res.status == nek.NEK_ERR_NOCONV and res.iters == 3
    with pytest.raises(nek.NekError):
        nek.cg_solve(_dev(m.D), _dev(m.g), gs, _dev(b), max_iter=3, rel_tol=1e-12)
    # zero rhs: x = 0 with no iterations
    x, res = nek.cg_solve(_dev(m.D), _dev(m.g), gs, _dev(np.zeros(m.P)), max_iter=5)
    assert res.iters == 0 and torch.count_nonzero(x).item() == 0
    gs.close()


def test_ax_argument_errors_on_device(nek):
    m = _mesh((2, 1, 1), 3)
    u = _dev(synth.local_uniform(m.P))
    with pytest.raises(nek.NekError) as ei:
        nek._check(nek._lib.nek_ax(m.E, 3, u.data_ptr(), _dev(m.D).data_ptr(), _dev(m.g).data_ptr(),
                                   u.data_ptr(), None), "nek_ax")
    assert ei.value.code == nek.NEK_ERR_ARG
    with pytest.raises(TypeError):
        nek.ax(u.float(), _dev(m.D), _dev(m.g), 3)


def test_cg_odd_point_count_and_interior_mask(nek):
    # N=2, 3x3x3 box: P = 27 * 27 is odd (vector tail); pin one element-interior
    # node with a Dirichlet flag, so element interiors are no longer exclusive
    # and the (p, w) product runs entirely through the gather-scatter
    for pin in (False, True):
        m = _mesh((3, 3, 3), 2)
        dr = m.dirichlet.copy()
        if pin:
            n = 3
            L = 13 * n ** 3 + 1 + n * (1 + n * 1)     # point (1,1,1) of element 13
            dr[L] = 1
        b = oracle.lattice_to_local(m, synth.lattice_uniform(3, 3, 3, 2))
        b = oracle.mask(dr, b)
        gs = nek.GatherScatter(m.E, 2, m.glo, dr)
        x, res = nek.cg_solve(_dev(m.D), _dev(m.g), gs, _dev(b), max_iter=30, true_residual=True)
        torch.cuda.synchronize()
        mm = oracle.BoxMesh(m.Ex, m.Ey, m.Ez, m.N, m.z, m.wq, m.D, m.X, m.g, m.bm, m.glo, dr, m.detmin)
        ref = oracle.cg(mm, b, max_iter=30)
        assert m.P % 2 == 1
        assert _rel(x, ref.x) <= TOL, pin
        gs.close()


@pytest.mark.parametrize("streaming", [False, True])
def test_bw_probe_sums_its_streams(nek, streaming):
    # dst[i] = sum over k of stream_k[i], summed in k order; odd n for the tail
    rng = np.random.default_rng(9)
    for nread, n, stride in ((1, 1001, 1002), (7, 40001, 40001 + 31 * 32 + 1), (8, 12345, 12346)):
        src = rng.uniform(-1, 1, (nread - 1) * stride + n)
        dst = torch.empty(n, dtype=torch.float64, device="cuda")
        nek.bw_probe(_dev(src), dst, nread, stride=stride, streaming=streaming)
        ref = np.zeros(n)
        for k in range(nread):
            ref = ref + src[k * stride:k * stride + n]
        np.testing.assert_array_equal(dst.cpu().numpy(), ref)
    # a capped grid walks the rest with a stride (streams 16-byte aligned: even stride)
    n, stride = 300001, 300002
    src = rng.uniform(-1, 1, 2 * stride + n)
    dst = torch.empty(n, dtype=torch.float64, device="cuda")
    nek.bw_probe(_dev(src), dst, 3, stride=stride, grid_cap=7, streaming=streaming)
    ref = src[:n] + src[stride:stride + n] + src[2 * stride:2 * stride + n]
    np.testing.assert_array_equal(dst.cpu().numpy(), ref)


@pytest.mark.parametrize("streaming", [False, True])
def test_bw_probe_blocked_layout(nek, streaming):
    # streams interleaved in blocks of NEK_PROBE_BLOCK doubles: block b of
    # stream k at (b * nread + k) * BLOCK; odd n and a ragged last block
    rng = np.random.default_rng(11)
    B = nek.NEK_PROBE_BLOCK
    for nread, n, cap in ((7, 40001, 0), (7, 3 * B, 2), (1, 12345, 0), (3, 300001, 13)):
        nb = (n + B - 1) // B
        src = rng.uniform(-1, 1, nek.bw_probe_src_doubles(n, nread, blocked=True))
        streams = src.reshape(nb, nread, B).transpose(1, 0, 2).reshape(nread, nb * B)[:, :n]
        dst = torch.empty(n, dtype=torch.float64, device="cuda")
        nek.bw_probe(_dev(src), dst, nread, grid_cap=cap, streaming=streaming, blocked=True)
        ref = np.zeros(n)
        for k in range(nread):
            ref = ref + streams[k]
        np.testing.assert_array_equal(dst.cpu().numpy(), ref)
        groups = nek.bw_probe_groups(n, cap)
        part = torch.empty(groups, dtype=torch.float64, device="cuda")
        nek.bw_probe(_dev(src), part, nread, n=n, grid_cap=cap, streaming=streaming, read_only=True, blocked=True)
        tot = streams[:, :n - (n & 1)].sum()
        assert abs(part.sum().item() - tot) <= 1e-9 * np.abs(streams).sum()


@pytest.mark.parametrize("streaming", [False, True])
def test_bw_probe_read_only_partials(nek, streaming):
    # one partial per workgroup; together they hold the sum of every stream
    # (the last value left out for odd n)
    rng = np.random.default_rng(10)
    for nread, n, cap in ((7, 40000, 0), (7, 300001, 13), (2, 5000, 1)):
        stride = (n + 34) // 2 * 2          # even: the streams stay 16-byte aligned
        src = rng.uniform(-1, 1, (nread - 1) * stride + n)
        groups = nek.bw_probe_groups(n, cap)
        dst = torch.empty(groups, dtype=torch.float64, device="cuda")
        nek.bw_probe(_dev(src), dst, nread, n=n, stride=stride, grid_cap=cap, streaming=streaming,
                     read_only=True)
        m = n - (n & 1)
        ref = sum(src[k * stride:k * stride + m].sum() for k in range(nread))
        got = dst.cpu().numpy().sum()
        assert abs(got - ref) <= 1e-12 * np.abs(src).sum(), (nread, n, cap)


def test_gs_dot_odd_and_unaligned_rejected(nek):
    m = _mesh((3, 1, 1), 2)
    gs = nek.GatherScatter(m.E, 2, m.glo, m.dirichlet)
    a = oracle.dssum(m.glo, synth.local_uniform(m.P, 1), m.U) / oracle.dssum(m.glo, np.ones(m.P), m.U)
    d = gs.dot(_dev(a), _dev(a)).item()
    assert abs(d - oracle.gdot(m.glo, a, a, m.U)) <= 1e-13 * d
    big = _dev(np.concatenate([[0.0], a]))
    with pytest.raises(nek.NekError):
        gs.dot(big[1:], big[1:])
    gs.close()
