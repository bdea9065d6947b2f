"""Served solves: admission by device footprint, resident CG state, shared
launches over all admitted solves (nek_server_*), against the oracle and
against the same request served alone.

* a served FP64 solve is bitwise nek_cg_solve of the same system (the same
  operator form, partials and reductions, whichever solves share the merged
  launches) and the oracle's converged solution to 1e-8;
* a request's solution is bitwise the same alone and in a mix with requests
  of other sizes, degrees and precisions that arrive while it runs (every
  solve's workgroups, reductions and tickets are its own);
* with a budget that holds one request, one waits until the other has
  finished (the order is that of their host preparation); with room for
  both, they are admitted and run at the same time;
* a prepared request that does not fit is not overtaken by a smaller one.
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


def _rhs(nek, box, N, seed):
    glo, dr = nek.box_numbering(*box, N)
    vals = synth.lattice_uniform(*box, N, seed=seed)
    b = vals[glo]
    b[dr == 1] = 0.0
    return b


GB = 1 << 30


def test_served_solve_matches_cg_and_oracle(nek):
    box, N = (4, 4, 4), 7
    a = synth.geom_coeffs()
    b = _rhs(nek, box, N, 5)
    srv = nek.Server(4 * GB)
    rid = srv.submit(*box, N, b, amp=synth.AMP, a=a, rel_tol=1e-10)
    res = srv.run_until_done([rid])[rid]
    x = srv.fetch(rid)
    srv.close()
    assert res["status"] == 0 and res["rel_res"] <= 1e-10 and res["rel_res_true"] <= 1e-9
    # the same system through nek_cg_solve with the library's own setup
    g, _, _ = nek.box_geometry(*box, N, synth.AMP, a)
    _, _, D = nek.gll(N)
    glo, dr = nek.box_numbering(*box, N)
    gs = nek.GatherScatter(64, N, glo, dr)
    xs, rs = nek.cg_solve(torch.from_numpy(D).cuda(), g, gs, torch.from_numpy(b).cuda(),
                          max_iter=10000, rel_tol=1e-10)
    assert rs.iters == res["iters"]
    np.testing.assert_array_equal(x, xs.cpu().numpy())
    # the oracle's converged solution on its own setup
    m = oracle.box_mesh(*box, N, synth.AMP, a)
    ref = oracle.cg(m, oracle.lattice_to_local(m, synth.lattice_uniform(*box, N, seed=5)),
                    max_iter=5000, rel_tol=1e-13)
    assert np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) <= 1e-8
    gs.close()


def _serve(nek, reqs, budget=8 * GB, stagger=0):
    """reqs: list of (box, N, precision, seed); request k is submitted after
    k*stagger steps.  Returns ({k: x}, {k: result}, server clock trace)."""
    srv = nek.Server(budget)
    ids, xs, res = {}, {}, {}
    a = synth.geom_coeffs()
    pending = list(enumerate(reqs))
    steps = 0
    trace = []
    while pending or len(res) < len(reqs):
        while pending and pending[0][0] * stagger <= steps:
            k, (box, N, prec, seed) = pending.pop(0)
            ids[srv.submit(*box, N, _rhs(nek, box, N, seed), amp=synth.AMP, a=a, precision=prec,
                           rel_tol=1e-10, max_iter=20000)] = k
        act, que = srv.step(1)
        trace.append((steps, act, que))
        steps += 1
        for r in srv.poll():
            k = ids[r["id"]]
            res[k] = r
            xs[k] = srv.fetch(r["id"])
        assert steps < 200000
    srv.close()
    return xs, res, trace


def test_alone_equals_in_the_mix_bitwise(nek):
    A = ((4, 4, 4), 7, nek.NEK_PREC_F64, 1)
    B = ((3, 3, 2), 5, nek.NEK_PREC_F32G32, 2)
    C = ((2, 2, 4), 9, nek.NEK_PREC_F64, 3)
    Dq = ((4, 2, 2), 7, nek.NEK_PREC_F32GBF16, 4)
    F = ((3, 2, 2), 9, nek.NEK_PREC_F64G32, 5)       # FP64 operator on FP32 g
    xa, ra, _ = _serve(nek, [A])
    xb, rb, _ = _serve(nek, [B])
    xf, rf, _ = _serve(nek, [F])
    xm, rm, trace = _serve(nek, [A, C, B, Dq, F], stagger=7)
    assert max(t[1] for t in trace) >= 2            # solves ran side by side
    np.testing.assert_array_equal(xm[0], xa[0])
    np.testing.assert_array_equal(xm[2], xb[0])
    np.testing.assert_array_equal(xm[4], xf[0])
    assert rm[0]["iters"] == ra[0]["iters"] and rm[2]["iters"] == rb[0]["iters"]
    assert rm[4]["iters"] == rf[0]["iters"]
    for k in rm:
        assert rm[k]["status"] == 0, rm[k]
        assert rm[k]["rel_res_true"] <= 1e-9
    assert rm[2]["n_replacements"] >= 1 and rm[3]["n_replacements"] >= 1 and rm[4]["n_replacements"] >= 1


def _cg_solve_box(nek, box, N, b, rel_tol=1e-10):
    """nek_cg_solve on the system a box request describes (the library's own
    geometry, numbering and D, as the server builds them)."""
    g, _, _ = nek.box_geometry(*box, N, synth.AMP, synth.geom_coeffs())
    _, _, D = nek.gll(N)
    glo, dr = nek.box_numbering(*box, N)
    gs = nek.GatherScatter(int(np.prod(box)), N, glo, dr)
    x, r = nek.cg_solve(torch.from_numpy(D).cuda(), g, gs, torch.from_numpy(b).cuda(), max_iter=20000,
                        rel_tol=rel_tol)
    torch.cuda.synchronize()
    gs.close()
    return x.cpu().numpy(), r


def test_mix_of_every_operator_form_bitwise_vs_cg_solve(nek):
    """FP64 requests that take each operator of the merged launches -- the
    one-thread-per-node form (N = 3, N = 9 on 64 elements), the pencil form
    at n = 2 and n = 10 (two parts per workgroup), the pencil form of the
    high degrees (N = 13) -- beside a larger request that makes the small
    ones run several iterations per round, and a BF16 request: every FP64
    solution is bitwise that of nek_cg_solve on the same system, with the
    same iteration count."""
    reqs = [((8, 8, 16), 9, nek.NEK_PREC_F64, 21),     # 1 M points: the heaviest, weight 1
            ((2, 2, 2), 3, nek.NEK_PREC_F64, 22),      # node form, n = 4
            ((4, 4, 4), 9, nek.NEK_PREC_F64, 23),      # node form, n = 10
            ((3, 3, 3), 1, nek.NEK_PREC_F64, 24),      # pencil, n = 2
            ((8, 8, 9), 9, nek.NEK_PREC_F64, 25),      # pencil, n = 10 (576 000 points)
            ((2, 2, 1), 13, nek.NEK_PREC_F64, 26),     # pencil, n = 14
            ((3, 2, 2), 7, nek.NEK_PREC_F32GBF16, 27)]
    print("serve mix of every operator form", flush=True)
    srv = nek.Server(16 * GB)
    a = synth.geom_coeffs()
    ids = {}

    def submit(k):
        box, N, prec, seed = reqs[k]
        ids[srv.submit(*box, N, _rhs(nek, box, N, seed), amp=synth.AMP, a=a, precision=prec,
                       rel_tol=1e-10, max_iter=20000)] = k

    submit(0)                         # the heavy one runs first, the rest join it
    for _ in range(100000):
        act, _ = srv.step(1)
        if act == 1:
            break
    assert act == 1
    for k in range(1, len(reqs)):
        submit(k)
    xs, res, most = {}, {}, 0
    for _ in range(1000000):
        act, _ = srv.step(1)
        most = max(most, act)
        for r in srv.poll():
            res[ids[r["id"]]] = r
            xs[ids[r["id"]]] = srv.fetch(r["id"])
        if len(res) == len(reqs):
            break
    srv.close()
    assert most >= 4                  # they ran side by side
    for k, (box, N, prec, seed) in enumerate(reqs):
        assert res[k]["status"] == 0, (k, res[k])
        if prec != nek.NEK_PREC_F64:
            assert res[k]["rel_res_true"] <= 1e-10
            continue
        print(f"serve mix: request {k} box={box} N={N}: {res[k]['iters']} iterations", flush=True)
        x, r = _cg_solve_box(nek, box, N, _rhs(nek, box, N, seed))
        assert r.iters == res[k]["iters"], (k, r.iters, res[k]["iters"])
        np.testing.assert_array_equal(xs[k], x)


def test_more_solves_than_the_by_value_slot_table_holds(nek):
    """Twelve small requests admitted together (eleven FP64, one with the FP32
    operator, whose w the assembly reads in FP32): their assembly is one
    batched launch over more slots than its kernel arguments carry, so it
    reads them from the device table.  Every FP64 solution is bitwise that of
    nek_cg_solve, with the same iteration count; the FP32-operator solve
    reaches its true residual."""
    reqs = [((2, 2, 2), 5, nek.NEK_PREC_F64, 60 + k) for k in range(11)]
    reqs.append(((2, 2, 2), 5, nek.NEK_PREC_F32G32, 71))
    print("serve 12 requests side by side", flush=True)
    xs, res, trace = _serve(nek, reqs, budget=16 * GB)
    assert max(act for _, act, _ in trace) == len(reqs)
    for k, (box, N, prec, seed) in enumerate(reqs):
        assert res[k]["status"] == 0, (k, res[k])
        if prec != nek.NEK_PREC_F64:
            assert res[k]["rel_res_true"] <= 1e-10, (k, res[k])
            continue
        x, r = _cg_solve_box(nek, box, N, _rhs(nek, box, N, seed))
        assert r.iters == res[k]["iters"], (k, r.iters, res[k]["iters"])
        np.testing.assert_array_equal(xs[k], x)


def test_admission_by_footprint(nek):
    box, N = (4, 4, 4), 7
    f = nek.server_footprint(*box, N)
    assert f > 0
    # room for one request: the second waits until the first has finished
    xs, res, trace = _serve(nek, [(box, N, nek.NEK_PREC_F64, 1), (box, N, nek.NEK_PREC_F64, 2)],
                            budget=int(1.5 * f))
    assert max(t[1] for t in trace) == 1
    assert any(t[2] >= 1 for t in trace)
    # whichever finished its host preparation first runs first; the other
    # is admitted only after it has finished
    first, second = sorted(res.values(), key=lambda r: r["t_admit"])
    assert second["t_admit"] >= first["t_done"] - 1e-9
    # room for both: admitted together, their lifetimes overlap
    xs2, res2, trace2 = _serve(nek, [(box, N, nek.NEK_PREC_F64, 1), (box, N, nek.NEK_PREC_F64, 2)],
                               budget=int(2.5 * f))
    assert max(t[1] for t in trace2) == 2
    assert res2[1]["t_admit"] < res2[0]["t_done"]
    np.testing.assert_array_equal(xs[0], xs2[0])
    np.testing.assert_array_equal(xs[1], xs2[1])


def test_waiting_request_that_does_not_fit_is_not_overtaken(nek):
    """X runs; Y (prepared, too large to join X) arrives before the small Z,
    which would fit beside X: Z waits behind Y."""
    import time
    X, Y, Z = ((4, 4, 4), 7), ((4, 4, 4), 9), ((2, 2, 2), 3)
    fX, fY, fZ = (nek.server_footprint(*box, N) for box, N in (X, Y, Z))
    budget = fY + 2 * fZ
    assert fX + fZ <= budget < fX + fY
    srv = nek.Server(budget)
    a = synth.geom_coeffs()
    sub = lambda box, N, seed: srv.submit(*box, N, _rhs(nek, box, N, seed), amp=synth.AMP, a=a,
                                          rel_tol=1e-10, max_iter=20000)
    ids = {sub(*X, 1): "X"}
    for _ in range(100000):
        act, _ = srv.step(1)
        if act == 1:
            break
    assert act == 1
    ids[sub(*Y, 2)] = "Y"
    ids[sub(*Z, 3)] = "Z"
    time.sleep(0.5)                 # both are prepared by now (tiny meshes)
    res = {}
    for _ in range(200000):
        srv.step(1)
        for r in srv.poll():
            res[ids[r["id"]]] = r
            srv.fetch(r["id"])
        if len(res) == 3:
            break
    srv.close()
    assert all(r["status"] == 0 for r in res.values())
    assert res["Y"]["t_admit"] >= res["X"]["t_done"] - 1e-9
    assert res["Z"]["t_admit"] >= res["Y"]["t_admit"]


def test_failing_requests_in_a_mix(nek):
    """A request whose rhs holds a NaN reports a breakdown, one that cannot
    reach its tolerance within max_iter reports non-convergence, and a healthy
    request served beside them is bitwise the same as served alone."""
    box, N = (3, 3, 3), 5
    a = synth.geom_coeffs()
    good = _rhs(nek, box, N, 11)
    bad = good.copy()
    glo, dr = nek.box_numbering(*box, N)
    bad[np.argmax(dr == 0)] = np.nan
    alone = nek.Server(4 * GB)
    rid = alone.submit(*box, N, good, amp=synth.AMP, a=a, rel_tol=1e-10)
    r_alone = alone.run_until_done([rid])[rid]
    x_alone = alone.fetch(rid)
    alone.close()
    srv = nek.Server(4 * GB)
    ids = {srv.submit(*box, N, bad, amp=synth.AMP, a=a, rel_tol=1e-10): "nan",
           srv.submit(*box, N, good, amp=synth.AMP, a=a, rel_tol=1e-14, max_iter=10): "cap",
           srv.submit(*box, N, good, amp=synth.AMP, a=a, rel_tol=1e-10): "good"}
    got = srv.run_until_done(list(ids))
    x_good = srv.fetch([k for k, v in ids.items() if v == "good"][0])
    srv.close()
    res = {ids[k]: v for k, v in got.items()}
    assert res["nan"]["status"] == nek.NEK_ERR_BREAKDOWN
    assert res["cap"]["status"] == nek.NEK_ERR_NOCONV and res["cap"]["iters"] == 10
    assert res["good"]["status"] == 0 and res["good"]["iters"] == r_alone["iters"]
    np.testing.assert_array_equal(x_good, x_alone)


def test_server_errors(nek):
    srv = nek.Server(1 << 20)
    b = np.zeros(8 ** 3 * 64)
    with pytest.raises(nek.NekError) as ei:
        srv.submit(4, 4, 4, 7, b)
    assert ei.value.code == nek.NEK_ERR_NOMEM
    with pytest.raises(nek.NekError) as ei:
        srv.submit(1, 1, 1, 16, np.zeros(17 ** 3))
    assert ei.value.code == nek.NEK_ERR_UNSUPPORTED
    # more than 2^31 local points: rejected before the rhs is touched
    req = nek.Request(1290, 1290, 1290, 1, 0.0, (nek.ctypes.c_double * 3)(0, 0, 0), b.ctypes.data,
                      nek.NEK_PREC_F64, 1e-10, 100)
    rid = nek.ctypes.c_uint64()
    big = nek.Server(1 << 62)
    assert nek._lib.nek_server_submit(big._h, nek.ctypes.byref(req), nek.ctypes.byref(rid)) == nek.NEK_ERR_ARG
    big.close()
    with pytest.raises(nek.NekError):
        srv.fetch(12345) if 12345 in srv._sizes else nek._check(
            nek._lib.nek_server_fetch(srv._h, nek.ctypes.c_uint64(12345), b.ctypes.data), "fetch")
    srv.close()


def _oracle_residual(m, b, x):
    """||b - mask(dssum(A_L x))|| / ||b|| over unique nodes, by the oracle."""
    r = b - oracle.masked_ax(m, x)
    return np.sqrt(oracle.gdot(m.glo, r, r, m.U) / oracle.gdot(m.glo, b, b, m.U))


def test_served_caller_mesh_host_and_device(nek):
    """The oracle's own arrays of a perturbed mesh, submitted once from host
    memory and once from device memory, beside a box request of another
    degree: both solutions are bitwise the same as the host request served
    alone, and the oracle's converged solution to 1e-8."""
    box, N = (4, 3, 3), 7
    m = oracle.box_mesh(*box, N, synth.AMP, synth.geom_coeffs(seed=31))
    b = oracle.lattice_to_local(m, synth.lattice_uniform(*box, N, seed=17))
    assert nek.server_footprint_mesh(m.E, N) == nek.server_footprint(*box, N)

    def run(with_device, with_box):
        srv = nek.Server(8 * GB)
        ids = {srv.submit_mesh(m.E, N, m.D, m.g, m.glo, m.dirichlet, b): "host"}
        if with_device:
            dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (m.D, m.g, m.glo, m.dirichlet, b)]
            ids[srv.submit_mesh(m.E, N, *dev)] = "device"
        if with_box:
            ids[srv.submit(3, 3, 3, 5, _rhs(nek, (3, 3, 3), 5, 2), amp=synth.AMP, a=synth.geom_coeffs())] = "box"
        got = srv.run_until_done(list(ids))
        xs = {ids[k]: srv.fetch(k) for k in got}
        res = {ids[k]: v for k, v in got.items()}
        srv.close()
        return xs, res

    xa, ra = run(False, False)
    xm, rm = run(True, True)
    for k in rm:
        assert rm[k]["status"] == 0 and rm[k]["rel_res"] <= 1e-10, (k, rm[k])
    assert rm["host"]["E"] == m.E and rm["host"]["N"] == N
    np.testing.assert_array_equal(xm["host"], xa["host"])
    np.testing.assert_array_equal(xm["device"], xa["host"])
    assert rm["device"]["iters"] == rm["host"]["iters"] == ra["host"]["iters"]
    ref = oracle.cg(m, b, max_iter=5000, rel_tol=1e-13)
    assert np.linalg.norm(xa["host"] - ref.x) / np.linalg.norm(ref.x) <= 1e-8
    assert _oracle_residual(m, b, xa["host"]) <= 1.01e-10


def test_served_paper_shape_fp64_and_large_mixed(nek):
    """One mix of the benchmark's shape in FP64 (E = 4096, N = 9) and the
    largest request of the served workload in the mixed form (E = 8192 as
    32x16x16, N = 11, FP32 operator with FP32 g), both from the oracle's own
    arrays: the FP64 solution is bitwise that of nek_cg_solve on the same
    arrays; the oracle evaluates b - A x of the mixed solution itself."""
    print("serve: building E=4096 N=9 and E=8192 N=11 meshes", flush=True)
    m9 = oracle.box_mesh(16, 16, 16, 9, synth.AMP, synth.geom_coeffs(seed=41))
    b9 = oracle.lattice_to_local(m9, synth.lattice_uniform(16, 16, 16, 9, seed=42))
    m11 = oracle.box_mesh(32, 16, 16, 11, synth.AMP, synth.geom_coeffs(seed=43))
    b11 = oracle.lattice_to_local(m11, synth.lattice_uniform(32, 16, 16, 11, seed=44))
    srv = nek.Server(16 * GB)
    ids = {srv.submit_mesh(m9.E, 9, m9.D, m9.g, m9.glo, m9.dirichlet, b9, rel_tol=1e-10): "fp64",
           srv.submit_mesh(m11.E, 11, m11.D, m11.g, m11.glo, m11.dirichlet, b11,
                           precision=nek.NEK_PREC_F32G32, rel_tol=1e-10, max_iter=20000): "mixed"}
    print("serve: running the mix", flush=True)
    got = srv.run_until_done(list(ids), iters=4)
    xs = {ids[k]: srv.fetch(k) for k in got}
    res = {ids[k]: v for k, v in got.items()}
    srv.close()
    print(f"serve: fp64 {res['fp64']['iters']} iterations, mixed {res['mixed']['iters']} "
          f"({res['mixed']['n_replacements']} replacements)", flush=True)
    for k in res:
        assert res[k]["status"] == 0, (k, res[k])
    # FP64: the same arrays through nek_cg_solve
    gs = nek.GatherScatter(m9.E, 9, m9.glo, m9.dirichlet)
    xs9, rs9 = nek.cg_solve(torch.from_numpy(m9.D).cuda(), torch.from_numpy(m9.g).cuda(), gs,
                            torch.from_numpy(b9).cuda(), max_iter=10000, rel_tol=1e-10, true_residual=True)
    torch.cuda.synchronize()
    gs.close()
    assert rs9.iters == res["fp64"]["iters"]
    np.testing.assert_array_equal(xs["fp64"], xs9.cpu().numpy())
    assert res["fp64"]["rel_res"] == rs9.rel_res
    # mixed: the oracle's own FP64 residual of the served solution
    print("serve: oracle residual of the mixed solution", flush=True)
    t = _oracle_residual(m11, b11, xs["mixed"])
    lib = res["mixed"]["rel_res_true"]
    print(f"serve: mixed true residual oracle {t:.4e} library {lib:.4e}", flush=True)
    assert t <= 1.01e-10
    assert abs(t - lib) <= 1e-3 * t
