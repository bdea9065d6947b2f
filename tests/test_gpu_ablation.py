"""The earlier GPU designs of the local operator (Sec. IV-A, IV-B, IV-C),
through nek_ax_variant, against the FP64 oracle.

Each computes Listing 1 in FP64 with its own summation order, so the bar is
the operator's (rel-L2 <= 1e-12 against the oracle).  Every degree the design
supports, on boxes with a ragged element count; the three designs and the
pencil kernel agree with each other to the same bar; SHARED3D refuses N > 9.
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


def _case(N):
    box = (3, 2, 2) if N > 6 else (5, 3, 3)     # 12 or 45 elements
    m = oracle.box_mesh(*box, N, synth.AMP, synth.geom_coeffs())
    u = synth.local_uniform(m.P, seed=70 + N)
    return m, u, oracle.ax(m.E, N, m.D, m.g, u)


def _variants(nek):
    return {"original": nek.NEK_AX_ORIGINAL, "shared3d": nek.NEK_AX_SHARED3D,
            "layer2d": nek.NEK_AX_LAYER2D, "pencil": nek.NEK_AX_PENCIL}


@pytest.mark.parametrize("N", list(range(1, 16)))
@pytest.mark.parametrize("name", ["original", "shared3d", "layer2d", "pencil"])
def test_variant_against_oracle(nek, N, name):
    if name == "shared3d" and N > 9:
        pytest.skip("SHARED3D takes one thread per node: N <= 9")
    m, u, ref = _case(N)
    w = nek.ax_variant(_dev(u), _dev(m.D), _dev(m.g), N, _variants(nek)[name])
    torch.cuda.synchronize()
    err = _rel(w, ref)
    print(f"{name} N={N} E={m.E}: rel-L2 {err:.2e}", flush=True)
    assert err <= TOL


def test_variants_agree_at_the_paper_shape(nek):
    N = 9
    m = oracle.box_mesh(16, 8, 8, N, synth.AMP, synth.geom_coeffs())
    u = _dev(synth.local_uniform(m.P, seed=5))
    D, g = _dev(m.D), _dev(m.g)
    outs = {k: nek.ax_variant(u, D, g, N, v) for k, v in _variants(nek).items()}
    torch.cuda.synchronize()
    base = outs["pencil"].cpu().numpy()
    assert np.array_equal(base, nek.ax(u, D, g, N).cpu().numpy())   # PENCIL is nek_ax
    for k, w in outs.items():
        assert _rel(w, base) <= TOL, k


def test_shared3d_refuses_high_degree(nek):
    m = oracle.box_mesh(2, 1, 1, 10, synth.AMP, synth.geom_coeffs())
    with pytest.raises(nek.NekError) as ei:
        nek.ax_variant(_dev(np.zeros(m.P)), _dev(m.D), _dev(m.g), 10, nek.NEK_AX_SHARED3D)
    assert ei.value.code == nek.NEK_ERR_UNSUPPORTED
