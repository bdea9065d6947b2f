"""CPU-side checks of the C ABI and of the library's host logic (no GPU work).

* libnek.so loads and exports every function that include/nek.h declares;
* status strings; argument checks that fail before any device call;
* the library's own host setup (GLL table, box numbering) against the oracle.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nek.h")
LIB = os.path.join(ROOT, "paper_2005_13425_amd", "libnek.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libnek.so not built")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(nek_\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("nek_ax", "nek_ax_f32", "nek_dssum", "nek_cg_solve", "nek_gs_create",
                 "nek_gs_destroy", "nek_strerror"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (nek_\w+)", out))
    assert set(_declared()) <= exported


@pytest.fixture(scope="module")
def nek():
    import paper_2005_13425_amd as nek
    return nek


def test_strerror_and_version(nek):
    assert nek.strerror(0) == "ok"
    assert "argument" in nek.strerror(-1)
    assert nek.strerror(-6) == "CG did not converge"
    assert nek.version() >= 10000


def test_argument_errors_before_device_work(nek):
    lib = nek._lib
    fake = ctypes.c_void_p(0x1000)
    assert lib.nek_ax(0, 9, fake, fake, fake, ctypes.c_void_p(0x9000), None) == nek.NEK_ERR_ARG
    assert lib.nek_ax(4, 16, fake, fake, fake, ctypes.c_void_p(0x9000), None) == nek.NEK_ERR_UNSUPPORTED
    assert lib.nek_ax(4, 0, fake, fake, fake, ctypes.c_void_p(0x9000), None) == nek.NEK_ERR_UNSUPPORTED
    assert lib.nek_ax(4, 9, None, fake, fake, ctypes.c_void_p(0x9000), None) == nek.NEK_ERR_ARG
    # misaligned u
    assert lib.nek_ax(4, 9, ctypes.c_void_p(0x1004), fake, fake, ctypes.c_void_p(0x9000000), None) == nek.NEK_ERR_ARG
    # u and w overlap (E*n^3*8 bytes from 0x1000)
    assert lib.nek_ax(4, 9, fake, fake, fake, ctypes.c_void_p(0x1008), None) == nek.NEK_ERR_ARG
    assert "overlap" in lib.nek_last_error().decode()
    assert lib.nek_ax_f32(4, 9, fake, fake, fake, 7, ctypes.c_void_p(0x9000000), None) == nek.NEK_ERR_UNSUPPORTED
    # the comparison designs: unknown variant, SHARED3D above N = 9, the nek_ax checks
    far = ctypes.c_void_p(0x9000000)
    assert lib.nek_ax_variant(4, 9, fake, fake, fake, far, 7, None) == nek.NEK_ERR_UNSUPPORTED
    assert lib.nek_ax_variant(4, 10, fake, fake, fake, far, nek.NEK_AX_SHARED3D, None) == nek.NEK_ERR_UNSUPPORTED
    assert "N <= 9" in lib.nek_last_error().decode()
    assert lib.nek_ax_variant(4, 9, fake, fake, fake, ctypes.c_void_p(0x1008), nek.NEK_AX_LAYER2D,
                              None) == nek.NEK_ERR_ARG
    assert lib.nek_ax_variant(0, 9, fake, fake, fake, far, nek.NEK_AX_ORIGINAL, None) == nek.NEK_ERR_ARG
    assert lib.nek_ax_variant(4, 16, fake, fake, fake, far, nek.NEK_AX_ORIGINAL, None) == nek.NEK_ERR_UNSUPPORTED
    assert lib.nek_dssum(None, fake, None) == nek.NEK_ERR_ARG
    assert lib.nek_gs_destroy(None) == nek.NEK_OK
    h = ctypes.c_void_p()
    assert lib.nek_gs_create(0, 3, fake, None, ctypes.byref(h)) == nek.NEK_ERR_ARG
    assert lib.nek_cg_solve(4, 9, fake, fake, None, fake, fake, None, None, None) == nek.NEK_ERR_ARG
    assert lib.nek_cg_workspace_bytes(0, 9) == 0
    assert lib.nek_cg_workspace_bytes(4096, 9) >= 3 * 4096 * 1000 * 8
    # the gather-scatter indexes local points with int32: E (N+1)^3 < 2^31
    big_E = (1 << 31) // 1000 + 1
    assert lib.nek_gs_create(big_E, 9, fake, None, ctypes.byref(h)) == nek.NEK_ERR_ARG
    assert "2^31" in lib.nek_last_error().decode()
    # bandwidth probe
    big = ctypes.c_void_p(0x100000)
    assert lib.nek_bw_probe(0, 7, fake, 0, big, 0, 0, None) == nek.NEK_ERR_ARG
    assert lib.nek_bw_probe(16, 9, fake, 16, big, 0, 0, None) == nek.NEK_ERR_ARG
    assert lib.nek_bw_probe(16, 0, fake, 16, big, 0, 1, None) == nek.NEK_ERR_ARG
    assert lib.nek_bw_probe(16, 1, ctypes.c_void_p(0x1008), 16, big, 0, 0, None) == nek.NEK_ERR_ARG
    assert lib.nek_bw_probe(16, 2, fake, 16, ctypes.c_void_p(0x1010), 0, 0, None) == nek.NEK_ERR_ARG   # overlap
    assert lib.nek_bw_probe(16, 2, fake, 15, big, 0, 0, None) == nek.NEK_ERR_ARG    # stride < n
    assert lib.nek_bw_probe(16, 2, fake, 17, big, 0, 0, None) == nek.NEK_ERR_ARG    # odd stride
    assert lib.nek_bw_probe(16, 2, fake, 16, big, 0, 8, None) == nek.NEK_ERR_ARG    # unknown flag
    # blocked streams: src holds nread whole blocks per block of n, whatever the stride
    blk = nek.NEK_PROBE_BLOCKED
    dst_in = ctypes.c_void_p(0x1000 + 8 * (2 * nek.NEK_PROBE_BLOCK - 16))
    assert lib.nek_bw_probe(16, 2, fake, 0, dst_in, 0, blk, None) == nek.NEK_ERR_ARG   # overlap
    assert "overlap" in lib.nek_last_error().decode()
    assert lib.nek_bw_probe(16, 2, fake, 16, big, -1, 0, None) == nek.NEK_ERR_ARG   # negative cap
    assert lib.nek_bw_probe_groups(10 ** 6, 0) == (10 ** 6 + 2047) // 2048
    assert lib.nek_bw_probe_groups(10 ** 6, 100) == 100
    assert lib.nek_bw_probe_groups(1, 0) == 0
    # Jacobi setup
    assert lib.nek_jacobi_inverse(0, 9, fake, fake, fake, fake, None) == nek.NEK_ERR_ARG
    assert lib.nek_jacobi_inverse(4, 16, fake, fake, fake, fake, None) == nek.NEK_ERR_UNSUPPORTED
    assert lib.nek_jacobi_inverse(4, 9, fake, fake, None, fake, None) == nek.NEK_ERR_ARG
    assert lib.nek_jacobi_inverse(4, 9, fake, fake, fake, ctypes.c_void_p(0x1008), None) == nek.NEK_ERR_ARG
    # served footprint: positive, growing with E and N, larger for the mixed forms
    f = [lib.nek_server_footprint(4, 4, 4, N, nek.NEK_PREC_F64) for N in (3, 5, 7)]
    assert 0 < f[0] < f[1] < f[2]
    assert lib.nek_server_footprint(8, 4, 4, 7, nek.NEK_PREC_F64) > f[2]
    assert (lib.nek_server_footprint(4, 4, 4, 7, nek.NEK_PREC_F32G32)
            > lib.nek_server_footprint(4, 4, 4, 7, nek.NEK_PREC_F32GBF16) > f[2])


@pytest.mark.parametrize("N", list(range(1, 16)))
def test_host_gll_table_matches_oracle(nek, N):
    z, w, D = nek.gll(N)
    zo, wo = oracle.gll(N)
    np.testing.assert_allclose(z, zo, atol=2e-16 * 4)
    np.testing.assert_allclose(w, wo, rtol=1e-13)
    np.testing.assert_allclose(D, oracle.dxm1_flat(N, zo), atol=1e-12 * N * N)
    # exact node symmetry and zero row sums of the library's table
    np.testing.assert_array_equal(z, -z[::-1])
    n = N + 1
    assert np.max(np.abs(D.reshape(n, n).sum(axis=0))) < 1e-12 * N * N


@pytest.mark.parametrize("box,N", [((2, 3, 4), 1), ((3, 2, 2), 4), ((4, 4, 4), 7), ((2, 2, 5), 9)])
def test_host_box_numbering_matches_oracle(nek, box, N):
    glo, dr = nek.box_numbering(*box, N)
    m = oracle.box_mesh(*box, N)
    np.testing.assert_array_equal(glo, m.glo)
    np.testing.assert_array_equal(dr, m.dirichlet)
