"""FP64 CPU oracle for the Nekbone Poisson hot path (arXiv 2005.13425).

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only users.  The product package
never imports this module, and this module never imports the product.

The arithmetic lives in ``nek_oracle.c`` (plain C, FP64); this file only
marshals numpy arrays into it.  Each wrapper names the passage of the paper
that the C routine follows:

* :func:`gll`, :func:`dxm1` -- GLL points and the derivative matrix dxm1 of
  Listing 1 (Sec. III-A: n = degree + 1 GLL points per direction).
* :func:`box_mesh` -- box of hexahedra on the unit cube (Sec. III, Poisson on
  a cubic domain): coordinates, geometric factors gxyz of Listing 1, mass,
  global numbering and Dirichlet flags.
* :func:`ax` -- Listing 1.
* :func:`dssum`, :func:`mask` -- the communication step of Ax (Sec. III) and
  the boundary masking (Sec. VI-B).
* :func:`gdot`, :func:`cg` -- the CG solve of Sec. III / Sec. V.
* :func:`ax_diag`, :func:`jacobi_inverse`, :func:`pcg` -- the diagonal of the
  element operator of Listing 1 and CG preconditioned by the inverse of the
  assembled diagonal (Jacobi), the simplest form of the preconditioning that
  Sec. VII names as future work.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nek_oracle.c")
_LIB = os.path.join(_HERE, "libnek_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, -O2, OpenMP over elements)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


TIMED_FLAGS = ["-std=c11", "-O3", "-march=native", "-fopenmp"]


def use_timed_build(directory: str) -> str:
    """Compile the same source with TIMED_FLAGS for the host that runs it
    (-march=native, so it is built where it runs, into `directory`) and make
    every later call of this module use that build.  ISO C11 keeps gcc from
    contracting a*b+c into fused multiply-adds and the source has no
    reassociation, so the results are those of the default build."""
    global _lib
    os.makedirs(directory, exist_ok=True)
    path = os.path.join(directory, "libnek_oracle_timed.so")
    subprocess.run(["gcc", *TIMED_FLAGS, "-fPIC", "-shared", "-o", path, _SRC, "-lm"], check=True)
    _lib = _bind(path)
    return path


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    _lib = _bind(_LIB)
    return _lib


def _bind(path):
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    i64 = ctypes.c_int64
    ci = ctypes.c_int
    lib.or_gll.argtypes = [ci, dp, dp]
    lib.or_gll.restype = ci
    lib.or_dxm1.argtypes = [ci, dp, dp]
    lib.or_dxm1.restype = ci
    lib.or_box_coords.argtypes = [ci, ci, ci, ci, dp, ctypes.c_double, dp, dp]
    lib.or_box_coords.restype = None
    lib.or_geom.argtypes = [i64, ci, dp, dp, dp, dp, dp]
    lib.or_geom.restype = ctypes.c_double
    lib.or_box_glonum.argtypes = [ci, ci, ci, ci, i64p, u8p]
    lib.or_box_glonum.restype = None
    lib.or_ax.argtypes = [i64, ci, dp, dp, dp, dp, ci]
    lib.or_ax.restype = None
    lib.or_dssum.argtypes = [i64, i64p, i64, dp]
    lib.or_dssum.restype = ci
    lib.or_mask.argtypes = [i64, u8p, dp]
    lib.or_mask.restype = None
    lib.or_gdot.argtypes = [i64, i64p, i64, dp, dp]
    lib.or_gdot.restype = ctypes.c_double
    lib.or_cg.argtypes = [i64, ci, dp, dp, i64p, i64, u8p, dp, dp, ci,
                          ctypes.c_double, ctypes.POINTER(ci), dp, ci]
    lib.or_cg.restype = ci
    lib.or_ax_diag.argtypes = [i64, ci, dp, dp, dp]
    lib.or_ax_diag.restype = None
    lib.or_pcg.argtypes = [i64, ci, dp, dp, i64p, i64, u8p, dp, dp, dp, ci,
                           ctypes.c_double, ctypes.POINTER(ci), dp, ci]
    lib.or_pcg.restype = ci
    lib.or_max_threads.argtypes = []
    lib.or_max_threads.restype = ci
    return lib


def _d(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i64(a):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _u8(a):
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def max_threads() -> int:
    return int(_load().or_max_threads())


def gll(N: int):
    """GLL nodes and weights for degree N (n = N+1 points)."""
    z = np.zeros(N + 1)
    w = np.zeros(N + 1)
    if _load().or_gll(N, _d(z), _d(w)) != 0:
        raise ValueError(f"bad degree {N}")
    return z, w


def dxm1(N: int, z=None):
    """The derivative matrix as a numpy (n, n) array with ``D[i, l] = dxm1(i, l)``."""
    if z is None:
        z, _ = gll(N)
    n = N + 1
    flat = np.zeros(n * n)
    _load().or_dxm1(N, _d(z), _d(flat))
    # flat[i + n*l] = dxm1(i,l): reshape (l, i) then transpose to [i, l]
    return flat.reshape(n, n).T.copy()


def dxm1_flat(N: int, z=None):
    """dxm1 in the layout of Listing 1 (column-major): ``flat[i + n*l] = dxm1(i,l)``."""
    return np.ascontiguousarray(dxm1(N, z).T).reshape(-1)


@dataclass
class BoxMesh:
    """Box of Ex x Ey x Ez hexahedra of degree N on the unit cube."""
    Ex: int
    Ey: int
    Ez: int
    N: int
    z: np.ndarray        # GLL nodes (n,)
    wq: np.ndarray       # GLL weights (n,)
    D: np.ndarray        # dxm1 flat, D[i + n*l] = dxm1(i,l)
    X: np.ndarray        # (3, P) nodal coordinates
    g: np.ndarray        # (E*6*n^3,) geometric factors, gxyz(i,j,k,c,e)
    bm: np.ndarray       # (P,) diagonal mass W*detJ
    glo: np.ndarray      # (P,) int64 global ids
    dirichlet: np.ndarray  # (P,) uint8
    detmin: float

    @property
    def n(self):
        return self.N + 1

    @property
    def E(self):
        return self.Ex * self.Ey * self.Ez

    @property
    def P(self):
        return self.E * self.n ** 3

    @property
    def U(self):
        return (self.Ex * self.N + 1) * (self.Ey * self.N + 1) * (self.Ez * self.N + 1)


def box_mesh(Ex: int, Ey: int, Ez: int, N: int, amp: float = 0.0, a=(0.0, 0.0, 0.0)) -> BoxMesh:
    """Coordinates, geometric factors, mass, numbering and Dirichlet flags of a box."""
    lib = _load()
    n = N + 1
    E = Ex * Ey * Ez
    P = E * n ** 3
    z, wq = gll(N)
    D = dxm1_flat(N, z)
    av = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    X = np.zeros(3 * P)
    lib.or_box_coords(Ex, Ey, Ez, N, _d(z), float(amp), _d(av), _d(X))
    g = np.zeros(6 * P)
    bm = np.zeros(P)
    detmin = lib.or_geom(E, N, _d(wq), _d(D), _d(X), _d(g), _d(bm))
    glo = np.zeros(P, dtype=np.int64)
    dirichlet = np.zeros(P, dtype=np.uint8)
    lib.or_box_glonum(Ex, Ey, Ez, N, _i64(glo), _u8(dirichlet))
    return BoxMesh(Ex, Ey, Ez, N, z, wq, D, X.reshape(3, P), g, bm, glo, dirichlet, float(detmin))


def ax(E: int, N: int, D, g, u, nthreads: int = 0):
    """w = A_e u for every element (Listing 1); no summation, no mask."""
    D = np.ascontiguousarray(D, dtype=np.float64).reshape(-1)
    g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    n = N + 1
    assert D.size == n * n and u.size == E * n ** 3 and g.size == 6 * E * n ** 3
    w = np.zeros_like(u)
    _load().or_ax(E, N, _d(D), _d(g), _d(u), _d(w), int(nthreads))
    return w


def dssum(glo, w, U=None):
    """Every copy of a global node gets the sum of all copies (Sec. III)."""
    glo = np.ascontiguousarray(glo, dtype=np.int64)
    w = np.array(w, dtype=np.float64, copy=True).reshape(-1)
    if U is None:
        U = int(glo.max()) + 1
    rc = _load().or_dssum(w.size, _i64(glo), int(U), _d(w))
    if rc != 0:
        raise ValueError(f"or_dssum failed ({rc})")
    return w


def mask(dirichlet, w):
    """Zero the Dirichlet nodes (Sec. VI-B)."""
    dirichlet = np.ascontiguousarray(dirichlet, dtype=np.uint8)
    w = np.array(w, dtype=np.float64, copy=True).reshape(-1)
    _load().or_mask(w.size, _u8(dirichlet), _d(w))
    return w


def gdot(glo, a, b, U=None):
    """Inner product over unique global nodes of two continuous vectors."""
    glo = np.ascontiguousarray(glo, dtype=np.int64)
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
    if U is None:
        U = int(glo.max()) + 1
    return float(_load().or_gdot(a.size, _i64(glo), int(U), _d(a), _d(b)))


def masked_ax(mesh: BoxMesh, u, nthreads: int = 0):
    """mask(dssum(A_L u)): the assembled, masked operator on a local vector."""
    w = ax(mesh.E, mesh.N, mesh.D, mesh.g, u, nthreads)
    return mask(mesh.dirichlet, dssum(mesh.glo, w, mesh.U))


@dataclass
class CGResult:
    x: np.ndarray
    iters: int
    status: int
    res_hist: np.ndarray


def cg(mesh: BoxMesh, b, max_iter: int = 100, rel_tol: float = 0.0, nthreads: int = 0) -> CGResult:
    """Unpreconditioned CG on mask(dssum(A_L .)) x = b, x_0 = 0 (Sec. III, Sec. V)."""
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
    x = np.zeros_like(b)
    hist = np.zeros(max_iter + 1)
    it = ctypes.c_int(0)
    rc = _load().or_cg(mesh.E, mesh.N, _d(mesh.D), _d(mesh.g), _i64(mesh.glo), mesh.U,
                       _u8(mesh.dirichlet), _d(b), _d(x), int(max_iter), float(rel_tol),
                       ctypes.byref(it), _d(hist), int(nthreads))
    return CGResult(x, int(it.value), int(rc), hist[: it.value + 1].copy())


def ax_diag(E: int, N: int, D, g):
    """Diagonal of the element operator of Listing 1 at every local point."""
    D = np.ascontiguousarray(D, dtype=np.float64).reshape(-1)
    g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1)
    d = np.empty(E * (N + 1) ** 3)
    _load().or_ax_diag(E, N, _d(D), _d(g), _d(d))
    return d


def jacobi_inverse(mesh: BoxMesh):
    """Jacobi preconditioner M^-1 as a continuous local vector: one over the
    diagonal of the assembled operator (dssum of the element diagonals) at
    free nodes, zero at Dirichlet nodes."""
    dg = dssum(mesh.glo, ax_diag(mesh.E, mesh.N, mesh.D, mesh.g), mesh.U)
    inv = np.zeros_like(dg)
    free = mesh.dirichlet == 0
    inv[free] = 1.0 / dg[free]
    return inv


def pcg(mesh: BoxMesh, b, dinv, max_iter: int = 100, rel_tol: float = 0.0,
        nthreads: int = 0) -> CGResult:
    """CG preconditioned with M^-1 = dinv on mask(dssum(A_L .)) x = b, x_0 = 0;
    the residual history and the stopping test use ||r|| / ||b||."""
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
    dinv = np.ascontiguousarray(dinv, dtype=np.float64).reshape(-1)
    x = np.zeros_like(b)
    hist = np.zeros(max_iter + 1)
    it = ctypes.c_int(0)
    rc = _load().or_pcg(mesh.E, mesh.N, _d(mesh.D), _d(mesh.g), _i64(mesh.glo), mesh.U,
                        _u8(mesh.dirichlet), _d(dinv), _d(b), _d(x), int(max_iter),
                        float(rel_tol), ctypes.byref(it), _d(hist), int(nthreads))
    return CGResult(x, int(it.value), int(rc), hist[: it.value + 1].copy())


def lattice_to_local(mesh: BoxMesh, vals):
    """Scatter per-lattice-node values to the local layout (b_L = vals[glo[L]])
    and zero the Dirichlet nodes: the plain right-hand side."""
    vals = np.asarray(vals, dtype=np.float64)
    b = vals[mesh.glo]
    return mask(mesh.dirichlet, b)


def manufactured_rhs(mesh: BoxMesh):
    """b = mask(dssum(B_L f)) with f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z),
    so that the exact solution is sin(pi x) sin(pi y) sin(pi z)."""
    x, y, zc = mesh.X
    f = 3.0 * np.pi ** 2 * np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * zc)
    return mask(mesh.dirichlet, dssum(mesh.glo, mesh.bm * f, mesh.U))
