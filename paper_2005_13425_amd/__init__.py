"""nekmi: Nekbone's matrix-free Poisson operator on AMD MI355X (gfx950).

Thin Python binding over the C ABI of ``libnek.so`` (``include/nek.h``).  The
functions below only check and marshal arguments (torch tensors for device
memory, the current HIP stream of torch) and call the library; every step of
the path runs in the library's HIP kernels.  There is no fallback: if the
library is missing, importing this package raises.

Method: Karp et al., "Optimization of Tensor-product Operations in Nekbone on
GPUs" (arXiv 2005.13425) -- Listing 1 (local operator), Sec. III (dssum, CG),
Sec. VI-B (masking).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnek.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
        "(there is no CPU fallback)")

_lib = ctypes.CDLL(LIB_PATH)

NEK_OK = 0
NEK_ERR_ARG = -1
NEK_ERR_UNSUPPORTED = -2
NEK_ERR_DEVICE = -3
NEK_ERR_NOMEM = -4
NEK_ERR_BREAKDOWN = -5
NEK_ERR_NOCONV = -6
NEK_ERR_STATE = -7
NEK_MAX_DEGREE = 15
NEK_G_F32 = 1
NEK_G_BF16 = 2
NEK_PREC_F64 = 0
NEK_PREC_F32G32 = 1
NEK_PREC_F32GBF16 = 2
NEK_PREC_F64G32 = 3
NEK_PREC_F64GBF16 = 4
NEK_AX_PENCIL = 0
NEK_AX_ORIGINAL = 1
NEK_AX_SHARED3D = 2
NEK_AX_LAYER2D = 3
NEK_MEM_HOST = 0
NEK_MEM_DEVICE = 1

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_ci = ctypes.c_int
_dp = ctypes.POINTER(ctypes.c_double)


class CgOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int), ("rel_tol", ctypes.c_double),
                ("precision", ctypes.c_int), ("D32", _vp), ("g_lo", _vp),
                ("check_every", ctypes.c_int), ("true_residual", ctypes.c_int),
                ("reliable_drop", ctypes.c_double), ("workspace", _vp),
                ("workspace_bytes", ctypes.c_size_t), ("dinv", _vp)]


class CgStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("status", ctypes.c_int), ("rel_res", ctypes.c_double),
                ("rel_res_true", ctypes.c_double), ("n_replacements", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("Ex", ctypes.c_int), ("Ey", ctypes.c_int), ("Ez", ctypes.c_int), ("N", ctypes.c_int),
                ("amp", ctypes.c_double), ("a", ctypes.c_double * 3), ("b", _vp),
                ("precision", ctypes.c_int), ("rel_tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("E", ctypes.c_int64), ("D", _vp), ("g", _vp), ("glo", _vp), ("dirichlet", _vp),
                ("mem", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int), ("iters", ctypes.c_int),
                ("n_replacements", ctypes.c_int), ("rel_res", ctypes.c_double),
                ("rel_res_true", ctypes.c_double), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double), ("E", ctypes.c_int64),
                ("N", ctypes.c_int), ("footprint", ctypes.c_size_t)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("nek_strerror", ctypes.c_char_p, [_ci])
_sig("nek_last_error", ctypes.c_char_p, [])
_sig("nek_version", _ci, [])
_sig("nek_gll", _ci, [_ci, _vp, _vp, _vp])
_sig("nek_box_numbering", _ci, [_ci, _ci, _ci, _ci, _vp, _vp])
_sig("nek_box_geometry", _ci, [_ci, _ci, _ci, _ci, ctypes.c_double, _vp, _vp, _vp, _vp, _vp])
_sig("nek_ax", _ci, [_i64, _ci, _vp, _vp, _vp, _vp, _vp])
_sig("nek_ax_variant", _ci, [_i64, _ci, _vp, _vp, _vp, _vp, _ci, _vp])
_sig("nek_ax_f32", _ci, [_i64, _ci, _vp, _vp, _vp, _ci, _vp, _vp])
_sig("nek_convert_g", _ci, [_i64, _ci, _vp, _ci, _vp, _vp])
_sig("nek_gs_create", _ci, [_i64, _ci, _vp, _vp, ctypes.POINTER(_vp)])
_sig("nek_gs_destroy", _ci, [_vp])
_sig("nek_gs_info", _ci, [_vp] + [ctypes.POINTER(_i64)] * 4)
_sig("nek_dssum", _ci, [_vp, _vp, _vp])
_sig("nek_gs_dot", _ci, [_vp, _vp, _vp, _vp, _vp])
_sig("nek_bw_probe", _ci, [_i64, _ci, _vp, _i64, _vp, _ci, _ci, _vp])
_sig("nek_bw_probe_groups", _i64, [_i64, _ci])
_sig("nek_jacobi_inverse", _ci, [_i64, _ci, _vp, _vp, _vp, _vp, _vp])
_sig("nek_server_create", _ci, [ctypes.c_size_t, ctypes.POINTER(_vp)])
_sig("nek_server_submit", _ci, [_vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)])
_sig("nek_server_footprint", ctypes.c_size_t, [_ci, _ci, _ci, _ci, _ci])
_sig("nek_server_footprint_mesh", ctypes.c_size_t, [_i64, _ci, _ci])
_sig("nek_server_step", _ci, [_vp, _ci, ctypes.POINTER(_ci), ctypes.POINTER(_ci)])
_sig("nek_server_poll", _ci, [_vp, ctypes.POINTER(Result), _ci, ctypes.POINTER(_ci)])
_sig("nek_server_fetch", _ci, [_vp, ctypes.c_uint64, _vp])
_sig("nek_server_clock", ctypes.c_double, [_vp])
_sig("nek_server_destroy", _ci, [_vp])
_sig("nek_cg_default_opts", None, [ctypes.POINTER(CgOpts)])
_sig("nek_cg_workspace_bytes", ctypes.c_size_t, [_i64, _ci])
_sig("nek_cg_solve", _ci, [_i64, _ci, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(CgOpts),
                           ctypes.POINTER(CgStats), _vp])
_sig("nek_cg_solve_noalloc", _ci, [_i64, _ci, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(CgOpts),
                                   ctypes.POINTER(CgStats), _vp])

# workspace bytes of nek_cg_solve_noalloc's device array (NEK_CG_NOALLOC_BYTES)
CG_NOALLOC_BYTES = 64 << 20


class NekError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _lib.nek_last_error().decode() or _lib.nek_strerror(code).decode()
        super().__init__(f"{where}: {msg} (status {code})")
        self.code = code


def _check(code: int, where: str):
    if code != NEK_OK:
        raise NekError(code, where)


def strerror(code: int) -> str:
    return _lib.nek_strerror(code).decode()


def version() -> int:
    return int(_lib.nek_version())


# ------------------------------------------------------------------ helpers
def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype, name, numel=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _host_np(a, dtype, name, numel=None):
    a = np.ascontiguousarray(a, dtype=dtype)
    if numel is not None and a.size != numel:
        raise ValueError(f"{name} must have {numel} elements, got {a.size}")
    return a


def npts(E: int, N: int) -> int:
    return int(E) * (N + 1) ** 3


# ------------------------------------------------------------------ setup
def gll(N: int):
    """GLL nodes, weights and dxm1 (numpy, D[i + n*l] = dxm1(i,l)) for degree N."""
    n = N + 1
    z, w, D = np.zeros(n), np.zeros(n), np.zeros(n * n)
    _check(_lib.nek_gll(N, z.ctypes.data, w.ctypes.data, D.ctypes.data), "nek_gll")
    return z, w, D


def box_numbering(Ex: int, Ey: int, Ez: int, N: int):
    """(glo int64[P], dirichlet uint8[P]) of a box mesh, on the host."""
    P = Ex * Ey * Ez * (N + 1) ** 3
    glo = np.zeros(P, dtype=np.int64)
    dr = np.zeros(P, dtype=np.uint8)
    _check(_lib.nek_box_numbering(Ex, Ey, Ez, N, glo.ctypes.data, dr.ctypes.data), "nek_box_numbering")
    return glo, dr


def box_geometry(Ex: int, Ey: int, Ez: int, N: int, amp: float, a, device="cuda",
                 want_mass: bool = False, want_coords: bool = False, stream=None):
    """Geometric factors g (6P) and optionally mass (P) and coordinates (3P) on the device."""
    torch = _torch()
    P = Ex * Ey * Ez * (N + 1) ** 3
    av = _host_np(a, np.float64, "a", 3)
    g = torch.empty(6 * P, dtype=torch.float64, device=device)
    bm = torch.empty(P, dtype=torch.float64, device=device) if want_mass else None
    X = torch.empty(3 * P, dtype=torch.float64, device=device) if want_coords else None
    _check(_lib.nek_box_geometry(Ex, Ey, Ez, N, float(amp), av.ctypes.data,
                                 ctypes.c_void_p(g.data_ptr()),
                                 ctypes.c_void_p(bm.data_ptr()) if bm is not None else None,
                                 ctypes.c_void_p(X.data_ptr()) if X is not None else None,
                                 _stream_ptr(stream)), "nek_box_geometry")
    return g, bm, X


# ------------------------------------------------------------------ operator
def ax(u, D, g, N: int, out=None, stream=None):
    """w = A_e u for every element (Listing 1), FP64, on the device."""
    torch = _torch()
    n3 = (N + 1) ** 3
    if u.numel() % n3:
        raise ValueError("u size is not a multiple of (N+1)^3")
    E = u.numel() // n3
    if out is None:
        out = torch.empty_like(u)
    _check(_lib.nek_ax(E, N, _dev(u, torch.float64, "u"), _dev(D, torch.float64, "D", (N + 1) ** 2),
                       _dev(g, torch.float64, "g", 6 * E * n3), _dev(out, torch.float64, "w", E * n3),
                       _stream_ptr(stream)), "nek_ax")
    return out


def ax_variant(u, D, g, N: int, variant: int, out=None, stream=None):
    """w = A_e u with one of the earlier GPU designs of Sec. IV (NEK_AX_ORIGINAL,
    NEK_AX_SHARED3D, NEK_AX_LAYER2D) or the pencil kernel (NEK_AX_PENCIL)."""
    torch = _torch()
    n3 = (N + 1) ** 3
    if u.numel() % n3:
        raise ValueError("u size is not a multiple of (N+1)^3")
    E = u.numel() // n3
    if out is None:
        out = torch.empty_like(u)
    _check(_lib.nek_ax_variant(E, N, _dev(u, torch.float64, "u"), _dev(D, torch.float64, "D", (N + 1) ** 2),
                               _dev(g, torch.float64, "g", 6 * E * n3), _dev(out, torch.float64, "w", E * n3),
                               int(variant), _stream_ptr(stream)), "nek_ax_variant")
    return out


def convert_g(g, N: int, dtype: int, stream=None):
    """g rounded to FP32 (NEK_G_F32) or BF16 bits (NEK_G_BF16) on the device."""
    torch = _torch()
    n3 = (N + 1) ** 3
    E = g.numel() // (6 * n3)
    tdt = torch.float32 if dtype == NEK_G_F32 else torch.int16
    out = torch.empty(g.numel(), dtype=tdt, device=g.device)
    _check(_lib.nek_convert_g(E, N, _dev(g, torch.float64, "g", 6 * E * n3), dtype,
                              ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)), "nek_convert_g")
    return out


def ax_f32(u, D32, g_lo, g_dtype: int, N: int, out=None, stream=None):
    """The local operator computed in FP32 (g as FP32 or BF16), FP64 in and out."""
    torch = _torch()
    n3 = (N + 1) ** 3
    E = u.numel() // n3
    if out is None:
        out = torch.empty_like(u)
    gdt = torch.float32 if g_dtype == NEK_G_F32 else torch.int16
    _check(_lib.nek_ax_f32(E, N, _dev(u, torch.float64, "u"), _dev(D32, torch.float32, "D32", (N + 1) ** 2),
                           _dev(g_lo, gdt, "g_lo", 6 * E * n3), int(g_dtype),
                           _dev(out, torch.float64, "w", E * n3), _stream_ptr(stream)), "nek_ax_f32")
    return out


NEK_PROBE_NT = 1
NEK_PROBE_READ_ONLY = 2
NEK_PROBE_BLOCKED = 4
NEK_PROBE_BLOCK = 2048


def bw_probe_src_doubles(n: int, nread: int, stride: int | None = None, blocked: bool = False) -> int:
    """Doubles the probe's src must hold for these streams."""
    if blocked:
        return nread * NEK_PROBE_BLOCK * ((n + NEK_PROBE_BLOCK - 1) // NEK_PROBE_BLOCK)
    return (nread - 1) * (n if stride is None else int(stride)) + n


def bw_probe(src, dst, nread: int, n: int | None = None, stride: int | None = None, grid_cap: int = 0,
             streaming: bool = False, read_only: bool = False, blocked: bool = False, stream=None):
    """nread read streams of n doubles, stream k at src[k*stride:] (blocked:
    interleaved in blocks of NEK_PROBE_BLOCK doubles); without read_only
    dst[i] = sum_k stream_k[i] (n doubles), with read_only dst gets one
    partial per workgroup (bw_probe_groups(n, grid_cap) doubles).
    streaming: non-temporal loads and stores."""
    torch = _torch()
    if n is None:
        n = dst.numel()
    stride = n if stride is None else int(stride)
    ndst = bw_probe_groups(n, grid_cap) if read_only else n
    if src.numel() < bw_probe_src_doubles(n, nread, stride, blocked):
        raise ValueError("src is shorter than its streams")
    if dst.numel() < ndst:
        raise ValueError(f"dst must hold {ndst} doubles")
    flags = ((NEK_PROBE_NT if streaming else 0) | (NEK_PROBE_READ_ONLY if read_only else 0) |
             (NEK_PROBE_BLOCKED if blocked else 0))
    _check(_lib.nek_bw_probe(int(n), int(nread), _dev(src, torch.float64, "src"), stride,
                             _dev(dst, torch.float64, "dst"), int(grid_cap), flags, _stream_ptr(stream)),
           "nek_bw_probe")
    return dst


def bw_probe_groups(n: int, grid_cap: int = 0) -> int:
    return int(_lib.nek_bw_probe_groups(int(n), int(grid_cap)))


# ------------------------------------------------------------------ gather-scatter
class GatherScatter:
    """Direct-stiffness summation + Dirichlet mask of a mesh (nek_gs handle)."""

    def __init__(self, E: int, N: int, glo, dirichlet=None):
        P = npts(E, N)
        self.E, self.N, self.P = int(E), int(N), P
        glo = _host_np(glo, np.int64, "glo", P)
        dr = None if dirichlet is None else _host_np(dirichlet, np.uint8, "dirichlet", P)
        h = ctypes.c_void_p()
        _check(_lib.nek_gs_create(E, N, glo.ctypes.data, None if dr is None else dr.ctypes.data,
                                  ctypes.byref(h)), "nek_gs_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def info(self):
        vals = [_i64() for _ in range(4)]
        _check(_lib.nek_gs_info(self._h, *[ctypes.byref(v) for v in vals]), "nek_gs_info")
        return dict(n_unique=vals[0].value, n_rows=vals[1].value, n_entries=vals[2].value,
                    n_masked=vals[3].value)

    def dssum(self, w, stream=None):
        """In place: w <- mask(dssum(w))."""
        torch = _torch()
        _check(_lib.nek_dssum(self._h, _dev(w, torch.float64, "w", self.P), _stream_ptr(stream)), "nek_dssum")
        return w

    def dot(self, a, b, stream=None):
        """Inner product over unique nodes, returned as a 1-element device tensor."""
        torch = _torch()
        res = torch.empty(1, dtype=torch.float64, device=a.device)
        _check(_lib.nek_gs_dot(self._h, _dev(a, torch.float64, "a", self.P), _dev(b, torch.float64, "b", self.P),
                               ctypes.c_void_p(res.data_ptr()), _stream_ptr(stream)), "nek_gs_dot")
        return res

    def close(self):
        if getattr(self, "_h", None):
            _lib.nek_gs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ CG
@dataclass
class CgResult:
    iters: int
    status: int
    rel_res: float
    rel_res_true: float
    n_replacements: int


def cg_workspace_bytes(E: int, N: int) -> int:
    return int(_lib.nek_cg_workspace_bytes(E, N))


def _cg_call(fn, name, D, g, gs, b, x, max_iter, rel_tol, precision, D32, g_lo, check_every, true_residual,
             reliable_drop, workspace, raise_on_error, stream, dinv):
    torch = _torch()
    E, N = gs.E, gs.N
    P = gs.P
    if x is None:
        x = torch.empty_like(b)
    o = CgOpts()
    _lib.nek_cg_default_opts(ctypes.byref(o))
    o.max_iter = int(max_iter)
    o.rel_tol = float(rel_tol)
    o.precision = int(precision)
    if precision != NEK_PREC_F64:
        if precision in (NEK_PREC_F32G32, NEK_PREC_F32GBF16):   # the FP32 operator
            o.D32 = _dev(D32, torch.float32, "D32", (N + 1) ** 2)
        gdt = torch.float32 if precision in (NEK_PREC_F32G32, NEK_PREC_F64G32) else torch.int16
        o.g_lo = _dev(g_lo, gdt, "g_lo", 6 * P)
    o.check_every = int(check_every)
    o.true_residual = 1 if true_residual else 0
    o.reliable_drop = float(reliable_drop)
    if dinv is not None:
        o.dinv = _dev(dinv, torch.float64, "dinv", P)
    if workspace is not None:
        if workspace.numel() * workspace.element_size() < cg_workspace_bytes(E, N):
            raise ValueError("workspace too small")
        o.workspace = ctypes.c_void_p(workspace.data_ptr())
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    st = CgStats()
    rc = fn(E, N, _dev(D, torch.float64, "D", (N + 1) ** 2), _dev(g, torch.float64, "g", 6 * P),
            gs.handle, _dev(b, torch.float64, "b", P), _dev(x, torch.float64, "x", P),
            ctypes.byref(o), ctypes.byref(st), _stream_ptr(stream))
    res = CgResult(st.iters, st.status, st.rel_res, st.rel_res_true, st.n_replacements)
    if rc != NEK_OK and (raise_on_error or rc not in (NEK_ERR_BREAKDOWN, NEK_ERR_NOCONV)):
        raise NekError(rc, name)
    return x, res


def cg_solve(D, g, gs: GatherScatter, b, x=None, max_iter: int = 100, rel_tol: float = 0.0,
             precision: int = NEK_PREC_F64, D32=None, g_lo=None, check_every: int = 0,
             true_residual: bool = False, reliable_drop: float = 0.0, workspace=None,
             raise_on_error: bool = True, stream=None, dinv=None):
    """CG on mask(dssum(A_L x)) = b with x_0 = 0, on the device; with dinv (from
    jacobi_inverse) Jacobi-preconditioned CG.

    Returns (x, CgResult).  With raise_on_error=False a breakdown or
    non-convergence is reported in CgResult.status instead of raising."""
    return _cg_call(_lib.nek_cg_solve, "nek_cg_solve", D, g, gs, b, x, max_iter, rel_tol, precision, D32, g_lo,
                    check_every, true_residual, reliable_drop, workspace, raise_on_error, stream, dinv)


def cg_solve_noalloc(D, g, gs: GatherScatter, b, x, max_iter: int = 100, rel_tol: float = 0.0,
                     precision: int = NEK_PREC_F64, D32=None, g_lo=None, check_every: int = 0,
                     true_residual: bool = False, reliable_drop: float = 0.0, raise_on_error: bool = True,
                     stream=None, dinv=None):
    """cg_solve with the library's own fixed device workspace (CG_NOALLOC_BYTES
    per GPU): the call allocates nothing, so x must be given.  Calls that
    overlap on one GPU share that workspace and must not overlap."""
    if x is None:
        raise ValueError("cg_solve_noalloc: x must be given (the call allocates nothing)")
    return _cg_call(_lib.nek_cg_solve_noalloc, "nek_cg_solve_noalloc", D, g, gs, b, x, max_iter, rel_tol,
                    precision, D32, g_lo, check_every, true_residual, reliable_drop, None, raise_on_error,
                    stream, dinv)


def jacobi_inverse(D, g, gs: GatherScatter, out=None, stream=None):
    """The Jacobi preconditioner of the assembled, masked operator as a device
    vector: 1 / assembled diagonal at free nodes, 0 at masked nodes."""
    torch = _torch()
    E, N, P = gs.E, gs.N, gs.P
    if out is None:
        out = torch.empty(P, dtype=torch.float64, device=g.device)
    _check(_lib.nek_jacobi_inverse(E, N, _dev(D, torch.float64, "D", (N + 1) ** 2),
                                   _dev(g, torch.float64, "g", 6 * P), gs.handle,
                                   _dev(out, torch.float64, "dinv", P), _stream_ptr(stream)),
           "nek_jacobi_inverse")
    return out


def cg_workspace(E: int, N: int, device="cuda"):
    """A device buffer usable as the CG workspace (256-byte aligned by torch's allocator)."""
    torch = _torch()
    nbytes = cg_workspace_bytes(E, N)
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


# ------------------------------------------------------------------ served solves
def server_footprint(Ex: int, Ey: int, Ez: int, N: int, precision: int = NEK_PREC_F64) -> int:
    return int(_lib.nek_server_footprint(Ex, Ey, Ez, N, precision))


def server_footprint_mesh(E: int, N: int, precision: int = NEK_PREC_F64) -> int:
    return int(_lib.nek_server_footprint_mesh(int(E), N, precision))


class Server:
    """Served Poisson solves on the device (nek_server_*): submit box-mesh
    requests as they arrive, call step() to admit and advance them, poll()
    finished ones and fetch() their solutions."""

    def __init__(self, hbm_budget: int):
        h = ctypes.c_void_p()
        _check(_lib.nek_server_create(int(hbm_budget), ctypes.byref(h)), "nek_server_create")
        self._h = h
        self._sizes = {}
        self._rhs = {}

    def submit(self, Ex, Ey, Ez, N, b, amp=0.0, a=(0.0, 0.0, 0.0), precision=NEK_PREC_F64,
               rel_tol=1e-10, max_iter=10000) -> int:
        """Queue one solve; returns its id.  b is not copied: the server reads
        it after this returns, so it must not be modified until poll() has
        reported the request (the binding keeps it alive until then)."""
        P = Ex * Ey * Ez * (N + 1) ** 3
        b = _host_np(b, np.float64, "b", P)
        r = Request(Ex, Ey, Ez, N, float(amp), (ctypes.c_double * 3)(*a), b.ctypes.data,
                    int(precision), float(rel_tol), int(max_iter))
        rid = ctypes.c_uint64()
        _check(_lib.nek_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid)), "nek_server_submit")
        self._sizes[rid.value] = P
        self._rhs[rid.value] = b          # read by the server until the result is reported
        return rid.value

    def submit_mesh(self, E, N, D, g, glo, dirichlet, b, precision=NEK_PREC_F64, rel_tol=1e-10,
                    max_iter=10000) -> int:
        """Queue one solve of the caller's own mesh: D, g, glo, dirichlet (may
        be None) and b all numpy arrays (host) or all torch tensors on the
        server's device.  None of them is copied here; the binding keeps them
        alive until poll() has reported the request."""
        torch = _torch()
        P = int(E) * (N + 1) ** 3
        on_dev = isinstance(b, torch.Tensor)
        if on_dev:
            keep = (_dev(D, torch.float64, "D", (N + 1) ** 2), _dev(g, torch.float64, "g", 6 * P),
                    _dev(glo, torch.int64, "glo", P),
                    _dev(dirichlet, torch.uint8, "dirichlet", P) if dirichlet is not None else None,
                    _dev(b, torch.float64, "b", P))
            ptrs = [k.value if k is not None else None for k in keep]
            hold = (D, g, glo, dirichlet, b)
        else:
            arrs = (_host_np(D, np.float64, "D", (N + 1) ** 2), _host_np(g, np.float64, "g", 6 * P),
                    _host_np(glo, np.int64, "glo", P),
                    _host_np(dirichlet, np.uint8, "dirichlet", P) if dirichlet is not None else None,
                    _host_np(b, np.float64, "b", P))
            ptrs = [a.ctypes.data if a is not None else None for a in arrs]
            hold = arrs
        r = Request(0, 0, 0, N, 0.0, (ctypes.c_double * 3)(0.0, 0.0, 0.0), ptrs[4], int(precision),
                    float(rel_tol), int(max_iter), int(E), ptrs[0], ptrs[1], ptrs[2], ptrs[3],
                    NEK_MEM_DEVICE if on_dev else NEK_MEM_HOST)
        rid = ctypes.c_uint64()
        _check(_lib.nek_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid)), "nek_server_submit")
        self._sizes[rid.value] = P
        self._rhs[rid.value] = hold
        return rid.value

    def step(self, iters: int = 1):
        act, que = _ci(), _ci()
        _check(_lib.nek_server_step(self._h, int(iters), ctypes.byref(act), ctypes.byref(que)),
               "nek_server_step")
        return act.value, que.value

    def poll(self, max_results: int = 64):
        buf = (Result * max_results)()
        n = _ci()
        _check(_lib.nek_server_poll(self._h, buf, max_results, ctypes.byref(n)), "nek_server_poll")
        out = [{f: getattr(buf[i], f) for f, _ in Result._fields_} for i in range(n.value)]
        for r in out:
            self._rhs.pop(r["id"], None)
        return out

    def fetch(self, rid: int):
        x = np.empty(self._sizes[rid])
        _check(_lib.nek_server_fetch(self._h, ctypes.c_uint64(rid), x.ctypes.data), "nek_server_fetch")
        return x

    def clock(self) -> float:
        return float(_lib.nek_server_clock(self._h))

    def run_until_done(self, ids, iters: int = 1, max_steps: int = 10 ** 7):
        """Step until every id in ids has finished; returns {id: result}."""
        want, got = set(ids), {}
        for _ in range(max_steps):
            self.step(iters)
            for r in self.poll():
                got[r["id"]] = r
            if want <= set(got):
                return got
        raise RuntimeError("server did not finish")

    def close(self):
        if getattr(self, "_h", None):
            _lib.nek_server_destroy(self._h)
            self._h = None
            self._rhs = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
