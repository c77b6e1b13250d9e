"""Thin ctypes binding of ``libgamblet.so`` (the C ABI of ``include/gamblet.h``).

Argument marshalling only: device memory and streams come from PyTorch, every
step of the hierarchy build and of the solve runs in the library's HIP
kernels.  There is no CPU fallback; a missing library raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgamblet.so")

GBL_OK, GBL_EINVAL, GBL_ENOTSPD, GBL_ENOCONV, GBL_ENOMEM, GBL_EHIP = 0, -1, -2, -3, -4, -5
GBL_FP64, GBL_MIXED, GBL_MIXED_FP64_BUILD = 0, 1, 2
PRECISIONS = {"fp64": GBL_FP64, "f64": GBL_FP64, "double": GBL_FP64, "mixed": GBL_MIXED,
              "mixed-fp64-build": GBL_MIXED_FP64_BUILD}
_STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOTSPD", -3: "ENOCONV", -4: "ENOMEM", -5: "EHIP"}


class GblOpts(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_int), ("precision", ctypes.c_int), ("rtol", ctypes.c_double),
                ("max_outer", ctypes.c_int), ("inner_iters", ctypes.c_int), ("max_rhs", ctypes.c_int),
                ("inner_iters_coarse", ctypes.c_int), ("inner_kind", ctypes.c_int), ("kappa", ctypes.c_double),
                ("kappa_coarse", ctypes.c_double), ("level_q_mass", ctypes.c_int),
                ("rho_coarse", ctypes.c_int), ("window_tol", ctypes.c_double), ("exact", ctypes.c_int),
                ("geometry", ctypes.c_int), ("source", ctypes.c_int), ("w_kind", ctypes.c_int),
                ("dim", ctypes.c_int), ("autotune", ctypes.c_int), ("autotune_path", ctypes.c_char_p),
                ("tensor", ctypes.c_int)]


class GblSolveInfo(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int), ("status", ctypes.c_int),
                ("rel_update", ctypes.c_double), ("rel_residual", ctypes.c_double)]


class GblLevelDesc(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("nk", ctypes.c_int), ("s", ctypes.c_int), ("t", ctypes.c_int),
                ("rw", ctypes.c_int), ("rho", ctypes.c_int), ("elem_bytes", ctypes.c_int),
                ("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("R", ctypes.c_void_p),
                ("nwin", ctypes.c_int), ("wlist", ctypes.c_void_p), ("winv", ctypes.c_void_p),
                ("dense", ctypes.c_int), ("n", ctypes.c_int), ("nsub", ctypes.c_int),
                ("patch_kernel", ctypes.c_int), ("galerkin_kernel", ctypes.c_int)]


class GambletError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1503_03467_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.gbl_version.restype = i
        L.gbl_default_opts.argtypes = [ctypes.POINTER(GblOpts)]
        L.gbl_workspace_bytes.argtypes = [i, ctypes.POINTER(GblOpts), ctypes.POINTER(ctypes.c_size_t)]
        L.gbl_build.argtypes = [ctypes.POINTER(vp), i, vp, ctypes.POINTER(GblOpts), vp, ctypes.c_size_t, vp]
        L.gbl_solve.argtypes = [vp, i, vp, vp, ctypes.POINTER(GblSolveInfo), vp]
        L.gbl_adjoint.argtypes = [vp, i, vp, vp, vp, vp, vp, ctypes.POINTER(GblSolveInfo), vp]
        L.gbl_level_layout.argtypes = [vp, i, ctypes.POINTER(GblLevelDesc)]
        L.gbl_build_flags.argtypes = [vp, ctypes.POINTER(ctypes.c_uint)]
        L.gbl_build_batched.argtypes = [i, ctypes.POINTER(i), ctypes.POINTER(vp), ctypes.POINTER(GblOpts),
                                        ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(vp),
                                        ctypes.POINTER(i), vp]
        L.gbl_solve_batched.argtypes = [i, ctypes.POINTER(vp), ctypes.POINTER(i), ctypes.POINTER(vp),
                                        ctypes.POINTER(vp), ctypes.POINTER(GblSolveInfo), ctypes.POINTER(i), vp]
        L.gbl_destroy.argtypes = [vp]
        L.gbl_last_error.argtypes = [vp]
        L.gbl_last_error.restype = ctypes.c_char_p
        L.gbl_profile_enable.argtypes = [ctypes.c_uint]
        L.gbl_profile_reset.argtypes = []
        L.gbl_profile_read.argtypes = [i, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_long)]
        L.gbl_transform_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.gbl_transform.argtypes = [vp, vp, vp, vp]
        L.gbl_inverse_transform.argtypes = [vp, vp, vp, vp]
        L.gbl_compress.argtypes = [vp, vp, ctypes.c_long, ctypes.POINTER(ctypes.c_double), vp]
        L.gbl_energy_norm.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double), vp]
        L.gbl_compress_noalloc.argtypes = [vp, ctypes.c_long, ctypes.c_long, ctypes.POINTER(ctypes.c_double), vp]
        L.gbl_mass_inverse.argtypes = [i, i, vp, vp]
        L.gbl_level_q_gamblets.argtypes = [i, i, vp, vp, vp]
        L.gbl_level_q_load.argtypes = [i, i, vp, vp, vp, vp]
        L.gbl_level_q_operator.argtypes = [i, i, vp, vp, vp, vp]
        L.gbl_level_q_to_nodal.argtypes = [i, i, vp, vp, vp, vp]
        for name in ("gbl_default_opts", "gbl_workspace_bytes", "gbl_build", "gbl_solve", "gbl_adjoint",
                     "gbl_level_layout", "gbl_build_flags", "gbl_build_batched", "gbl_solve_batched",
                     "gbl_destroy", "gbl_profile_enable", "gbl_profile_reset", "gbl_profile_read",
                     "gbl_transform_size", "gbl_transform", "gbl_inverse_transform", "gbl_compress",
                     "gbl_energy_norm", "gbl_compress_noalloc", "gbl_mass_inverse", "gbl_level_q_gamblets", "gbl_level_q_load",
                     "gbl_level_q_operator", "gbl_level_q_to_nodal"):
            getattr(L, name).restype = i
        _lib = L
    return _lib


def _check(code: int, ctx=None):
    if code != GBL_OK:
        msg = lib().gbl_last_error(ctx).decode()
        raise GambletError(code, msg)


INNER_KINDS = {"chebyshev": 0, "cg": 1, "cheb-cg": 2}
SOURCES = {"cell": 0, "nodal": 1}


def make_opts(rho: int = 3, precision: str = "mixed", rtol: float = 1e-8, max_outer: int = 100,
              inner_iters: int | None = None, max_rhs: int = 1, inner_iters_coarse: int | None = None,
              inner: str | None = None, kappa: float | None = None, kappa_coarse: float | None = None,
              level_q_mass: int = 0, rho_coarse: int = 0, window_tol: float = 0.0, exact: bool = False,
              geometry: int = 0, source: str = "cell", w_kind: int = 0, dim: int = 2, autotune: bool = False,
              autotune_path: str | None = None, tensor: bool = False) -> GblOpts:
    o = GblOpts()
    _check(lib().gbl_default_opts(ctypes.byref(o)))
    if inner is not None:
        o.inner_kind = INNER_KINDS[inner]
    if kappa is not None:
        o.kappa = float(kappa)
    if kappa_coarse is not None:
        o.kappa_coarse = float(kappa_coarse)
    o.rho = int(rho)
    o.precision = PRECISIONS[precision]
    o.rtol = float(rtol)
    o.max_outer = int(max_outer)
    if inner_iters is not None:
        o.inner_iters = int(inner_iters)
    if inner_iters_coarse is not None:
        o.inner_iters_coarse = int(inner_iters_coarse)
    o.max_rhs = int(max_rhs)
    o.level_q_mass = int(level_q_mass)
    o.rho_coarse = int(rho_coarse)
    o.window_tol = float(window_tol)
    o.exact = 1 if exact else 0
    o.geometry = int(geometry)
    o.source = SOURCES[source]
    o.w_kind = int(w_kind)
    o.dim = int(dim)
    o.autotune = 1 if autotune else 0
    o.autotune_path = autotune_path.encode() if autotune_path else None
    o.tensor = 1 if tensor else 0
    return o


def workspace_bytes(q: int, opts: GblOpts) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().gbl_workspace_bytes(int(q), ctypes.byref(opts), ctypes.byref(b)))
    return int(b.value)


def _stream_ptr(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _require(t: torch.Tensor, shape, name):
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


@dataclass
class SolveInfo:
    outer_iters: int
    status: int
    rel_update: float
    rel_residual: float


class Hierarchy:
    """Gamblet hierarchy of one coefficient field, built on the GPU: localized
    (the default) or, with ``exact=True``, the dense FP64 hierarchy of
    Algorithm 1 (``geometry=1``: the mesh of Example 5.1, a of shape
    [2^q + 1][2^q + 1]; ``source="nodal"``: sources given at the interior
    nodes and loaded with the mass matrix).  A three-dimensional ``a``
    ([n][n][n]) selects the problem on the unit cube (exact hierarchy only)."""

    def __init__(self, a: torch.Tensor, rho: int = 3, precision: str = "mixed", rtol: float = 1e-8,
                 max_outer: int = 100, inner_iters: int | None = None, max_rhs: int = 1,
                 inner_iters_coarse: int | None = None, inner: str | None = None, kappa: float | None = None,
                 kappa_coarse: float | None = None, level_q_mass: int = 0, rho_coarse: int = 0,
                 window_tol: float = 0.0, exact: bool = False, geometry: int = 0, source: str = "cell",
                 w_kind: int = 0, autotune: bool = False, autotune_path: str | None = None, tensor: bool = False):
        n = a.shape[0]
        q = (n - geometry).bit_length() - 1
        self.dim = 2 if tensor else a.dim()
        if n - geometry != (1 << q) or q < 2 or self.dim not in (2, 3):
            raise ValueError("a must be [2^q]^d (geometry 0) or [2^q + 1]^d (geometry 1), d = 2 or 3, q >= 2")
        _require(a, (n, n, 3) if tensor else (n,) * self.dim, "a")
        self.q, self.n, self.device = q, n, a.device
        self.exact = bool(exact)
        self.source = source
        self.opts = make_opts(rho, "fp64" if exact else precision, rtol, max_outer, inner_iters, max_rhs,
                              inner_iters_coarse, inner, kappa, kappa_coarse, level_q_mass, rho_coarse, window_tol,
                              exact, geometry, source, w_kind, self.dim, autotune, autotune_path, tensor)
        self.ws = torch.empty(workspace_bytes(q, self.opts), dtype=torch.uint8, device=a.device)
        self.ctx = ctypes.c_void_p()
        with torch.cuda.device(a.device):
            _check(lib().gbl_build(ctypes.byref(self.ctx), q, ctypes.c_void_p(a.data_ptr()),
                                   ctypes.byref(self.opts), ctypes.c_void_p(self.ws.data_ptr()),
                                   ctypes.c_size_t(self.ws.numel()), _stream_ptr(a.device)))
        self.last_info: SolveInfo | None = None

    def close(self):
        if getattr(self, "ctx", None) and self.ctx.value:
            lib().gbl_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, g: torch.Tensor, u_boundary: torch.Tensor | None = None, check: bool = True) -> torch.Tensor:
        """Solve for cell sources ``g`` ([n][n] or [nrhs][n][n]; nodal sources [n-1][n-1] when the
        hierarchy was built with ``source="nodal"``); returns nodal u ([.., n+1, n+1])."""
        d = self.dim
        single = g.dim() == d
        gg = g.unsqueeze(0) if single else g
        nrhs = gg.shape[0]
        gs = self.n - 1 if self.source == "nodal" else self.n
        _require(gg, (nrhs,) + (gs,) * d, "g")
        m = self.n + 1
        if u_boundary is None:
            u = torch.zeros((nrhs,) + (m,) * d, dtype=torch.float64, device=self.device)
        else:
            u = u_boundary.reshape((-1,) + (m,) * d).expand((nrhs,) + (m,) * d).clone().contiguous()
        info = GblSolveInfo()
        with torch.cuda.device(self.device):
            code = lib().gbl_solve(self.ctx, nrhs, ctypes.c_void_p(gg.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                   ctypes.byref(info), _stream_ptr(self.device))
        self.last_info = SolveInfo(info.outer_iters, info.status, info.rel_update, info.rel_residual)
        if check or code not in (GBL_OK, GBL_ENOCONV):
            _check(code, self.ctx)
        return u[0] if single else u

    def adjoint(self, u: torch.Tensor, dJdu: torch.Tensor, check: bool = True):
        """Return (dJ/dlog a, dJ/dg, lambda) for the solution u and nodal gradient dJ/du."""
        single = u.dim() == 2
        uu = u.unsqueeze(0) if single else u
        dd = dJdu.unsqueeze(0) if single else dJdu
        nrhs = uu.shape[0]
        m = self.n + 1
        _require(uu, (nrhs, m, m), "u")
        _require(dd, (nrhs, m, m), "dJdu")
        dloga = torch.empty((nrhs, self.n, self.n), dtype=torch.float64, device=self.device)
        dg = torch.empty_like(dloga)
        lam = torch.empty((nrhs, m, m), dtype=torch.float64, device=self.device)
        info = GblSolveInfo()
        with torch.cuda.device(self.device):
            code = lib().gbl_adjoint(self.ctx, nrhs, ctypes.c_void_p(uu.data_ptr()), ctypes.c_void_p(dd.data_ptr()),
                                     ctypes.c_void_p(dloga.data_ptr()), ctypes.c_void_p(dg.data_ptr()),
                                     ctypes.c_void_p(lam.data_ptr()), ctypes.byref(info), _stream_ptr(self.device))
        self.last_info = SolveInfo(info.outer_iters, info.status, info.rel_update, info.rel_residual)
        if check or code not in (GBL_OK, GBL_ENOCONV):
            _check(code, self.ctx)
        if single:
            return dloga[0], dg[0], lam[0]
        return dloga, dg, lam

    @property
    def build_flags(self) -> int:
        """GBL_FLAG_* bits of the build (1: FP32 pivots raised to the floor)."""
        f = ctypes.c_uint(0)
        _check(lib().gbl_build_flags(self.ctx, ctypes.byref(f)), self.ctx)
        return int(f.value)

    def transform_size(self) -> int:
        """Number of gamblet coefficients, 4^q."""
        c = ctypes.c_size_t(0)
        _check(lib().gbl_transform_size(self.ctx, ctypes.byref(c)), self.ctx)
        return int(c.value)

    def transform(self, u: torch.Tensor) -> torch.Tensor:
        """Normalized gamblet coefficients of a nodal u ([n+1]^d FP64; layout in ``gamblet.h``)."""
        m = self.n + 1
        _require(u, (m,) * self.dim, "u")
        c = torch.empty(self.transform_size(), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().gbl_transform(self.ctx, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(c.data_ptr()),
                                       _stream_ptr(self.device)), self.ctx)
        return c

    def inverse_transform(self, c: torch.Tensor) -> torch.Tensor:
        """Nodal u ([n+1]^d, zero boundary) from normalized gamblet coefficients."""
        _require(c, (self.transform_size(),), "coefficients")
        m = self.n + 1
        u = torch.empty((m,) * self.dim, dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().gbl_inverse_transform(self.ctx, ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                               _stream_ptr(self.device)), self.ctx)
        return u

    def compress(self, c: torch.Tensor, keep: int) -> float:
        """Keep the ``keep`` largest |c| in place (others zero); returns the smallest kept magnitude."""
        _require(c, (self.transform_size(),), "coefficients")
        thr = ctypes.c_double(0.0)
        with torch.cuda.device(self.device):
            _check(lib().gbl_compress(self.ctx, ctypes.c_void_p(c.data_ptr()), int(keep), ctypes.byref(thr),
                                      _stream_ptr(self.device)), self.ctx)
        return float(thr.value)

    def energy_norm(self, u: torch.Tensor) -> float:
        """sqrt(u^T A u) of a nodal u with the FP64 fine stiffness matrix."""
        m = self.n + 1
        _require(u, (m,) * self.dim, "u")
        out = ctypes.c_double(0.0)
        with torch.cuda.device(self.device):
            _check(lib().gbl_energy_norm(self.ctx, ctypes.c_void_p(u.data_ptr()), ctypes.byref(out),
                                         _stream_ptr(self.device)), self.ctx)
        return float(out.value)

    def level(self, k: int) -> dict:
        """A^(k) [S,S,nk,nk] and R^(k-1,k) [rw,rw,nc,nc] as device views, B^(k) as a
        [T,T,3,3,np,np] copy (the library stores it block-interleaved, see ``gamblet.h``).
        For the exact hierarchy: dense views A [n][n], B [nsub][nsub], R [n_{k-1}][n]."""
        d = GblLevelDesc()
        _check(lib().gbl_level_layout(self.ctx, int(k), ctypes.byref(d)), self.ctx)
        dt = torch.float64 if d.elem_bytes == 8 else torch.float32
        base = self.ws.data_ptr()

        def view(ptr, count):
            off = ptr - base
            return self.ws[off: off + count * d.elem_bytes].view(dt)

        if d.dense:
            out = {"k": d.k, "n": d.n, "nsub": d.nsub, "A": view(d.A, d.n * d.n).view(d.n, d.n)}
            if k >= 2:
                npar = d.nsub // ((1 << self.dim) - 1)
                out["B"] = view(d.B, d.nsub * d.nsub).view(d.nsub, d.nsub)
                out["R"] = view(d.R, npar * d.n).view(npar, d.n)
            return out

        nk = d.nk
        S = 2 * d.s + 1
        out = {"k": d.k, "nk": nk, "s": d.s, "t": d.t, "rw": d.rw, "rho": d.rho,
               "patch_kernel": d.patch_kernel, "galerkin_kernel": d.galerkin_kernel,
               "A": view(d.A, S * S * nk * nk).view(S, S, nk, nk)}
        if k >= 2:
            np_ = nk // 2
            T = 2 * d.t + 1
            ng = (np_ * np_ + 63) // 64
            Bg = view(d.B, ng * T * T * 9 * 64).view(ng, T, T, 3, 3, 64)
            out["B"] = Bg.permute(1, 2, 3, 4, 0, 5).reshape(T, T, 3, 3, ng * 64)[..., :np_ * np_].reshape(
                T, T, 3, 3, np_, np_)
            out["R"] = view(d.R, d.rw * d.rw * np_ * np_).view(d.rw, d.rw, np_, np_)
            out["nwin"] = d.nwin
            if d.nwin > 0:
                out["wlist"] = self.ws[d.wlist - base: d.wlist - base + 4 * d.nwin].view(torch.int32)
                wdt = torch.float64 if self.opts.precision == GBL_FP64 else torch.float32
                wb = 8 if wdt == torch.float64 else 4
                out["winv"] = self.ws[d.winv - base: d.winv - base + wb * d.nwin * 27 * 27].view(wdt).view(
                    d.nwin, 27, 27)
        return out


PROF_KERNELS = ["assemble", "subband_operator", "patch_solve", "galerkin", "restrict", "cg_init", "cg_spmv",
                "cg_update", "prolong", "fine_apply", "gradient", "fine_cg", "patch_band"]


class LevelQ:
    """Level-q gamblets from the localized mass inverse (Algorithm 2;
    Definition 5.2) on the 2^q x 2^q cell grid, patch radius ``rho_q`` node
    steps.  Holds the table of one-dimensional factors on the device; every
    method is one C-ABI call on the current stream.  Interior vectors are
    float64 ``[(2^q - 1)^2]`` tensors."""

    def __init__(self, q: int, rho_q: int = 3, device=None):
        self.q, self.rho_q = int(q), int(rho_q)
        self.n = 1 << self.q
        self.m = self.n - 1
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        w = 2 * self.rho_q + 1
        self.table = torch.empty((max(self.m, 1), w), dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            _check(lib().gbl_mass_inverse(self.q, self.rho_q, ctypes.c_void_p(self.table.data_ptr()),
                                          _stream_ptr(self.device)))

    def _call(self, name, *ptrs):
        with torch.cuda.device(self.device):
            _check(getattr(lib(), name)(self.q, self.rho_q, *[ctypes.c_void_p(p) for p in ptrs],
                                        _stream_ptr(self.device)))

    def gamblets(self) -> torch.Tensor:
        """psi^(q)_i in the nodal basis, ``[m^2][(2 rho_q + 1)^2]``."""
        w = 2 * self.rho_q + 1
        out = torch.empty((self.m * self.m, w * w), dtype=torch.float64, device=self.device)
        self._call("gbl_level_q_gamblets", self.table.data_ptr(), out.data_ptr())
        return out

    def load(self, b: torch.Tensor) -> torch.Tensor:
        """g^(q) = Minv^T b for the nodal load b (``[m^2]``)."""
        _require(b, (self.m * self.m,), "b")
        out = torch.empty_like(b)
        self._call("gbl_level_q_load", self.table.data_ptr(), b.data_ptr(), out.data_ptr())
        return out

    def operator(self, a: torch.Tensor) -> torch.Tensor:
        """A^(q) = Minv^T A Minv as stencil rows ``[m^2][(2S + 1)^2]``, S = 2 rho_q + 1."""
        _require(a, (self.n, self.n), "a")
        W = 4 * self.rho_q + 3
        out = torch.empty((self.m * self.m, W * W), dtype=torch.float64, device=self.device)
        self._call("gbl_level_q_operator", a.data_ptr(), self.table.data_ptr(), out.data_ptr())
        return out

    def to_nodal(self, U: torch.Tensor) -> torch.Tensor:
        """Nodal values Minv U of sum_i U_i psi^(q)_i."""
        _require(U, (self.m * self.m,), "U")
        out = torch.empty_like(U)
        self._call("gbl_level_q_to_nodal", self.table.data_ptr(), U.data_ptr(), out.data_ptr())
        return out


def compress_noalloc(c: torch.Tensor, keep: int) -> float:
    """Keep the ``keep`` largest |c| of an FP64 device vector in place (others zero) through
    ``gbl_compress_noalloc``, which allocates no device memory; returns the smallest kept magnitude."""
    if not (isinstance(c, torch.Tensor) and c.is_cuda and c.dtype == torch.float64 and c.dim() == 1
            and c.is_contiguous()):
        raise ValueError("c must be a contiguous 1-D float64 CUDA tensor")
    thr = ctypes.c_double(0.0)
    with torch.cuda.device(c.device):
        _check(lib().gbl_compress_noalloc(ctypes.c_void_p(c.data_ptr()), int(c.numel()), int(keep),
                                          ctypes.byref(thr), _stream_ptr(c.device)))
    return float(thr.value)


def profile_enable(kernels="all"):
    """Time launches of the named kernel classes with HIP events (``"all"``, a list, or None to stop)."""
    if kernels is None:
        mask = 0
    elif kernels == "all":
        mask = (1 << len(PROF_KERNELS)) - 1
    else:
        mask = 0
        for k in kernels:
            mask |= 1 << PROF_KERNELS.index(k)
    _check(lib().gbl_profile_enable(mask))


def profile_reset():
    _check(lib().gbl_profile_reset())


def profile_read() -> dict:
    """{kernel: (total_ms, launches)} accumulated since the last reset."""
    out = {}
    for i, name in enumerate(PROF_KERNELS):
        ms, n = ctypes.c_double(), ctypes.c_long()
        _check(lib().gbl_profile_read(i, ctypes.byref(ms), ctypes.byref(n)))
        out[name] = (ms.value, n.value)
    return out


class GambletSolve(torch.autograd.Function):
    """u = solve(exp(log_a), g) with a hand-written adjoint.

    Forward builds the hierarchy for ``a = exp(log_a)`` and solves; backward
    reuses the same hierarchy for the symmetric adjoint system and returns
    dJ/dlog a and dJ/dg per cell.
    """

    @staticmethod
    def forward(ctx, log_a, g, rho=3, precision="mixed", rtol=1e-8):
        a = torch.exp(log_a.detach()).contiguous()
        H = Hierarchy(a, rho=rho, precision=precision, rtol=rtol, max_rhs=g.shape[0] if g.dim() == 3 else 1)
        u = H.solve(g.detach().contiguous())
        ctx.H = H
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        (u,) = ctx.saved_tensors
        # The hierarchy stays open: a graph kept with retain_graph may run
        # backward again; it is released with the autograd context.
        dloga, dg, _ = ctx.H.adjoint(u, grad_u.contiguous())
        return dloga, dg, None, None, None


def _adopt(ctx_value: int, q: int, ws: torch.Tensor, opts: GblOpts) -> Hierarchy:
    """Wrap a context built by gbl_build_batched in a Hierarchy (which then owns it)."""
    h = Hierarchy.__new__(Hierarchy)
    h.q, h.n, h.device = q, 1 << q, ws.device
    h.opts, h.ws = opts, ws
    h.exact, h.source, h.dim = False, "cell", 2
    h.ctx = ctypes.c_void_p(ctx_value)
    h.last_info = None
    return h


def build_batched(coeffs: list, rho: int = 3, precision: str = "mixed", rtol: float = 1e-8,
                  max_outer: int = 100, inner_iters: int | None = None, max_rhs: int = 1,
                  inner_iters_coarse: int | None = None, inner: str | None = None, kappa: float | None = None,
                  kappa_coarse: float | None = None, autotune: bool = False,
                  autotune_path: str | None = None) -> list:
    """Build the hierarchies of independent problems of uneven depth concurrently
    (``gbl_build_batched``); ``coeffs`` holds [2^q][2^q] float64 CUDA tensors."""
    P = len(coeffs)
    if P == 0:
        return []
    opts = make_opts(rho, precision, rtol, max_outer, inner_iters, max_rhs, inner_iters_coarse, inner, kappa,
                     kappa_coarse, autotune=autotune, autotune_path=autotune_path)
    qs, wss = [], []
    for a in coeffs:
        n = a.shape[0]
        q = n.bit_length() - 1
        if n != (1 << q) or q < 2:
            raise ValueError("every coefficient must be [2^q][2^q] with q >= 2")
        _require(a, (n, n), "a")
        qs.append(q)
        wss.append(torch.empty(workspace_bytes(q, opts), dtype=torch.uint8, device=a.device))
    vp = ctypes.c_void_p
    q_arr = (ctypes.c_int * P)(*qs)
    a_arr = (vp * P)(*[a.data_ptr() for a in coeffs])
    ws_arr = (vp * P)(*[w.data_ptr() for w in wss])
    wb_arr = (ctypes.c_size_t * P)(*[w.numel() for w in wss])
    ctx_arr = (vp * P)()
    st_arr = (ctypes.c_int * P)()
    dev = coeffs[0].device
    with torch.cuda.device(dev):
        code = lib().gbl_build_batched(P, q_arr, a_arr, ctypes.byref(opts), ws_arr, wb_arr, ctx_arr, st_arr,
                                       _stream_ptr(dev))
    hs = [_adopt(ctx_arr[i], qs[i], wss[i], opts) if ctx_arr[i] else None for i in range(P)]
    if code != GBL_OK:
        for h in hs:
            if h is not None:
                h.close()
        _check(code)
    return hs


def solve_batched(hiers: list, sources: list, check: bool = True) -> list:
    """Solve problem i for the cell sources ``sources[i]`` ([nrhs][n][n]) with
    ``hiers[i]``, all problems concurrently (``gbl_solve_batched``); returns the
    nodal solutions and sets each hierarchy's ``last_info``."""
    P = len(hiers)
    if P == 0:
        return []
    us, nr = [], []
    for h, g in zip(hiers, sources):
        gg = g.unsqueeze(0) if g.dim() == 2 else g
        _require(gg, (gg.shape[0], h.n, h.n), "g")
        nr.append(gg.shape[0])
        us.append(torch.zeros((gg.shape[0], h.n + 1, h.n + 1), dtype=torch.float64, device=h.device))
    srcs = [g.unsqueeze(0) if g.dim() == 2 else g for g in sources]
    vp = ctypes.c_void_p
    ctx_arr = (vp * P)(*[h.ctx.value for h in hiers])
    nr_arr = (ctypes.c_int * P)(*nr)
    g_arr = (vp * P)(*[g.data_ptr() for g in srcs])
    u_arr = (vp * P)(*[u.data_ptr() for u in us])
    info_arr = (GblSolveInfo * P)()
    st_arr = (ctypes.c_int * P)()
    dev = hiers[0].device
    with torch.cuda.device(dev):
        code = lib().gbl_solve_batched(P, ctx_arr, nr_arr, g_arr, u_arr, info_arr, st_arr, _stream_ptr(dev))
    for h, inf in zip(hiers, info_arr):
        h.last_info = SolveInfo(inf.outer_iters, inf.status, inf.rel_update, inf.rel_residual)
    if check or code not in (GBL_OK, GBL_ENOCONV):
        _check(code)
    return us
