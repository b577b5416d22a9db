"""Thin ctypes binding of libpomm (the C ABI in include/pomm.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Orbital blocks are torch tensors on the GPU of shape (ncols, n)
(row c = orbital column c, so the memory is the library's column-major n x ncols
layout), dtype complex128 (or complex64 for the FP32 H apply).

Importing this module loads libpomm.so; it raises ImportError when the library
has not been built (python -m paper_1603_09724_amd.build).
"""

from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpomm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libpomm.so is not built; run `python -m paper_1603_09724_amd.build` (hipcc, gfx950)")
_lib = ctypes.CDLL(LIB_PATH)

# ------------------------------------------------------------------ constants (pomm.h)
OK, EINVAL, ENOTNEGDEF, ESPECTRUM, ENOMEM, EHIP, ENOCONV, EBREAKDOWN, EUNSUPPORTED = range(9)
PREC_FP64, PREC_FP32 = 0, 1
FP64, MIXED = 0, 1
INNER_SPP, INNER_PP = 0, 1
POLES_ELLIPTIC, POLES_CIRCLE = 0, 1
SIDE_AUTO, SIDE_RIGHT, SIDE_LEFT = 0, 1, 2
PRODUCTS_SPLIT16, PRODUCTS_FP32, PRODUCTS_F16 = 0, 1, 2
OUTER_FERMI, OUTER_LAPLACE, OUTER_TPA = 0, 1, 2
STOP_GRAD, STOP_ENERGY, STOP_MAXIT = 1, 2, 3
STOP_NAMES = {STOP_GRAD: "grad", STOP_ENERGY: "energy", STOP_MAXIT: "maxit"}

EXPORTED = ["ommDefaultOptions", "ommSetup", "ommApplyH", "ommPrecondition", "ommPrecompute", "ommSolveBatched",
            "ommEstimateSpectrum", "ommApplyInner", "ommSolve",
            "ommGetPoles",
            "ommGetStencil", "ommGetInfo", "ommGetSpectrum", "ommGetCounters", "ommSetProfiling", "ommSetProfilingClasses",
            "ommGetProfile",
            "ommProfileClassName", "ommDestroy", "ommStatusString", "ommLastError"]
PROF_CLASSES = 7


class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("m", ctypes.c_int * 3)]


class Spectrum(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double), ("homo", ctypes.c_double), ("lumo", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("inner", ctypes.c_int), ("poles", ctypes.c_int),
                ("npoles", ctypes.c_int), ("gmres_rtol", ctypes.c_double), ("gmres_restart", ctypes.c_int),
                ("gmres_cycles", ctypes.c_int), ("filter_rtol", ctypes.c_double), ("tol", ctypes.c_double),
                ("maxit", ctypes.c_int), ("stall", ctypes.c_int), ("filter", ctypes.c_int),
                ("pole_tol", ctypes.c_double), ("gmres_side", ctypes.c_int), ("spp_products", ctypes.c_int),
                ("outer", ctypes.c_int), ("tau", ctypes.c_double), ("gmres_verify", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("status", ctypes.c_int), ("stop_rule", ctypes.c_int),
                ("energy", ctypes.c_double), ("rel_grad", ctypes.c_double), ("gmres_steps", ctypes.c_longlong),
                ("precond_calls", ctypes.c_longlong), ("sigma", ctypes.c_double)]


class EstimateInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("applies", ctypes.c_int), ("converged", ctypes.c_int),
                ("res_homo", ctypes.c_double), ("res_lumo", ctypes.c_double)]


_vp = ctypes.c_void_p
_lib.ommDefaultOptions.argtypes = [ctypes.POINTER(Options)]
_lib.ommDefaultOptions.restype = None
_lib.ommSetup.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_double,
                          ctypes.POINTER(Spectrum), ctypes.POINTER(Options), _vp, ctypes.POINTER(_vp)]
_lib.ommSetup.restype = ctypes.c_int
_lib.ommApplyH.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int]
_lib.ommApplyH.restype = ctypes.c_int
_lib.ommPrecondition.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_double]
_lib.ommPrecondition.restype = ctypes.c_int
_lib.ommPrecompute.argtypes = [_vp, _vp, ctypes.c_int, ctypes.c_double]
_lib.ommPrecompute.restype = ctypes.c_int
_lib.ommEstimateSpectrum.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(ctypes.c_double), ctypes.c_int, _vp,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, _vp,
                                     ctypes.POINTER(Spectrum), ctypes.POINTER(EstimateInfo)]
_lib.ommEstimateSpectrum.restype = ctypes.c_int
_lib.ommApplyInner.argtypes = [_vp, ctypes.c_int, _vp, _vp, ctypes.c_int]
_lib.ommApplyInner.restype = ctypes.c_int
_lib.ommSolve.argtypes = [_vp, _vp, ctypes.POINTER(Info)]
_lib.ommSolveBatched.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(_vp), ctypes.POINTER(Info)]
_lib.ommSolveBatched.restype = ctypes.c_int
_lib.ommSolve.restype = ctypes.c_int
_lib.ommGetPoles.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
_lib.ommGetPoles.restype = ctypes.c_int
_lib.ommGetStencil.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
_lib.ommGetStencil.restype = ctypes.c_int
_lib.ommGetInfo.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int),
                            ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
_lib.ommGetInfo.restype = ctypes.c_int
_lib.ommGetSpectrum.argtypes = [_vp, ctypes.POINTER(Spectrum)]
_lib.ommGetSpectrum.restype = ctypes.c_int
_lib.ommGetCounters.argtypes = [_vp, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)]
_lib.ommGetCounters.restype = ctypes.c_int
_lib.ommSetProfiling.argtypes = [_vp, ctypes.c_int]
_lib.ommSetProfiling.restype = ctypes.c_int
_lib.ommSetProfilingClasses.argtypes = [_vp, ctypes.c_uint]
_lib.ommSetProfilingClasses.restype = ctypes.c_int
_lib.ommGetProfile.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong)]
_lib.ommGetProfile.restype = ctypes.c_int
_lib.ommProfileClassName.argtypes = [ctypes.c_int]
_lib.ommProfileClassName.restype = ctypes.c_char_p
_lib.ommDestroy.argtypes = [_vp]
_lib.ommDestroy.restype = ctypes.c_int
_lib.ommStatusString.argtypes = [ctypes.c_int]
_lib.ommStatusString.restype = ctypes.c_char_p
_lib.ommLastError.argtypes = [_vp]
_lib.ommLastError.restype = ctypes.c_char_p


class PommError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_lib.ommStatusString(code).decode(), code, msg))
        self.code = code


def library():
    """The loaded ctypes library (for symbol checks)."""
    return _lib


def default_options(**overrides) -> Options:
    o = Options()
    _lib.ommDefaultOptions(ctypes.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _ptr(t):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous GPU tensor")
    return ctypes.c_void_p(t.data_ptr())


class Handle:
    """One ommSetup handle (RAII: destroyed with the object or by close())."""

    def __init__(self, dim: int, m: int, V: np.ndarray, N: int, spectrum, shift: float | None = None,
                 options: Options | None = None, stream=None):
        g = Grid()
        g.dim = dim
        for i in range(3):
            g.m[i] = m if i < dim else 0
        V = np.ascontiguousarray(V, dtype=np.float64)
        spec = None if spectrum is None else ctypes.byref(Spectrum(*[float(x) for x in spectrum]))
        opts = options if options is not None else default_options()
        h = _vp()
        self._stream = _stream_ptr(stream)
        rc = _lib.ommSetup(ctypes.byref(g), V.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(N),
                           float("nan") if shift is None else float(shift), spec,
                           ctypes.byref(opts), self._stream, ctypes.byref(h))
        if rc != OK:
            raise PommError(rc, _lib.ommLastError(None).decode())
        self._h = h
        self.dim, self.m, self.N = dim, m, N
        self.n = m ** dim
        self.options = opts

    def spectrum(self):
        """The window (lo, homo, lumo) the pole set was built from (given, or estimated when the
        handle was created with spectrum=None)."""
        sp = Spectrum()
        self._check(_lib.ommGetSpectrum(self._h, ctypes.byref(sp)))
        return sp.lo, sp.homo, sp.lumo

    def close(self):
        if getattr(self, "_h", None):
            _lib.ommDestroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, rc):
        if rc != OK:
            raise PommError(rc, _lib.ommLastError(self._h).decode())

    # -------------------------------------------------------------- calls
    def apply_h(self, X, HX, ncols: int | None = None):
        import torch
        prec = PREC_FP64 if X.dtype == torch.complex128 else PREC_FP32
        ncols = X.shape[0] if ncols is None else ncols
        self._check(_lib.ommApplyH(self._h, _ptr(X), _ptr(HX), int(ncols), prec))

    def precondition(self, G, PG, ncols: int | None = None, rtol: float = 0.0):
        ncols = G.shape[0] if ncols is None else ncols
        self._check(_lib.ommPrecondition(self._h, _ptr(G), _ptr(PG), int(ncols), float(rtol)))

    def precompute(self, B, rtol: float = 0.0):
        """Algorithm 2: U U^H from the real Gaussian block B (torch float64 on the device, shape
        (ncols, n), N <= ncols <= 2N); afterwards precondition/solve apply U U^H.  B = None
        returns to the pole expansion."""
        if B is None:
            self._check(_lib.ommPrecompute(self._h, None, 0, 0.0))
        else:
            self._check(_lib.ommPrecompute(self._h, _ptr(B), int(B.shape[0]), float(rtol)))

    def apply_inner(self, pole: int, B, Y, ncols: int | None = None):
        """Y = M_pole^{-1} B (inner preconditioner of one pole); complex128 blocks."""
        ncols = B.shape[0] if ncols is None else ncols
        self._check(_lib.ommApplyInner(self._h, int(pole), _ptr(B), _ptr(Y), int(ncols)))

    def solve(self, X) -> dict:
        info = Info()
        rc = _lib.ommSolve(self._h, _ptr(X), ctypes.byref(info))
        if rc not in (OK, ENOCONV):
            self._check(rc)
        return {"iters": info.iters, "status": info.status, "stop_rule": STOP_NAMES.get(info.stop_rule, "?"),
                "energy": info.energy, "rel_grad": info.rel_grad, "gmres_steps": info.gmres_steps,
                "precond_calls": info.precond_calls, "sigma": info.sigma}

    def poles(self):
        p = self.npoles
        z = (ctypes.c_double * (2 * p))()
        w = (ctypes.c_double * (2 * p))()
        self._check(_lib.ommGetPoles(self._h, z, w))
        z = np.array(z[:]).reshape(p, 2)
        w = np.array(w[:]).reshape(p, 2)
        return z[:, 0] + 1j * z[:, 1], w[:, 0] + 1j * w[:, 1]

    def stencil(self, pole: int):
        """(q, t) of the sparsifying preconditioner of one pole, 9 complex values each."""
        q = (ctypes.c_double * 18)()
        t = (ctypes.c_double * 18)()
        self._check(_lib.ommGetStencil(self._h, int(pole), q, t))
        q = np.array(q[:]).reshape(9, 2)
        t = np.array(t[:]).reshape(9, 2)
        return q[:, 0] + 1j * q[:, 1], t[:, 0] + 1j * t[:, 1]

    def set_profiling(self, on: bool = True, classes=None):
        """Record kernel-class timings: every class (on), or only the named classes."""
        if classes is None:
            self._check(_lib.ommSetProfiling(self._h, int(bool(on))))
            return
        names = [_lib.ommProfileClassName(i).decode() for i in range(PROF_CLASSES)]
        mask = 0
        for c in classes:
            mask |= 1 << names.index(c)
        self._check(_lib.ommSetProfilingClasses(self._h, mask if on else 0))

    def profile(self) -> dict:
        """Per kernel class: ms, algorithmic bytes and flops, launches (events on the handle's stream)."""
        k = PROF_CLASSES
        ms = (ctypes.c_double * k)()
        by = (ctypes.c_double * k)()
        fl = (ctypes.c_double * k)()
        la = (ctypes.c_longlong * k)()
        self._check(_lib.ommGetProfile(self._h, ms, by, fl, la))
        return {_lib.ommProfileClassName(i).decode(): {"ms": ms[i], "bytes": by[i], "flops": fl[i],
                                                        "launches": la[i]} for i in range(k)}

    @property
    def npoles(self) -> int:
        p = ctypes.c_int()
        self._check(_lib.ommGetInfo(self._h, None, None, None, ctypes.byref(p)))
        return p.value

    @property
    def sigma(self) -> float:
        s = ctypes.c_double()
        self._check(_lib.ommGetInfo(self._h, ctypes.byref(s), None, None, None))
        return s.value

    def counters(self):
        a, b = ctypes.c_longlong(), ctypes.c_longlong()
        self._check(_lib.ommGetCounters(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value


def solve_batched(handles, Xs) -> list:
    """ommSolveBatched: independent solves of several instances at once (each handle ideally
    on its own stream).  Returns one info dict per instance; raises on the first failure."""
    count = len(handles)
    if count != len(Xs):
        raise ValueError("one orbital block per handle")
    hs = (_vp * count)(*[h._h for h in handles])
    xs = (_vp * count)(*[_ptr(X).value for X in Xs])
    infos = (Info * count)()
    rc = _lib.ommSolveBatched(hs, count, xs, infos)
    out = [{"iters": i.iters, "status": i.status, "stop_rule": STOP_NAMES.get(i.stop_rule, "?"),
            "energy": i.energy, "rel_grad": i.rel_grad, "gmres_steps": i.gmres_steps,
            "precond_calls": i.precond_calls, "sigma": i.sigma} for i in infos]
    if rc not in (OK, ENOCONV):
        bad = next((k for k, i in enumerate(infos) if i.status not in (OK, ENOCONV)), 0)
        handles[bad]._check(rc)
    return out


def estimate_spectrum(dim: int, m: int, V: np.ndarray, N: int, B, degree: int = 0, tol: float = 0.0,
                      maxit: int = 0, stream=None) -> dict:
    """ommEstimateSpectrum: the window (lo, homo, lumo) for ommSetup from a Chebyshev-filtered
    subspace iteration started from B (a real float64 GPU tensor of shape (ncols, n), one row
    per column).  Raises unless the Ritz residuals met tol."""
    g = Grid()
    g.dim = dim
    for i in range(3):
        g.m[i] = m if i < dim else 0
    V = np.ascontiguousarray(V, dtype=np.float64)
    spec = Spectrum()
    info = EstimateInfo()
    rc = _lib.ommEstimateSpectrum(ctypes.byref(g), V.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(N),
                                  _ptr(B), int(B.shape[0]), int(degree), float(tol), int(maxit),
                                  _stream_ptr(stream), ctypes.byref(spec), ctypes.byref(info))
    if rc != OK:
        raise PommError(rc, _lib.ommLastError(None).decode())
    return {"lo": spec.lo, "homo": spec.homo, "lumo": spec.lumo, "iters": info.iters, "applies": info.applies,
            "converged": bool(info.converged), "res_homo": info.res_homo, "res_lumo": info.res_lumo}


def spectrum_window(lo: float, homo: float, lumo: float):
    if not (lo < homo < lumo) or not all(math.isfinite(x) for x in (lo, homo, lumo)):
        raise ValueError("need lo < homo < lumo")
    return (lo, homo, lumo)
