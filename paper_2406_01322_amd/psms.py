"""Thin ctypes binding of the psms C ABI (include/psms.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
``libpsms.so``.  PyTorch provides device memory (the workspace and the I/O
tensors) and the stream.  If the library is missing the calls raise; there is
no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpsms.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "psms.h")

PSMS_OK = 0
ERRORS = {-1: "PSMS_E_INVAL", -2: "PSMS_E_WORKSPACE", -3: "PSMS_E_DEVICE", -4: "PSMS_E_NOTSUP",
          -5: "PSMS_E_NONFINITE", -6: "PSMS_E_STATE", -7: "PSMS_E_LAUNCH"}
BOX, CHANNEL = 0, 1
FP64, MIXED = 0, 1
DEALIAS, DERIV_X, DERIV_Y, DERIV_Z = 1, 2, 4, 8


class PsmsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "error"), code, msg))
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("geometry", ctypes.c_int32), ("n", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("re", ctypes.c_double), ("we", ctypes.c_double),
                ("ch", ctypes.c_double), ("pe", ctypes.c_double), ("dt", ctypes.c_double),
                ("s", ctypes.c_double)]


class Diag(ctypes.Structure):
    _fields_ = [("mean_phi", ctypes.c_double), ("ke", ctypes.c_double), ("grad2", ctypes.c_double),
                ("max_div", ctypes.c_double), ("nonfinite", ctypes.c_int32), ("nstep", ctypes.c_int32)]


_lib = None

_SIGS = {
    "psms_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)]),
    "psms_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(Params), ctypes.c_void_p,
                                   ctypes.c_size_t, ctypes.c_void_p]),
    "psms_init_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "psms_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_int32]),
    "psms_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "psms_get_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "psms_transform": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_uint32]),
    "psms_solve_helmholtz": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                            ctypes.c_void_p, ctypes.c_void_p]),
    "psms_diagnostics": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Diag)]),
    "psms_index_maps": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "psms_band_modes": (ctypes.c_int64, [ctypes.c_void_p]),
    "psms_stage_times": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "psms_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "psms_last_error": (ctypes.c_char_p, []),
    "psms_version": (ctypes.c_char_p, []),
}


def lib():
    """Load libpsms.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpsms.so is not built; run `python -m paper_2406_01322_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def header_functions(path: str = HEADER):
    """Names of the functions declared in include/psms.h."""
    src = open(path).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z0-9_]+\s*\*?\s*(psms_[a-z0-9_]+)\s*\(", src, re.M)))


def _check(code: int):
    if code != PSMS_OK:
        raise PsmsError(code, lib().psms_last_error().decode())


def make_params(n, re, we, ch, pe, dt, s=0.0, precision="fp64", geometry=BOX) -> Params:
    prec = {"fp64": FP64, "mixed": MIXED}[precision] if isinstance(precision, str) else int(precision)
    return Params(geometry, int(n), prec, 0, float(re), float(we), float(ch), float(pe), float(dt), float(s or 0.0))


def workspace_bytes(params: Params) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().psms_workspace_bytes(ctypes.byref(params), ctypes.byref(b)))
    return int(b.value)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """One periodic-box NS+CH context on the current GPU and torch stream."""

    def __init__(self, n, re, we, ch, pe, dt, s=0.0, precision="fp64", device="cuda", stream=None):
        import torch
        self.torch = torch
        self.params = make_params(n, re, we, ch, pe, dt, s, precision)
        self.n = int(n)
        self.precision = precision
        self.device = torch.device(device)
        nbytes = workspace_bytes(self.params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        _check(lib().psms_create(ctypes.byref(ctx), ctypes.byref(self.params), _ptr(self.workspace), nbytes,
                                 ctypes.c_void_p(self.stream.cuda_stream)))
        self.ctx = ctx

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            lib().psms_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _spec_shape(self, nf):
        n = self.n
        return (nf, n, n, n // 2 + 1) if nf > 1 else (n, n, n // 2 + 1)

    def _need(self, t, dtype, shape):
        t = self.torch.as_tensor(t)
        if t.dtype != dtype or tuple(t.shape) != tuple(shape):
            raise ValueError("expected %s %s, got %s %s" % (dtype, shape, t.dtype, tuple(t.shape)))
        if t.device != self.device and not (t.device.type == self.device.type):
            raise ValueError("tensor on %s, context on %s" % (t.device, self.device))
        return t.contiguous()

    # -- calls of the C ABI -----------------------------------------------
    def init_state(self, u, phi):
        n = self.n
        u = self._need(u, self.torch.float64, (3, n, n, n))
        phi = self._need(phi, self.torch.float64, (n, n, n))
        _check(lib().psms_init_state(self.ctx, _ptr(u), _ptr(phi)))

    def set_state(self, uhat, phihat, hist=None, nstep=0):
        c128 = self.torch.complex128
        uhat = self._need(uhat, c128, self._spec_shape(3))
        phihat = self._need(phihat, c128, self._spec_shape(1))
        hp = None
        if hist is not None:
            hist = self._need(hist, c128, self._spec_shape(4))
            hp = _ptr(hist)
        self._keep = (uhat, phihat, hist)
        _check(lib().psms_set_state(self.ctx, _ptr(uhat), _ptr(phihat), hp, int(nstep)))

    def step(self, nsteps=1):
        _check(lib().psms_step(self.ctx, int(nsteps)))

    def stage_times(self, nsteps):
        """Run nsteps steps and return the average ms of each of the 4 stage kernels."""
        ms = (ctypes.c_double * 4)()
        _check(lib().psms_stage_times(self.ctx, int(nsteps), ms))
        return [float(v) for v in ms]

    def get_state(self, with_history=False):
        c128 = self.torch.complex128
        uhat = self.torch.empty(self._spec_shape(3), dtype=c128, device=self.device)
        phihat = self.torch.empty(self._spec_shape(1), dtype=c128, device=self.device)
        hist = self.torch.empty(self._spec_shape(4), dtype=c128, device=self.device) if with_history else None
        _check(lib().psms_get_state(self.ctx, _ptr(uhat), _ptr(phihat), _ptr(hist) if hist is not None else None))
        return (uhat, phihat, hist) if with_history else (uhat, phihat)

    def transform(self, direction, x, flags=0):
        torch = self.torch
        n = self.n
        real = torch.float64 if self.precision == "fp64" else torch.float32
        cplx = torch.complex128 if self.precision == "fp64" else torch.complex64
        if direction > 0:
            x = x.contiguous()
            if x.dtype != real or tuple(x.shape[-3:]) != (n, n, n):
                raise ValueError("forward transform needs %s [...,%d,%d,%d]" % (real, n, n, n))
            nf = x.numel() // (n * n * n)
            out = torch.empty(tuple(x.shape[:-3]) + (n, n, n // 2 + 1), dtype=cplx, device=self.device)
        else:
            x = x.contiguous()
            if x.dtype != cplx or tuple(x.shape[-3:]) != (n, n, n // 2 + 1):
                raise ValueError("inverse transform needs %s [...,%d,%d,%d]" % (cplx, n, n, n // 2 + 1))
            nf = x.numel() // (n * n * (n // 2 + 1))
            out = torch.empty(tuple(x.shape[:-3]) + (n, n, n), dtype=real, device=self.device)
        _check(lib().psms_transform(self.ctx, 1 if direction > 0 else -1, nf, _ptr(x), _ptr(out), int(flags)))
        return out

    def solve_helmholtz(self, rhs, lambdas):
        torch = self.torch
        n = self.n
        rhs = rhs.contiguous()
        if rhs.dtype != torch.complex128 or tuple(rhs.shape[-3:]) != (n, n, n // 2 + 1):
            raise ValueError("rhs must be complex128 [...,%d,%d,%d]" % (n, n, n // 2 + 1))
        nf = rhs.numel() // (n * n * (n // 2 + 1))
        lam = (ctypes.c_double * max(nf, 1))(*[float(v) for v in lambdas])
        out = torch.empty_like(rhs)
        _check(lib().psms_solve_helmholtz(self.ctx, nf, lam, _ptr(rhs), _ptr(out)))
        return out

    def diagnostics(self):
        d = Diag()
        _check(lib().psms_diagnostics(self.ctx, ctypes.byref(d)))
        return dict(mean_phi=d.mean_phi, ke=d.ke, grad2=d.grad2, max_div=d.max_div,
                    nonfinite=int(d.nonfinite), nstep=int(d.nstep))

    def index_maps(self):
        m = int(lib().psms_band_modes(self.ctx))
        out = self.torch.empty((m, 4), dtype=self.torch.int32, device=self.device)
        _check(lib().psms_index_maps(self.ctx, _ptr(out)))
        return out
