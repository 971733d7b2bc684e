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
                ("cube", ctypes.c_int32), ("re", ctypes.c_double), ("we", ctypes.c_double),
                ("ch", ctypes.c_double), ("pe", ctypes.c_double), ("dt", ctypes.c_double),
                ("s", ctypes.c_double)]


class Diag(ctypes.Structure):
    _fields_ = [("mean_phi", ctypes.c_double), ("ke", ctypes.c_double), ("grad2", ctypes.c_double),
                ("max_div", ctypes.c_double), ("nonfinite", ctypes.c_int32), ("nstep", ctypes.c_int32),
                ("cfl", ctypes.c_double), ("sphi0_re", ctypes.c_double), ("sphi0_im", ctypes.c_double)]


class WallArgs(ctypes.Structure):
    _fields_ = [("nc", ctypes.c_int32), ("reserved", ctypes.c_int32), ("nlines", ctypes.c_int64),
                ("d_kx", ctypes.c_void_p), ("d_ky", ctypes.c_void_p), ("beta_ns", ctypes.c_double),
                ("beta_a", ctypes.c_double), ("beta_b", ctypes.c_double), ("d_g_om", ctypes.c_void_p),
                ("d_g_w", ctypes.c_void_p), ("d_g_phi", ctypes.c_void_p), ("d_om", ctypes.c_void_p),
                ("d_w", ctypes.c_void_p), ("d_phi", ctypes.c_void_p), ("d_u", ctypes.c_void_p),
                ("d_v", ctypes.c_void_p)]


class ChannelParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nc", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("re", ctypes.c_double), ("we", ctypes.c_double),
                ("ch", ctypes.c_double), ("pe", ctypes.c_double), ("dt", ctypes.c_double), ("s", ctypes.c_double),
                ("forcing", ctypes.c_double), ("single_phase", ctypes.c_int32), ("free_slip", ctypes.c_int32)]


DIRICHLET, NEUMANN = 1, 2

_lib = None

_SIGS = {
    "psms_channel_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(ChannelParams), ctypes.POINTER(ctypes.c_size_t)]),
    "psms_channel_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ChannelParams),
                                           ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "psms_channel_init_state": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 4),
    "psms_channel_set_state": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 4 + [ctypes.c_int32]),
    "psms_channel_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "psms_channel_get_state": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 4),
    "psms_channel_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "psms_channel_diagnostics": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Diag)]),
    "psms_channel_set_graphs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
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
    "psms_pressure": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "psms_index_maps": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "psms_band_modes": (ctypes.c_int64, [ctypes.c_void_p]),
    "psms_stage_times": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "psms_cheb_transform": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "psms_cheb_deriv": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "psms_cheb_helmholtz": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p]),
    "psms_cheb_helmholtz_noalloc": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32,
                                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_void_p]),
    "psms_wall_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]),
    "psms_wall_solve": (ctypes.c_int, [ctypes.POINTER(WallArgs), ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.c_void_p]),
    "psms_batch_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(Params),
                                                  ctypes.POINTER(ctypes.c_size_t)]),
    "psms_batch_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.POINTER(Params),
                                         ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "psms_batch_init_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "psms_batch_get_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "psms_batch_diagnostics": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(Diag)]),
    "psms_batch_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "psms_batch_groups": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "psms_batch_set_variants": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "psms_batch_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_double)]),
    "psms_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "psms_adjoint_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int32, ctypes.c_int32,
                                                    ctypes.POINTER(ctypes.c_size_t)]),
    "psms_adjoint_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(Params), ctypes.c_int32,
                                           ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "psms_adjoint_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_double)]),
    "psms_adjoint_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "psms_adjoint_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "psms_set_graphs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
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


def make_params(n, re, we, ch, pe, dt, s=0.0, precision="fp64", geometry=BOX, cube="grid") -> Params:
    prec = {"fp64": FP64, "mixed": MIXED}[precision] if isinstance(precision, str) else int(precision)
    cb = {"grid": 0, "exact": 1}[cube] if isinstance(cube, str) else int(cube)
    return Params(geometry, int(n), prec, cb, float(re), float(we), float(ch), float(pe), float(dt), float(s or 0.0))


def workspace_bytes(params: Params) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().psms_workspace_bytes(ctypes.byref(params), ctypes.byref(b)))
    return int(b.value)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """One periodic-box NS+CH context on the current GPU and torch stream."""

    def __init__(self, n, re, we, ch, pe, dt, s=0.0, precision="fp64", device="cuda", stream=None, cube="grid"):
        import torch
        self.torch = torch
        self.params = make_params(n, re, we, ch, pe, dt, s, precision, cube=cube)
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

    def set_graphs(self, enable):
        _check(lib().psms_set_graphs(self.ctx, 1 if enable else 0))

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
                    nonfinite=int(d.nonfinite), nstep=int(d.nstep), cfl=d.cfl,
                    sphi0=complex(d.sphi0_re, d.sphi0_im))

    def pressure(self):
        """p_hat of the current state, complex128 [n, n, n/2+1]."""
        n = self.n
        out = self.torch.empty((n, n, n // 2 + 1), dtype=self.torch.complex128, device=self.device)
        _check(lib().psms_pressure(self.ctx, _ptr(out)))
        return out

    def index_maps(self):
        m = int(lib().psms_band_modes(self.ctx))
        out = self.torch.empty((m, 4), dtype=self.torch.int32, device=self.device)
        _check(lib().psms_index_maps(self.ctx, _ptr(out)))
        return out


# ---------------------------------------------------------------------------
# wall-normal (Chebyshev) operations: stateless calls on torch's current stream
# ---------------------------------------------------------------------------

def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def cheb_transform(x, direction):
    """DCT-I Chebyshev transform of lines x [nc+1, nlines] (complex128 or complex64, on the GPU).
    direction +1: values at the CGL points -> coefficients; -1: coefficients -> values."""
    import torch
    x = x.contiguous()
    prec = {torch.complex128: FP64, torch.complex64: MIXED}[x.dtype]
    out = torch.empty_like(x)
    nc = x.shape[0] - 1
    nl = x.numel() // (nc + 1)
    _check(lib().psms_cheb_transform(nc, nl, 1 if direction > 0 else -1, prec, _ptr(x), _ptr(out), _stream()))
    return out


def cheb_deriv(a):
    """Coefficients of d/dz of a [nc+1, nlines] complex128."""
    import torch
    a = a.contiguous()
    if a.dtype != torch.complex128:
        raise ValueError("complex128 required")
    out = torch.empty_like(a)
    nc = a.shape[0] - 1
    _check(lib().psms_cheb_deriv(nc, a.numel() // (nc + 1), _ptr(a), _ptr(out), _stream()))
    return out


def cheb_helmholtz(g, beta, bc="dirichlet", bcval=None):
    """Chebyshev-tau solve of (D^2 - beta_l) f = g per line (FP64).  g [nc+1, nlines] complex128,
    beta [nlines] float64, bcval [nlines, 2] complex128 (top, bottom) or None."""
    import torch
    g = g.contiguous()
    if g.dtype != torch.complex128:
        raise ValueError("complex128 required")
    nc = g.shape[0] - 1
    nl = g.numel() // (nc + 1)
    beta = beta.to(dtype=torch.float64).contiguous()
    out = torch.empty_like(g)
    work = torch.empty((nc + 1) * max(nl, 1), dtype=torch.float64, device=g.device)
    bv = None
    if bcval is not None:
        bcval = bcval.to(dtype=torch.complex128).contiguous()
        bv = _ptr(bcval)
    kind = {"dirichlet": DIRICHLET, "neumann": NEUMANN}[bc]
    _check(lib().psms_cheb_helmholtz(nc, nl, _ptr(beta), kind, bv, _ptr(g), _ptr(out), _ptr(work), _stream()))
    return out


def cheb_helmholtz_noalloc(g, beta, bc="dirichlet", bcval=None, out=None):
    """cheb_helmholtz with the library's own device scratch (no workspace): for
    callers that cannot allocate.  `out` (same shape and dtype as g) may be given
    so that the call itself allocates nothing."""
    import torch
    if g.dtype != torch.complex128 or beta.dtype != torch.float64:
        raise ValueError("complex128 g and float64 beta required")
    if not (g.is_contiguous() and beta.is_contiguous()):
        raise ValueError("contiguous g and beta required")
    nc = g.shape[0] - 1
    nl = g.numel() // (nc + 1)
    if out is None:
        out = torch.empty_like(g)
    bv = None
    if bcval is not None:
        if bcval.dtype != torch.complex128 or not bcval.is_contiguous():
            raise ValueError("contiguous complex128 bcval required")
        bv = _ptr(bcval)
    kind = {"dirichlet": DIRICHLET, "neumann": NEUMANN}[bc]
    _check(lib().psms_cheb_helmholtz_noalloc(nc, nl, _ptr(beta), kind, bv, _ptr(g), _ptr(out), _stream()))
    return out


def wall_solve(kx, ky, beta_ns, beta_a, beta_b, g_om, g_w, g_phi):
    """The implicit wall-normal solves of a channel step for every (kx, ky) line.
    kx, ky [nlines] float64; g_* [nc+1, nlines] complex128.  Returns dict of
    omega, w, phi, u, v coefficient arrays."""
    import torch
    nc = g_om.shape[0] - 1
    nl = g_om.numel() // (nc + 1)
    kx = kx.to(torch.float64).contiguous()
    ky = ky.to(torch.float64).contiguous()
    g = [t.contiguous() for t in (g_om, g_w, g_phi)]
    outs = {k: torch.empty_like(g[0]) for k in ("omega", "w", "phi", "u", "v")}
    nbytes = ctypes.c_size_t(0)
    _check(lib().psms_wall_workspace_bytes(nc, nl, ctypes.byref(nbytes)))
    work = torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device=g_om.device)
    a = WallArgs(nc, 0, nl, kx.data_ptr(), ky.data_ptr(), float(beta_ns), float(beta_a), float(beta_b),
                 g[0].data_ptr(), g[1].data_ptr(), g[2].data_ptr(), outs["omega"].data_ptr(), outs["w"].data_ptr(),
                 outs["phi"].data_ptr(), outs["u"].data_ptr(), outs["v"].data_ptr())
    _check(lib().psms_wall_solve(ctypes.byref(a), _ptr(work), int(nbytes.value), _stream()))
    return outs


# ---------------------------------------------------------------------------
# batches of independent boxes
# ---------------------------------------------------------------------------

class Batch:
    """Many independent periodic boxes of uneven size stepped together.

    params: list of dicts with n, re, we, ch, pe, dt (and optionally s).  All
    boxes share `precision`.  The batch runs on `stream` (default: a new
    torch stream, which graph capture needs (step(use_graph=True)); use it with torch.cuda.stream).
    """

    def __init__(self, params, precision="mixed", device="cuda", stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.precision = precision
        self.nbox = len(params)
        arr = (Params * self.nbox)(*[make_params(q["n"], q["re"], q["we"], q["ch"], q["pe"], q["dt"],
                                                 q.get("s", 0.0), precision) for q in params])
        self._params = arr
        self.ns = [int(q["n"]) for q in params]
        nbytes = ctypes.c_size_t(0)
        _check(lib().psms_batch_workspace_bytes(self.nbox, arr, ctypes.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        torch.cuda.current_stream(self.device).synchronize()
        h = ctypes.c_void_p()
        _check(lib().psms_batch_create(ctypes.byref(h), self.nbox, arr, _ptr(self.workspace), int(nbytes.value),
                                       ctypes.c_void_p(self.stream.cuda_stream)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().psms_batch_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _on_stream(self, t):
        # make the batch stream wait for work queued on the caller's stream
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        return t

    def init_state(self, box, u, phi):
        n = self.ns[box]
        u = u.to(self.device, self.torch.float64).contiguous()
        phi = phi.to(self.device, self.torch.float64).contiguous()
        assert tuple(u.shape) == (3, n, n, n) and tuple(phi.shape) == (n, n, n)
        self._on_stream(u)
        _check(lib().psms_batch_init_state(self.h, int(box), _ptr(u), _ptr(phi)))
        self.stream.synchronize()

    def step(self, nsteps=1, use_graph=False):
        _check(lib().psms_batch_step(self.h, int(nsteps), 1 if use_graph else 0))

    def get_state(self, box):
        torch = self.torch
        n = self.ns[box]
        uh = torch.empty((3, n, n, n // 2 + 1), dtype=torch.complex128, device=self.device)
        ph = torch.empty((n, n, n // 2 + 1), dtype=torch.complex128, device=self.device)
        self._on_stream(uh)
        _check(lib().psms_batch_get_state(self.h, int(box), _ptr(uh), _ptr(ph)))
        self.stream.synchronize()
        return uh, ph

    def diagnostics(self, box):
        d = Diag()
        _check(lib().psms_batch_diagnostics(self.h, int(box), ctypes.byref(d)))
        return dict(mean_phi=d.mean_phi, ke=d.ke, grad2=d.grad2, max_div=d.max_div,
                    nonfinite=int(d.nonfinite), nstep=int(d.nstep), cfl=d.cfl,
                    sphi0=complex(d.sphi0_re, d.sphi0_im))

    def groups(self):
        ng = ctypes.c_int32(0)
        _check(lib().psms_batch_groups(self.h, ctypes.byref(ng), None, None))
        ns = (ctypes.c_int32 * ng.value)()
        cnt = (ctypes.c_int32 * ng.value)()
        _check(lib().psms_batch_groups(self.h, ctypes.byref(ng), ns, cnt))
        return [(int(ns[i]), int(cnt[i])) for i in range(ng.value)]

    def set_variants(self, variants):
        arr = (ctypes.c_int32 * len(variants))(*variants)
        _check(lib().psms_batch_set_variants(self.h, arr))

    def autotune(self, reps=5, cache_path=None):
        """Pick the workgroup-size variant of every stage of every group by timing (HIP
        events), or reuse the choices stored in the JSON file `cache_path`.  Keys are
        "<precision>/N<n>x<count>"; values are the 4 per-stage variants."""
        import json
        groups = self.groups()
        keys = ["%s/N%dx%d" % (self.precision, n, c) for n, c in groups]
        cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        if all(k in cache for k in keys):
            flat = [v for k in keys for v in cache[k]]
            self.set_variants(flat)
            return {"source": "cache", "variants": dict(zip(keys, [cache[k] for k in keys]))}
        var = (ctypes.c_int32 * (4 * len(groups)))()
        ms = (ctypes.c_double * (12 * len(groups)))()
        _check(lib().psms_batch_autotune(self.h, int(reps), var, ms))
        res = {}
        for i, k in enumerate(keys):
            cache[k] = [int(var[4 * i + s]) for s in range(4)]
            res[k] = {"variants": cache[k], "ms": [[float(ms[(4 * i + s) * 3 + v]) for v in range(3)]
                                                  for s in range(4)]}
        if cache_path:
            with open(cache_path, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
        return {"source": "timed", "groups": res}


# ---------------------------------------------------------------------------
# discrete adjoint and torch.autograd
# ---------------------------------------------------------------------------

class Adjoint:
    """Primal run with FP64 checkpoints every seg_len steps and the hand-written
    discrete adjoint (recomputing each segment in FP64)."""

    def __init__(self, n, re, we, ch, pe, dt, s=0.0, precision="fp64", max_steps=50, seg_len=10, device="cuda"):
        import torch
        self.torch = torch
        self.n = int(n)
        self.device = torch.device(device)
        self.params = make_params(n, re, we, ch, pe, dt, s, precision)
        nb = ctypes.c_size_t(0)
        _check(lib().psms_adjoint_workspace_bytes(ctypes.byref(self.params), int(max_steps), int(seg_len),
                                                  ctypes.byref(nb)))
        self.workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(lib().psms_adjoint_create(ctypes.byref(h), ctypes.byref(self.params), int(max_steps), int(seg_len),
                                         _ptr(self.workspace), int(nb.value), ctypes.c_void_p(self.stream.cuda_stream)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().psms_adjoint_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, u0, phi0, nsteps):
        torch = self.torch
        n = self.n
        u0 = u0.to(self.device, torch.float64).contiguous()
        phi0 = phi0.to(self.device, torch.float64).contiguous()
        assert tuple(u0.shape) == (3, n, n, n) and tuple(phi0.shape) == (n, n, n)
        J = ctypes.c_double(0.0)
        _check(lib().psms_adjoint_forward(self.h, _ptr(u0), _ptr(phi0), int(nsteps), ctypes.byref(J)))
        return float(J.value)

    def backward(self):
        torch = self.torch
        n = self.n
        d = torch.empty((n, n, n), dtype=torch.float64, device=self.device)
        dwe = ctypes.c_double(0.0)
        _check(lib().psms_adjoint_backward(self.h, _ptr(d), ctypes.byref(dwe)))
        return d, float(dwe.value)


def _objective_function():
    import torch

    class NSCHObjective(torch.autograd.Function):
        """J(phi0, We) = int |grad phi|^2 + 1/2 int |u|^2 after nsteps, with the gradient
        from the hand-written discrete adjoint (segment checkpointing)."""

        @staticmethod
        def forward(ctx, phi0, we, u0, cfg):
            a = Adjoint(cfg["n"], cfg["re"], float(we), cfg["ch"], cfg["pe"], cfg["dt"], cfg.get("s", 0.0),
                        cfg.get("precision", "fp64"), cfg["nsteps"], cfg.get("seg_len", 10), device=phi0.device)
            J = a.forward(u0, phi0, cfg["nsteps"])
            ctx.adj = a
            return torch.tensor(J, dtype=torch.float64, device=phi0.device)

        @staticmethod
        def backward(ctx, gJ):
            d, dwe = ctx.adj.backward()
            ctx.adj.close()
            g = gJ.to(torch.float64)
            return g * d, g * torch.tensor(dwe, dtype=torch.float64, device=d.device), None, None

    return NSCHObjective


def objective(phi0, we, u0, cfg):
    """Differentiable J(phi0, We): cfg holds n, re, ch, pe, dt, nsteps (and s, precision,
    seg_len).  phi0 [n,n,n] and we (0-d) are float64 tensors on the GPU."""
    return _objective_function().apply(phi0, we, u0, cfg)


# ---------------------------------------------------------------------------
# the channel step
# ---------------------------------------------------------------------------

class Channel:
    """One channel NS+CH context (x, y periodic, Chebyshev in z between walls).

    Spectral arrays: complex128 [..., nc+1, 2 Ky + 1, Kx + 1] (Chebyshev index,
    ky in band order 0..Ky, -Ky..-1, kx = 0..Kx); mean lines [2, nc+1] (U, V);
    physical fields float64 [nc+1, ny, nx] at z_j = cos(pi j / nc).
    single_phase=True steps Navier-Stokes alone (phi stays zero; we, ch, pe, s unused).
    walls = (top, bottom) wall conditions, each "noslip" or "freeslip".
    """

    def __init__(self, nx, ny, nc, re, we, ch, pe, dt, s=0.0, precision="fp64", lx=4 * 3.141592653589793,
                 ly=2 * 3.141592653589793, forcing=1.0, single_phase=False, walls=("noslip", "noslip"),
                 device="cuda", stream=None):
        import torch
        self.torch = torch
        prec = {"fp64": FP64, "mixed": MIXED}[precision]
        self.single_phase = bool(single_phase)
        self.params = ChannelParams(int(nx), int(ny), int(nc), prec, float(lx), float(ly), float(re),
                                    float(we or 0.0), float(ch or 0.0), float(pe or 0.0), float(dt), float(s or 0.0),
                                    float(forcing), int(self.single_phase),
                                    sum(1 << j for j, wl in enumerate(walls) if wl == "freeslip"))
        if any(wl not in ("noslip", "freeslip") for wl in walls) or len(walls) != 2:
            raise ValueError("walls = (top, bottom), each 'noslip' or 'freeslip'")
        self.nx, self.ny, self.nc = int(nx), int(ny), int(nc)
        self.band = (self.nc + 1, 2 * ((self.ny - 1) // 3) + 1, (self.nx - 1) // 3 + 1)
        self.device = torch.device(device)
        b = ctypes.c_size_t(0)
        _check(lib().psms_channel_workspace_bytes(ctypes.byref(self.params), ctypes.byref(b)))
        self.workspace = torch.empty(int(b.value), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(lib().psms_channel_create(ctypes.byref(h), ctypes.byref(self.params), _ptr(self.workspace),
                                         int(b.value), ctypes.c_void_p(self.stream.cuda_stream)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().psms_channel_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, x, dtype):
        t = self.torch
        return x.to(device=self.device, dtype=dtype).contiguous()

    def init_state(self, u, v, w, phi=None):
        """phi may be None in single phase."""
        t = self.torch
        f = [self._dev(x, t.float64) if x is not None else None for x in (u, v, w, phi)]
        _check(lib().psms_channel_init_state(self.h, *[_ptr(x) if x is not None else None for x in f]))

    def set_state(self, state, mean, hist=None, hmean=None, nstep=0):
        t = self.torch
        st = self._dev(state, t.complex128)
        mn = self._dev(mean, t.complex128)
        hs = self._dev(hist, t.complex128) if hist is not None else None
        hm = self._dev(hmean, t.complex128) if hmean is not None else None
        _check(lib().psms_channel_set_state(self.h, _ptr(st), _ptr(mn), _ptr(hs) if hs is not None else None,
                                            _ptr(hm) if hm is not None else None, int(nstep)))
        self._keep = (st, mn, hs, hm)

    def step(self, nsteps=1):
        _check(lib().psms_channel_step(self.h, int(nsteps)))

    def get_state(self, with_history=False):
        t = self.torch
        st = t.empty((3,) + self.band, dtype=t.complex128, device=self.device)
        mn = t.empty((2, self.nc + 1), dtype=t.complex128, device=self.device)
        hs = t.empty_like(st) if with_history else None
        hm = t.empty_like(mn) if with_history else None
        _check(lib().psms_channel_get_state(self.h, _ptr(st), _ptr(mn), _ptr(hs) if hs is not None else None,
                                            _ptr(hm) if hm is not None else None))
        return (st, mn, hs, hm) if with_history else (st, mn)

    def set_graphs(self, enable):
        _check(lib().psms_channel_set_graphs(self.h, 1 if enable else 0))

    def diagnostics(self):
        d = Diag()
        _check(lib().psms_channel_diagnostics(self.h, ctypes.byref(d)))
        return dict(mean_phi=d.mean_phi, ke=d.ke, grad2=d.grad2, max_div=d.max_div,
                    nonfinite=int(d.nonfinite), nstep=int(d.nstep), cfl=d.cfl,
                    sphi0=complex(d.sphi0_re, d.sphi0_im))
