"""Plain FP64 CPU oracle for the triply periodic Navier-Stokes + Cahn-Hilliard step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP implementation.

The paper (Roccon, "A GPU-ready pseudo-spectral method for direct numerical
simulations of multiphase turbulence") solves a channel; this module is the
Fourier x Fourier x Fourier reduction of the same scheme on the box
[0, 2 pi)^3, where every wall-normal Helmholtz problem becomes a division per
wavenumber and the wall-normal velocity/vorticity pair (Sec. 2.2, equations
``omegaz``, ``ww``, ``omegadef``) is equivalent to the Leray projection of the
nonlinear term.  The step follows Sec. 2.2:

* the nonlinear terms are formed in physical space (pseudo-spectral, Sec. 2.2)
  and transformed back, with the 2/3 rule (cut-off K = floor((N-1)/3) on every
  axis) applied to every product;
* Navier-Stokes (equation ``NSE``): Adams-Bashforth for S, Crank-Nicolson for
  the viscous term (Sec. 2.2, IMEX paragraph);
* Cahn-Hilliard (equations ``CHE`` and ``phisplit``): Adams-Bashforth for
  S_phi, implicit Euler for (s Ch^2 / Pe) lap(phi) - (Ch^2 / Pe) lap^2(phi).

Conventions (fixed here because the paper is silent):
* u(x) = sum_k u_k exp(i k.x); the forward transform carries 1/N^3
  (numpy ``norm="forward"``); a derivative d/dx_j is multiplication by i k_j.
* Arrays are [z][y][x] in physical space and [kz][ky][kx] (kx = 0..N/2) in
  spectral space; all spectral arrays hold the full half spectrum with zeros
  outside the retained band.
* The first step after initialisation uses Adams-Bashforth order 1.
* s defaults to sqrt(4 Pe / (Ch^2 dt)), the smallest value for which the
  implicit CH operator factors into two real Helmholtz operators.
* The oracle evaluates u.grad(u) and u.grad(phi) in the convective form the
  paper writes, and the surface force as the divergence of the Korteweg
  tensor (equation ``kort``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


# ---------------------------------------------------------------------------
# index maps and the dealiasing mask (Sec. 2.2, pseudo-spectral discretisation)
# ---------------------------------------------------------------------------

def cutoff(n: int) -> int:
    """Largest retained integer wavenumber K under the 2/3 rule: K = floor((N-1)/3).

    With K modes kept, a quadratic product has modes up to 2K, whose aliases
    land at |k| >= N - 2K > K, i.e. outside the retained band.
    """
    return (n - 1) // 3


def wavenumbers(n: int):
    """Integer wavenumbers for a 2 pi box: (kz, ky, kx) 1-D arrays.

    kz, ky follow FFT order 0, 1, ..., N/2-1, -N/2, ..., -1; kx = 0..N/2.
    """
    k = np.fft.fftfreq(n, 1.0 / n).astype(np.int64)
    kx = np.arange(n // 2 + 1, dtype=np.int64)
    return k.copy(), k.copy(), kx


def kgrid(n: int):
    kz, ky, kx = wavenumbers(n)
    KZ, KY, KX = np.meshgrid(kz.astype(np.float64), ky.astype(np.float64),
                             kx.astype(np.float64), indexing="ij")
    return KX, KY, KZ


def dealias_mask(n: int) -> np.ndarray:
    """Boolean [kz][ky][kx] mask of retained modes: |kx|,|ky|,|kz| <= K."""
    K = cutoff(n)
    kz, ky, kx = wavenumbers(n)
    return ((np.abs(kz)[:, None, None] <= K) & (np.abs(ky)[None, :, None] <= K)
            & (kx[None, None, :] <= K))


# ---------------------------------------------------------------------------
# transforms (library primitive: numpy pocketfft)
# ---------------------------------------------------------------------------

_FFT_WORKERS = 1


def set_fft_workers(n: int) -> None:
    """Transforms by numpy (n = 1, the default) or by scipy.fft with n threads:
    the same FP64 transforms, used only to time the oracle on several cores."""
    global _FFT_WORKERS
    _FFT_WORKERS = max(1, int(n))


def fwd(f: np.ndarray) -> np.ndarray:
    """Physical -> spectral over the last three axes, with the 1/N^3 factor."""
    if _FFT_WORKERS > 1:
        import scipy.fft
        return scipy.fft.rfftn(f, axes=(-3, -2, -1), norm="forward", workers=_FFT_WORKERS)
    return np.fft.rfftn(f, axes=(-3, -2, -1), norm="forward")


def inv(fh: np.ndarray, n: int) -> np.ndarray:
    """Spectral -> physical over the last three axes, unnormalised sum."""
    if _FFT_WORKERS > 1:
        import scipy.fft
        return scipy.fft.irfftn(fh, s=(n, n, n), axes=(-3, -2, -1), norm="forward", workers=_FFT_WORKERS)
    return np.fft.irfftn(fh, s=(n, n, n), axes=(-3, -2, -1), norm="forward")


def deriv(fh: np.ndarray, axis: int) -> np.ndarray:
    """Spectral derivative along x (0), y (1) or z (2): multiply by i k."""
    n = fh.shape[-2]
    KX, KY, KZ = kgrid(n)
    return 1j * (KX, KY, KZ)[axis] * fh


def project(vh: np.ndarray) -> np.ndarray:
    """Leray projection P v = v - k (k.v) / |k|^2 of a spectral vector field.

    On the box this is what the wall-normal velocity-vorticity system of
    Sec. 2.2 computes: it removes the pressure gradient so that continuity
    (equation ``cont``) holds.  The k = 0 mode is set to zero.
    """
    n = vh.shape[-2]
    KX, KY, KZ = kgrid(n)
    k2 = KX * KX + KY * KY + KZ * KZ
    k2s = k2.copy()
    k2s[0, 0, 0] = 1.0
    kdotv = KX * vh[0] + KY * vh[1] + KZ * vh[2]
    out = np.stack([vh[0] - KX * kdotv / k2s,
                    vh[1] - KY * kdotv / k2s,
                    vh[2] - KZ * kdotv / k2s])
    out[:, 0, 0, 0] = 0.0
    return out


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------

@dataclass
class Params:
    """Dimensionless numbers of Sec. 2.1 and the time step.

    re: friction Reynolds number (equation ``Re``); we: Weber number
    (equation ``We``); ch: Cahn number; pe: Peclet number; dt: time step;
    s: CH splitting coefficient of equation ``phisplit`` (None -> default).
    """
    n: int
    re: float
    we: float
    ch: float
    pe: float
    dt: float
    s: float | None = None
    cube: str = "grid"   # phi^3: "grid" = pointwise cube on the N grid, then truncated;
                         # "exact" = the truncation of the exact cube (cube_exact)

    def split_s(self) -> float:
        if self.s is not None and self.s > 0.0:
            return float(self.s)
        return default_s(self.ch, self.pe, self.dt)

    def capillary(self) -> float:
        """Coefficient of the Korteweg force, (3 / sqrt 8) Ch / We (equation ``kort``)."""
        return 3.0 / math.sqrt(8.0) * self.ch / self.we


def default_s(ch: float, pe: float, dt: float) -> float:
    """s such that 1 + dt (Ch^2/Pe)(k^4 + s k^2) has a double real root in k^2.

    The implicit CH factor (Pe / (dt Ch^2)) + s k^2 + k^4 factors as
    (k^2 + a)(k^2 + b) with a b = Pe / (dt Ch^2) and a + b = s; a and b are
    real iff s^2 >= 4 Pe / (dt Ch^2).
    """
    return math.sqrt(4.0 * pe / (ch * ch * dt))


# ---------------------------------------------------------------------------
# the step (Sec. 2.2, steps i-v)
# ---------------------------------------------------------------------------

def init_state(u: np.ndarray, phi: np.ndarray, prm: Params) -> dict:
    """Step (i): transform u^0, phi^0 to spectral space.

    The spectra are truncated to the retained band and the velocity is
    projected onto divergence-free fields.  The history is empty, so the next
    step uses Adams-Bashforth order 1.
    """
    n = prm.n
    D = dealias_mask(n)
    uh = project(fwd(np.asarray(u, dtype=np.float64)) * D)
    ph = fwd(np.asarray(phi, dtype=np.float64)) * D
    return dict(uh=uh, ph=ph, hS=np.zeros_like(uh), hphi=np.zeros_like(ph), nstep=0)


def nonlinear_terms(uh: np.ndarray, ph: np.ndarray, prm: Params):
    """Steps (ii) and (vi): the explicit right-hand sides, in spectral space.

    Returns (S_hat, Sphi_hat, Sphi0) where
      S      = -u.grad(u) + (3/sqrt8)(Ch/We) div(|grad phi|^2 I - grad phi (x) grad phi)
      S_phi  = -u.grad(phi) + (1/Pe) lap(phi^3) - ((1 + s Ch^2)/Pe) lap(phi)
    (equations ``NSE``, ``kort``, ``CHE`` and ``phisplit``, with
    mu = phi^3 - phi - Ch^2 lap phi).  Every physical-space product is
    truncated to the retained band.  S_hat(0) and S_phi_hat(0) are set to zero
    (the mean of each term is a divergence); Sphi0 is the value S_phi_hat(0)
    had before that, a consistency check that should be at rounding level.
    """
    n = prm.n
    D = dealias_mask(n)
    KX, KY, KZ = kgrid(n)
    kvec = (KX, KY, KZ)
    k2 = KX * KX + KY * KY + KZ * KZ
    s = prm.split_s()

    u = inv(uh, n)                                   # u_i on the grid
    phi = inv(ph, n)
    g = np.stack([inv(1j * kvec[j] * ph, n) for j in range(3)])   # grad phi
    # convective term u.grad(u): (u.grad u)_i = sum_j u_j d_j u_i
    conv = np.zeros_like(u)
    for i in range(3):
        for j in range(3):
            conv[i] += u[j] * inv(1j * kvec[j] * uh[i], n)
    # Korteweg tensor tau_ij = |g|^2 delta_ij - g_i g_j
    g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2]
    S = np.zeros_like(uh)
    csig = prm.capillary()
    for i in range(3):
        div_tau = np.zeros_like(ph)
        for j in range(3):
            tau_ij = (g2 if i == j else 0.0) - g[i] * g[j]
            div_tau = div_tau + 1j * kvec[j] * (fwd(tau_ij) * D)
        S[i] = -fwd(conv[i]) * D + csig * div_tau
    S[:, 0, 0, 0] = 0.0

    adv = fwd(u[0] * g[0] + u[1] * g[1] + u[2] * g[2]) * D      # u.grad(phi)
    if prm.cube == "exact":
        cube = cube_exact(ph, n)                                 # phi^3 without aliasing
    else:
        cube = fwd(phi * phi * phi) * D                          # phi^3 on the N grid
    Sphi = -adv - (k2 / prm.pe) * cube + ((1.0 + s * prm.ch ** 2) / prm.pe) * k2 * ph
    Sphi0 = complex(Sphi[0, 0, 0])
    Sphi[0, 0, 0] = 0.0
    return S, Sphi, Sphi0


def cube_exact(ph: np.ndarray, n: int, m: int | None = None) -> np.ndarray:
    """The retained band of the exact cube of the band-limited phi (chemical
    potential mu = phi^3 - phi - Ch^2 lap phi, Sec. 2.1.1): phi is evaluated on
    an m^3 grid (default 2n), cubed there and transformed back, and the modes
    |k_i| <= K of the n grid kept.  The cube of modes |k| <= K reaches 3K; on
    the m grid its aliases land at |k| >= m - 3K > K once m > 4K, so the kept
    modes are those of the exact product (for any such m)."""
    K = cutoff(n)
    m = 2 * n if m is None else m
    if m <= 4 * K:
        raise ValueError("m must exceed 4K")
    kz, ky, _ = wavenumbers(n)
    kzm, kym, _ = wavenumbers(m)
    band = np.abs(kz) <= K
    pos_n = np.nonzero(band)[0]                      # rows / planes of the band on the n grid
    pos_m = np.array([np.nonzero(kzm == kz[p])[0][0] for p in pos_n])   # the same k on the m grid
    big = np.zeros((m, m, m // 2 + 1), dtype=complex)
    big[np.ix_(pos_m, pos_m, np.arange(K + 1))] = ph[np.ix_(pos_n, pos_n, np.arange(K + 1))]
    f = inv(big, m)
    cm = fwd(f * f * f)
    out = np.zeros_like(ph)
    out[np.ix_(pos_n, pos_n, np.arange(K + 1))] = cm[np.ix_(pos_m, pos_m, np.arange(K + 1))]
    return out


def pressure(state: dict, prm: Params) -> np.ndarray:
    """The pressure that the projection removes (eq. cont): lap p = div S, i.e.
    p_hat = -i k.S_hat / k^2 with S the unprojected nonlinear term of the state
    (convective and Korteweg parts, ``nonlinear_terms``); p_hat(0) = 0."""
    n = prm.n
    S, _, _ = nonlinear_terms(state["uh"], state["ph"], prm)
    KX, KY, KZ = kgrid(n)
    k2 = KX * KX + KY * KY + KZ * KZ
    k2[0, 0, 0] = 1.0
    p = -1j * (KX * S[0] + KY * S[1] + KZ * S[2]) / k2
    p[0, 0, 0] = 0.0
    return p


def step(state: dict, prm: Params) -> dict:
    """Advance (u_hat, phi_hat) from n to n+1 (steps ii-v of Sec. 2.2).

    NS (step iv), Crank-Nicolson + Adams-Bashforth 2 (AB1 on the first step):
      (1 + dt k^2/(2 Re)) u^{n+1} = (1 - dt k^2/(2 Re)) u^n + dt (3/2 P S^n - 1/2 P S^{n-1})
    CH (step v), implicit Euler + Adams-Bashforth 2:
      (1 + dt (Ch^2/Pe)(k^4 + s k^2)) phi^{n+1} = phi^n + dt (3/2 S_phi^n - 1/2 S_phi^{n-1})
    Both right-hand sides are built from the fields at time n.
    """
    n = prm.n
    D = dealias_mask(n)
    KX, KY, KZ = kgrid(n)
    k2 = KX * KX + KY * KY + KZ * KZ
    s = prm.split_s()
    dt, nu = prm.dt, 1.0 / prm.re

    S, Sphi, _ = nonlinear_terms(state["uh"], state["ph"], prm)
    PS = project(S)
    if state["nstep"] == 0:
        expl_u, expl_p = PS, Sphi
    else:
        expl_u = 1.5 * PS - 0.5 * state["hS"]
        expl_p = 1.5 * Sphi - 0.5 * state["hphi"]
    uh = ((1.0 - 0.5 * dt * nu * k2) * state["uh"] + dt * expl_u) / (1.0 + 0.5 * dt * nu * k2)
    ph = (state["ph"] + dt * expl_p) / (1.0 + dt * (prm.ch ** 2 / prm.pe) * (k2 * k2 + s * k2))
    return dict(uh=uh * D, ph=ph * D, hS=PS, hphi=Sphi, nstep=state["nstep"] + 1)


def run(state: dict, prm: Params, nsteps: int) -> dict:
    for _ in range(nsteps):
        state = step(state, prm)
    return state


# ---------------------------------------------------------------------------
# single-stage operations used by the transform / Helmholtz entry points
# ---------------------------------------------------------------------------

def transform_forward(f: np.ndarray, dealias: bool = False, deriv_axis: int | None = None):
    """Forward 3-D transform of real fields (..., N, N, N), optional mask and i k_j."""
    n = f.shape[-1]
    fh = fwd(np.asarray(f, dtype=np.float64))
    if deriv_axis is not None:
        fh = deriv(fh, deriv_axis)
    if dealias:
        fh = fh * dealias_mask(n)
    return fh


def transform_inverse(fh: np.ndarray, dealias: bool = False, deriv_axis: int | None = None):
    """Inverse 3-D transform of half spectra (..., N, N, N/2+1)."""
    n = fh.shape[-2]
    if dealias:
        fh = fh * dealias_mask(n)
    if deriv_axis is not None:
        fh = deriv(fh, deriv_axis)
    return inv(fh, n)


def solve_helmholtz(gh: np.ndarray, lam: float) -> np.ndarray:
    """Solve (lap - lam) f = g on the box: f_hat = -g_hat / (k^2 + lam).

    Modes with k^2 + lam = 0 (only k = 0 when lam = 0) are set to zero.
    """
    n = gh.shape[-2]
    KX, KY, KZ = kgrid(n)
    den = KX * KX + KY * KY + KZ * KZ + lam
    out = np.zeros_like(gh)
    nz = den != 0.0
    out[..., nz] = -gh[..., nz] / den[nz]
    return out


# ---------------------------------------------------------------------------
# diagnostics
# ---------------------------------------------------------------------------

def half_weights(n: int) -> np.ndarray:
    """Parseval weights of the half spectrum: 1 at kx = 0 and kx = N/2, else 2."""
    w = np.full(n // 2 + 1, 2.0)
    w[0] = 1.0
    w[-1] = 1.0
    return w


def diagnostics(state: dict, n: int, dt: float | None = None) -> dict:
    """Volume averages: mean phi, kinetic energy 1/2 <|u|^2>, <|grad phi|^2>,
    and max |k.u_hat| (continuity, equation ``cont``); with dt, also the CFL
    number dt max_x (|u| + |v| + |w|) / dx on the physical grid, dx = 2 pi / N."""
    uh, ph = state["uh"], state["ph"]
    KX, KY, KZ = kgrid(n)
    k2 = KX * KX + KY * KY + KZ * KZ
    w = half_weights(n)[None, None, :]
    ke = 0.5 * float(np.sum(w * (np.abs(uh) ** 2).sum(axis=0)))
    grad2 = float(np.sum(w * k2 * np.abs(ph) ** 2))
    div = float(np.max(np.abs(KX * uh[0] + KY * uh[1] + KZ * uh[2])))
    finite = bool(np.all(np.isfinite(uh)) and np.all(np.isfinite(ph)))
    out = dict(mean_phi=float(ph[0, 0, 0].real), ke=ke, grad2=grad2, max_div=div, finite=finite)
    if dt is not None:
        u = inv(uh, n)
        out["cfl"] = float(dt * np.max(np.abs(u).sum(axis=0)) / (2.0 * math.pi / n))
    return out
