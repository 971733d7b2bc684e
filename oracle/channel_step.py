"""Plain FP64 CPU oracle for one coupled NS + CH step of the plane channel.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP implementation.

The paper's geometry (Sec. 2.1-2.2): x and y periodic (lengths Lx, Ly, Fourier),
z in [-1, 1] between two walls (Chebyshev, collocation at the Chebyshev-Gauss-
Lobatto points).  The velocity is carried as the wall-normal vorticity omega_z
and the wall-normal velocity w (eqs. omegaz, ww, omegadef), plus the mean
(kx = ky = 0) velocities U(z), V(z); the phase field phi obeys the split CH
equation (eq. phisplit).  One step (Sec. 2.2):

1. u, v from continuity and the definition of omega_z; U, V on the mean line;
2. u, v, w, phi and grad(phi) to physical space;
3. products at the collocation points: T_ij = -u_i u_j + c_sigma (|g|^2 delta_ij
   - g_i g_j) (eqs. NSE, kort; c_sigma = 3 Ch / (sqrt(8) We)), a = u.grad(phi),
   c = phi^3;
4. back to spectral space, 2/3 rule in x and y (K = floor((n-1)/3)) and in z
   (Chebyshev modes n <= floor((2 nc - 1) / 3), the 2/3 rule of the 2 nc-point
   even extension);
5. S_i = d_j T_ij (i kx, i ky, and the Chebyshev derivative D);
   S_phi = -a + (1/Pe) lap(c) - ((1 + s Ch^2)/Pe) lap(phi), lap = D^2 - k^2;
   H_omega = i kx S_y - i ky S_x;  H_w = -k^2 S_z - D(i kx S_x + i ky S_y);
6. Adams-Bashforth (order 1 on the first step) for H_omega, H_w, S_phi and the
   mean S_x, S_y; Crank-Nicolson for the viscous terms, implicit Euler for the
   split CH operator, so that every (kx, ky) pair needs the Helmholtz problems
   of `channel.wall_normal_solve` with
     g_om  = -(lap + beta) omega^n - (2 Re) AB(H_omega),
     g_w   = -(lap + beta) lap(w^n) - (2 Re) AB(H_w),
     g_phi = (Pe / (dt Ch^2)) (phi^n + dt AB(S_phi)),
   beta = 2 Re / dt, and the mean flow
     (D^2 - beta) U = -(D^2 + beta) U^n - 2 Re (AB(S_x(0)) + F), U(+-1) = 0
   (V likewise without the driving F = -dP/dx, here 1 in wall units).
   Each wall is no-slip (the conditions above) or free-slip (Sec. 2.1: w = 0
   and du/dz = dv/dz = 0, hence omega_z' = 0, w'' = 0 and U' = V' = 0 there).

Readings fixed here (the paper is silent): the momentum nonlinearity is taken
in divergence form (in the channel the Chebyshev products are aliased, so the
form is part of the discrete scheme); the state keeps every Chebyshev mode
(the tau solutions have full degree) and the 2/3 band in x and y; Re is the
friction Reynolds number Re_tau = 1/nu with u_tau = h = 1.

Arrays: physical [z][y][x] with z_j = cos(pi j / nc) (z_0 = +1); spectral band
[n][ky][kx] with kx = 0..Kx and ky = 0..Ky, -Ky..-1 (2 Ky + 1 entries).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import channel as ch


@dataclass
class ChannelParams:
    nx: int
    ny: int
    nc: int
    re: float           # Re_tau = 1 / nu
    we: float
    ch: float
    pe: float
    dt: float
    s: float = 0.0      # CH splitting coefficient; 0 selects sqrt(4 Pe / (Ch^2 dt))
    lx: float = 4.0 * math.pi
    ly: float = 2.0 * math.pi
    forcing: float = 1.0  # mean pressure gradient -dP/dx
    walls: tuple = ("noslip", "noslip")   # (top z = +1, bottom z = -1): "noslip" or "freeslip"

    @property
    def split_s(self) -> float:
        return self.s if self.s > 0.0 else math.sqrt(4.0 * self.pe / (self.ch ** 2 * self.dt))

    @property
    def capillary(self) -> float:
        return 3.0 / math.sqrt(8.0) * self.ch / self.we

    @property
    def beta(self) -> float:
        return 2.0 * self.re / self.dt

    def ch_factors(self):
        """a, b with a + b = s and a b = Pe / (dt Ch^2) (real when s^2 >= 4 a b)."""
        s = self.split_s
        p = self.pe / (self.dt * self.ch ** 2)
        d = math.sqrt(max(s * s - 4.0 * p, 0.0))
        return 0.5 * (s - d), 0.5 * (s + d)


def cut(n: int) -> int:
    return (n - 1) // 3


def zcut(nc: int) -> int:
    """Largest Chebyshev mode kept in the products: the 2/3 rule of the 2 nc extension."""
    return (2 * nc - 1) // 3


def band_wavenumbers(p: ChannelParams):
    """kx (Hx entries) and ky (Cy entries, band order) as physical wavenumbers."""
    kxm = cut(p.nx)
    kym = cut(p.ny)
    mx = np.arange(kxm + 1)
    my = np.concatenate([np.arange(kym + 1), np.arange(-kym, 0)])
    return mx * (2.0 * math.pi / p.lx), my * (2.0 * math.pi / p.ly)


def band_shape(p: ChannelParams):
    return (p.nc + 1, 2 * cut(p.ny) + 1, cut(p.nx) + 1)


# ---------------------------------------------------------------------------
# transforms between the collocation grid and the spectral band
# ---------------------------------------------------------------------------

def _ky_positions(p: ChannelParams):
    kym = cut(p.ny)
    return np.concatenate([np.arange(kym + 1), p.ny - np.arange(kym, 0, -1)])


def to_spectral(f: np.ndarray, p: ChannelParams) -> np.ndarray:
    """Physical [nc+1][ny][nx] -> band [nc+1][Cy][Hx] (Fourier with 1/(nx ny),
    Chebyshev coefficients in z); modes outside the x/y band are dropped."""
    fh = np.fft.rfft(f, axis=2, norm="forward")
    fh = np.fft.fft(fh, axis=1, norm="forward")
    fh = ch.values_to_coeffs(fh, axis=0)
    return fh[:, _ky_positions(p), : cut(p.nx) + 1]


def to_physical(a: np.ndarray, p: ChannelParams) -> np.ndarray:
    """Band [nc+1][Cy][Hx] -> physical [nc+1][ny][nx]."""
    full = np.zeros((p.nc + 1, p.ny, p.nx // 2 + 1), dtype=complex)
    full[:, _ky_positions(p), : cut(p.nx) + 1] = a
    v = ch.coeffs_to_values(full, axis=0)
    v = np.fft.ifft(v, axis=1, norm="forward")
    v[:, :, 0] = v[:, :, 0].real   # kx = 0 (and Nyquist) taken as real
    return np.fft.irfft(v, n=p.nx, axis=2, norm="forward")


def dz(a: np.ndarray) -> np.ndarray:
    """Chebyshev derivative along axis 0."""
    return ch.deriv(a, axis=0)


def lap(a: np.ndarray, p: ChannelParams) -> np.ndarray:
    kx, ky = band_wavenumbers(p)
    k2 = ky[:, None] ** 2 + kx[None, :] ** 2
    return dz(dz(a)) - k2[None] * a


# ---------------------------------------------------------------------------
# state
# ---------------------------------------------------------------------------

def init_state(u, v, w, phi, p: ChannelParams) -> dict:
    """Spectral state from the physical fields on the collocation grid."""
    kx, ky = band_wavenumbers(p)
    uh, vh, wh, ph = (to_spectral(np.asarray(x, float), p) for x in (u, v, w, phi))
    om = 1j * kx[None, None, :] * vh - 1j * ky[None, :, None] * uh
    mean = np.stack([uh[:, 0, 0], vh[:, 0, 0]])
    wh = wh.copy()
    wh[:, 0, 0] = 0.0
    om[:, 0, 0] = 0.0
    shp = band_shape(p)
    return dict(om=om, w=wh, phi=ph, mean=mean,
                h_om=np.zeros(shp, complex), h_w=np.zeros(shp, complex), h_phi=np.zeros(shp, complex),
                h_mean=np.zeros((2, p.nc + 1), complex), nstep=0)


def velocities(st: dict, p: ChannelParams):
    """u, v (band) from continuity and the definition of omega_z; the mean line
    carries U, V."""
    kx, ky = band_wavenumbers(p)
    KX = kx[None, None, :]
    KY = ky[None, :, None]
    k2 = KX ** 2 + KY ** 2
    k2s = np.where(k2 == 0.0, 1.0, k2)
    dw = dz(st["w"])
    u = 1j * (KX * dw + KY * st["om"]) / k2s
    v = 1j * (KY * dw - KX * st["om"]) / k2s
    u[:, 0, 0] = st["mean"][0]
    v[:, 0, 0] = st["mean"][1]
    return u, v


def nonlinear(st: dict, p: ChannelParams):
    """(S_x, S_y, S_z, S_phi) of the state, band arrays (Sec. 2.2 items i-iii)."""
    kx, ky = band_wavenumbers(p)
    KX = kx[None, None, :]
    KY = ky[None, :, None]
    u, v = velocities(st, p)
    w, ph = st["w"], st["phi"]
    U, Vv, W, PH = (to_physical(x, p) for x in (u, v, w, ph))
    GX = to_physical(1j * KX * ph, p)
    GY = to_physical(1j * KY * ph, p)
    GZ = to_physical(dz(ph), p)
    cs = p.capillary
    g2 = GX * GX + GY * GY + GZ * GZ
    T = {
        "xx": -U * U + cs * (g2 - GX * GX), "yy": -Vv * Vv + cs * (g2 - GY * GY), "zz": -W * W + cs * (g2 - GZ * GZ),
        "xy": -U * Vv - cs * GX * GY, "xz": -U * W - cs * GX * GZ, "yz": -Vv * W - cs * GY * GZ,
    }
    A = U * GX + Vv * GY + W * GZ
    C = PH * PH * PH
    kz = zcut(p.nc)

    def fwd(f):
        a = to_spectral(f, p)
        a[kz + 1:] = 0.0
        return a

    Th = {k: fwd(x) for k, x in T.items()}
    ah, chh = fwd(A), fwd(C)
    sx = 1j * KX * Th["xx"] + 1j * KY * Th["xy"] + dz(Th["xz"])
    sy = 1j * KX * Th["xy"] + 1j * KY * Th["yy"] + dz(Th["yz"])
    sz = 1j * KX * Th["xz"] + 1j * KY * Th["yz"] + dz(Th["zz"])
    sphi = -ah + lap(chh, p) / p.pe - (1.0 + p.split_s * p.ch ** 2) / p.pe * lap(ph, p)
    return sx, sy, sz, sphi


def step(st: dict, p: ChannelParams, lines=None) -> dict:
    """One step from time n.  `lines` (optional list of (iy, ix) band indices)
    restricts the wall-normal solves to those pairs (the other entries of the
    returned om, w, phi are NaN); the mean flow is always solved."""
    kx, ky = band_wavenumbers(p)
    KX = kx[None, None, :]
    KY = ky[None, :, None]
    k2 = KX ** 2 + KY ** 2
    sx, sy, sz, sphi = nonlinear(st, p)
    h_om = 1j * KX * sy - 1j * KY * sx
    h_w = -k2 * sz - dz(1j * KX * sx + 1j * KY * sy)
    h_mean = np.stack([sx[:, 0, 0], sy[:, 0, 0]])
    if st["nstep"] == 0:
        e_om, e_w, e_phi, e_mean = h_om, h_w, sphi, h_mean
    else:
        e_om = 1.5 * h_om - 0.5 * st["h_om"]
        e_w = 1.5 * h_w - 0.5 * st["h_w"]
        e_phi = 1.5 * sphi - 0.5 * st["h_phi"]
        e_mean = 1.5 * h_mean - 0.5 * st["h_mean"]
    beta = p.beta
    g_om = -(lap(st["om"], p) + beta * st["om"]) - 2.0 * p.re * e_om
    psi = lap(st["w"], p)
    g_w = -(lap(psi, p) + beta * psi) - 2.0 * p.re * e_w
    g_phi = p.pe / (p.dt * p.ch ** 2) * (st["phi"] + p.dt * e_phi)
    a, b = p.ch_factors()
    shp = band_shape(p)
    if lines is None:
        lines = [(iy, ix) for iy in range(shp[1]) for ix in range(shp[2])]
        om = np.zeros(shp, complex)
        w = np.zeros(shp, complex)
        ph = np.zeros(shp, complex)
    else:
        om = np.full(shp, np.nan + 0j)
        w = np.full(shp, np.nan + 0j)
        ph = np.full(shp, np.nan + 0j)
    iy = np.array([l[0] for l in lines], dtype=int)
    ix = np.array([l[1] for l in lines], dtype=int)
    kk = kx[ix] ** 2 + ky[iy] ** 2
    # every (kx, ky) pair's problems, solved together (each line its own dense systems)
    r = ch.wall_normal_solve_lines(g_om[:, iy, ix], g_w[:, iy, ix], g_phi[:, iy, ix], kx[ix], ky[iy],
                                   kk + beta, kk + a, kk + b, p.walls)
    om[:, iy, ix] = r["omega"]
    w[:, iy, ix] = r["w"]
    ph[:, iy, ix] = r["phi"]
    d2 = dz(dz(st["mean"].T)).T
    mean = np.zeros((2, p.nc + 1), complex)
    drive = np.zeros(p.nc + 1)
    drive[0] = p.forcing          # the constant -dP/dx is the coefficient of T_0
    for c in range(2):
        g = -(d2[c] + beta * st["mean"][c]) - 2.0 * p.re * (e_mean[c] + (drive if c == 0 else 0.0))
        mean[c] = ch.helmholtz(g, beta, ch.wall_kinds(p.walls))
    return dict(om=om, w=w, phi=ph, mean=mean, h_om=h_om, h_w=h_w, h_phi=sphi, h_mean=h_mean,
                nstep=st["nstep"] + 1)


def run(st: dict, p: ChannelParams, nsteps: int) -> dict:
    for _ in range(nsteps):
        st = step(st, p)
    return st


# ---------------------------------------------------------------------------
# diagnostics (volume averages over [0, Lx) x [0, Ly) x [-1, 1])
# ---------------------------------------------------------------------------

def cheb_integrals(nc: int) -> np.ndarray:
    """int_{-1}^{1} T_n(z) dz = 2 / (1 - n^2) for even n, 0 for odd n."""
    n = np.arange(nc + 1)
    out = np.zeros(nc + 1)
    ev = n % 2 == 0
    out[ev] = 2.0 / (1.0 - n[ev].astype(float) ** 2)
    return out


def cheb_gram(nc: int) -> np.ndarray:
    """G[m, n] = int_{-1}^{1} T_m T_n dz = (I(m + n) + I(|m - n|)) / 2 with
    I(k) = int T_k (the product rule T_m T_n = (T_{m+n} + T_{|m-n|}) / 2)."""
    I = cheb_integrals(2 * nc)
    m = np.arange(nc + 1)
    return 0.5 * (I[m[:, None] + m[None, :]] + I[np.abs(m[:, None] - m[None, :])])


def local_spacing(nc: int) -> np.ndarray:
    """Grid spacing at each CGL point: (z_{j-1} - z_{j+1}) / 2 inside, the one-sided
    spacing at the two walls."""
    z = ch.cgl(nc)
    dz_ = np.empty(nc + 1)
    dz_[1:-1] = 0.5 * (z[:-2] - z[2:])
    dz_[0] = z[0] - z[1]
    dz_[-1] = z[-2] - z[-1]
    return dz_


def diagnostics(st: dict, p: ChannelParams) -> dict:
    """Volume averages of the state (eqs. cont and CHE):
      mean_phi = <phi> = (1/2) int phi_00(z) dz (the mean line, kx = ky = 0);
      ke    = 1/2 <|u|^2>, grad2 = <|grad phi|^2>: Parseval in x and y (half-spectrum
              weights 1 at kx = 0, 2 otherwise) and the exact Chebyshev integral
              (1/2) int conj(f) g dz = (1/2) a^H G b in z (cheb_gram);
      max_div = max |i kx u + i ky v + D w| over the band (continuity);
      nonfinite = number of non-finite entries of the state and mean lines;
      cfl   = dt max (|u| / dx + |v| / dy + |w| / dz_j) over the collocation grid,
              dx = Lx / nx, dy = Ly / ny, dz_j the local spacing (local_spacing)."""
    kx, ky = band_wavenumbers(p)
    KX = kx[None, None, :]
    KY = ky[None, :, None]
    u, v = velocities(st, p)
    w, ph = st["w"], st["phi"]
    G = cheb_gram(p.nc)
    wx = np.where(kx == 0.0, 1.0, 2.0)[None, :]

    def avg_sq(a):
        """<|f|^2> of a band field a [n][ky][kx]."""
        per_line = np.einsum("mij,mn,nij->ij", np.conj(a), G, a).real
        return 0.5 * float(np.sum(wx * per_line))

    ke = 0.5 * (avg_sq(u) + avg_sq(v) + avg_sq(w))
    grad2 = avg_sq(1j * KX * ph) + avg_sq(1j * KY * ph) + avg_sq(dz(ph))
    mean_phi = 0.5 * float(np.dot(cheb_integrals(p.nc), ph[:, 0, 0].real))
    div = 1j * KX * u + 1j * KY * v + dz(w)
    arrays = [st["om"], st["w"], st["phi"], st["mean"]]
    nonfinite = int(sum(np.count_nonzero(~np.isfinite(a)) for a in arrays))
    U, V, W = (to_physical(x, p) for x in (u, v, w))
    dzl = local_spacing(p.nc)[:, None, None]
    speed = np.abs(U) / (p.lx / p.nx) + np.abs(V) / (p.ly / p.ny) + np.abs(W) / dzl
    return dict(mean_phi=mean_phi, ke=ke, grad2=grad2, max_div=float(np.max(np.abs(div))),
                nonfinite=nonfinite, cfl=float(p.dt * np.max(speed)))
