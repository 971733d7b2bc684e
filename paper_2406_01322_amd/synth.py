"""Seeded synthetic inputs for the coupled Navier-Stokes + Cahn-Hilliard step.

This module is shared by the CPU oracle tests, the GPU tests and the benchmark.
It only *draws* inputs; it contains none of the method's arithmetic (no
dealiasing rule, no projection, no time stepping).  Every generator returns
plain float64 host arrays in physical space with layout ``[z][y][x]`` (x
fastest) on the triply periodic box ``[0, 2*pi)^3``.

Inputs stand in for the paper's drop-laden turbulence (Sec. 4): a random-phase
solenoidal velocity with energy spectrum E(k) ~ k^4 exp(-2 (k/k0)^2) and
spherical drops with the equilibrium tanh interface profile of Sec. 2.1.1
(equation ``width``).  The velocity is made solenoidal by taking the curl of a
random vector potential, which is input synthesis, not the method's Leray
projection.
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft

_WORKERS = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else 1))

TWO_PI = 2.0 * math.pi


def grid_coords(n: int, length: float = TWO_PI) -> np.ndarray:
    """Uniform collocation points x_j = j L / n, j = 0..n-1."""
    return np.arange(n, dtype=np.float64) * (length / n)


def _int_wavenumbers(n: int):
    kz = np.fft.fftfreq(n, 1.0 / n)
    ky = np.fft.fftfreq(n, 1.0 / n)
    kx = np.fft.rfftfreq(n, 1.0 / n)
    return np.meshgrid(kz, ky, kx, indexing="ij")


def random_velocity(n: int, rng: np.random.Generator, k0: float = 4.0,
                    u_rms: float = 1.0, kmax: float | None = None) -> np.ndarray:
    """Random-phase solenoidal velocity, shape (3, n, n, n), float64.

    A white-noise vector potential A is given the shell amplitude
    |A(k)| ~ exp(-(k/k0)^2) (random phases from the noise), u = curl A is
    formed spectrally, modes with |k| > kmax (default n/3 - 1, a sphere) are
    dropped, and the field is scaled so that sqrt(<|u|^2>/3) = u_rms.
    """
    if kmax is None:
        kmax = n / 3.0 - 1.0
    KZ, KY, KX = _int_wavenumbers(n)
    kmag = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    noise = rng.standard_normal((3, n, n, n))
    a_hat = scipy.fft.rfftn(noise, axes=(1, 2, 3), workers=_WORKERS)
    mag = np.abs(a_hat)
    mag[mag == 0.0] = 1.0
    amp = np.exp(-(kmag / k0) ** 2)
    amp[kmag > kmax] = 0.0
    amp[kmag == 0.0] = 0.0
    a_hat = a_hat / mag * amp
    ax, ay, az = a_hat[0], a_hat[1], a_hat[2]
    # curl in Fourier space: (i k) x A, components ordered (x, y, z)
    ux = 1j * (KY * az - KZ * ay)
    uy = 1j * (KZ * ax - KX * az)
    uz = 1j * (KX * ay - KY * ax)
    u = np.stack([scipy.fft.irfftn(c, s=(n, n, n), axes=(0, 1, 2), workers=_WORKERS)
                  for c in (ux, uy, uz)])
    rms = math.sqrt(float(np.mean(u * u)))
    if rms > 0.0:
        u *= u_rms / rms
    return u


def drop_centres(rng: np.random.Generator, ndrops: int, radius: float,
                 ch: float, length: float = TWO_PI, max_tries: int = 200000):
    """Seeded rejection sampling of non-overlapping drop centres.

    Two centres are accepted when their minimum-image distance is at least
    2 R + 8 sqrt(2) Ch, so interfaces stay several widths apart.
    """
    gap = 2.0 * radius + 8.0 * math.sqrt(2.0) * ch
    centres: list[np.ndarray] = []
    tries = 0
    while len(centres) < ndrops:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place %d drops of radius %g" % (ndrops, radius))
        c = rng.uniform(0.0, length, size=3)
        ok = True
        for d in centres:
            delta = np.abs(c - d)
            delta = np.minimum(delta, length - delta)
            if float(np.sqrt(np.sum(delta ** 2))) < gap:
                ok = False
                break
        if ok:
            centres.append(c)
    return np.array(centres)


def drops_phi(n: int, centres: np.ndarray, radius: float, ch: float,
              length: float = TWO_PI) -> np.ndarray:
    """Phase field of spherical drops, +1 inside, -1 outside.

    phi = max_i tanh((R - d_i) / (sqrt(2) Ch)), d_i the minimum-image
    distance to centre i (equilibrium profile of Sec. 2.1.1).
    """
    x = grid_coords(n, length)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    phi = np.full((n, n, n), -1.0)
    w = math.sqrt(2.0) * ch
    for c in np.atleast_2d(centres):
        dz = np.abs(Z - c[2]); dz = np.minimum(dz, length - dz)
        dy = np.abs(Y - c[1]); dy = np.minimum(dy, length - dy)
        dx = np.abs(X - c[0]); dx = np.minimum(dx, length - dx)
        d = np.sqrt(dx * dx + dy * dy + dz * dz)
        phi = np.maximum(phi, np.tanh((radius - d) / w))
    return phi


# ---------------------------------------------------------------------------
# named workloads (box)
# ---------------------------------------------------------------------------

def box_case(name: str):
    """Return (params dict, u (3,n,n,n), phi (n,n,n)) for a named box workload.

    ``single_drop_32``: 32^3, Re=100, We=1, Ch=0.05, Pe=1/Ch, dt=1e-3, one
    centred drop of radius 0.8, seed 1.
    ``drops16_128``: 128^3, Re=300, We=1, Ch=0.025, Pe=1/Ch, dt=5e-4, 16 drops
    of radius 0.4 at seeded non-overlapping centres, seed 2.
    Smaller variants (``drops4_48``, ``drops2_64``) keep the second recipe on
    grids the oracle steps in well under a second.
    """
    if name == "single_drop_32":
        n, seed = 32, 1
        p = dict(n=n, re=100.0, we=1.0, ch=0.05, pe=20.0, dt=1e-3)
        rng = np.random.default_rng(seed)
        u = random_velocity(n, rng, k0=4.0)
        c = np.array([[math.pi, math.pi, math.pi]])
        phi = drops_phi(n, c, 0.8, p["ch"])
        return p, u, phi
    recipes = {
        "drops16_128": (128, 2, 16, 0.4, 300.0, 1.0, 0.025, 5e-4),
        "drops2_64": (64, 12, 2, 0.6, 300.0, 1.0, 0.05, 5e-4),
        "drops4_48": (48, 11, 4, 0.5, 200.0, 2.0, 0.06, 5e-4),
        "drops3_96": (96, 13, 3, 0.5, 300.0, 1.0, 0.04, 5e-4),
        "drops2_256": (256, 14, 2, 0.5, 300.0, 1.0, 0.02, 2.5e-4),
    }
    if name not in recipes:
        raise KeyError(name)
    n, seed, nd, r, re, we, ch, dt = recipes[name]
    p = dict(n=n, re=re, we=we, ch=ch, pe=1.0 / ch, dt=dt)
    rng = np.random.default_rng(seed)
    u = random_velocity(n, rng, k0=4.0)
    c = drop_centres(rng, nd, r, ch)
    phi = drops_phi(n, c, r, ch)
    return p, u, phi


def batch_cases(nbox: int = 96, seed: int = 4, sizes=(32, 48, 64, 96)):
    """Independent boxes of uneven size: per box, drawn in this order, N from
    `sizes`, the number of drops in [1, 8], Re ~ U[50, 400], We ~ U[0.5, 5];
    Ch = 0.05, drop radius 0.4, Pe = 1/Ch, dt = 1e-3, k0 = 4.
    Returns a list of (params, u, phi)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nbox):
        n = int(rng.choice(sizes))
        nd = int(rng.integers(1, 9))
        re = float(rng.uniform(50.0, 400.0))
        we = float(rng.uniform(0.5, 5.0))
        ch = 0.05
        p = dict(n=n, re=re, we=we, ch=ch, pe=1.0 / ch, dt=1e-3)
        u = random_velocity(n, rng, k0=4.0)
        c = drop_centres(rng, nd, 0.4, ch)
        phi = drops_phi(n, c, 0.4, ch)
        out.append((p, u, phi))
    return out


# ---------------------------------------------------------------------------
# the channel: x, y periodic (lengths lx, ly), z in [-1, 1] at the
# Chebyshev-Gauss-Lobatto points z_j = cos(pi j / nc)
# ---------------------------------------------------------------------------

def channel_grid(nx: int, ny: int, nc: int, lx: float, ly: float):
    """Coordinates X, Y, Z of shape (nc+1, ny, nx)."""
    z = np.cos(math.pi * np.arange(nc + 1) / nc)
    x = grid_coords(nx, lx)
    y = grid_coords(ny, ly)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def channel_perturbation(X, Y, Z, lx: float, ly: float, rng: np.random.Generator, mmax: int, amp: float):
    """Divergence-free velocity vanishing at the walls with its normal derivative:
    the curl of A = (f(z) r_x(x, y), f(z) r_y(x, y), 0), f = (1 - z^2)^2, with r_x,
    r_y random-phase sums of the modes 1 <= |m_x|, |m_y| <= mmax; scaled so that the
    largest rms over an (x, y) plane of the streamwise component is `amp`."""
    f = (1.0 - Z ** 2) ** 2
    fp = -4.0 * Z * (1.0 - Z ** 2)
    X2, Y2 = X[0], Y[0]          # r_x, r_y depend on (x, y) only
    rx = np.zeros_like(X2)
    ry = np.zeros_like(X2)
    drx_dy = np.zeros_like(X2)
    dry_dx = np.zeros_like(X2)
    for mx in range(-mmax, mmax + 1):
        for my in range(-mmax, mmax + 1):
            if abs(mx) < 1 or abs(my) < 1:
                continue
            kx, ky = TWO_PI * mx / lx, TWO_PI * my / ly
            ax, ay = rng.standard_normal(2)
            px, py = rng.uniform(0.0, TWO_PI, 2)
            sx = kx * X2 + ky * Y2 + px
            sy = kx * X2 + ky * Y2 + py
            rx += ax * np.cos(sx)
            drx_dy += -ax * ky * np.sin(sx)
            ry += ay * np.cos(sy)
            dry_dx += -ay * kx * np.sin(sy)
    u = -fp * ry[None]
    v = fp * rx[None]
    w = f * (dry_dx - drx_dy)[None]
    scale = amp / np.max(np.sqrt(np.mean(u * u, axis=(1, 2))))
    return u * scale, v * scale, w * scale


def channel_drops(X, Y, Z, lx: float, ly: float, rng: np.random.Generator, ndrops: int, radius: float, ch: float):
    """phi = max_i tanh((R - d_i)/(sqrt(2) Ch)), d_i the distance to centre i with
    periodic images in x and y; centres drawn uniformly with |z_c| <= 1 - R -
    4 sqrt(2) Ch and pairwise distances >= 2R + 8 sqrt(2) Ch (rejection)."""
    zmax = 1.0 - radius - 4.0 * math.sqrt(2.0) * ch
    sep = 2.0 * radius + 8.0 * math.sqrt(2.0) * ch
    cs = []
    tries = 0
    while len(cs) < ndrops:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place the drops")
        c = np.array([rng.uniform(0, lx), rng.uniform(0, ly), rng.uniform(-zmax, zmax)])
        ok = True
        for d in cs:
            dx = abs(c[0] - d[0]); dx = min(dx, lx - dx)
            dy = abs(c[1] - d[1]); dy = min(dy, ly - dy)
            if math.sqrt(dx * dx + dy * dy + (c[2] - d[2]) ** 2) < sep:
                ok = False
                break
        if ok:
            cs.append(c)
    phi = np.full(X.shape, -1.0)
    w = math.sqrt(2.0) * ch
    # beyond R + 20 w from a centre, tanh((R - d)/w) rounds to -1 in FP64: only
    # the points inside that box are evaluated
    reach = radius + 20.0 * w
    x1, y1, z1 = X[0, 0, :], Y[0, :, 0], Z[:, 0, 0]
    for c in cs:
        dx = np.abs(x1 - c[0]); dx = np.minimum(dx, lx - dx)
        dy = np.abs(y1 - c[1]); dy = np.minimum(dy, ly - dy)
        dz = np.abs(z1 - c[2])
        ix, iy, iz = np.nonzero(dx < reach)[0], np.nonzero(dy < reach)[0], np.nonzero(dz < reach)[0]
        sub = np.ix_(iz, iy, ix)
        d = np.sqrt(dx[ix][None, None, :] ** 2 + dy[iy][None, :, None] ** 2 + dz[iz][:, None, None] ** 2)
        phi[sub] = np.maximum(phi[sub], np.tanh((radius - d) / w))
    return phi


def channel_case(name: str):
    """(params, u, v, w, phi): laminar profile U = Re (1 - z^2)/2 (wall units,
    -dP/dx = 1) plus a wall-bounded random perturbation of 10% of the centreline
    velocity, and drops.  params: nx, ny, nc, lx, ly, re, we, ch, pe, dt.
      chan_small: 16 x 12 x 17, Re_tau 20, 2 drops R = 0.4, Ch 0.1 (seed 11);
      chan_mid:   32 x 24 x 33, Re_tau 50, 4 drops R = 0.3, Ch 0.05 (seed 12);
      chan_256:   256 x 128 x 129 on 4 pi x 2 pi x 2, Re_tau 150, 64 drops R = 0.2,
                  Ch 0.02, We 3, Pe 50, dt 1e-4 (seed 3).
    Single-phase cases (no drops, phi = 0; params carry single_phase=True and
    placeholder we = ch = pe = 1, which do not enter a step with phi = 0):
      chan_sp_small: 16 x 12 x 257, Re_tau 150, dt 1e-4 (seed 13);
      chan_sp_256:   256 x 256 x 257 on 4 pi x 2 pi x 2, Re_tau 150, dt 1e-4 (seed 7),
                     the grid of the single-phase timing runs of Sec. 3.4."""
    table = {
        "chan_small": (dict(nx=16, ny=12, nc=16, re=20.0, we=1.0, ch=0.1, pe=10.0, dt=1e-3), 2, 0.4, 11),
        "chan_mid": (dict(nx=32, ny=24, nc=32, re=50.0, we=2.0, ch=0.05, pe=20.0, dt=5e-4), 4, 0.3, 12),
        "chan_256": (dict(nx=256, ny=128, nc=128, re=150.0, we=3.0, ch=0.02, pe=50.0, dt=1e-4), 64, 0.2, 3),
        "chan_sp_small": (dict(nx=16, ny=12, nc=256, re=150.0, we=1.0, ch=1.0, pe=1.0, dt=1e-4), 0, 0.0, 13),
        "chan_sp_256": (dict(nx=256, ny=256, nc=256, re=150.0, we=1.0, ch=1.0, pe=1.0, dt=1e-4), 0, 0.0, 7),
    }
    p, nd, radius, seed = table[name]
    p = dict(p, lx=4.0 * math.pi, ly=2.0 * math.pi)
    rng = np.random.default_rng(seed)
    X, Y, Z = channel_grid(p["nx"], p["ny"], p["nc"], p["lx"], p["ly"])
    mmax = min(4, (p["nx"] - 1) // 3, (p["ny"] - 1) // 3)
    uc = p["re"] / 2.0
    up, vp, wp = channel_perturbation(X, Y, Z, p["lx"], p["ly"], rng, mmax, 0.1 * uc)
    u = uc * (1.0 - Z ** 2) + up
    if nd == 0:
        p["single_phase"] = True
        return p, u, vp, wp, np.zeros_like(u)
    phi = channel_drops(X, Y, Z, p["lx"], p["ly"], rng, nd, radius, p["ch"])
    return p, u, vp, wp, phi


def band_limited_box(n: int, seed: int = 21):
    """u = curl A with A made of a few Fourier modes |k_i| <= 2, phi = -0.2 plus modes
    |k_i| <= 3, on the n^3 grid: every product the step forms (quadratic terms up to
    |k_i| = 5, phi^3 up to 9) is represented exactly from n = 32 up, and lies in the
    2/3 band there, so one step gives the same spectral state at every such n.  Each
    field is Re(sum_k c_k exp(i k.x)), synthesised by one inverse FFT."""
    rng = np.random.default_rng(seed)
    modes = [(kz, ky, kx) for kz in range(-2, 3) for ky in range(-2, 3) for kx in range(0, 3)
             if (kz, ky, kx) != (0, 0, 0)]
    U = np.zeros((4, n, n, n), complex)
    for kz, ky, kx in modes[::3]:
        k = (kx, ky, kz)
        ab = [0.1 * rng.standard_normal(2) for _ in range(3)]   # A_c = a_c cos(k.x) + b_c sin(k.x)
        # u_c = d_j1 A_c1 - d_j2 A_c2 with d_j A_c = k_j (b_c cos - a_c sin)
        for c, (j1, c1), (j2, c2) in ((0, (1, 2), (2, 1)), (1, (2, 0), (0, 2)), (2, (0, 1), (1, 0))):
            cc = k[j1] * ab[c1][1] - k[j2] * ab[c2][1]
            ss = -(k[j1] * ab[c1][0] - k[j2] * ab[c2][0])
            U[c, kz % n, ky % n, kx % n] += cc - 1j * ss      # Re((cc - i ss) e^{i k.x})
    for (kz, ky, kx), a in (((0, 0, 0), -0.2), ((0, 2, 1), 0.3), ((3, -1, 0), -0.2j), ((-3, 0, 2), 0.1)):
        U[3, kz % n, ky % n, kx % n] += a
    f = np.real(np.fft.ifftn(U, axes=(1, 2, 3))) * float(n) ** 3
    return f[:3], f[3]
