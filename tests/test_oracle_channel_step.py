"""Pins of the channel-step oracle (oracle/channel_step.py) against closed forms and
invariants of the equations (Sec. 2.1-2.2), independent of the oracle's own code.

* laminar Poiseuille flow U = Re (1 - z^2) / 2 with a single phase is a fixed point
  (pins the driving -dP/dx = 1, the mean-flow Crank-Nicolson update, beta = 2 Re/dt);
* a cos(pi z / 2) perturbation of U decays by the Crank-Nicolson factor of its
  eigenvalue -pi^2/4 (pins the mean viscous term);
* a small wall-normal vorticity mode cos(pi z / 2) cos(kx x) decays by the
  Crank-Nicolson factor of -(kx^2 + pi^2/4) (pins the omega equation);
* a small wall-normal velocity mode converges at second order in dt and decays
  (pins the w equation's explicit part against inconsistent variants);
* a flat interface tanh(z / (sqrt 2 Ch)) parallel to the walls is a CH equilibrium
  and drives no flow (pins the split CH operator and the Korteweg stress);
* a small phase mode cos(pi z) on the mean line follows the IE/AB1 amplification
  (1 + dt (1 + s Ch^2) pi^2 / Pe) / (1 + dt (Ch^2/Pe)(pi^4 + s pi^2));
* u, v recovered from omega_z and w satisfy continuity exactly;
* on low-degree fields that the bands represent exactly, the nonlinear terms S_i,
  S_phi and the forcings H_omega = (curl S)_z and H_w = lap_h S_z - d_z(d_x S_x +
  d_y S_y) equal the continuous operators applied by the product rule (sympy);
* from rest, one small step under capillary forcing gives omega = dt H_omega and
  lap(w) = dt H_w in the interior.
Ten planted mistakes in the oracle (signs, factors of 2, the constant forcing on
every Chebyshev coefficient) each fail one of these.
"""
import math

import numpy as np

from oracle import channel as ch
from oracle import channel_step as cs


def _grid(p):
    z = ch.cgl(p.nc)
    x = np.arange(p.nx) * p.lx / p.nx
    y = np.arange(p.ny) * p.ly / p.ny
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return z, Z, Y, X


def _params(**kw):
    d = dict(nx=8, ny=8, nc=16, re=10.0, we=1.0, ch=0.1, pe=10.0, dt=1e-2)
    d.update(kw)
    return cs.ChannelParams(**d)


def test_laminar_poiseuille_is_a_fixed_point():
    p = _params()
    z, Z, Y, X = _grid(p)
    u = p.re * (1 - Z ** 2) / 2
    zero = np.zeros_like(u)
    st0 = cs.init_state(u, zero, zero, -np.ones_like(u), p)
    st = cs.run(st0, p, 3)
    assert np.max(np.abs(st["mean"][0] - st0["mean"][0])) < 1e-13 * np.max(np.abs(st0["mean"][0]))
    assert np.max(np.abs(st["mean"][1])) == 0.0
    assert np.max(np.abs(st["om"])) == 0.0 and np.max(np.abs(st["w"])) == 0.0
    assert np.max(np.abs(st["phi"] - st0["phi"])) < 1e-13


def test_open_channel_profile_is_a_fixed_point():
    """A free-slip top wall over a no-slip bottom wall (Sec. 2.1): the laminar profile
    U = Re (1 + z)(3 - z) / 2 solves U'' = -Re with U(-1) = 0 and U'(+1) = 0, and is a
    fixed point of the step."""
    p = _params(walls=("freeslip", "noslip"))
    z, Z, Y, X = _grid(p)
    u = p.re * (1 + Z) * (3 - Z) / 2
    zero = np.zeros_like(u)
    st0 = cs.init_state(u, zero, zero, -np.ones_like(u), p)
    st = cs.run(st0, p, 3)
    assert np.max(np.abs(st["mean"][0] - st0["mean"][0])) < 1e-12 * np.max(np.abs(st0["mean"][0]))
    # and the no-slip profile is not: it is accelerated at the free-slip wall
    st1 = cs.step(cs.init_state(p.re * (1 - Z ** 2) / 2, zero, zero, -np.ones_like(u), p), p)
    top = np.sum(st1["mean"][0])
    assert top.real > 1e-3 * p.re * p.dt


def test_mean_flow_crank_nicolson_decay():
    p = _params(nc=24)
    z, Z, Y, X = _grid(p)
    base = p.re * (1 - Z ** 2) / 2
    eps = 1e-3
    zero = np.zeros_like(base)
    st = cs.init_state(base + eps * np.cos(math.pi * Z / 2), zero, zero, -np.ones_like(base), p)
    st1 = cs.step(st, p)
    a = (1.0 / p.re) * p.dt * (math.pi ** 2 / 4) / 2
    r = (1 - a) / (1 + a)
    want = cs.to_spectral(base + eps * r * np.cos(math.pi * Z / 2), p)[:, 0, 0]
    assert np.max(np.abs(st1["mean"][0] - want)) < 1e-10 * eps


def test_wall_normal_vorticity_mode_decay():
    p = _params()
    z, Z, Y, X = _grid(p)
    kx = 2 * math.pi / p.lx
    eps = 1e-8
    v = eps * np.cos(math.pi * Z / 2) * np.cos(kx * X)   # w = 0, div u = 0, omega = dv/dx
    zero = np.zeros_like(v)
    st = cs.init_state(zero, v, zero, -np.ones_like(v), p)
    st1 = cs.step(st, p)
    a = (1.0 / p.re) * p.dt * (kx ** 2 + math.pi ** 2 / 4) / 2
    r = (1 - a) / (1 + a)
    assert np.max(np.abs(st1["om"] - r * st["om"])) < 1e-12 * np.max(np.abs(st["om"]))


def _w_mode(dt, T=0.04):
    p = _params(nc=24, dt=dt, forcing=0.0)
    z, Z, Y, X = _grid(p)
    ky = 2 * math.pi / p.ly
    eps = 1e-8
    w = eps * (1 - Z ** 2) ** 2 * np.cos(ky * Y)
    v = eps * 4 * Z * (1 - Z ** 2) * np.sin(ky * Y) / ky      # continuity: dv/dy = -dw/dz
    st0 = cs.init_state(np.zeros_like(w), v, w, -np.ones_like(w), p)
    st = cs.run(st0, p, int(round(T / dt)))
    return st0["w"][:, 1, 0] / eps, st["w"][:, 1, 0] / eps


def test_wall_normal_velocity_mode_converges_at_second_order():
    w0, a = _w_mode(0.01)
    _, b = _w_mode(0.005)
    _, c = _w_mode(0.0025)
    ratio = np.linalg.norm(a - b) / np.linalg.norm(b - c)
    assert 2.8 < ratio < 4.5, ratio
    # viscous decay, no change of sign
    assert np.linalg.norm(c) < np.linalg.norm(w0)
    assert np.real(np.vdot(c, w0)) > 0.9 * np.linalg.norm(c) * np.linalg.norm(w0)


def test_flat_interface_is_an_equilibrium_without_flow():
    p = _params(nx=4, ny=4, nc=128, dt=1e-3, forcing=0.0)
    z, Z, Y, X = _grid(p)
    phi = np.tanh(Z / (math.sqrt(2) * p.ch))
    zero = np.zeros_like(phi)
    st = cs.init_state(zero, zero, zero, phi, p)
    st1 = cs.step(st, p)
    assert np.max(np.abs(st1["phi"] - st["phi"])) < 2e-6
    assert np.max(np.abs(st1["mean"])) < 1e-14
    assert np.max(np.abs(st1["om"])) < 1e-14 and np.max(np.abs(st1["w"])) < 1e-14


def test_phase_mode_follows_the_ie_ab1_amplification():
    p = _params(nc=32, dt=1e-3)
    z, Z, Y, X = _grid(p)
    eps = 1e-6
    phi = eps * np.cos(math.pi * Z)          # phi' = phi''' = 0 at the walls
    zero = np.zeros_like(phi)
    st = cs.init_state(zero, zero, zero, phi, p)
    st1 = cs.step(st, p)
    lam, s = math.pi ** 2, p.split_s
    g = (1 + p.dt * (1 + s * p.ch ** 2) * lam / p.pe) / (1 + p.dt * p.ch ** 2 / p.pe * (lam ** 2 + s * lam))
    assert np.max(np.abs(st1["phi"] - g * st["phi"])) < 1e-12 * eps


def test_recovered_velocity_satisfies_continuity():
    p = _params(nx=12, ny=8, nc=16)
    rng = np.random.default_rng(3)
    shp = cs.band_shape(p)
    st = cs.init_state(*(np.zeros((p.nc + 1, p.ny, p.nx)) for _ in range(3)), np.zeros((p.nc + 1, p.ny, p.nx)), p)
    st["om"] = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    st["w"] = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    st["om"][:, 0, 0] = 0
    st["w"][:, 0, 0] = 0
    u, v = cs.velocities(st, p)
    kx, ky = cs.band_wavenumbers(p)
    div = 1j * kx[None, None, :] * u + 1j * ky[None, :, None] * v + cs.dz(st["w"])
    div[:, 0, 0] = 0
    assert np.max(np.abs(div)) < 1e-12 * np.max(np.abs(cs.dz(st["w"])))
    om = 1j * kx[None, None, :] * v - 1j * ky[None, :, None] * u
    om[:, 0, 0] = 0
    assert np.max(np.abs(om - st["om"])) < 1e-12 * np.max(np.abs(st["om"]))


# ---------------------------------------------------------------------------
# nonlinear terms and their assembly against the continuous operators
# (product rule by sympy on low-degree fields that the 2/3 bands represent
# exactly)
# ---------------------------------------------------------------------------

def _analytic_case(with_velocity=True, nc=16, dt=1e-3):
    sp = __import__("sympy")
    x, y, z = sp.symbols("x y z", real=True)
    p = _params(nx=8, ny=8, nc=nc, dt=dt)
    kx, ky = 2 * sp.pi / p.lx, 2 * sp.pi / p.ly
    if with_velocity:
        C = (1 - z ** 2) ** 2
        u = (1 - z ** 2) - sp.diff(C, z) / kx * sp.sin(kx * x)
        w = C * sp.cos(kx * x)
        v = sp.Rational(1, 2) * z * (1 - z ** 2)
    else:
        u = v = w = sp.Integer(0)
    phi = sp.Rational(3, 10) * z + sp.Rational(1, 5) * (1 - z ** 2) * sp.cos(ky * y) \
        + sp.Rational(1, 10) * (1 - z ** 2) * sp.sin(kx * x)
    g = [sp.diff(phi, s) for s in (x, y, z)]
    vel = [u, v, w]
    cs_ = sp.Rational(3, 1) / sp.sqrt(8) * sp.Float(p.ch) / sp.Float(p.we)
    g2 = g[0] ** 2 + g[1] ** 2 + g[2] ** 2
    T = [[-vel[i] * vel[j] + cs_ * ((g2 if i == j else 0) - g[i] * g[j]) for j in range(3)] for i in range(3)]
    X = (x, y, z)
    S = [sum(sp.diff(T[i][j], X[j]) for j in range(3)) for i in range(3)]
    lapl = lambda f: sum(sp.diff(f, s, 2) for s in X)
    a = sum(vel[i] * g[i] for i in range(3))
    s_ = sp.Float(p.split_s)
    sphi = -a + lapl(phi ** 3) / p.pe - (1 + s_ * p.ch ** 2) / p.pe * lapl(phi)
    h_om = sp.diff(S[1], x) - sp.diff(S[0], y)
    h_w = sp.diff(S[2], x, 2) + sp.diff(S[2], y, 2) - sp.diff(sp.diff(S[0], x) + sp.diff(S[1], y), z)
    zz, Zg, Yg, Xg = _grid(p)

    def ev(f):
        return np.broadcast_to(np.asarray(sp.lambdify((x, y, z), f, "numpy")(Xg, Yg, Zg), float), Xg.shape)

    fields = [ev(f) for f in (u, v, w, phi)]
    st = cs.init_state(*fields, p)
    want = {k: cs.to_spectral(ev(f), p) for k, f in
            dict(sx=S[0], sy=S[1], sz=S[2], sphi=sphi, h_om=h_om, h_w=h_w).items()}
    return p, st, want


def test_nonlinear_terms_match_the_continuous_operators():
    p, st, want = _analytic_case()
    sx, sy, sz, sphi = cs.nonlinear(st, p)
    for k, got in dict(sx=sx, sy=sy, sz=sz, sphi=sphi).items():
        ref = want[k]   # phi^3 carries kx, ky = 3, outside the band: both sides keep the band
        assert np.max(np.abs(got - ref)) < 1e-11 * np.max(np.abs(ref)), k


def test_vorticity_and_wall_normal_forcing_assembly():
    p, st, want = _analytic_case()
    st1 = cs.step(st, p)
    for k in ("h_om", "h_w"):
        assert np.max(np.abs(st1[k] - want[k])) < 1e-11 * np.max(np.abs(want[k])), k


def test_small_step_response_to_capillary_forcing():
    """From rest, one small step gives omega = dt H_omega and lap(w) = dt H_w, up to
    O(nu dt k^2), away from the wall layers of width (2 Re / dt)^(-1/2), which nc = 64
    resolves (pins the weight of the explicit terms in both solves)."""
    p, st, want = _analytic_case(with_velocity=False, nc=64, dt=1e-3)
    st1 = cs.step(st, p)
    zz = ch.cgl(p.nc)
    inner = np.abs(zz) < 0.5
    om = cs.to_physical(st1["om"], p)[inner] / p.dt
    ref = cs.to_physical(want["h_om"], p)[inner]
    assert np.max(np.abs(om - ref)) < 1e-3 * np.max(np.abs(ref))
    lw = cs.to_physical(cs.lap(st1["w"], p), p)[inner] / p.dt
    ref = cs.to_physical(want["h_w"], p)[inner]
    assert np.max(np.abs(lw - ref)) < 1e-3 * np.max(np.abs(ref))


# ---------------------------------------------------------------------------
# diagnostics: volume averages of fields whose averages are known in closed form
# ---------------------------------------------------------------------------

def _diag_fields(p, A=3.0, B=0.7, c0=0.25):
    """A solenoidal velocity and a phase field with closed-form volume averages:
    U(z) = A (1 - z^2) (mean flow); u' = f'(z) sin(kx x), w = -kx f(z) cos(kx x) from
    the stream function f(z) sin(kx x), f = (1 - z^2)^2; v = B (1 - z^2) cos(kx x)
    (divergence free on its own); phi = c0 + z^2 / 2 + h(z) cos(kx x + ky y),
    h = z (1 - z^2)."""
    import sympy as sp
    zs = sp.symbols("z")
    f = (1 - zs ** 2) ** 2
    h = zs * (1 - zs ** 2)
    kx, ky = 2 * math.pi / p.lx, 2 * math.pi / p.ly
    z, Z, Y, X = _grid(p)
    lam = lambda e: sp.lambdify(zs, e, "numpy")
    fz, dfz, hz = lam(f)(Z), lam(sp.diff(f, zs))(Z), lam(h)(Z)
    u = A * (1 - Z ** 2) + dfz * np.sin(kx * X)
    w = -kx * fz * np.cos(kx * X)
    v = B * (1 - Z ** 2) * np.cos(kx * X)
    phi = c0 + 0.5 * Z ** 2 + hz * np.cos(kx * X + ky * Y)
    half = lambda e: float(sp.integrate(e, (zs, -1, 1))) / 2.0     # (1/2) int dz
    # <u^2> = <U^2> + <u'^2> (cross term averages to zero in x), <sin^2> = <cos^2> = 1/2
    ke = 0.5 * (A * A * half((1 - zs ** 2) ** 2) + 0.5 * half(sp.diff(f, zs) ** 2)
                + 0.5 * kx * kx * half(f ** 2) + 0.5 * B * B * half((1 - zs ** 2) ** 2))
    # grad phi = (-kx h sin, -ky h sin, z + h' cos): <|grad phi|^2>
    grad2 = (0.5 * (kx * kx + ky * ky) * half(h ** 2) + half(zs ** 2) + 0.5 * half(sp.diff(h, zs) ** 2))
    mean_phi = c0 + half(zs ** 2 / 2)
    # CFL on the grid, from the closed-form fields
    dzl = cs.local_spacing(p.nc)[:, None, None]
    cfl = p.dt * np.max(np.abs(u) / (p.lx / p.nx) + np.abs(v) / (p.ly / p.ny) + np.abs(w) / dzl)
    return (u, v, w, phi), dict(ke=ke, grad2=grad2, mean_phi=mean_phi, cfl=cfl)


def test_diagnostics_closed_form_volume_averages():
    """Pins the half-spectrum weights, the Chebyshev integrals (cheb_gram, cheb_integrals),
    the 1/2 of the z-average, the local spacing of the CFL number and the continuity
    check on fields whose averages sympy integrates exactly."""
    p = _params(nx=12, ny=8, nc=16, lx=4 * math.pi, ly=2 * math.pi, dt=1e-3)
    f, want = _diag_fields(p)
    st = cs.init_state(*f, p)
    d = cs.diagnostics(st, p)
    for k in ("ke", "grad2", "mean_phi", "cfl"):
        assert abs(d[k] - want[k]) <= 1e-13 * abs(want[k]), (k, d[k], want[k])
    assert d["max_div"] < 1e-13 and d["nonfinite"] == 0


def test_diagnostics_gram_matrix_and_nonfinite_count():
    """cheb_gram against numpy's Chebyshev product and integral, and the non-finite count."""
    from numpy.polynomial import chebyshev as npcheb
    nc = 9
    G = cs.cheb_gram(nc)
    for m in range(nc + 1):
        for n in range(nc + 1):
            em = np.zeros(m + 1)
            em[m] = 1.0
            en = np.zeros(n + 1)
            en[n] = 1.0
            integ = npcheb.chebint(npcheb.chebmul(em, en), lbnd=-1)
            assert abs(G[m, n] - npcheb.chebval(1.0, integ)) < 1e-14
    p = _params(nc=8)
    f, _ = _diag_fields(p)
    st = cs.init_state(*f, p)
    st["om"][3, 1, 1] = np.nan
    st["mean"][0, 2] = np.inf
    assert cs.diagnostics(st, p)["nonfinite"] == 2
