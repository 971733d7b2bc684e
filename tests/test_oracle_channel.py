"""Pins of the Chebyshev / wall-normal oracle against closed forms and invariants."""
import numpy as np
import pytest
import scipy.fft
from numpy.polynomial import chebyshev as npcheb

from oracle import channel as ch


@pytest.mark.parametrize("nc", [8, 16, 32, 128])
def test_transform_of_single_polynomials(nc):
    z = ch.cgl(nc)
    assert z[0] == 1.0 and z[-1] == -1.0
    for m in [0, 1, 3, nc // 2, nc - 1, nc]:
        f = np.cos(m * np.arccos(np.clip(z, -1, 1)))     # T_m on the grid
        a = ch.values_to_coeffs(f)
        e = np.zeros(nc + 1)
        e[m] = 1.0
        assert np.max(np.abs(a - e)) < 1e-12


@pytest.mark.parametrize("nc", [16, 64, 128])
def test_transform_matches_scipy_dct1_and_roundtrips(nc):
    rng = np.random.default_rng(nc)
    f = rng.standard_normal(nc + 1) + 1j * rng.standard_normal(nc + 1)
    a = ch.values_to_coeffs(f)
    # DCT-I (scipy, unnormalised): y_n = f_0 + (-1)^n f_nc + 2 sum f_j cos(pi n j / nc)
    y = scipy.fft.dct(f.real, type=1) + 1j * scipy.fft.dct(f.imag, type=1)
    cb = np.ones(nc + 1)
    cb[0] = cb[-1] = 2.0
    assert np.max(np.abs(a - y / (nc * cb))) < 1e-13
    assert np.max(np.abs(ch.coeffs_to_values(a) - f)) < 1e-13


@pytest.mark.parametrize("nc", [16, 64])
def test_derivative_closed_form(nc):
    """T_n'(z) = n U_{n-1}(z) = n sin(n t) / sin t, z = cos t."""
    t = np.linspace(0.1, 3.0, 7)
    z = np.cos(t)
    for n in [1, 2, 5, nc - 1, nc]:
        a = np.zeros(nc + 1)
        a[n] = 1.0
        d = ch.deriv(a)
        got = npcheb.chebval(z, d)
        assert np.max(np.abs(got - n * np.sin(n * t) / np.sin(t))) < 1e-9 * n * n


@pytest.mark.parametrize("kind", ["dirichlet", "neumann"])
@pytest.mark.parametrize("beta", [0.5, 40.0, 4000.0])
def test_helmholtz_manufactured_polynomial_is_exact(kind, beta):
    nc = 32
    rng = np.random.default_rng(3)
    u = np.zeros(nc + 1, complex)
    u[: nc - 1] = rng.standard_normal(nc - 1) + 1j * rng.standard_normal(nc - 1)   # degree <= nc-2
    u[: nc - 1] /= (1.0 + np.arange(nc - 1)) ** 2
    d2 = npcheb.chebder(u, 2)
    g = -beta * u
    g[: d2.shape[0]] += d2
    top, bot, dtop, dbot = ch.wall_values(u)
    if kind == "dirichlet":
        f = ch.helmholtz(g, beta, kind, top, bot)
    else:
        f = ch.helmholtz(g, beta, kind, dtop, dbot)
    assert np.max(np.abs(f - u)) < 1e-12 * max(1.0, np.max(np.abs(u)))


@pytest.mark.parametrize("kinds", [("dirichlet", "neumann"), ("neumann", "dirichlet")])
@pytest.mark.parametrize("beta", [0.5, 40.0, 3e6])
def test_helmholtz_mixed_conditions_manufactured_polynomial_is_exact(kinds, beta):
    """A different condition at each wall (a no-slip and a free-slip wall): the tau
    solution of a manufactured polynomial is exact; the wall values come from numpy's
    Chebyshev evaluation, not from the oracle's boundary rows."""
    nc = 32
    rng = np.random.default_rng(5)
    u = np.zeros(nc + 1, complex)
    u[: nc - 1] = rng.standard_normal(nc - 1) + 1j * rng.standard_normal(nc - 1)
    u[: nc - 1] /= (1.0 + np.arange(nc - 1)) ** 2
    d2 = npcheb.chebder(u, 2)
    g = -beta * u
    g[: d2.shape[0]] += d2
    du = npcheb.chebder(u)
    val = {("dirichlet", 1): npcheb.chebval(1.0, u), ("dirichlet", -1): npcheb.chebval(-1.0, u),
           ("neumann", 1): npcheb.chebval(1.0, du), ("neumann", -1): npcheb.chebval(-1.0, du)}
    f = ch.helmholtz(g, beta, kinds, val[(kinds[0], 1)], val[(kinds[1], -1)])
    assert np.max(np.abs(f - u)) < 1e-12 * max(1.0, np.max(np.abs(u)))


@pytest.mark.parametrize("beta", [1.0, 25.0])
def test_helmholtz_exponential_solutions(beta):
    """g = 0: Dirichlet f(+1)=1, f(-1)=0 -> sinh(k(1+z))/sinh(2k); Neumann f'(+1)=1,
    f'(-1)=0 -> cosh(k(1+z))/(k sinh(2k)), k = sqrt(beta)."""
    nc = 48
    k = np.sqrt(beta)
    z = np.linspace(-1, 1, 11)
    f = ch.helmholtz(np.zeros(nc + 1), beta, "dirichlet", 1.0, 0.0)
    assert np.max(np.abs(npcheb.chebval(z, f) - np.sinh(k * (1 + z)) / np.sinh(2 * k))) < 1e-12
    f = ch.helmholtz(np.zeros(nc + 1), beta, "neumann", 1.0, 0.0)
    assert np.max(np.abs(npcheb.chebval(z, f) - np.cosh(k * (1 + z)) / (k * np.sinh(2 * k)))) < 1e-12


def _dense_fourth_order(g, k2, beta, nc):
    """(D^2 - k2)(D^2 - beta) w = g with w = w' = 0 at both walls, one dense tau system
    (rows n = 0..nc-4 of the fourth-order operator plus four boundary rows)."""
    D2 = ch.d2_matrix(nc)
    I = np.eye(nc + 1)
    A = (D2 - k2 * I) @ (D2 - beta * I)
    rt, rb = ch.bc_rows(nc, "dirichlet")
    nt, nb = ch.bc_rows(nc, "neumann")
    A[nc - 3], A[nc - 2], A[nc - 1], A[nc] = rt, rb, nt, nb
    rhs = np.array(g, dtype=complex)
    rhs[nc - 3:] = 0.0
    return np.linalg.solve(A, rhs)


def test_wall_normal_solve_invariants_and_dense_fourth_order():
    """Invariants of the influence-matrix solve, and agreement with one dense fourth-order
    tau system: the two discretisations drop different top coefficients, so they agree to
    the truncation level, spectrally small for a smooth right-hand side."""
    nc = 48
    rng = np.random.default_rng(11)
    cplx = lambda: (rng.standard_normal(nc + 1) + 1j * rng.standard_normal(nc + 1)) * np.exp(-0.6 * np.arange(nc + 1))
    g_om, g_w, g_phi = cplx(), cplx(), cplx()
    kx, ky = 2.0, -3.0
    k2 = kx * kx + ky * ky
    beta_ns = k2 + 100.0
    beta_a, beta_b = k2 + 30.0, k2 + 50.0
    r = ch.wall_normal_solve(g_om, g_w, g_phi, kx, ky, beta_ns, beta_a, beta_b)
    om, w, phi, u, v = r["omega"], r["w"], r["phi"], r["u"], r["v"]
    t, b, _, _ = ch.wall_values(om)
    assert abs(t) < 1e-13 and abs(b) < 1e-13
    wt, wb, dwt, dwb = ch.wall_values(w)
    assert max(abs(wt), abs(wb), abs(dwt), abs(dwb)) < 1e-11
    _, _, pt, pb = ch.wall_values(phi)
    assert abs(pt) < 1e-11 and abs(pb) < 1e-11
    # the influence-matrix route equals a dense fourth-order tau solve
    wd = _dense_fourth_order(g_w, k2, beta_ns, nc)
    assert np.max(np.abs(w - wd)) < 1e-11 * np.max(np.abs(wd))
    # continuity and the definition of omega_z, coefficient by coefficient
    dw = ch.deriv(w)
    assert np.max(np.abs(1j * kx * u + 1j * ky * v + dw)) < 1e-12 * np.max(np.abs(dw))
    assert np.max(np.abs(1j * kx * v - 1j * ky * u - om)) < 1e-12 * np.max(np.abs(om))
    # the CH pair: (D^2 - beta_b) phi satisfies the first Helmholtz problem
    D2 = ch.d2_matrix(nc)
    xi = D2 @ phi - beta_b * phi
    res = D2 @ xi - beta_a * xi - g_phi
    assert np.max(np.abs(res[: nc - 3])) < 1e-9 * np.max(np.abs(g_phi))


def _wall_derivative_rows(nc, order):
    """Rows evaluating the order-th z-derivative at z = +1 and z = -1, from numpy's
    Chebyshev derivative of each basis polynomial."""
    rows = np.zeros((2, nc + 1))
    for n in range(nc + 1):
        e = np.zeros(nc + 1)
        e[n] = 1.0
        d = npcheb.chebder(e, order) if order else e
        rows[0, n] = npcheb.chebval(1.0, d)
        rows[1, n] = npcheb.chebval(-1.0, d)
    return rows


@pytest.mark.parametrize("walls", [("freeslip", "noslip"), ("noslip", "freeslip"), ("freeslip", "freeslip")])
def test_wall_normal_solve_free_slip_walls(walls):
    """Free-slip walls (Sec. 2.1): omega' = 0 and w = w'' = 0 there; w' = 0 and
    omega = 0 at a no-slip wall; w agrees with one dense fourth-order tau system
    whose four boundary rows are written from numpy's Chebyshev derivatives."""
    nc = 48
    rng = np.random.default_rng(17)
    cplx = lambda: (rng.standard_normal(nc + 1) + 1j * rng.standard_normal(nc + 1)) * np.exp(-0.6 * np.arange(nc + 1))
    g_om, g_w, g_phi = cplx(), cplx(), cplx()
    kx, ky = 1.0, 2.0
    k2 = kx * kx + ky * ky
    beta_ns = k2 + 100.0
    r = ch.wall_normal_solve(g_om, g_w, g_phi, kx, ky, beta_ns, k2 + 30.0, k2 + 50.0, walls)
    om, w = r["omega"], r["w"]
    R0, R1, R2 = (_wall_derivative_rows(nc, k) for k in (0, 1, 2))
    scale_o, scale_w = np.max(np.abs(om)), np.max(np.abs(w))
    for j, wall in enumerate(walls):
        if wall == "noslip":
            assert abs(R0[j] @ om) < 1e-12 * scale_o
            assert abs(R1[j] @ w) < 1e-10 * scale_w
        else:
            assert abs(R1[j] @ om) < 1e-10 * scale_o
            assert abs(R2[j] @ w) < 1e-9 * scale_w
        assert abs(R0[j] @ w) < 1e-12 * scale_w
    D2 = ch.d2_matrix(nc)
    I = np.eye(nc + 1)
    A = (D2 - k2 * I) @ (D2 - beta_ns * I)
    rows = [R0[0], R0[1]] + [(R1 if wall == "noslip" else R2)[j] for j, wall in enumerate(walls)]
    A[nc - 3:] = np.array(rows)
    rhs = np.array(g_w, dtype=complex)
    rhs[nc - 3:] = 0.0
    wd = np.linalg.solve(A, rhs)
    assert np.max(np.abs(w - wd)) < 1e-11 * np.max(np.abs(wd))
    # u, v still satisfy continuity and the definition of omega_z
    dw = ch.deriv(w)
    assert np.max(np.abs(1j * kx * r["u"] + 1j * ky * r["v"] + dw)) < 1e-12 * np.max(np.abs(dw))


def test_mean_mode_has_no_wall_normal_velocity():
    nc = 16
    g = np.ones(nc + 1, complex)
    r = ch.wall_normal_solve(g, g, g, 0.0, 0.0, 100.0, 30.0, 50.0)
    assert np.all(r["w"] == 0) and np.all(r["u"] == 0) and np.all(r["v"] == 0)


@pytest.mark.parametrize("walls", [("noslip", "noslip"), ("freeslip", "noslip"), ("freeslip", "freeslip")])
def test_stacked_line_solves_equal_the_per_line_solves(walls):
    """The stacked solve of many (kx, ky) pairs builds, per line, the matrices of the
    one-line solve: their results agree to rounding (the w combination cancels to
    about 1e-13 of its terms at large k), including the mean pair k = 0."""
    nc, L = 32, 9
    rng = np.random.default_rng(11)
    g = [rng.standard_normal((nc + 1, L)) + 1j * rng.standard_normal((nc + 1, L)) for _ in range(3)]
    kx = np.array([0.0, 0.5, 0.0, 1.0, 2.5, 3.0, 0.5, 7.0, 10.5])
    ky = np.array([0.0, 0.0, 1.0, -1.0, 2.0, -3.0, 4.0, 0.0, -6.0])
    k2 = kx * kx + ky * ky
    b_ns, b_a, b_b = k2 + 2e5, k2 + 900.0, k2 + 2500.0
    got = ch.wall_normal_solve_lines(*g, kx, ky, b_ns, b_a, b_b, walls)
    for l in range(L):
        want = ch.wall_normal_solve(g[0][:, l], g[1][:, l], g[2][:, l], kx[l], ky[l], b_ns[l], b_a[l], b_b[l], walls)
        for k in ("omega", "w", "phi", "u", "v"):
            scale = max(np.max(np.abs(want[k])), 1e-300)
            assert np.max(np.abs(got[k][:, l] - want[k])) <= 1e-12 * scale, (k, l)
