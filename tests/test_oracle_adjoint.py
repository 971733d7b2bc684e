"""Pins of the oracle's discrete adjoint: dot-product (transpose) tests against
central differences of the oracle's own step, and the gradient of J against
central finite differences with eps = 1e-4 in seeded directions."""
import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import box
from paper_2406_01322_amd import synth


def _state(n=16, nprev=2, seed=3):
    cases = synth.batch_cases(nbox=1, seed=seed, sizes=(n,))
    p, u, phi = cases[0]
    prm = box.Params(**p)
    st = box.run(box.init_state(u, phi, prm), prm, nprev)
    return prm, st, u, phi


def _rand_spec(rng, shape, D):
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return x * D


@pytest.mark.parametrize("nprev", [0, 2])
def test_step_adjoint_dot_product(nprev):
    """<(F(x + e d) - F(x - e d)) / 2e, y> = <d, F^T y> for the full step map
    (state and history in, state and history out)."""
    prm, st, _, _ = _state(nprev=nprev)
    n = prm.n
    D = box.dealias_mask(n)
    rng = np.random.default_rng(7)
    # real-field perturbations: transform random real fields so Hermitian symmetry holds
    d = {k: box.fwd(rng.standard_normal(v.shape[:-3] + (n, n, n))) * D for k, v in st.items() if k != "nstep"}
    y = {k: box.fwd(rng.standard_normal(v.shape[:-3] + (n, n, n))) * D for k, v in st.items() if k != "nstep"}
    scale = {k: np.max(np.abs(st[k])) + 1e-3 for k in d}
    eps = 1e-6

    def shifted(sign):
        s2 = {k: (st[k] + sign * eps * scale[k] * d[k]) if k != "nstep" else st[k] for k in st}
        return box.step(s2, prm)

    fp, fm = shifted(+1), shifted(-1)
    jd = {k: (fp[k] - fm[k]) / (2 * eps) for k in d}
    lhs = sum(adj.inner(jd[k], y[k]) for k in d)
    lu, lp, mu, mp, _ = adj.step_adjoint(st, prm, y["uh"], y["ph"], y["hS"], y["hphi"])
    if st["nstep"] == 0:
        mu, mp = mu * 0, mp * 0            # the first step does not read the history
    rhs = (adj.inner(scale["uh"] * d["uh"], lu) + adj.inner(scale["ph"] * d["ph"], lp)
           + adj.inner(scale["hS"] * d["hS"], mu) + adj.inner(scale["hphi"] * d["hphi"], mp))
    assert abs(lhs - rhs) < 1e-7 * max(abs(lhs), abs(rhs))


def test_we_derivative_dot_product():
    """<d out / d We, y> = dJ/dWe from the adjoint, for cotangents y on the new state and
    the new history (the history carries the capillary term directly)."""
    prm, st, _, _ = _state()
    n = prm.n
    D = box.dealias_mask(n)
    rng = np.random.default_rng(9)
    y = [box.fwd(rng.standard_normal(sh)) * D for sh in ((3, n, n, n), (n, n, n), (3, n, n, n), (n, n, n))]
    eps = 1e-5 * prm.we

    def out(we):
        q = box.Params(n=n, re=prm.re, we=we, ch=prm.ch, pe=prm.pe, dt=prm.dt, s=prm.s)
        return box.step(st, q)

    fp, fm = out(prm.we + eps), out(prm.we - eps)
    lhs = sum(adj.inner((fp[k] - fm[k]) / (2 * eps), yk) for k, yk in zip(("uh", "ph", "hS", "hphi"), y))
    _, _, _, _, dwe = adj.step_adjoint(st, prm, *y)
    assert abs(lhs - dwe) < 1e-7 * abs(lhs)


def test_gradient_matches_central_differences():
    """dJ/dphi0 and dJ/dWe against central differences, eps = 1e-4, 8 seeded directions."""
    prm, _, u0, phi0 = _state(n=16, nprev=0, seed=5)
    nsteps = 4
    J, dphi0, dwe, _ = adj.gradient(u0, phi0, prm, nsteps)
    n = prm.n
    rng = np.random.default_rng(6)
    D = box.dealias_mask(n)
    eps = 1e-4
    for _ in range(8):
        d = box.inv(box.fwd(rng.standard_normal((n, n, n))) * D, n)
        d /= np.sqrt(np.mean(d * d))
        dw = rng.standard_normal()
        def Jat(s):
            q = box.Params(n=n, re=prm.re, we=prm.we + s * eps * dw, ch=prm.ch, pe=prm.pe, dt=prm.dt, s=prm.s)
            return adj.run_objective(u0, phi0 + s * eps * d, q, nsteps)
        fd = (Jat(+1) - Jat(-1)) / (2 * eps)
        ad = float(np.sum(dphi0 * d)) + dwe * dw
        assert abs(fd - ad) < 1e-6 * max(abs(fd), 1e-8 * abs(J)), (fd, ad)


def _objective_closed_form():
    """The trigonometric fields of the box diagnostics pin: J = (2 pi)^3 (<|grad phi|^2>
    + 1/2 <|u|^2>) with both averages in closed form."""
    import math
    n = 16
    x = 2.0 * np.pi * np.arange(n) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    A, B, C = 0.7, -0.4, 0.9
    u = np.stack([A * np.sin(2 * Y + Z), B * np.cos(X - 3 * Z), C * np.sin(2 * X + Y)])
    modes = [((1, 2, 0), 0.3, 0.4), ((0, -1, 3), 0.2, -1.1), ((2, 0, 0), 0.1, 0.0)]
    phi = np.full((n, n, n), 0.1)
    for (kx, ky, kz), a, t in modes:
        phi += a * np.cos(kx * X + ky * Y + kz * Z + t)
    g2 = sum(a * a * (kx * kx + ky * ky + kz * kz) / 2.0 for (kx, ky, kz), a, _ in modes)
    u2 = (A * A + B * B + C * C) / 2.0
    J = (2.0 * math.pi) ** 3 * (g2 + 0.5 * u2)
    prm = box.Params(n=n, re=100.0, we=1.0, ch=0.05, pe=20.0, dt=1e-3)
    return box.init_state(u, phi, prm), J


def test_objective_closed_form():
    """J of the terminal state equals int |grad phi|^2 + 1/2 int |u|^2 over the
    (2 pi)^3 box, in closed form for trigonometric fields (pins the Parseval
    weights, the factor 1/2 and the volume)."""
    st, J = _objective_closed_form()
    assert abs(adj.objective(st, 16) - J) < 1e-13 * J


@pytest.mark.parametrize("plant", ["weight2_at_kx0", "unit_volume"])
def test_objective_pin_catches_planted_mistakes(monkeypatch, plant):
    if plant == "weight2_at_kx0":
        monkeypatch.setattr(box, "half_weights", lambda n: np.full(n // 2 + 1, 2.0))
    else:
        monkeypatch.setattr(adj, "VOLUME", 1.0)
    st, J = _objective_closed_form()
    assert abs(adj.objective(st, 16) - J) > 1e-3 * J


def test_objective_gradient_is_the_derivative_of_j():
    """objective_grad is the Riesz representative of dJ under the half-spectrum inner
    product: <grad, d> equals the central difference of J along d (J is quadratic, so
    the difference is exact up to rounding)."""
    st, _ = _objective_closed_form()
    n = 16
    D = box.dealias_mask(n)
    rng = np.random.default_rng(4)
    du = box.fwd(rng.standard_normal((3, n, n, n))) * D
    dp = box.fwd(rng.standard_normal((n, n, n))) * D
    gu, gp = adj.objective_grad(st, n)
    eps = 1e-3
    sp = dict(st, uh=st["uh"] + eps * du, ph=st["ph"] + eps * dp)
    sm = dict(st, uh=st["uh"] - eps * du, ph=st["ph"] - eps * dp)
    fd = (adj.objective(sp, n) - adj.objective(sm, n)) / (2 * eps)
    an = adj.inner(gu, du) + adj.inner(gp, dp)
    assert abs(fd - an) < 1e-10 * abs(an)
