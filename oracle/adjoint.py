"""Discrete adjoint of the oracle's box step (FP64, numpy).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP implementation.

Discretise-then-differentiate: this is the exact transpose of `oracle.box.step`
(the Jacobian-transpose product), with respect to the real inner product of
the half spectrum

    <a, b> = sum_{k in band, kx >= 0} w_k Re(conj(a_k) b_k),   w = 1 at kx = 0, 2 otherwise,

which equals the grid inner product of the real fields divided by N^3.  Under
it every per-mode real factor is self-adjoint, (i k)^T = -i k, the forward
transform (with 1/N^3 and the 2/3 truncation) has transpose inv / N^3 and the
inverse transform has transpose N^3 fwd.

One step (AB2; AB1 has alpha = 1, beta = 0):
    S^n = R(x^n; We),  x^{n+1} = A x^n + B (alpha S^n + beta h^n),  h^{n+1} = S^n.
Its adjoint, given lam = dJ/dx^{n+1} and mu = dJ/dh^{n+1}:
    Sbar = alpha B lam + mu,   mu^n = beta B lam,
    lam^n = A lam + (dR/dx)^T Sbar,   dJ/dWe += (dR/dWe)^T Sbar.

Objective (the adjoint workload): J = int |grad phi|^2 dV + 1/2 int |u|^2 dV at
the final step, on the box of volume (2 pi)^3.
"""
from __future__ import annotations

import math

import numpy as np

from . import box


VOLUME = (2.0 * math.pi) ** 3


def inner(a: np.ndarray, b: np.ndarray) -> float:
    """<a, b> over the half spectrum with weights 1 (kx = 0) / 2 (kx > 0)."""
    n = a.shape[-2]
    w = box.half_weights(n)
    return float(np.sum(w * np.real(np.conj(a) * b)))


def objective(state: dict, n: int) -> float:
    """J = int |grad phi|^2 + 1/2 int |u|^2 (Parseval on the half spectrum)."""
    KX, KY, KZ = box.kgrid(n)
    k2 = KX * KX + KY * KY + KZ * KZ
    w = box.half_weights(n)
    jp = VOLUME * float(np.sum(w * k2 * np.abs(state["ph"]) ** 2))
    ju = 0.5 * VOLUME * float(np.sum(w * (np.abs(state["uh"]) ** 2).sum(axis=0)))
    return jp + ju


def objective_grad(state: dict, n: int):
    """dJ/d(u_hat, phi_hat) as Riesz representatives of <.,.>."""
    KX, KY, KZ = box.kgrid(n)
    k2 = KX * KX + KY * KY + KZ * KZ
    return VOLUME * state["uh"], 2.0 * VOLUME * k2 * state["ph"]


def nonlinear_adjoint(uh, ph, prm: box.Params, s_bar, sphi_bar):
    """Transpose of (uh, ph) -> (P S, S_phi) of `box.nonlinear_terms` applied to
    (s_bar, sphi_bar); returns (uh_bar, ph_bar, dWe)."""
    n = prm.n
    D = box.dealias_mask(n)
    KX, KY, KZ = box.kgrid(n)
    kv = (KX, KY, KZ)
    k2 = KX * KX + KY * KY + KZ * KZ
    s = prm.split_s()
    csig = prm.capillary()
    fwd = lambda f: box.fwd(f) * D      # forward transform with truncation
    inv = lambda f: box.inv(f, n)

    sb = box.project(s_bar)             # P is self-adjoint
    sb[:, 0, 0, 0] = 0.0                # S(0) was set to zero
    spb = np.array(sphi_bar, dtype=complex)
    spb[0, 0, 0] = 0.0                  # S_phi(0) was set to zero

    u = inv(uh)
    phi = inv(ph)
    g = np.stack([inv(1j * kv[j] * ph) for j in range(3)])

    uh_bar = np.zeros_like(uh)
    ph_bar = np.zeros_like(ph)
    u_bar = np.zeros_like(u)           # physical cotangents, scaled by N^3
    g_bar = np.zeros_like(g)
    phi_bar = np.zeros_like(phi)

    # -u.grad(u): conv_i = sum_j u_j d_j u_i, S_i gets -fwd(conv_i)
    for i in range(3):
        cb = -inv(sb[i])
        for j in range(3):
            G_ij = inv(1j * kv[j] * uh[i])
            u_bar[j] += cb * G_ij
            uh_bar[i] += -1j * kv[j] * fwd(cb * u[j])
    # Korteweg: S_i gets csig sum_j i k_j fwd(tau_ij), tau = |g|^2 I - g g
    dwe = 0.0
    g2 = g[0] ** 2 + g[1] ** 2 + g[2] ** 2
    for i in range(3):
        div_tau = np.zeros_like(ph)
        for j in range(3):
            tb = -csig * inv(1j * kv[j] * sb[i])      # tau_ij bar (scaled)
            if i == j:
                for m in range(3):
                    g_bar[m] += 2.0 * tb * g[m]
            g_bar[i] += -tb * g[j]
            g_bar[j] += -tb * g[i]
            tau_ij = (g2 if i == j else 0.0) - g[i] * g[j]
            div_tau = div_tau + 1j * kv[j] * fwd(tau_ij)
        dwe += inner(sb[i], -(csig / prm.we) * div_tau)
    # CH: S_phi = -fwd(u.g) - (k^2/Pe) fwd(phi^3) + ((1 + s Ch^2)/Pe) k^2 phi_hat
    ab = -inv(spb)
    cb = -inv((k2 / prm.pe) * spb)
    for j in range(3):
        u_bar[j] += ab * g[j]
        g_bar[j] += ab * u[j]
    phi_bar += 3.0 * phi * phi * cb
    ph_bar += ((1.0 + s * prm.ch ** 2) / prm.pe) * k2 * spb
    # back to spectral space (transpose of the inverse transforms)
    for j in range(3):
        uh_bar[j] += fwd(u_bar[j])
        ph_bar += -1j * kv[j] * fwd(g_bar[j])
    ph_bar += fwd(phi_bar)
    return uh_bar, ph_bar, dwe


def step_adjoint(state: dict, prm: box.Params, lam_u, lam_p, mu_u, mu_p):
    """Adjoint of `box.step(state)`: (lam, mu) at n+1 -> (lam, mu) at n and dJ/dWe."""
    n = prm.n
    KX, KY, KZ = box.kgrid(n)
    k2 = KX * KX + KY * KY + KZ * KZ
    dt, nu = prm.dt, 1.0 / prm.re
    s = prm.split_s()
    A_u = (1.0 - 0.5 * dt * nu * k2) / (1.0 + 0.5 * dt * nu * k2)
    B_u = dt / (1.0 + 0.5 * dt * nu * k2)
    B_p = dt / (1.0 + dt * (prm.ch ** 2 / prm.pe) * (k2 * k2 + s * k2))
    A_p = B_p / dt
    alpha, beta = (1.0, 0.0) if state["nstep"] == 0 else (1.5, -0.5)
    D = box.dealias_mask(n)
    lam_u = lam_u * D
    lam_p = lam_p * D
    sbar_u = alpha * B_u * lam_u + mu_u
    sbar_p = alpha * B_p * lam_p + mu_p
    mu_u_n = beta * B_u * lam_u
    mu_p_n = beta * B_p * lam_p
    ub, pb, dwe = nonlinear_adjoint(state["uh"], state["ph"], prm, sbar_u, sbar_p)
    lam_u_n = (A_u * lam_u + ub) * D
    lam_p_n = (A_p * lam_p + pb) * D
    return lam_u_n, lam_p_n, mu_u_n * D, mu_p_n * D, dwe


def gradient(u0, phi0, prm: box.Params, nsteps: int):
    """J after nsteps from (u0, phi0), dJ/dphi0 (physical array) and dJ/dWe."""
    n = prm.n
    states = [box.init_state(u0, phi0, prm)]
    for _ in range(nsteps):
        states.append(box.step(states[-1], prm))
    J = objective(states[-1], n)
    lam_u, lam_p = objective_grad(states[-1], n)
    mu_u = np.zeros_like(lam_u)
    mu_p = np.zeros_like(lam_p)
    dwe = 0.0
    for m in range(nsteps - 1, -1, -1):
        lam_u, lam_p, mu_u, mu_p, d = step_adjoint(states[m], prm, lam_u, lam_p, mu_u, mu_p)
        dwe += d
    # phi_hat^0 = D fwd(phi0): the transpose maps lam_p to inv(lam_p) / N^3 on the grid
    dphi0 = box.inv(lam_p * box.dealias_mask(n), n) / n ** 3
    return J, dphi0, dwe, (lam_u, lam_p)


def run_objective(u0, phi0, prm: box.Params, nsteps: int) -> float:
    st = box.run(box.init_state(u0, phi0, prm), prm, nsteps)
    return objective(st, prm.n)
