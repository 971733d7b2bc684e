"""Plain FP64 CPU oracle for the wall-normal (Chebyshev) operations of the channel.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP implementation.

The paper represents every quantity along the wall-normal direction z in [-1, 1]
by Chebyshev polynomials on a grid refined near the walls (Sec. 2.2), obtains
the Chebyshev transform as a DCT-I (Sec. 3.2.1), and reduces the implicit
parts of the velocity-vorticity and Cahn-Hilliard equations to independent 1-D
Helmholtz problems per Fourier pair (kx, ky) (Sec. 2.2, eqs. omegaz, ww,
phisplit; Sec. 3.2.2).  This module writes those operations out densely:

* collocation at the Chebyshev-Gauss-Lobatto points z_j = cos(pi j / nc),
  j = 0..nc (the paper's stretched grid, read as CGL);
* f(z) = sum_n a_n T_n(z); transforms by explicit cosine sums;
* derivative of a coefficient vector by numpy's Chebyshev derivative;
* Helmholtz problems (D^2 - beta) f = g by the Chebyshev-tau method: the
  equations for n = 0..nc-2 plus two boundary rows, assembled from the
  explicit second-derivative formula and solved by a dense LU (numpy);
* the fourth-order wall-normal velocity problem by the influence-matrix
  method; u and v from continuity and the definition of omega_z (eq. omegadef).
"""
from __future__ import annotations

import functools

import numpy as np
from numpy.polynomial import chebyshev as npcheb


def cgl(nc: int) -> np.ndarray:
    """Chebyshev-Gauss-Lobatto points z_j = cos(pi j / nc), j = 0..nc (z_0 = +1)."""
    return np.cos(np.pi * np.arange(nc + 1) / nc)


def _cbar(nc: int) -> np.ndarray:
    c = np.ones(nc + 1)
    c[0] = 2.0
    c[-1] = 2.0
    return c


def values_to_coeffs(f: np.ndarray, axis: int = 0) -> np.ndarray:
    """a_n = 2/(nc cbar_n) sum_j f_j cos(pi n j / nc) / cbar_j (cbar_0 = cbar_nc = 2)."""
    f = np.moveaxis(np.asarray(f), axis, 0)
    nc = f.shape[0] - 1
    n = np.arange(nc + 1)
    cb = _cbar(nc)
    Cm = np.cos(np.pi * np.outer(n, n) / nc) / cb[None, :]
    a = (2.0 / (nc * cb))[:, None] * (Cm @ f.reshape(nc + 1, -1))
    return np.moveaxis(a.reshape(f.shape), 0, axis)


def coeffs_to_values(a: np.ndarray, axis: int = 0) -> np.ndarray:
    """f_j = sum_n a_n T_n(z_j) = sum_n a_n cos(pi n j / nc)."""
    a = np.moveaxis(np.asarray(a), axis, 0)
    nc = a.shape[0] - 1
    n = np.arange(nc + 1)
    Cm = np.cos(np.pi * np.outer(n, n) / nc)
    f = Cm @ a.reshape(nc + 1, -1)
    return np.moveaxis(f.reshape(a.shape), 0, axis)


def deriv(a: np.ndarray, axis: int = 0) -> np.ndarray:
    """Coefficients of df/dz (same length, last entry zero)."""
    a = np.moveaxis(np.asarray(a), axis, 0)
    d = npcheb.chebder(a, axis=0)
    out = np.zeros_like(a)
    out[: d.shape[0]] = d
    return np.moveaxis(out, 0, axis)


def d2_matrix(nc: int) -> np.ndarray:
    """(D^2 a)_n = (1/c_n) sum_{p >= n+2, p+n even} p (p^2 - n^2) a_p, c_0 = 2, c_n = 1."""
    D2 = np.zeros((nc + 1, nc + 1))
    for n in range(nc + 1):
        cn = 2.0 if n == 0 else 1.0
        for p in range(n + 2, nc + 1, 2):
            D2[n, p] = p * (p * p - n * n) / cn
    return D2


@functools.lru_cache(maxsize=None)
def _d2_fixed(nc: int) -> np.ndarray:
    """d2_matrix(nc), built once per nc and kept read-only."""
    m = d2_matrix(nc)
    m.setflags(write=False)
    return m


def _wall_row(nc: int, kind: str, wall: int) -> np.ndarray:
    """Row evaluating f (Dirichlet) or f' (Neumann) at z = wall (+1 or -1):
    T_n(+-1) = (+-1)^n, T_n'(+-1) = (+-1)^(n+1) n^2."""
    n = np.arange(nc + 1, dtype=float)
    if kind == "dirichlet":
        return np.ones(nc + 1) if wall > 0 else (-1.0) ** n
    if kind == "neumann":
        return n * n if wall > 0 else (-1.0) ** (n + 1) * n * n
    raise ValueError(kind)


def bc_rows(nc: int, kind):
    """Rows of the top (z = +1) and bottom (z = -1) conditions.  kind is one
    condition for both walls ("dirichlet" or "neumann") or a pair (top, bottom)."""
    kt, kb = (kind, kind) if isinstance(kind, str) else kind
    return _wall_row(nc, kt, +1), _wall_row(nc, kb, -1)


def helmholtz(g: np.ndarray, beta: float, kind="dirichlet", top=0.0, bottom=0.0) -> np.ndarray:
    """Chebyshev-tau solution of (D^2 - beta) f = g on [-1, 1] with
    f(+1) = top, f(-1) = bottom (Dirichlet) or f'(+1) = top, f'(-1) = bottom
    (Neumann); kind may also be a pair (top kind, bottom kind).  g holds nc+1
    Chebyshev coefficients (entries n > nc-2 are dropped, as the tau method
    does).  Dense LU."""
    g = np.asarray(g)
    nc = g.shape[0] - 1
    A = _d2_fixed(nc) - beta * np.eye(nc + 1)
    rt, rb = bc_rows(nc, kind)
    A[nc - 1] = rt
    A[nc] = rb
    rhs = np.array(g, dtype=complex)
    rhs[nc - 1] = top
    rhs[nc] = bottom
    return np.linalg.solve(A, rhs)


def helmholtz_lines(g: np.ndarray, beta, kind="dirichlet", top=0.0, bottom=0.0, chunk: int = 512) -> np.ndarray:
    """`helmholtz` for many independent lines at once: g [nc+1][L] (one line per
    column), beta [L] (or a scalar), the same kind for every line, top and
    bottom scalars or [L].  Each line gets exactly the matrix `helmholtz` builds
    for it; the L dense systems are solved as one stacked LU call, `chunk`
    lines at a time (only to bound memory).  The matrices are real, so the real
    and imaginary parts of each right-hand side share one real factorisation."""
    g = np.asarray(g)
    nc = g.shape[0] - 1
    L = g.shape[1]
    beta = np.broadcast_to(np.asarray(beta, dtype=float), (L,))
    top = np.broadcast_to(np.asarray(top), (L,))
    bottom = np.broadcast_to(np.asarray(bottom), (L,))
    rt, rb = bc_rows(nc, kind)
    eye = np.eye(nc + 1)
    out = np.empty((nc + 1, L), dtype=complex)
    for s in range(0, L, chunk):
        e = min(L, s + chunk)
        A = _d2_fixed(nc)[None] - beta[s:e, None, None] * eye[None]
        A[:, nc - 1] = rt
        A[:, nc] = rb
        rhs = np.array(g[:, s:e].T, dtype=complex)
        rhs[:, nc - 1] = top[s:e]
        rhs[:, nc] = bottom[s:e]
        # the matrix is real: one real LU per line, the real and imaginary parts of
        # the right-hand side as its two columns
        x = np.linalg.solve(A, np.stack([rhs.real, rhs.imag], axis=-1))
        out[:, s:e] = (x[..., 0] + 1j * x[..., 1]).T
    return out


def wall_values(a: np.ndarray):
    """(f(+1), f(-1), f'(+1), f'(-1)) of a coefficient vector."""
    nc = a.shape[0] - 1
    n = np.arange(nc + 1, dtype=float)
    return (np.sum(a), np.sum((-1.0) ** n * a), np.sum(n * n * a), np.sum((-1.0) ** (n + 1) * n * n * a))


def wall_kinds(walls) -> tuple:
    """Condition of omega_z and of the mean velocities at each wall (top, bottom):
    zero value at a no-slip wall, zero normal derivative at a free-slip wall."""
    return tuple("dirichlet" if w == "noslip" else "neumann" for w in walls)


def wall_normal_solve(g_om, g_w, g_phi, kx, ky, beta_ns, beta_a, beta_b, walls=("noslip", "noslip")):
    """The implicit wall-normal solves of one (kx, ky) pair (Sec. 2.2, items iv and v).

    walls = (top, bottom), each "noslip" (u = v = w = 0) or "freeslip"
    (w = 0, du/dz = dv/dz = 0; Sec. 2.1 allows either, or one of each).
    omega_z: (D^2 - beta_ns) omega = g_om,  omega = 0 at a no-slip wall,
             omega' = 0 at a free-slip wall (the z-derivative of
             dv/dx - du/dy).
    w:       (D^2 - beta_ns) psi = g_w, (D^2 - k^2) w = psi, w(+-1) = 0
             (k^2 = kx^2 + ky^2), and w' = 0 at a no-slip wall, w'' = 0 at a
             free-slip wall (continuity with du/dz = dv/dz = 0), i.e. psi = 0
             there.  psi = psi_p + sum c_j psi_j: psi_p vanishes at both
             walls, each homogeneous psi_j takes the unit value at one no-slip
             wall and 0 at the other wall, and the c_j make w' = 0 at the
             no-slip walls (influence matrix).  For k = 0, w = 0 (continuity).
    phi:     (D^2 - beta_a) xi = g_phi, (D^2 - beta_b) phi = xi, both with zero
             normal derivative at the walls (no-flux: phi' = phi''' = 0).
    u, v:    from continuity and eq. omegadef:
             u = i (kx w' + ky omega) / k^2,  v = i (ky w' - kx omega) / k^2
             (for k = 0 they are left to the mean-flow solve and returned as 0).
    Returns dict(omega, w, phi, u, v) of coefficient vectors.
    """
    nc = len(g_om) - 1
    k2 = float(kx * kx + ky * ky)
    om = helmholtz(g_om, beta_ns, wall_kinds(walls))
    if k2 == 0.0:
        w = np.zeros(nc + 1, complex)
    else:
        zero = np.zeros(nc + 1)
        psi_p = helmholtz(g_w, beta_ns, "dirichlet")
        w_p = helmholtz(psi_p, k2, "dirichlet")
        # one homogeneous solution per no-slip wall; the condition w' = 0 there
        clamped = [j for j in range(2) if walls[j] == "noslip"]
        if clamped:
            w_h = []
            for j in clamped:
                psi_j = helmholtz(zero, beta_ns, "dirichlet", 1.0 if j == 0 else 0.0, 1.0 if j == 1 else 0.0)
                w_h.append(helmholtz(psi_j, k2, "dirichlet"))
            dwall = lambda a: (wall_values(a)[2], wall_values(a)[3])   # w'(+1), w'(-1)
            M = np.array([[dwall(wh)[i] for wh in w_h] for i in clamped])
            c = np.linalg.solve(M, -np.array([dwall(w_p)[i] for i in clamped]))
            w = w_p + sum(cj * wh for cj, wh in zip(c, w_h))
        else:
            w = w_p
    xi = helmholtz(g_phi, beta_a, "neumann")
    phi = helmholtz(xi, beta_b, "neumann")
    if k2 == 0.0:
        u = np.zeros(nc + 1, complex)
        v = np.zeros(nc + 1, complex)
    else:
        dw = deriv(w)
        u = 1j * (kx * dw + ky * om) / k2
        v = 1j * (ky * dw - kx * om) / k2
    return dict(omega=om, w=w, phi=phi, u=u, v=v)


def wall_normal_solve_lines(g_om, g_w, g_phi, kx, ky, beta_ns, beta_a, beta_b, walls=("noslip", "noslip")):
    """`wall_normal_solve` for L pairs at once: g_* [nc+1][L], kx, ky, beta_* [L].
    The same problems, the same matrices and the same influence-matrix
    combination per line; every Helmholtz problem of the set is one stacked
    dense solve (`helmholtz_lines`).  Returns dict(omega, w, phi, u, v) of
    [nc+1][L] arrays."""
    g_om, g_w, g_phi = (np.asarray(g) for g in (g_om, g_w, g_phi))
    nc, L = g_om.shape[0] - 1, g_om.shape[1]
    kx = np.asarray(kx, dtype=float)
    ky = np.asarray(ky, dtype=float)
    beta_ns = np.broadcast_to(np.asarray(beta_ns, dtype=float), (L,))
    k2 = kx * kx + ky * ky
    om = helmholtz_lines(g_om, beta_ns, wall_kinds(walls))
    w = np.zeros((nc + 1, L), complex)
    nz = np.nonzero(k2 != 0.0)[0]
    if len(nz):
        bn, kn = beta_ns[nz], k2[nz]
        psi_p = helmholtz_lines(g_w[:, nz], bn, "dirichlet")
        w_p = helmholtz_lines(psi_p, kn, "dirichlet")
        clamped = [j for j in range(2) if walls[j] == "noslip"]
        n = np.arange(nc + 1, dtype=float)
        dwall = (n * n, (-1.0) ** (n + 1) * n * n)          # rows of w'(+1), w'(-1)
        if clamped:
            zero = np.zeros((nc + 1, len(nz)))
            w_h = []
            for j in clamped:
                psi_j = helmholtz_lines(zero, bn, "dirichlet", 1.0 if j == 0 else 0.0, 1.0 if j == 1 else 0.0)
                w_h.append(helmholtz_lines(psi_j, kn, "dirichlet"))
            M = np.empty((len(nz), len(clamped), len(clamped)), complex)
            for a, i in enumerate(clamped):
                for b, wh in enumerate(w_h):
                    M[:, a, b] = dwall[i] @ wh
            r = -np.stack([dwall[i] @ w_p for i in clamped], axis=1)
            c = np.linalg.solve(M, r[..., None])[..., 0]
            acc = 0
            for b, wh in enumerate(w_h):
                acc = acc + c[:, b][None, :] * wh
            w[:, nz] = w_p + acc
        else:
            w[:, nz] = w_p
    xi = helmholtz_lines(g_phi, beta_a, "neumann")
    phi = helmholtz_lines(xi, beta_b, "neumann")
    u = np.zeros((nc + 1, L), complex)
    v = np.zeros((nc + 1, L), complex)
    if len(nz):
        dw = deriv(w[:, nz])
        u[:, nz] = 1j * (kx[nz] * dw + ky[nz] * om[:, nz]) / k2[nz]
        v[:, nz] = 1j * (ky[nz] * dw - kx[nz] * om[:, nz]) / k2[nz]
    return dict(omega=om, w=w, phi=phi, u=u, v=v)
