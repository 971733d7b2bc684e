"""GPU parity of the wall-normal (Chebyshev) kernels against the dense FP64 oracle.

Lines are stored [n][line].  The channel workload has Fourier pairs
kx = 0..85 (2/3 of 256 in x, half spectrum) and ky = -42..42 (2/3 of 128 in y),
7310 lines of nc + 1 = 129 Chebyshev coefficients; Re_tau = 150, dt = 1e-4
give the Crank-Nicolson shift beta_ns = 2 Re/dt = 3e6, and Ch = 0.02,
Pe = 50 with the default splitting give the CH factors a = b = sqrt(Pe/(dt Ch^2)).
"""
import math

import numpy as np
import pytest

from oracle import channel as ch

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NCS = [4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 256]
BETA_NS = 2.0 * 150.0 / 1e-4
BETA_CH = math.sqrt(50.0 / (1e-4 * 0.02 ** 2))


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _lines(nc, nl, seed, decay=0.0):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((nc + 1, nl)) + 1j * rng.standard_normal((nc + 1, nl))
    if decay:
        x *= np.exp(-decay * np.arange(nc + 1))[:, None]
    return x


@pytest.mark.parametrize("nc", NCS)
@pytest.mark.parametrize("nl", [1, 37, 300])
def test_cheb_transform_parity(nc, nl):
    from paper_2406_01322_amd import psms
    f = _lines(nc, nl, nc + nl)
    a = _host(psms.cheb_transform(_dev(f), +1))
    want = ch.values_to_coeffs(f)
    assert np.max(np.abs(a - want)) < 1e-14 * nc * np.max(np.abs(want))
    back = _host(psms.cheb_transform(_dev(want), -1))
    assert np.max(np.abs(back - ch.coeffs_to_values(want))) < 1e-14 * nc * np.max(np.abs(f))
    # FP32
    a32 = _host(psms.cheb_transform(_dev(f.astype(np.complex64)), +1)).astype(np.complex128)
    want32 = ch.values_to_coeffs(f.astype(np.complex64).astype(np.complex128))
    assert np.max(np.abs(a32 - want32)) < 3e-7 * max(1.0, math.log2(nc)) * np.max(np.abs(want32))


@pytest.mark.parametrize("nc", [4, 16, 128, 256])
def test_cheb_deriv_parity(nc):
    from paper_2406_01322_amd import psms
    a = _lines(nc, 53, 7, decay=0.05)
    got = _host(psms.cheb_deriv(_dev(a)))
    want = ch.deriv(a, axis=0)
    assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(want))


def _kappa(nc, beta, kind):
    """Condition number ||A||_inf ||A^-1||_inf of the oracle's tau matrix."""
    A = ch.d2_matrix(nc) - beta * np.eye(nc + 1)
    A[nc - 1], A[nc] = ch.bc_rows(nc, kind)
    return float(np.linalg.cond(A, np.inf))


@pytest.mark.parametrize("kind", ["dirichlet", "neumann"])
@pytest.mark.parametrize("nc", [8, 32, 128, 256])
@pytest.mark.parametrize("beta_scale", [1.0, 1e3, BETA_CH, BETA_NS])
def test_cheb_helmholtz_parity(kind, nc, beta_scale, record_error):
    from paper_2406_01322_amd import psms
    nl = 24
    rng = np.random.default_rng(nc)
    g = _lines(nc, nl, 3 * nc, decay=0.03)
    beta = beta_scale * (0.5 + rng.random(nl))
    bcv = rng.standard_normal((nl, 2)) + 1j * rng.standard_normal((nl, 2))
    got = _host(psms.cheb_helmholtz(_dev(g), _dev(beta), kind, _dev(bcv)))
    want = np.stack([ch.helmholtz(g[:, l], beta[l], kind, bcv[l, 0], bcv[l, 1]) for l in range(nl)], axis=1)
    # The oracle's dense LU (partial pivoting) is normwise backward stable, so the two
    # solutions differ by rounding amplified by the normwise conditioning of the tau
    # system: 10 kappa_inf(A) u, and at most 1e-11 (the zero-boundary-value problems at
    # large beta, whose solutions are ~g / beta, reach 2e-12).
    bar = min(1e-11, 10.0 * max(_kappa(nc, beta[l], kind) for l in range(nl)) * 2.0 ** -53)
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    record_error("helmholtz", err, bar)
    assert err < bar, (err, bar)
    # zero boundary values when bcval is omitted
    got0 = _host(psms.cheb_helmholtz(_dev(g), _dev(beta), kind))
    want0 = np.stack([ch.helmholtz(g[:, l], beta[l], kind) for l in range(nl)], axis=1)
    err0 = np.max(np.abs(got0 - want0)) / np.max(np.abs(want0))
    record_error("helmholtz, zero boundary values", err0, bar)
    assert err0 < bar, (err0, bar)


# The full wall solve chains up to four tau problems (psi, then w; the influence
# combination of three of them; u, v by a derivative), each solved to ~1e-15 here:
# 1e-11 of each line's largest coefficient (measured: 3.3e-13 at worst).


def _kgrid(nkx, nky):
    kx = np.repeat(np.arange(nkx, dtype=float), nky)
    ky = np.tile(np.arange(-(nky // 2), nky // 2 + 1, dtype=float), nkx)
    return kx, ky


@pytest.mark.parametrize("nc,nkx,nky", [(16, 3, 5), (32, 4, 7), (128, 3, 3), (256, 2, 3)])
def test_wall_solve_parity(nc, nkx, nky, record_error):
    from paper_2406_01322_amd import psms
    kx, ky = _kgrid(nkx, nky)              # includes the mean line kx = ky = 0
    nl = len(kx)
    g = [_lines(nc, nl, s, decay=0.05) for s in (1, 2, 3)]
    r = psms.wall_solve(_dev(kx), _dev(ky), BETA_NS, BETA_CH, BETA_CH, *[_dev(x) for x in g])
    got = {k: _host(v) for k, v in r.items()}
    worst = 0.0
    for l in range(nl):
        ref = ch.wall_normal_solve(g[0][:, l], g[1][:, l], g[2][:, l], kx[l], ky[l],
                                   kx[l] ** 2 + ky[l] ** 2 + BETA_NS, kx[l] ** 2 + ky[l] ** 2 + BETA_CH,
                                   kx[l] ** 2 + ky[l] ** 2 + BETA_CH)
        for key in ("omega", "w", "phi", "u", "v"):
            scale = max(np.max(np.abs(ref[key])), 1e-300)
            err = np.max(np.abs(got[key][:, l] - ref[key])) / scale
            worst = max(worst, err if scale > 1e-300 else 0.0)
            assert (err < 1e-11) or (scale == 1e-300 and np.max(np.abs(got[key][:, l])) == 0.0), (key, l, err)
    record_error("wall solve (per line)", worst, 1e-11)


def test_wall_solve_channel_size_sampled_lines():
    """The channel workload's full line set (kx 0..85, ky -42..42, nc = 128), checked on
    sampled lines against the dense oracle, and on every line by the wall conditions."""
    from paper_2406_01322_amd import psms
    nc = 128
    kx, ky = _kgrid(86, 85)
    nl = len(kx)
    g = [_lines(nc, nl, s, decay=0.08) for s in (4, 5, 6)]
    r = psms.wall_solve(_dev(kx), _dev(ky), BETA_NS, BETA_CH, BETA_CH, *[_dev(x) for x in g])
    got = {k: _host(v) for k, v in r.items()}
    n = np.arange(nc + 1, dtype=float)
    w = got["w"]
    assert np.max(np.abs(np.sum(w, axis=0))) < 1e-12 * np.max(np.abs(w))
    assert np.max(np.abs(np.sum(((-1.0) ** n)[:, None] * w, axis=0))) < 1e-12 * np.max(np.abs(w))
    assert np.max(np.abs(np.sum((n * n)[:, None] * w, axis=0))) < 1e-9 * np.max(np.abs(w))
    for l in [0, 1, 42, 43, 1000, 3654, 7309]:
        k2 = kx[l] ** 2 + ky[l] ** 2
        ref = ch.wall_normal_solve(g[0][:, l], g[1][:, l], g[2][:, l], kx[l], ky[l], k2 + BETA_NS, k2 + BETA_CH,
                                   k2 + BETA_CH)
        for key in ("omega", "w", "phi", "u", "v"):
            scale = np.max(np.abs(ref[key]))
            if scale == 0.0:
                assert np.max(np.abs(got[key][:, l])) == 0.0
            else:
                assert np.max(np.abs(got[key][:, l] - ref[key])) < 1e-11 * scale, (key, l)


def test_zero_lines_is_a_noop():
    from paper_2406_01322_amd import psms
    x = torch.zeros((17, 0), dtype=torch.complex128, device="cuda")
    assert psms.cheb_transform(x, +1).shape == (17, 0)
