"""GPU parity of the HIP step against the FP64 oracle, through the C ABI.

Tolerances: FP64 path rel-L2 <= 1e-12 per field per step (transforms 1e-13);
MIXED path (FP32 transforms and products, FP64 state, RHS assembly and
projection) rel-L2 <= 1e-5 per field per step.  Index maps are compared
bit-exactly.
"""
import functools

import numpy as np
import pytest

from oracle import box
from paper_2406_01322_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _solver(p, precision="fp64"):
    from paper_2406_01322_amd.psms import Solver
    return Solver(p["n"], p["re"], p["we"], p["ch"], p["pe"], p["dt"], s=p.get("s", 0.0), precision=precision)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_l2(a, b):
    d = np.linalg.norm((a - b).ravel())
    r = np.linalg.norm(b.ravel())
    return d / r if r > 0 else d


def _params(n, **kw):
    p = dict(n=n, re=100.0, we=1.0, ch=0.05, pe=20.0, dt=1e-3)
    p.update(kw)
    return p


def _oracle_state(case):
    p, u, phi = synth.box_case(case)
    prm = box.Params(**p)
    return p, u, phi, prm


# ------------------------------------------------------------------ index maps

@pytest.mark.parametrize("n", [8, 12, 16, 24, 32, 48, 96, 128])
def test_index_maps_bit_exact(n):
    s = _solver(_params(n))
    maps = _host(s.index_maps()).astype(np.int64)
    K = box.cutoff(n)
    assert maps.shape == ((2 * K + 1) ** 2 * (K + 1), 4)
    kz, ky, kx = box.wavenumbers(n)
    nh = n // 2 + 1
    D = box.dealias_mask(n)
    off = maps[:, 3]
    assert len(np.unique(off)) == len(off) == int(D.sum())
    assert np.all(D.ravel()[off])
    pz, rem = off // (n * nh), off % (n * nh)
    py, px = rem // nh, rem % nh
    assert np.array_equal(maps[:, 0], kz[pz])
    assert np.array_equal(maps[:, 1], ky[py])
    assert np.array_equal(maps[:, 2], kx[px])


# ------------------------------------------------------------------ transforms

@pytest.mark.parametrize("n", [8, 12, 16, 24, 32, 48, 64, 96, 128])
@pytest.mark.parametrize("flags", [0, 1, 2, 4 | 1, 8])
def test_forward_transform_parity_fp64(n, flags):
    from paper_2406_01322_amd import psms
    rng = np.random.default_rng(n + 31 * flags)
    f = rng.standard_normal((2, n, n, n))
    s = _solver(_params(n))
    got = _host(s.transform(+1, _dev(f), flags))
    axis = 0 if flags & psms.DERIV_X else 1 if flags & psms.DERIV_Y else 2 if flags & psms.DERIV_Z else None
    want = box.transform_forward(f, dealias=bool(flags & psms.DEALIAS), deriv_axis=axis)
    scale = np.max(np.abs(want))
    assert np.max(np.abs(got - want)) <= 1e-13 * scale * max(1, n // 16)


@pytest.mark.parametrize("n", [8, 12, 16, 24, 32, 48, 64, 96, 128])
@pytest.mark.parametrize("flags", [0, 1, 4, 8 | 1])
def test_inverse_transform_parity_fp64(n, flags):
    from paper_2406_01322_amd import psms
    rng = np.random.default_rng(7 * n + flags)
    fh = box.fwd(rng.standard_normal((3, n, n, n)))
    s = _solver(_params(n))
    got = _host(s.transform(-1, _dev(fh), flags))
    axis = 0 if flags & psms.DERIV_X else 1 if flags & psms.DERIV_Y else 2 if flags & psms.DERIV_Z else None
    want = box.transform_inverse(fh, dealias=bool(flags & psms.DEALIAS), deriv_axis=axis)
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want)) * max(1, n // 16)


@pytest.mark.parametrize("n", [16, 48, 128])
def test_transform_parity_mixed(n):
    rng = np.random.default_rng(n)
    f = rng.standard_normal((n, n, n))
    s = _solver(_params(n), precision="mixed")
    got = _host(s.transform(+1, _dev(f.astype(np.float32)), 1)).astype(np.complex128)
    want = box.transform_forward(f.astype(np.float32).astype(np.float64), dealias=True)
    assert rel_l2(got, want) < 1e-6
    back = _host(s.transform(-1, _dev(want.astype(np.complex64)), 0)).astype(np.float64)
    assert rel_l2(back, box.transform_inverse(want)) < 1e-6


def test_transform_zero_fields_is_a_noop():
    n = 16
    s = _solver(_params(n))
    x = torch.zeros((0, n, n, n), dtype=torch.float64, device="cuda")
    out = s.transform(+1, x, 0)
    assert out.shape == (0, n, n, n // 2 + 1)


# ------------------------------------------------------------------ init, Helmholtz, diagnostics

@pytest.mark.parametrize("case", ["single_drop_32", "drops4_48"])
def test_init_state_parity(case):
    p, u, phi, prm = _oracle_state(case)
    st = box.init_state(u, phi, prm)
    s = _solver(p)
    s.init_state(_dev(u), _dev(phi))
    uh, ph = s.get_state()
    assert rel_l2(_host(uh), st["uh"]) < 1e-13
    assert rel_l2(_host(ph), st["ph"]) < 1e-13
    d = s.diagnostics()
    od = box.diagnostics(st, prm.n, prm.dt)
    assert abs(d["mean_phi"] - od["mean_phi"]) < 1e-14
    assert abs(d["cfl"] - od["cfl"]) < 1e-12 * od["cfl"]
    assert abs(d["ke"] - od["ke"]) < 1e-12 * od["ke"]
    assert abs(d["grad2"] - od["grad2"]) < 1e-12 * od["grad2"]
    assert d["max_div"] < 1e-13 and d["nonfinite"] == 0


def test_init_rejects_nonfinite_input():
    from paper_2406_01322_amd.psms import PsmsError
    p, u, phi, prm = _oracle_state("single_drop_32")
    phi = phi.copy()
    phi[3, 4, 5] = np.nan
    s = _solver(p)
    with pytest.raises(PsmsError) as e:
        s.init_state(_dev(u), _dev(phi))
    assert e.value.code == -5


def test_step_before_init_is_rejected():
    from paper_2406_01322_amd.psms import PsmsError
    s = _solver(_params(16))
    with pytest.raises(PsmsError) as e:
        s.step(1)
    assert e.value.code == -6


@pytest.mark.parametrize("n", [16, 48])
def test_helmholtz_parity(n):
    rng = np.random.default_rng(5)
    g = box.fwd(rng.standard_normal((2, n, n, n)))
    s = _solver(_params(n))
    got = _host(s.solve_helmholtz(_dev(g), [0.0, 3.5]))
    want = np.stack([box.solve_helmholtz(g[0], 0.0), box.solve_helmholtz(g[1], 3.5)])
    assert rel_l2(got, want) < 1e-15


# ------------------------------------------------------------------ the step

def _prepare(case, nprev):
    """Oracle state after init and `nprev` oracle steps (history populated if nprev > 0)."""
    p, u, phi, prm = _oracle_state(case)
    st = box.init_state(u, phi, prm)
    st = box.run(st, prm, nprev)
    return p, prm, st


def _load(s, st):
    hist = np.concatenate([st["hS"], st["hphi"][None]])
    s.set_state(_dev(st["uh"]), _dev(st["ph"]), _dev(hist), st["nstep"])


@pytest.mark.parametrize("case", ["single_drop_32", "drops4_48", "drops2_64", "drops3_96"])
@pytest.mark.parametrize("nprev", [0, 1])
def test_one_step_parity_fp64(case, nprev):
    p, prm, st = _prepare(case, nprev)
    ref = box.step(st, prm)
    s = _solver(p)
    _load(s, st)
    s.step(1)
    uh, ph, hist = s.get_state(with_history=True)
    uh, ph, hist = _host(uh), _host(ph), _host(hist)
    for i in range(3):
        assert rel_l2(uh[i], ref["uh"][i]) < 1e-12, i
        assert rel_l2(hist[i], ref["hS"][i]) < 1e-12, i
    assert rel_l2(ph, ref["ph"]) < 1e-12
    assert rel_l2(hist[3], ref["hphi"]) < 1e-12
    # mean phi is carried bitwise
    assert ph[0, 0, 0] == st["ph"][0, 0, 0]


@pytest.mark.parametrize("case", ["single_drop_32", "drops4_48", "drops2_64", "drops3_96"])
@pytest.mark.parametrize("nprev", [0, 1])
def test_one_step_parity_mixed(case, nprev):
    p, prm, st = _prepare(case, nprev)
    ref = box.step(st, prm)
    s = _solver(p, precision="mixed")
    _load(s, st)
    s.step(1)
    uh, ph = (_host(t) for t in s.get_state())
    for i in range(3):
        assert rel_l2(uh[i], ref["uh"][i]) < 1e-5, i
    assert rel_l2(ph, ref["ph"]) < 1e-5
    assert ph[0, 0, 0] == st["ph"][0, 0, 0]


def test_ten_steps_single_drop_32_fp64():
    """The 32^3 single-drop workload: 10 steps from the initial fields."""
    p, u, phi, prm = _oracle_state("single_drop_32")
    st = box.run(box.init_state(u, phi, prm), prm, 10)
    s = _solver(p)
    s.init_state(_dev(u), _dev(phi))
    s.step(10)
    uh, ph = (_host(t) for t in s.get_state())
    assert rel_l2(uh, st["uh"]) < 1e-12
    assert rel_l2(ph, st["ph"]) < 1e-12
    d = s.diagnostics()
    assert d["nstep"] == 10 and d["nonfinite"] == 0 and d["max_div"] < 1e-13


def test_step_is_deterministic():
    p, prm, st = _prepare("drops4_48", 1)
    outs = []
    for _ in range(2):
        s = _solver(p)
        _load(s, st)
        s.step(3)
        outs.append([_host(t) for t in s.get_state()])
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


@functools.lru_cache(maxsize=2)
def _low_mode_fields(n):
    return synth.band_limited_box(n, seed=21)


def _low_modes(a, k_to):
    """Entries |k_i| <= k_to (kx = 0..k_to) of a half-spectrum array [..., N, N, N/2+1],
    in the order ky, kz = 0..k_to, -k_to..-1, and the largest entry elsewhere."""
    n = a.shape[-2]
    idx = list(range(0, k_to + 1)) + [n - m for m in range(k_to, 0, -1)]
    sub = a[..., idx, :, :][..., :, idx, :][..., :, :, : k_to + 1]
    rest = a.copy()
    rest[..., : k_to + 1] = np.where(np.isin(np.arange(n), idx)[:, None, None] & np.isin(np.arange(n), idx)[None, :, None],
                                     0.0, rest[..., : k_to + 1])
    return sub, np.max(np.abs(rest))


@pytest.mark.parametrize("n", [192, 256])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_large_n_band_limited_steps_match_the_oracle_at_32(n, precision, tol):
    """N = 192 and 256 (the radix-3 plans and the x stage's direct-to-LDS staging at
    N = 256): a band-limited state steps to the same spectral state as at N = 32,
    where the oracle computes it; two steps (Adams-Bashforth 1, then 2).  After the
    first step every mode outside |k_i| <= 10 is zero; the second step's products
    reach beyond the N = 32 band, whose phi^3 then aliases at the 4e-14 level (checked
    on the oracle at N = 48 and 64), so only the modes |k_i| <= 10 are compared."""
    p = _params(32, re=200.0, we=2.0, ch=0.05, pe=20.0, dt=2e-3)
    prm = box.Params(**p)
    u32, phi32 = _low_mode_fields(32)
    st1 = box.step(box.init_state(u32, phi32, prm), prm)
    st2 = box.step(st1, prm)
    u, phi = _low_mode_fields(n)
    s = _solver(dict(p, n=n), precision=precision)
    s.init_state(_dev(u), _dev(phi))
    K32 = (32 - 1) // 3
    for i, ref in enumerate((st1, st2)):
        s.step(1)
        uh, ph = (_host(t) for t in s.get_state())
        su, ru = _low_modes(uh, K32)
        sp, rp = _low_modes(ph, K32)
        wu, _ = _low_modes(ref["uh"], K32)
        wp, _ = _low_modes(ref["ph"], K32)
        assert rel_l2(su, wu) < tol, rel_l2(su, wu)
        assert rel_l2(sp, wp) < tol, rel_l2(sp, wp)
        if i == 0:
            assert ru < tol * np.max(np.abs(wu)) and rp < tol * np.max(np.abs(wp))


@pytest.fixture(scope="module")
def drops256():
    """The 256^3 two-drop case (full state, every mode of the band populated): the
    oracle's state after init and one step, and its second (Adams-Bashforth 2) step."""
    p, u, phi, prm = _oracle_state("drops2_256")
    st = box.step(box.init_state(u, phi, prm), prm)
    ref = box.step(st, prm)
    return p, st, ref


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_full_state_256_one_step(drops256, precision, tol, record_error):
    """N = 256 on a full state (the band edge K = 85, the radix-2 plans and the x
    stage's direct-to-LDS staging on real data): one AB2 step against the oracle."""
    p, st, ref = drops256
    s = _solver(p, precision=precision)
    _load(s, st)
    s.step(1)
    uh, ph, hist = (_host(t) for t in s.get_state(with_history=True))
    for i in range(3):
        assert record_error("u%d" % i, rel_l2(uh[i], ref["uh"][i]), tol) < tol, i
        assert record_error("hS%d" % i, rel_l2(hist[i], ref["hS"][i]), tol) < tol, i
    assert record_error("phi", rel_l2(ph, ref["ph"]), tol) < tol
    assert record_error("hphi", rel_l2(hist[3], ref["hphi"]), tol) < tol
    assert ph[0, 0, 0] == st["ph"][0, 0, 0]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_full_size_128_one_step(precision, tol):
    """The 128^3 sixteen-drop workload at full size, one step from the oracle's state."""
    p, u, phi, prm = _oracle_state("drops16_128")
    st = box.init_state(u, phi, prm)
    st = box.step(st, prm)
    ref = box.step(st, prm)
    s = _solver(p, precision=precision)
    _load(s, st)
    s.step(1)
    uh, ph = (_host(t) for t in s.get_state())
    for i in range(3):
        assert rel_l2(uh[i], ref["uh"][i]) < tol, i
    assert rel_l2(ph, ref["ph"]) < tol


def test_graph_replay_matches_eager_steps():
    """Steps replayed from a captured hipGraph (non-default stream) equal eager steps
    bitwise, with host work between replays."""
    p, prm, st = _prepare("drops4_48", 0)
    eager = _solver(p)
    eager.set_graphs(False)
    _load(eager, st)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        g = _solver(p)
        g.set_graphs(True)
        _load(g, st)
    for k in (1, 2, 3):
        eager.step(k)
        with torch.cuda.stream(side):
            g.step(k)
            a = g.get_state()
        side.synchronize()
        b = eager.get_state()
        torch.cuda.synchronize()
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


@pytest.mark.parametrize("graphs", [False, True])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_diagnostics_between_steps_leave_the_trajectory_unchanged(precision, graphs):
    """psms_diagnostics reuses the step's scratch for the CFL transforms; the next
    step must rebuild its input (bitwise the same trajectory, eager and graph)."""
    p, prm, st = _prepare("drops4_48", 0)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        a = _solver(p, precision)
        a.set_graphs(graphs)
        _load(a, st)
        a.step(4)
        ua = a.get_state()
        b = _solver(p, precision)
        b.set_graphs(graphs)
        _load(b, st)
        b.step(2)
        d = b.diagnostics()
        b.step(2)
        ub = b.get_state()
    side.synchronize()
    assert d["nstep"] == 2 and d["cfl"] > 0.0
    assert torch.equal(ua[0], ub[0]) and torch.equal(ua[1], ub[1])


# ------------------------------------------------------------------ exact cube, pressure

def _solver_cube(p, precision="fp64", stream=None):
    from paper_2406_01322_amd.psms import Solver
    return Solver(p["n"], p["re"], p["we"], p["ch"], p["pe"], p["dt"], precision=precision, cube="exact",
                  stream=stream)


@pytest.mark.parametrize("case", ["single_drop_32", "drops4_48", "drops2_64", "drops3_96"])
@pytest.mark.parametrize("nprev", [0, 1])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_exact_cube_one_step_parity(case, nprev, precision, tol, record_error):
    """phi^3 formed on the padded grid (48, 64, 96, 128 points for N = 32, 48, 64, 96)
    against the oracle's exact cube, one step from the oracle's state."""
    p, u, phi, _ = _oracle_state(case)
    prm = box.Params(**p, cube="exact")
    st = box.run(box.init_state(u, phi, prm), prm, nprev)
    ref = box.step(st, prm)
    s = _solver_cube(p, precision)
    _load(s, st)
    s.step(1)
    uh, ph, hist = (_host(t) for t in s.get_state(with_history=True))
    for i in range(3):
        assert record_error("u%d" % i, rel_l2(uh[i], ref["uh"][i]), tol) < tol, i
    assert record_error("phi", rel_l2(ph, ref["ph"]), tol) < tol
    assert record_error("hphi", rel_l2(hist[3], ref["hphi"]), tol) < tol
    assert ph[0, 0, 0] == st["ph"][0, 0, 0]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_exact_cube_full_size_128(precision, tol):
    """The 128^3 sixteen-drop workload with the exact cube (padded grid 192^3)."""
    p, u, phi, _ = _oracle_state("drops16_128")
    prm = box.Params(**p, cube="exact")
    st = box.step(box.init_state(u, phi, prm), prm)
    ref = box.step(st, prm)
    s = _solver_cube(p, precision)
    _load(s, st)
    s.step(1)
    uh, ph = (_host(t) for t in s.get_state())
    for i in range(3):
        assert rel_l2(uh[i], ref["uh"][i]) < tol, i
    assert rel_l2(ph, ref["ph"]) < tol


def test_exact_cube_graph_replay_matches_eager_steps():
    p, prm, st = _prepare("drops4_48", 0)
    eager = _solver_cube(p)
    eager.set_graphs(False)
    _load(eager, st)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        g = _solver_cube(p, stream=side)
        g.set_graphs(True)
        _load(g, st)
    for k in (1, 2, 3):
        eager.step(k)
        with torch.cuda.stream(side):
            g.step(k)
            a = g.get_state()
        side.synchronize()
        b = eager.get_state()
        torch.cuda.synchronize()
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_exact_cube_is_refused_where_unsupported():
    from paper_2406_01322_amd import psms
    from paper_2406_01322_amd.psms import PsmsError
    with pytest.raises(PsmsError) as e:
        _solver_cube(_params(256))
    assert e.value.code == -4
    prm = psms.make_params(32, 100, 1, 0.05, 20, 1e-3, cube="exact")
    import ctypes
    b = ctypes.c_size_t(0)
    assert psms.lib().psms_batch_workspace_bytes(1, ctypes.byref(prm), ctypes.byref(b)) == -4
    assert psms.lib().psms_adjoint_workspace_bytes(ctypes.byref(prm), 4, 2, ctypes.byref(b)) == -4


@pytest.mark.parametrize("case", ["single_drop_32", "drops4_48", "drops2_64"])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_pressure_parity(case, precision, tol, record_error):
    p, prm, st = _prepare(case, 1)
    want = box.pressure(st, prm)
    s = _solver(p, precision)
    _load(s, st)
    got = _host(s.pressure())
    assert record_error("p", rel_l2(got, want), tol) < tol
    # the step after a pressure evaluation is unchanged
    s.step(1)
    uh, ph = (_host(t) for t in s.get_state())
    ref = box.step(st, prm)
    assert rel_l2(uh, ref["uh"]) < tol and rel_l2(ph, ref["ph"]) < tol


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_laplace_pressure_jump_on_the_gpu(precision):
    """A resting spherical drop (R = 1.5, Ch = 0.12, We = 2, N = 64): the pressure jump
    between the drop's centre and the far corner is the Laplace pressure 2 / (We R) to 1%,
    i.e. the Korteweg force carries surface tension 1/We (eq. kort)."""
    n, ch, we, R = 64, 0.12, 2.0, 1.5
    p = dict(n=n, re=100.0, we=we, ch=ch, pe=10.0, dt=1e-3)
    phi = synth.drops_phi(n, np.array([[np.pi, np.pi, np.pi]]), R, ch)
    s = _solver(p, precision)
    s.init_state(_dev(np.zeros((3, n, n, n))), _dev(phi))
    pr = np.fft.irfftn(_host(s.pressure()), s=(n, n, n), norm="forward")
    jump = pr[n // 2, n // 2, n // 2] - pr[0, 0, 0]
    assert abs(jump - 2.0 / (we * R)) < 0.01 * 2.0 / (we * R), jump


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_recorded_sphi0_is_at_rounding_level(precision):
    """The z stage records S_phi(k = 0) before setting it to zero (every CH term is a
    divergence): like the oracle's record, it sits at the rounding level of S_phi."""
    p, prm, st = _prepare("drops4_48", 1)
    _, sphi, sphi0 = box.nonlinear_terms(st["uh"], st["ph"], prm)
    scale = np.max(np.abs(sphi))
    s = _solver(p, precision)
    _load(s, st)
    assert s.diagnostics()["sphi0"] == 0.0
    s.step(1)
    got = s.diagnostics()["sphi0"]
    bar = (1e-13 if precision == "fp64" else 1e-6) * scale
    assert abs(sphi0) < 1e-13 * scale
    assert abs(got) < bar, (got, sphi0, scale)
