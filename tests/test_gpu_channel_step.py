"""GPU parity of the channel step (psms_channel_*) with the FP64 oracle
(oracle/channel_step.py), through the C ABI.

Per step from the same state: FP64 max error <= 1e-9 of each field's maximum
(omega_z, w, phi, U, V: the wall-normal solves of the tau systems at
beta = 2 Re / dt differ from the oracle's dense LU by rounding amplified by the
conditioning, as in the wall-solve tests, and the explicit terms carry fourth
Chebyshev derivatives); MIXED (FP32 transforms and products) rel-L2 <= 1e-5.
The full channel workload (256 x 128 x 129) is checked on sampled (kx, ky) lines,
whose wall-normal solves the oracle performs one by one, and on the mean flow.
"""
import numpy as np
import pytest

from oracle import channel_step as cs
from paper_2406_01322_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _gpu(p, precision, single_phase=None, walls=("noslip", "noslip")):
    from paper_2406_01322_amd.psms import Channel
    sp = p.get("single_phase", False) if single_phase is None else single_phase
    return Channel(p["nx"], p["ny"], p["nc"], p["re"], p["we"], p["ch"], p["pe"], p["dt"], precision=precision,
                   lx=p["lx"], ly=p["ly"], single_phase=sp, walls=walls)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _load(c, st):
    state = np.stack([st["om"], st["w"], st["phi"]])
    hist = np.stack([st["h_om"], st["h_w"], st["h_phi"]])
    c.set_state(_dev(state), _dev(st["mean"]), _dev(hist), _dev(st["h_mean"]), st["nstep"])


def _rel_max(a, b):
    s = np.max(np.abs(b))
    return np.max(np.abs(a - b)) / s if s > 0 else np.max(np.abs(a))


def _rel_l2(a, b):
    s = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / s if s > 0 else np.linalg.norm(a.ravel())


def _case(name):
    p, u, v, w, phi = synth.channel_case(name)
    return p, cs.ChannelParams(**{k: x for k, x in p.items() if k != "single_phase"}), (u, v, w, phi)


@pytest.mark.parametrize("name", ["chan_small", "chan_mid"])
def test_channel_init_state_parity(name):
    p, prm, f = _case(name)
    ref = cs.init_state(*f, prm)
    c = _gpu(p, "fp64")
    c.init_state(*[_dev(x) for x in f])
    state, mean = (_host(t) for t in c.get_state())
    for i, k in enumerate(("om", "w", "phi")):
        assert _rel_max(state[i], ref[k]) < 1e-12, k
    assert _rel_max(mean, ref["mean"]) < 1e-12


@pytest.mark.parametrize("name", ["chan_small", "chan_mid"])
@pytest.mark.parametrize("nprev", [0, 1])
def test_channel_one_step_parity_fp64(name, nprev):
    p, prm, f = _case(name)
    st = cs.run(cs.init_state(*f, prm), prm, nprev)
    ref = cs.step(st, prm)
    c = _gpu(p, "fp64")
    _load(c, st)
    c.step(1)
    state, mean, hist, hmean = (_host(t) for t in c.get_state(with_history=True))
    for i, k in enumerate(("om", "w", "phi")):
        assert _rel_max(state[i], ref[k]) < 1e-9, (k, _rel_max(state[i], ref[k]))
    for i, k in enumerate(("h_om", "h_w", "h_phi")):
        assert _rel_max(hist[i], ref[k]) < 1e-9, (k, _rel_max(hist[i], ref[k]))
    assert _rel_max(mean, ref["mean"]) < 1e-9
    assert _rel_max(hmean, ref["h_mean"]) < 1e-9


@pytest.mark.parametrize("name", ["chan_small", "chan_mid"])
def test_channel_one_step_parity_mixed(name):
    p, prm, f = _case(name)
    st = cs.run(cs.init_state(*f, prm), prm, 1)
    ref = cs.step(st, prm)
    c = _gpu(p, "mixed")
    _load(c, st)
    c.step(1)
    state, mean = (_host(t) for t in c.get_state())
    for i, k in enumerate(("om", "w", "phi")):
        assert _rel_l2(state[i], ref[k]) < 1e-5, (k, _rel_l2(state[i], ref[k]))
    assert _rel_l2(mean, ref["mean"]) < 1e-5


def test_channel_ten_steps_fp64():
    p, prm, f = _case("chan_small")
    ref = cs.run(cs.init_state(*f, prm), prm, 10)
    c = _gpu(p, "fp64")
    c.init_state(*[_dev(x) for x in f])
    c.step(10)
    state, mean = (_host(t) for t in c.get_state())
    for i, k in enumerate(("om", "w", "phi")):
        assert _rel_max(state[i], ref[k]) < 1e-8, (k, _rel_max(state[i], ref[k]))
    assert _rel_max(mean, ref["mean"]) < 1e-8


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("mixed", 1e-5)])
def test_channel_workload_256_sampled_lines(precision, tol):
    """256 x 128 x 129 (the channel workload), one step after one oracle step;
    sampled lines (the mean line, low and band-edge wavenumbers) and the mean flow."""
    p, prm, f = _case("chan_256")
    st = cs.step(cs.init_state(*f, prm), prm)
    lines = [(0, 0), (1, 0), (0, 1), (1, 1), (42, 85), (43, 85), (84, 3), (20, 40)]
    ref = cs.step(st, prm, lines=lines)
    c = _gpu(p, precision)
    _load(c, st)
    c.step(1)
    state, mean = (_host(t) for t in c.get_state())
    for i, k in enumerate(("om", "w", "phi")):
        a = np.stack([state[i][:, iy, ix] for iy, ix in lines])
        b = np.stack([ref[k][:, iy, ix] for iy, ix in lines])
        if precision == "fp64":   # every sampled line to its own scale
            for j, (iy, ix) in enumerate(lines):
                scale = np.max(np.abs(b[j]))
                assert np.max(np.abs(a[j] - b[j])) <= tol * scale or scale == 0.0, (k, iy, ix)
        else:                     # FP32 transforms: errors scale with the field, not the line
            assert _rel_l2(a, b) < tol, (k, _rel_l2(a, b))
    assert _rel_max(mean, ref["mean"]) < tol


def test_channel_step_before_init_is_rejected():
    from paper_2406_01322_amd.psms import PsmsError
    p, prm, f = _case("chan_small")
    c = _gpu(p, "fp64")
    with pytest.raises(PsmsError) as e:
        c.step(1)
    assert e.value.code == -6


# ---------------------------------------------------------------------------
# single phase (Navier-Stokes alone): the oracle's step with phi = 0, in which
# every Korteweg and CH term vanishes identically
# ---------------------------------------------------------------------------

def test_single_phase_equals_two_phase_with_zero_phi():
    """The single-phase path (3 fields to physical space, 6 products back, no CH
    solves) gives the two-phase step with phi = 0, up to rounding."""
    p, prm, f = _case("chan_small")
    u, v, w, _ = f
    zero = np.zeros_like(u)
    out = []
    for sp in (False, True):
        c = _gpu(p, "fp64", single_phase=sp)
        c.init_state(_dev(u), _dev(v), _dev(w), _dev(zero) if not sp else None)
        c.step(3)
        out.append([_host(t) for t in c.get_state(with_history=True)])
    for a, b in zip(out[0], out[1]):
        assert _rel_max(b, a) < 1e-13
    assert np.all(out[1][0][2] == 0.0)


@pytest.mark.parametrize("nprev", [0, 1])
def test_single_phase_nc256_parity_fp64(nprev):
    """16 x 12 x 257 (the 512-point Chebyshev extension), Re_tau 150, dt 1e-4.
    The history holds H_w = lap_h S_z - D div_h S: the norm of D grows as nc^2, so the
    rounding of the transformed products reaches it 4 times amplified from nc = 128,
    where the bound is 1e-9: 4e-9 here."""
    p, prm, f = _case("chan_sp_small")
    st = cs.run(cs.init_state(*f, prm), prm, nprev)
    ref = cs.step(st, prm)
    c = _gpu(p, "fp64")
    _load(c, st)
    c.step(1)
    state, mean, hist, hmean = (_host(t) for t in c.get_state(with_history=True))
    tol = 1e-9 * (p["nc"] / 128) ** 2
    for i, k in enumerate(("om", "w")):
        assert _rel_max(state[i], ref[k]) < tol, (k, _rel_max(state[i], ref[k]))
        assert _rel_max(hist[i], ref["h_" + k]) < tol, (k, _rel_max(hist[i], ref["h_" + k]))
    assert np.all(state[2] == 0.0)
    assert _rel_max(mean, ref["mean"]) < tol
    assert _rel_max(hmean, ref["h_mean"]) < tol


def test_single_phase_nc256_parity_mixed():
    p, prm, f = _case("chan_sp_small")
    st = cs.run(cs.init_state(*f, prm), prm, 1)
    ref = cs.step(st, prm)
    c = _gpu(p, "mixed")
    _load(c, st)
    c.step(1)
    state, mean = (_host(t) for t in c.get_state())
    for i, k in enumerate(("om", "w")):
        assert _rel_l2(state[i], ref[k]) < 1e-5, (k, _rel_l2(state[i], ref[k]))
    assert _rel_l2(mean, ref["mean"]) < 1e-5


@pytest.fixture(scope="module")
def sp256():
    """256 x 256 x 257 single phase: the oracle's first (Adams-Bashforth 1) step from
    the initial state, on sampled lines."""
    p, prm, f = _case("chan_sp_256")
    st = cs.init_state(*f, prm)
    lines = [(0, 0), (1, 0), (0, 1), (1, 1), (85, 85), (84, 85), (3, 84), (40, 20)]
    ref = cs.step(st, prm, lines=lines)
    return p, f, lines, ref


@pytest.mark.parametrize("precision,tol", [("fp64", 4e-9), ("mixed", 1e-5)])
def test_single_phase_256_sampled_lines(sp256, precision, tol):
    """FP64: each sampled line to its own scale (the nc = 256 bound above); the
    band-edge lines, which the first step from modes |k| <= 4 leaves at zero up to
    rounding, to the rounding level of the field (1e-14 of its largest line)."""
    p, f, lines, ref = sp256
    c = _gpu(p, precision)
    c.init_state(*[_dev(x) for x in f[:3]])
    c.step(1)
    state, mean = (_host(t) for t in c.get_state())
    for i, k in enumerate(("om", "w")):
        a = np.stack([state[i][:, iy, ix] for iy, ix in lines])
        b = np.stack([ref[k][:, iy, ix] for iy, ix in lines])
        if precision == "fp64":
            floor = 1e-14 * np.max(np.abs(b))
            for j, (iy, ix) in enumerate(lines):
                scale = np.max(np.abs(b[j]))
                assert np.max(np.abs(a[j] - b[j])) <= tol * scale + floor, (k, iy, ix)
        else:
            assert _rel_l2(a, b) < tol, (k, _rel_l2(a, b))
    assert _rel_max(mean, ref["mean"]) < tol


# ---------------------------------------------------------------------------
# free-slip walls (a different tau row at that wall: omega_z' = 0, psi = 0,
# U' = 0), alone or with a no-slip wall (the two parities of the tau chains
# couple)
# ---------------------------------------------------------------------------

WALLS = [("freeslip", "noslip"), ("noslip", "freeslip"), ("freeslip", "freeslip")]


@pytest.mark.parametrize("walls", WALLS)
@pytest.mark.parametrize("nprev", [0, 1])
def test_free_slip_walls_one_step_parity_fp64(walls, nprev):
    import dataclasses
    p, prm, f = _case("chan_mid")
    prm = dataclasses.replace(prm, walls=walls)
    st = cs.run(cs.init_state(*f, prm), prm, nprev)
    ref = cs.step(st, prm)
    c = _gpu(p, "fp64", walls=walls)
    _load(c, st)
    c.step(1)
    state, mean, hist, hmean = (_host(t) for t in c.get_state(with_history=True))
    for i, k in enumerate(("om", "w", "phi")):
        assert _rel_max(state[i], ref[k]) < 1e-9, (k, _rel_max(state[i], ref[k]))
    assert _rel_max(mean, ref["mean"]) < 1e-9
    assert _rel_max(hmean, ref["h_mean"]) < 1e-9


@pytest.mark.parametrize("walls", WALLS)
def test_free_slip_walls_one_step_parity_mixed(walls):
    import dataclasses
    p, prm, f = _case("chan_small")
    prm = dataclasses.replace(prm, walls=walls)
    st = cs.run(cs.init_state(*f, prm), prm, 1)
    ref = cs.step(st, prm)
    c = _gpu(p, "mixed", walls=walls)
    _load(c, st)
    c.step(1)
    state, mean = (_host(t) for t in c.get_state())
    for i, k in enumerate(("om", "w", "phi")):
        assert _rel_l2(state[i], ref[k]) < 1e-5, (k, _rel_l2(state[i], ref[k]))
    assert _rel_l2(mean, ref["mean"]) < 1e-5


def test_free_slip_ten_steps_fp64():
    import dataclasses
    p, prm, f = _case("chan_small")
    walls = ("freeslip", "noslip")
    prm = dataclasses.replace(prm, walls=walls)
    ref = cs.run(cs.init_state(*f, prm), prm, 10)
    c = _gpu(p, "fp64", walls=walls)
    c.init_state(*[_dev(x) for x in f])
    c.step(10)
    state, mean = (_host(t) for t in c.get_state())
    for i, k in enumerate(("om", "w", "phi")):
        assert _rel_max(state[i], ref[k]) < 1e-8, (k, _rel_max(state[i], ref[k]))
    assert _rel_max(mean, ref["mean"]) < 1e-8


def test_bad_wall_flags_are_rejected():
    from paper_2406_01322_amd.psms import Channel
    p, prm, f = _case("chan_small")
    with pytest.raises(ValueError):
        Channel(p["nx"], p["ny"], p["nc"], p["re"], p["we"], p["ch"], p["pe"], p["dt"], walls=("slip", "noslip"))


def test_single_phase_open_channel_parity_fp64():
    """Single phase under a free-slip top wall (both switches at once), one AB2 step
    against the oracle's step with phi = 0 and the same walls."""
    import dataclasses
    p, prm, f = _case("chan_mid")
    walls = ("freeslip", "noslip")
    prm = dataclasses.replace(prm, walls=walls)
    u, v, w, _ = f
    zero = np.zeros_like(u)
    st = cs.run(cs.init_state(u, v, w, zero, prm), prm, 1)
    ref = cs.step(st, prm)
    c = _gpu(p, "fp64", single_phase=True, walls=walls)
    _load(c, st)
    c.step(1)
    state, mean = (_host(t) for t in c.get_state())
    for i, k in enumerate(("om", "w")):
        assert _rel_max(state[i], ref[k]) < 1e-9, (k, _rel_max(state[i], ref[k]))
    assert np.all(state[2] == 0.0)
    assert _rel_max(mean, ref["mean"]) < 1e-9
