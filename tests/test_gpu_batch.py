"""Batches of uneven boxes: grouped launches and hipGraph replays against single-box runs.

Every box of a batch is advanced by the same kernels as a single-box context,
so batch results (eager or graph-replayed, any workgroup-size variant) must be
bitwise identical to single-box results; one box is also checked against the
FP64 oracle.
"""
import numpy as np
import pytest

from oracle import box as obox
from paper_2406_01322_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _cases(seed=21, nbox=6, sizes=(16, 24, 32, 48)):
    return synth.batch_cases(nbox=nbox, seed=seed, sizes=sizes)


def _single(p, u, phi, nsteps, precision):
    from paper_2406_01322_amd.psms import Solver
    s = Solver(p["n"], p["re"], p["we"], p["ch"], p["pe"], p["dt"], precision=precision)
    s.init_state(torch.from_numpy(u).cuda(), torch.from_numpy(phi).cuda())
    s.step(nsteps)
    uh, ph = s.get_state()
    torch.cuda.synchronize()
    return uh.cpu().numpy(), ph.cpu().numpy()


def _batch(cases, precision):
    from paper_2406_01322_amd.psms import Batch
    b = Batch([c[0] for c in cases], precision=precision)
    for i, (p, u, phi) in enumerate(cases):
        b.init_state(i, torch.from_numpy(u), torch.from_numpy(phi))
    return b


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_graph_replays_match_single_box_runs(precision):
    cases = _cases()
    b = _batch(cases, precision)
    assert [n for n, _ in b.groups()] == sorted(set(c[0]["n"] for c in cases))
    done = 0
    for k in (1, 2, 3):      # eager AB1 step, then graph replays with host work in between
        b.step(k, use_graph=True)
        done += k
        for i in (0, len(cases) - 1):
            got = b.get_state(i)
            ref = _single(*cases[i], done, precision)
            assert np.array_equal(got[0].cpu().numpy(), ref[0]), (i, done)
            assert np.array_equal(got[1].cpu().numpy(), ref[1]), (i, done)
    for i in range(len(cases)):
        d = b.diagnostics(i)
        assert d["nstep"] == done and d["nonfinite"] == 0


def test_batch_box_matches_oracle():
    cases = _cases(nbox=3, sizes=(16, 24))
    b = _batch(cases, "fp64")
    b.step(4)
    for i, (p, u, phi) in enumerate(cases):
        prm = obox.Params(**p)
        ref = obox.run(obox.init_state(u, phi, prm), prm, 4)
        uh, ph = b.get_state(i)
        uh, ph = uh.cpu().numpy(), ph.cpu().numpy()
        assert np.linalg.norm(uh - ref["uh"]) <= 1e-12 * np.linalg.norm(ref["uh"])
        assert np.linalg.norm(ph - ref["ph"]) <= 1e-12 * np.linalg.norm(ref["ph"])


def test_autotune_and_variants_do_not_change_results(tmp_path):
    from paper_2406_01322_amd.psms import Batch
    cases = _cases(seed=5, nbox=4, sizes=(16, 32))
    b = Batch([c[0] for c in cases], precision="mixed")
    info = b.autotune(reps=2, cache_path=str(tmp_path / "tune.json"))
    assert info["source"] == "timed"
    for g in info["groups"].values():
        assert all(0 <= v <= 2 for v in g["variants"])
    for i, (p, u, phi) in enumerate(cases):
        b.init_state(i, torch.from_numpy(u), torch.from_numpy(phi))
    b.step(3)
    got = [b.get_state(i) for i in range(len(cases))]
    for variants in ([0] * 8, [1] * 8):
        b2 = Batch([c[0] for c in cases], precision="mixed")
        b2.set_variants(variants)
        for i, (p, u, phi) in enumerate(cases):
            b2.init_state(i, torch.from_numpy(u), torch.from_numpy(phi))
        b2.step(3)
        for i in range(len(cases)):
            x = b2.get_state(i)
            assert torch.equal(x[0], got[i][0]) and torch.equal(x[1], got[i][1])
    # a second batch of the same shape reuses the cached choice
    b3 = Batch([c[0] for c in cases], precision="mixed")
    assert b3.autotune(reps=2, cache_path=str(tmp_path / "tune.json"))["source"] == "cache"


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_64_96_groups_match_single_boxes_under_every_variant(precision):
    """Groups of 64^3 and 96^3 boxes (most of the batched workload's points): the
    default, autotuned and each forced workgroup-size variant give, after an AB1 step
    and two graph replays, bitwise the single-box result of every box."""
    from paper_2406_01322_amd.psms import Batch
    cases = [c for c in synth.batch_cases(nbox=12, seed=4) if c[0]["n"] in (64, 96)][:4]
    assert sorted(set(c[0]["n"] for c in cases)) == [64, 96]
    refs = [_single(*c, 3, precision) for c in cases]
    runs = {"default": None, "v0": [0] * 8, "v1": [1] * 8, "v2": [2] * 8, "tuned": "tune"}
    for name, variants in runs.items():
        b = Batch([c[0] for c in cases], precision=precision)
        if variants == "tune":
            b.autotune(reps=1, cache_path=None)
        elif variants is not None:
            b.set_variants(variants)
        for i, (p, u, phi) in enumerate(cases):
            b.init_state(i, torch.from_numpy(u), torch.from_numpy(phi))
        b.step(1, use_graph=True)
        b.step(2, use_graph=True)
        for i in range(len(cases)):
            got = b.get_state(i)
            assert np.array_equal(got[0].cpu().numpy(), refs[i][0]), (name, i)
            assert np.array_equal(got[1].cpu().numpy(), refs[i][1]), (name, i)
        b.close()


def test_batch_96_box_matches_oracle():
    """A 96^3 box of a batch with a 64^3 box (FP64), two steps, against the oracle."""
    cases = [c for c in synth.batch_cases(nbox=12, seed=4) if c[0]["n"] in (64, 96)]
    cases = [next(c for c in cases if c[0]["n"] == 64), next(c for c in cases if c[0]["n"] == 96)]
    b = _batch(cases, "fp64")
    b.step(2)
    for i, (p, u, phi) in enumerate(cases):
        prm = obox.Params(**p)
        ref = obox.run(obox.init_state(u, phi, prm), prm, 2)
        uh, ph = b.get_state(i)
        uh, ph = uh.cpu().numpy(), ph.cpu().numpy()
        assert np.linalg.norm(uh - ref["uh"]) <= 1e-12 * np.linalg.norm(ref["uh"])
        assert np.linalg.norm(ph - ref["ph"]) <= 1e-12 * np.linalg.norm(ref["ph"])
