"""Host-side checks of bench.py: the clock-settling loop, the byte models and the
single-GPU refusal (no GPU, no library call)."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


class _Stream:
    def __init__(self):
        self.syncs = 0

    def synchronize(self):
        self.syncs += 1


def test_settle_runs_whole_chunks_until_the_time_has_passed():
    calls = []
    st = _Stream()
    n = bench.settle(lambda k: calls.append(k), st, ms=5.0, chunk=7)
    assert n == 7 * len(calls) and n >= 7
    assert set(calls) == {7}
    assert st.syncs == len(calls)      # one synchronisation per chunk, the time read after it


def test_settle_with_zero_time_still_runs_one_chunk():
    calls = []
    assert bench.settle(lambda k: calls.append(k), _Stream(), ms=0.0, chunk=3) == 3
    assert calls == [3]


def test_stage_bytes_follow_the_band_layout():
    n = 128
    K, C, H, Q, M = bench.band(n)
    assert (K, C, H) == (42, 85, 43) and Q == C * H and M == C * C * H
    for cb in (8, 16):
        sb = bench.stage_bytes(n, cb)
        nq, nnh = n * Q * cb, n * n * H * cb
        assert sb["y_inverse"] == 5 * nq + 6 * nnh
        assert sb["x_products"] == 14 * nnh
        assert sb["y_forward"] == 8 * nnh + 8 * nq
        assert sb["z_update"] == 13 * nq + 16 * M * 16
    # FP64 moves twice the transform bytes of MIXED; the state terms are FP64 in both
    assert bench.step_model_bytes(n, False) > bench.step_model_bytes(n, True)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
