"""Throughput of the coupled NS + CH pseudo-spectral step on one MI355X.

Workload: triply periodic box, 128^3 Fourier grid, 16 drops of radius 0.4 at
seeded non-overlapping centres, random-phase solenoidal velocity with
E(k) ~ k^4 exp(-2 (k/4)^2), u_rms = 1; Re = 300, We = 1, Ch = 0.025,
Pe = 1/Ch, dt = 5e-4 (seed 2).  One "step" is one full time step (all
transforms, products, RHS assembly, projection and implicit updates).

`value` is the MIXED path (FP32 transforms and products, FP64 state, RHS
assembly, projection and update) in grid-points x time-steps per second; the
plain FP64 path is reported beside it.  The dominant kernel's HBM roofline is
measured live with HIP events on the library's stream; `cpu_baseline` times
the FP64 oracle on the host on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps 200] [--warmup 10] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "grid-points·timesteps/s for NS+CH step (FP64 vs mixed) + % HBM roofline"
HBM_PEAK_GBS = 8000.0
STAGES = ["y_inverse", "x_products", "y_forward", "z_update"]
KERNELS = {"y_inverse": "k_ystep<+1>", "x_products": "k_xstep", "y_forward": "k_ystep<-1>",
           "z_update": "k_zstep"}


def band(n):
    K = (n - 1) // 3
    C, H = 2 * K + 1, K + 1
    return K, C, H, C * H, C * C * H


def stage_bytes(n, cplx_bytes):
    """Algorithmic HBM bytes of one launch of each stage kernel: every array the
    kernel must read or write, counted once, at its stored (retained-band) size."""
    K, C, H, Q, M = band(n)
    t = cplx_bytes
    nq, nnh = n * Q, n * n * H
    return {
        "y_inverse": (5 * nq + 6 * nnh) * t,
        "x_products": (6 * nnh + 8 * nnh) * t,
        "y_forward": (8 * nnh + 8 * nq) * t,
        "z_update": (8 * nq + 5 * nq) * t + 4 * 4 * M * 16,  # + state and history read and written, FP64
    }


def step_model_bytes(n, mixed):
    """Whole-step byte model: every method-defined intermediate written once and read
    once, spectral arrays at their retained size (7 inverse outputs, 8 products,
    8 forward inputs; state read twice and written once, history read and written,
    8 RHS fields written and read)."""
    P = n ** 3
    M = band(n)[4]
    w_phys = 4 if mixed else 8      # bytes per real word, physical fields
    w_rhs = 4 if mixed else 8       # bytes per real word, RHS fields
    w_state = 8                     # FP64 state and history
    return w_phys * 30 * P + w_state * 2 * 20 * M + w_rhs * 2 * 16 * M


def measured_traffic(stage, precision="mixed"):
    """HBM bytes per launch of a stage kernel from the committed counter record
    (profiles/box128_<precision>_hbm_counters.json), or None if the kernel sources
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "box128_%s_hbm_counters.json" % precision)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec["source_sha256"]:
        return None
    return rec["hbm_bytes_per_launch"].get(stage)


SETTLE_MS = 40.0


def settle(step, stream, ms=SETTLE_MS, chunk=25):
    """Advance the workload `chunk` steps at a time until `ms` of wall time have passed,
    before the warm-up steps of a timed leg.  From idle, the GPU's clocks ramp over
    about 20 ms of load and the step time with them (128^3 MIXED step, 5-step regions
    from a cold start: 0.089-0.098 ms over the first 7 ms, 0.0815 ms from 20 ms on);
    the steps run here are reported (`settle_steps`) and not counted as warm-up."""
    t0 = time.perf_counter()
    done = 0
    while True:
        step(chunk)
        done += chunk
        stream.synchronize()
        if (time.perf_counter() - t0) * 1e3 >= ms:
            return done


def run_gpu(precision, n, p, u, phi, steps, warmup):
    """Time `steps` steps (the step's four kernels launched directly, which measured
    faster than replaying a captured hipGraph of them; HIP events bracketing the region
    on the library's stream, plus the wall clock), then the same number of steps with an
    event around every kernel for the per-kernel durations."""
    import torch
    from paper_2406_01322_amd.psms import Solver
    stream = torch.cuda.Stream()       # the library's stream (not the legacy default one)
    with torch.cuda.stream(stream):
        s = Solver(n, p["re"], p["we"], p["ch"], p["pe"], p["dt"], precision=precision)
        s.init_state(torch.from_numpy(u).cuda(), torch.from_numpy(phi).cuda())
        nset = settle(s.step, stream)
        s.step(warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        s.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ev_ms = e0.elapsed_time(e1)
        reps = []                      # four more timed regions of the same length
        for _ in range(4):
            e0.record(stream)
            s.step(steps)
            e1.record(stream)
            e1.synchronize()
            reps.append(e0.elapsed_time(e1) / steps)
        ms = s.stage_times(steps)      # per-kernel HIP events, eager launches of the same kernels
        torch.cuda.synchronize()
        d = s.diagnostics()
    if d["nonfinite"] or not (d["max_div"] < 1e-8):
        raise RuntimeError("%s run produced a bad state: %s" % (precision, d))
    wall = t1 - t0
    med = sorted(reps + [ev_ms / steps])[2]
    return dict(wall=wall, ms_per_step=1e3 * wall / steps, value=n ** 3 * steps / wall,
                event_ms_per_step=ev_ms / steps, median_of_5_ms_per_step=med, settle_steps=nset,
                stage_ms=dict(zip(STAGES, ms)), diag=d)


def mixed_error(n, p, u, phi, nsteps=(1, 20)):
    """Per-field rel-L2 of the MIXED state against the FP64 GPU state (the FP64 path is
    held to 1e-12 of the FP64 oracle by the parity tests), after each count in nsteps."""
    import torch
    from paper_2406_01322_amd.psms import Solver
    out = {}
    ss = {}
    for prec in ("fp64", "mixed"):
        s = Solver(n, p["re"], p["we"], p["ch"], p["pe"], p["dt"], precision=prec)
        s.init_state(torch.from_numpy(u).cuda(), torch.from_numpy(phi).cuda())
        ss[prec] = s
    done = 0
    for k in nsteps:
        for s in ss.values():
            s.step(k - done)
        done = k
        a = ss["fp64"].get_state()
        b = ss["mixed"].get_state()
        torch.cuda.synchronize()
        rel = {}
        for name, x, y in (("u", a[0][0], b[0][0]), ("v", a[0][1], b[0][1]), ("w", a[0][2], b[0][2]),
                           ("phi", a[1], b[1])):
            rel[name] = float(torch.linalg.norm(y - x) / torch.linalg.norm(x))
        out["after_%d_steps" % k] = rel
    return out


def copy_peak(nbytes=1 << 30, reps=10):
    """Measured device-to-device copy bandwidth (read + write bytes / time) of a 1 GiB
    buffer, HIP events around `reps` copies: the practical HBM ceiling beside the
    8 TB/s peak."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return gbs


def bench_batch(steps=100, nbox=96):
    """The batched form: 96 independent boxes, N drawn from {32, 48, 64, 96}, 1-8 drops,
    Re ~ U[50, 400], We ~ U[0.5, 5], MIXED; workgroup sizes autotuned; each stage is one
    launch per group of equal N.  Timed with HIP events on the batch stream."""
    import torch
    from paper_2406_01322_amd import synth
    from paper_2406_01322_amd.psms import Batch
    cases = synth.batch_cases(nbox=nbox, seed=4)
    b = Batch([c[0] for c in cases], precision="mixed")
    tune = b.autotune(reps=3)
    for i, (p, u, phi) in enumerate(cases):
        b.init_state(i, torch.from_numpy(u), torch.from_numpy(phi))
    b.step(2)                                   # AB1 step and one AB2 step
    nset = settle(b.step, b.stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(b.stream)
    b.step(steps)
    e1.record(b.stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    pts = sum(c[0]["n"] ** 3 for c in cases)
    bad = [i for i in range(nbox) if b.diagnostics(i)["nonfinite"]]
    if bad:
        raise RuntimeError("batched boxes went non-finite: %s" % bad)
    return {"boxes": nbox, "groups": b.groups(), "total_points": pts, "steps": steps, "settle_steps": nset,
            "ms_per_step": ms / steps, "value": pts * steps / (ms * 1e-3), "unit": "grid-points*timesteps/s",
            "variants": {k: v["variants"] for k, v in tune["groups"].items()}}


def bench_adjoint(nsteps=50, seg_len=10):
    """The adjoint form: 128^3 16-drop workload, MIXED primal with FP64 checkpoints every
    seg_len steps, FP64 segment recompute and discrete adjoint; J = int |grad phi|^2 +
    1/2 int |u|^2; gradient with respect to phi0 and We."""
    import torch
    from paper_2406_01322_amd import synth
    from paper_2406_01322_amd.psms import Adjoint
    p, u, phi = synth.box_case("drops16_128")
    a = Adjoint(p["n"], p["re"], p["we"], p["ch"], p["pe"], p["dt"], precision="mixed", max_steps=nsteps,
                seg_len=seg_len)
    u_d, phi_d = torch.from_numpy(u).cuda(), torch.from_numpy(phi).cuda()
    a.forward(u_d, phi_d, nsteps)
    a.backward()                                 # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = a.forward(u_d, phi_d, nsteps)
    t1 = time.perf_counter()
    d, dwe = a.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    if not (torch.isfinite(d).all() and math.isfinite(dwe)):
        raise RuntimeError("adjoint produced non-finite values")
    return {"n": p["n"], "steps": nsteps, "checkpoint_every": seg_len, "J": J, "dJ_dWe": dwe,
            "forward_ms": 1e3 * (t1 - t0), "backward_ms": 1e3 * (t2 - t1),
            "backward_over_forward": (t2 - t1) / (t1 - t0)}


def bench_exact_cube(steps=50, precision="mixed"):
    """The 128^3 workload with the exact cube of phi (formed on the padded 192^3 grid)
    instead of the grid cube: ms per step (HIP events)."""
    import torch
    from paper_2406_01322_amd import synth
    from paper_2406_01322_amd.psms import Solver
    p, u, phi = synth.box_case("drops16_128")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        s = Solver(p["n"], p["re"], p["we"], p["ch"], p["pe"], p["dt"], precision=precision, cube="exact",
                   stream=stream)
        s.init_state(torch.from_numpy(u).cuda(), torch.from_numpy(phi).cuda())
        s.step(3)
        nset = settle(s.step, stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        s.step(steps)
        e1.record(stream)
        e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    return {"n": p["n"], "padded_grid": 192, "precision": precision, "steps": steps, "settle_steps": nset,
            "ms_per_step": ms,
            "value": p["n"] ** 3 / (ms * 1e-3), "unit": "grid-points*timesteps/s"}


def bench_wall_solve(reps=20):
    """The channel's implicit wall-normal solves (omega_z, w with the influence matrix,
    the two CH Helmholtz problems, u and v) for kx = 0..85, ky = -42..42 (7310 lines) of
    nc + 1 = 129 Chebyshev coefficients, Re_tau = 150, dt = 1e-4, Ch = 0.02, Pe = 50."""
    import numpy as np
    import torch
    from paper_2406_01322_amd import psms
    nc = 128
    kx = np.repeat(np.arange(86, dtype=float), 85)
    ky = np.tile(np.arange(-42, 43, dtype=float), 86)
    nl = len(kx)
    rng = np.random.default_rng(3)
    g = [torch.from_numpy((rng.standard_normal((nc + 1, nl)) + 1j * rng.standard_normal((nc + 1, nl)))
                          * np.exp(-0.05 * np.arange(nc + 1))[:, None]).cuda() for _ in range(3)]
    kxd, kyd = torch.from_numpy(kx).cuda(), torch.from_numpy(ky).cuda()
    beta_ns = 2.0 * 150.0 / 1e-4
    beta_ch = math.sqrt(50.0 / (1e-4 * 0.02 ** 2))
    psms.wall_solve(kxd, kyd, beta_ns, beta_ch, beta_ch, *g)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        psms.wall_solve(kxd, kyd, beta_ns, beta_ch, beta_ch, *g)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"lines": nl, "nc": nc, "ms_per_solve_set": ms,
            "lines_per_s": nl / (ms * 1e-3)}


def bench_channel(steps=20, warmup=2, case="chan_256"):
    """The channel step, MIXED and FP64: ms per step (HIP events on the stream) after
    `warmup` steps from the synthetic initial state.  chan_256: 256 x 128 x 129
    (4 pi x 2 pi x 2, Re_tau 150, 64 drops R = 0.2, Ch 0.02, We 3, Pe 50, dt 1e-4);
    chan_sp_256: 256 x 256 x 257 single phase (Re_tau 150, dt 1e-4), the grid of the
    paper's single-phase timing runs."""
    import torch
    from paper_2406_01322_amd import psms, synth
    p, u, v, w, phi = synth.channel_case(case)
    sp = p.get("single_phase", False)
    npts = (p["nc"] + 1) * p["ny"] * p["nx"]
    out = {"grid": [p["nx"], p["ny"], p["nc"] + 1], "points": npts, "steps": steps, "single_phase": sp}
    f = [torch.from_numpy(x).cuda() for x in ((u, v, w) if sp else (u, v, w, phi))]
    del u, v, w, phi
    stream = torch.cuda.Stream()       # the library's stream (not the legacy default one)
    torch.cuda.synchronize()
    for prec in ("mixed", "fp64"):
        with torch.cuda.stream(stream):
            c = psms.Channel(p["nx"], p["ny"], p["nc"], p["re"], p["we"], p["ch"], p["pe"], p["dt"], precision=prec,
                             lx=p["lx"], ly=p["ly"], single_phase=sp, stream=stream)
            c.init_state(*f)
            nset = settle(c.step, stream, chunk=5)
            c.step(warmup)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            c.step(steps)
            e1.record(stream)
            e1.synchronize()
        ms = e0.elapsed_time(e1) / steps
        d = c.diagnostics()
        if d["nonfinite"]:
            raise RuntimeError("channel %s run produced a bad state: %s" % (prec, d))
        out[prec] = {"ms_per_step": ms, "value": npts / (ms * 1e-3), "settle_steps": nset}
        c.close()
        del c
    out["unit"] = "grid-points*timesteps/s"
    return out


def cpu_baseline_threaded(n, p, u, phi, budget_s=10.0):
    """The same oracle with its transforms on all the host's cores (scipy.fft,
    workers = the cores this process may use): a second CPU row beside the
    single-threaded one."""
    from oracle import box
    cores = min(len(os.sched_getaffinity(0)), 16)
    box.set_fft_workers(cores)
    try:
        prm = box.Params(**p)
        st = box.init_state(u, phi, prm)
        t0 = time.perf_counter()
        steps = 0
        while True:
            st = box.step(st, prm)
            steps += 1
            el = time.perf_counter() - t0
            if el > budget_s or steps >= 20:
                break
    finally:
        box.set_fft_workers(1)
    return dict(value=n ** 3 * steps / el, unit="grid-points*timesteps/s", cores=cores, kind="oracle",
                sample="%d FP64 oracle steps of the %d^3 workload after init, transforms by scipy.fft with "
                       "%d workers, %.1f s" % (steps, n, cores, el))


def channel_oracle_timing(case="chan_256"):
    """One FP64 oracle step of the channel workload from its initial state (every
    (kx, ky) line's tau problems by dense LU, one stacked numpy solve)."""
    from oracle import channel_step as cs
    from paper_2406_01322_amd import synth
    p, u, v, w, phi = synth.channel_case(case)
    prm = cs.ChannelParams(**{k: x for k, x in p.items() if k != "single_phase"})
    st = cs.init_state(u, v, w, phi, prm)
    t0 = time.perf_counter()
    cs.step(st, prm)
    el = time.perf_counter() - t0
    npts = (p["nc"] + 1) * p["ny"] * p["nx"]
    return dict(value=npts / el, unit="grid-points*timesteps/s", cores=1, kind="oracle (dense LU)",
                sample="1 FP64 oracle step of the %d x %d x %d channel from its initial state "
                       "(wall-normal tau problems by dense LU), %.1f s" % (p["nx"], p["ny"], p["nc"] + 1, el))


def channel_model_bytes(nx, ny, nc, mixed):
    """The step byte model of the channel in the box's convention: 30 physical passes,
    the FP64 state (omega_z, w, phi on every Chebyshev mode) read twice and written once
    with its history read and written, 8 right-hand-side fields written and read at
    the products' Chebyshev cut."""
    hx, cy = (nx - 1) // 3 + 1, 2 * ((ny - 1) // 3) + 1
    kz = (2 * nc - 1) // 3
    P = (nc + 1) * ny * nx
    w_phys = 4 if mixed else 8
    return w_phys * 30 * P + 8 * 2 * 20 * hx * cy * (nc + 1) + w_phys * 2 * 16 * hx * cy * (kz + 1)


def roofline_entry(nbytes, ms, traffic=None):
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "traffic": traffic, "model_bytes_per_step": nbytes, "ms_per_step": ms}


def step_traffic(precision):
    """Counted HBM bytes of one box step (the four stage kernels), or None."""
    t = [measured_traffic(st, precision) for st in STAGES]
    return None if any(v is None for v in t) else sum(t)


def channel_traffic(precision):
    """Counted HBM bytes of one 256 x 128 x 129 channel step from the committed counter
    record (profiles/channel256_hbm_counters.json), or None if the sources it was taken
    with have changed."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "channel256_hbm_counters.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec["source_sha256"]:
        return None
    return rec["hbm_bytes_per_step"].get(precision)


def cpu_baseline(n, p, u, phi, budget_s=20.0):
    """The FP64 oracle on the host: init, then as many steps as fit in ~budget_s.
    Also returns the oracle's states after its first and second steps, from which the
    GPU's per-step error is measured."""
    from oracle import box
    prm = box.Params(**p)
    st = box.init_state(u, phi, prm)
    t0 = time.perf_counter()
    steps = 0
    kept = []
    while True:
        st = box.step(st, prm)
        steps += 1
        if steps <= 2:
            kept.append(st)
        el = time.perf_counter() - t0
        if el > budget_s or steps >= 20:
            break
    return dict(value=n ** 3 * steps / el, unit="grid-points*timesteps/s", cores=1, kind="oracle",
                sample="%d FP64 oracle steps of the %d^3 workload after init (numpy pocketfft, "
                       "single-threaded), %.1f s" % (steps, n, el)), kept


def oracle_error(n, p, st1, st2):
    """Per-field rel-L2 of one GPU step (FP64 and MIXED) from the oracle's state after
    its first step, against the oracle's second step (an AB2 step)."""
    import numpy as np
    import torch
    from paper_2406_01322_amd.psms import Solver
    hist = np.concatenate([st1["hS"], st1["hphi"][None]])
    out = {}
    for prec in ("fp64", "mixed"):
        s = Solver(n, p["re"], p["we"], p["ch"], p["pe"], p["dt"], precision=prec)
        s.set_state(torch.from_numpy(st1["uh"]).cuda(), torch.from_numpy(st1["ph"]).cuda(),
                    torch.from_numpy(hist).cuda(), st1["nstep"])
        s.step(1)
        uh, ph = (t.cpu().numpy() for t in s.get_state())
        rel = {}
        for name, a, b in (("u", uh[0], st2["uh"][0]), ("v", uh[1], st2["uh"][1]), ("w", uh[2], st2["uh"][2]),
                           ("phi", ph, st2["ph"])):
            rel[name] = float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
        out[prec] = rel
        s.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only", choices=["fp64", "mixed"], default=None)
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the batched, adjoint, channel wall-solve and channel-step measurements")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="first copy a buffer of this many MiB 3 times (HBM counter calibration)")
    ap.add_argument("--channel-only", action="store_true",
                    help="measure only the 256 x 128 x 129 channel step (--steps timed after --warmup, "
                         "both precisions) and print its JSON record (for profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr, flush=True)
        sys.exit(2)
    import torch
    from paper_2406_01322_amd import synth

    if args.copy_mb > 0:
        src = torch.ones(args.copy_mb * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.channel_only:
        print(json.dumps(bench_channel(args.steps, args.warmup)), flush=True)
        return
    name = "drops16_128"
    p, u, phi = synth.box_case(name)
    n = p["n"]
    precs = [args.only] if args.only else ["fp64", "mixed"]
    res = {}
    for prec in precs:
        res[prec] = run_gpu(prec, n, p, u, phi, args.steps, args.warmup)
        print("[bench] %s: %.4f ms/step, stages %s" % (prec, res[prec]["ms_per_step"],
              {k: round(v, 4) for k, v in res[prec]["stage_ms"].items()}), file=sys.stderr, flush=True)
    head = "mixed" if "mixed" in res else "fp64"
    r = res[head]
    cb = 8 if head == "mixed" else 16
    sb = stage_bytes(n, cb)
    dom = max(r["stage_ms"], key=lambda k: r["stage_ms"][k])
    achieved = sb[dom] / (r["stage_ms"][dom] * 1e-3) / 1e9
    step_bytes = step_model_bytes(n, head == "mixed")
    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "grid-points*timesteps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "periodic box 128^3, 16 drops R=0.4, Re=300, We=1, Ch=0.025, Pe=40, dt=5e-4, seed 2",
                   "n": n, "precision": head,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": KERNELS[dom], "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom, head),
                     "algorithmic_bytes_per_launch": sb[dom]},
        "event_ms_per_step": r["event_ms_per_step"],
        "median_of_5": {"ms_per_step": r["median_of_5_ms_per_step"],
                        "value": n ** 3 / (r["median_of_5_ms_per_step"] * 1e-3)},
        "settle": {"ms": SETTLE_MS, "steps": r["settle_steps"],
                   "note": "steps run for SETTLE_MS of wall time before the warm-up steps, so that the "
                           "timed steps run at the clocks the GPU holds under sustained load"},
        "stage_ms": r["stage_ms"],
        "stage_gbs": {k: sb[k] / (r["stage_ms"][k] * 1e-3) / 1e9 for k in STAGES},
        "copy_peak_gbs": copy_peak(),
        "step_model": {"bytes_per_step": step_bytes,
                       "frac_of_hbm": step_bytes * r["value"] / n ** 3 / (HBM_PEAK_GBS * 1e9)},
    }
    if "fp64" in res and "mixed" in res:
        out["fp64"] = {"value": res["fp64"]["value"], "ms_per_step": res["fp64"]["ms_per_step"],
                       "stage_ms": res["fp64"]["stage_ms"]}
        out["speedup_mixed_vs_fp64"] = res["fp64"]["ms_per_step"] / res["mixed"]["ms_per_step"]
    if "fp64" in res and "mixed" in res:
        out["mixed_vs_fp64_rel_l2"] = mixed_error(n, p, u, phi)
    if not args.no_forms:
        out["forms"] = {}
        for name, fn in (("batched", bench_batch), ("adjoint", bench_adjoint), ("channel_wall_solve", bench_wall_solve),
                         ("channel_step", bench_channel), ("box_exact_cube", bench_exact_cube),
                         ("channel_single_phase_step", lambda: bench_channel(10, 2, "chan_sp_256"))):
            out["forms"][name] = fn()
            print("[bench] %s: %s" % (name, {k: v for k, v in out["forms"][name].items() if k != "groups"}),
                  file=sys.stderr, flush=True)
    # step-level HBM rooflines of the other paths (byte model / step time)
    out["rooflines"] = {}
    if "fp64" in res:
        out["rooflines"]["box_fp64_step"] = roofline_entry(step_model_bytes(n, False), res["fp64"]["ms_per_step"],
                                                           step_traffic("fp64"))
    out["rooflines"]["box_%s_step" % head] = roofline_entry(step_bytes, r["ms_per_step"], step_traffic(head))
    forms = out.get("forms", {})
    if "channel_step" in forms:
        cf = forms["channel_step"]
        nx, ny, nz = cf["grid"]
        for prec in ("mixed", "fp64"):
            out["rooflines"]["channel_%s_step" % prec] = roofline_entry(
                channel_model_bytes(nx, ny, nz - 1, prec == "mixed"), cf[prec]["ms_per_step"],
                channel_traffic(prec) if (nx, ny, nz) == (256, 128, 129) else None)
    if "batched" in forms:
        bf = forms["batched"]
        nb = sum(cnt * step_model_bytes(nn, True) for nn, cnt in bf["groups"])
        out["rooflines"]["batch_mixed_step"] = roofline_entry(nb, bf["ms_per_step"])
    if not args.no_cpu:
        out["cpu_baseline"], kept = cpu_baseline(n, p, u, phi)
        out["cpu_baseline_threaded"] = cpu_baseline_threaded(n, p, u, phi)
        out["vs_oracle_rel_l2_one_step"] = oracle_error(n, p, kept[0], kept[1])
        if not args.no_forms:
            out["cpu_channel_oracle"] = channel_oracle_timing()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
