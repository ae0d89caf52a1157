"""Benchmark of the longitudinal tracking hot path on one MI355X.

Default: one step = tracking 1e6 particles for 1e4
turns with FP64 leap-frog and moments after every turn (host constants, the
fused turn kernels and the moment finalize: the whole hot path) of a seeded
Gaussian bunch already resident in HBM, restored from a resident copy before
each step outside the step's timer (each step is bracketed by device
synchronisations; `value` is K steps of particle-turns over the sum of their
times). Per-launch kernel times come from HIP events inside a timed copy of
the launch graph, replayed for a few more steps after the K timed ones (its
event nodes cost ~1% of a step, so the timed steps replay the plain graph).
The default 20 warm-up steps (~0.15 s) cover the graph build and the first
steps of a process, over which the GPU clock is still rising.
Prints ONE JSON line on stdout; progress goes to stderr.

    python bench.py [--gpus 1] [--steps 20] [--warmup 20]

Other workloads (--workload): unfused (one launch per turn, HBM roofline
sweep), precision (FP32+Kahan vs FP64, 1e7 particles), batched (256 uneven
bunches), serving (Poisson request stream through the engine), ksweep,
schemes (every integrator), rf2 (double-harmonic RF, slip factor to second
order in dp), program (per-turn RF settings and a momentum ramp), 6d
(transverse linear map with chromaticity plus the longitudinal step), wake
(longitudinal resonator wake kick every turn), nsweep (the paper's
small-n table: 1 ... 8192 and up to 1e6 particles against the single-core
oracle, S and S_pure).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("particle-turns/sec, FP64 leap-frog, 10^6 particles; FP32 vs FP64; "
          "p50/p99 latency")
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VECTOR_PEAK_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz



def _sin_terms() -> int:
    import re
    with open(os.path.join(ROOT, "paper_1610_05801_amd", "csrc", "sinpi_coeffs.h")) as f:
        return int(re.search(r"kSinPiTerms = (\d+);", f.read()).group(1))


# Algorithmic FP64 flops per particle-turn (FMA = 2), the method's count:
# sin(k z) = phase multiply + reduction subtract + r^2 + (terms - 1) FMA + final
# multiply by r.
SIN_FLOPS = 4 + 2 * (_sin_terms() - 1)
FLOPS_PER_PT = {
    "euler_cromer": 2 + 2 + SIN_FLOPS + 8,
    "leapfrog": 4 + 2 + SIN_FLOPS + 8,
    "ruth4": 8 + 6 + 3 * SIN_FLOPS + 8,
    "rk4": 32 + 4 * SIN_FLOPS + 8,
}
# Extended map (two RF harmonics with phase offsets, slip factor quadratic in
# dp): drift = 2 FMA for eta(dp) + 1 FMA = 6; kick per harmonic = the sine
# above + phase offset add + the FMA into dp = SIN_FLOPS + 3.
RF2_DRIFT, RF2_KICK = 6, 2 * (SIN_FLOPS + 3)
RF2_FLOPS_PER_PT = {
    "euler_cromer": RF2_DRIFT + RF2_KICK + 8,
    "leapfrog": 2 * RF2_DRIFT + RF2_KICK + 8,
    "ruth4": 4 * RF2_DRIFT + 3 * RF2_KICK + 8,
    "rk4": 4 * RF2_DRIFT + 4 * RF2_KICK + 26 + 8,
}
# RF programme: one more FMA per kick (the reference step (p/p') delta + (p - p')/p').
RF2_REF_STEP = {"euler_cromer": 2, "leapfrog": 2, "ruth4": 6, "rk4": 0}
# 6-D map, per transverse plane: phase FMA 2, reduction subtract 1, r^2 1,
# t = 1/2 - |r| 1, t^2 1, two sine polynomials (7 FMA + final multiply each)
# 30, Twiss matrix (2 FMA for the diagonal, 2 multiplies, 2 x (multiply + FMA))
# 12 = 48; the longitudinal step without its moments, plus 5 sums (8 flops)
# for each of the three planes.
POLY_FLOPS = 2 * (_sin_terms() - 1) + 1
PLANE_FLOPS = 2 + 1 + 1 + 1 + 1 + 2 * POLY_FLOPS + 12
SIXD_FLOPS_PER_PT = {k: 2 * PLANE_FLOPS + (v - 8) + 3 * 8 for k, v in RF2_FLOPS_PER_PT.items()}
STATE_BYTES_PER_PARTICLE = 16  # z, dp FP64 (or FP32 hi + comp for both)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the sources the benchmark kernel is built from, with comments
    and blank space removed (a comment edit does not change the kernel)."""
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1610_05801_amd", "csrc")
    for f in ("kernels.hip", "wave.h", "ltrk_device.h", "sinpi_coeffs.h", "sinpi32_coeffs.h"):
        with open(os.path.join(csrc, f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)   # block comments
        text = re.sub(r"//[^\n]*", " ", text)                # line comments
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def load_traffic(name: str, launch_units: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when missing or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", name)
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != kernel_source_hash():
        return None
    per_unit = d.get("hbm_bytes_per_particle_turn")
    return None if per_unit is None else per_unit * launch_units


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q))


def _oracle_rate(z0, dp0, turns_total, ring, threads, budget_s):
    """Oracle particle-turns/s on `threads` threads over the first turns of the
    workload that fit in about budget_s seconds; returns (rate, turns, seconds)."""
    import oracle
    t0 = time.perf_counter()
    oracle.track(z0, dp0, 2, ring, "leapfrog", threads=threads)
    per_turn = (time.perf_counter() - t0) / 2
    turns = int(max(2, min(turns_total, budget_s / max(per_turn, 1e-9))))
    t0 = time.perf_counter()
    oracle.track(z0, dp0, turns, ring, "leapfrog", threads=threads)
    dt = time.perf_counter() - t0
    return z0.size * turns / dt, turns, dt


def host_cpu_model() -> str:
    """The CPU model name from /proc/cpuinfo with its family, model and
    stepping numbers (a virtual machine may report only a generic name); the
    machine type where there is none."""
    import platform
    fields = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if not line.strip():
                    break  # the first processor's block
                key, _, val = line.partition(":")
                fields[key.strip()] = val.strip()
    except OSError:
        pass
    name = fields.get("model name")
    if not name:
        return platform.processor() or platform.machine()
    ids = ", ".join("%s %s" % (k.replace("cpu ", ""), fields[k])
                    for k in ("cpu family", "model", "stepping") if k in fields)
    return "%s (%s)" % (name, ids) if ids else name


def cpu_baseline(n, turns_total, ring, seed, budget_s=10.0):
    """The FP64 oracle on the host cores: a bounded sample of the workload
    (the same bunch, its first T turns), scaled to particle-turns/s; also on
    one core (a tenth of the bunch, a third of the budget)."""
    from synth import SIGMA_DP, SIGMA_Z, gaussian_bunch
    z0, dp0 = gaussian_bunch(n, SIGMA_Z, SIGMA_DP, seed)
    threads = len(os.sched_getaffinity(0))
    rate, turns, dt = _oracle_rate(z0, dp0, turns_total, ring, threads, budget_s)
    n1 = max(1, n // 10)
    rate1, turns1, dt1 = _oracle_rate(z0[:n1], dp0[:n1], turns_total, ring, 1, budget_s / 3)
    return {"value": rate, "unit": "particle-turns/s", "cores": threads, "kind": "oracle",
            "sample": "%d particles x first %d of %d turns, leap-frog FP64 with moments every "
                      "turn, OpenMP over particles, %.1f s wall" % (n, turns, turns_total, dt),
            "ns_per_particle_turn": 1e9 / rate,
            "single_core": {"value": rate1, "ns_per_particle_turn": 1e9 / rate1,
                            "sample": "%d particles x first %d turns on 1 thread, %.1f s wall"
                                      % (n1, turns1, dt1)},
            "host_cpu": host_cpu_model(), "nproc": os.cpu_count(),
            "threads_available": threads}


TIMING_STEPS = 5   # steps replayed with launch timing on, for the per-launch kernel times


def bench_default(args):
    import torch
    import paper_1610_05801_amd as ltrk
    from synth import SIGMA_DP, SIGMA_Z, SPS_RING, SEEDS, gaussian_bunch, split_f32c

    n, T = args.particles, args.turns
    integ = "leapfrog"
    seed = SEEDS["paper_scale"]
    log("bench: %d particles x %d turns, %s FP64" % (n, T, integ))
    # Stages outside the rate, as the paper's stage profile lists them
    # (host timers around device-synchronised stages): device init, device
    # allocation, host-to-device copy of the initial state, the first call
    # (scratch allocation and launch-graph build), one tracking step (the
    # median of the timed steps), device-to-host copy of the final state and
    # the moment rows, and freeing the device memory.
    stages = {}
    t0 = time.perf_counter()
    torch.cuda.init()
    dev = torch.device("cuda:0")
    torch.empty(1, device=dev)
    torch.cuda.synchronize()
    stages["init"] = (time.perf_counter() - t0) * 1e3
    stream = torch.cuda.Stream(device=dev)
    z0, dp0 = gaussian_bunch(n, SIGMA_Z, SIGMA_DP, seed)
    zt, dt = torch.as_tensor(z0), torch.as_tensor(dp0)
    if args.tune:
        plan = ltrk.ltrk_autotune(integ, "f64", n, stream=stream)
        log("autotuned plan", plan)
    plan = ltrk.ltrk_get_plan(integ, "f64", n)
    # Every step tracks the initial bunch from the same device buffers: before
    # each step (outside its timer) the buffers are restored from a resident
    # copy, so every step does the same work and replays the same cached
    # graph (built in the first warm-up step). Launch timing is off in the
    # timed steps; the per-launch kernel times come from TIMING_STEPS more
    # steps with timing on (a second, timed graph: event-record nodes between
    # its segments), after one step that builds that graph.
    t0 = time.perf_counter()
    z_init, d_init = torch.empty(n, dtype=torch.float64, device=dev), torch.empty_like(zt, device=dev)
    z_run, d_run = torch.empty_like(z_init), torch.empty_like(d_init)
    mom = torch.empty((T, 5), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    stages["alloc"] = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    z_init.copy_(zt)
    d_init.copy_(dt)
    torch.cuda.synchronize()
    stages["h2d"] = (time.perf_counter() - t0) * 1e3
    moms = [mom]

    def restore():
        z_run.copy_(z_init)
        d_run.copy_(d_init)
        stream.synchronize()

    with torch.cuda.stream(stream):
        ltrk.ltrk_timing_enable(False)
        for i in range(args.warmup):
            restore()
            t0 = time.perf_counter()
            ltrk.ltrk_track_f64(z_run, d_run, T, SPS_RING, integ, mom, stream=stream)
            if i == 0:
                stream.synchronize()
                stages["first_call"] = (time.perf_counter() - t0) * 1e3
        stream.synchronize()
        step_ms = []
        for i in range(args.steps):
            restore()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ltrk.ltrk_track_f64(z_run, d_run, T, SPS_RING, integ, mom, stream=stream)
            torch.cuda.synchronize()   # every stream of the device, ours included
            step_ms.append((time.perf_counter() - t0) * 1e3)
        elapsed = sum(step_ms) * 1e-3
        ltrk.ltrk_timing_enable(True)
        for i in range(TIMING_STEPS + 1):
            if i == 1:
                ltrk.ltrk_timing_take()  # the first of these steps built the timed graph
            restore()
            ltrk.ltrk_track_f64(z_run, d_run, T, SPS_RING, integ, mom, stream=stream)
        stream.synchronize()
        tm = ltrk.ltrk_timing_take()
        ltrk.ltrk_timing_enable(False)
    value = n * T * args.steps / elapsed
    log("fused: %.4e particle-turns/s, %.3f ms/step" % (value, elapsed / args.steps * 1e3))
    avg_track_ms = tm["track_ms"] / max(tm["track_launches"], 1)
    launch_turns = T * TIMING_STEPS / max(tm["track_launches"], 1)
    launch_pt = n * launch_turns
    flops = FLOPS_PER_PT[integ] * launch_pt
    achieved = flops / (avg_track_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                "traffic": load_traffic("fused_leapfrog_f64_1e6_traffic.json", launch_pt),
                "kernel": "k_track_single<leapfrog,f64,P=%d>" % plan["ppl"],
                "avg_launch_ms": avg_track_ms, "turns_per_launch": launch_turns,
                "flops_per_particle_turn": FLOPS_PER_PT[integ],
                "finalize_ms_per_step": tm["finalize_ms"] / TIMING_STEPS,
                "timing_steps": TIMING_STEPS}

    extras = {}
    if not args.quick:
        # FP32 + Kahan state on the same workload (2 steps); its moment rows
        # against those of the FP64 steps (same initial bunch)
        m64 = mom.cpu().numpy()
        zh, zc = split_f32c(z0)
        dh, dc = split_f32c(dp0)
        f32 = [torch.as_tensor(a).to(dev) for a in (zh, dh, zc, dc)]
        f32_run = [torch.empty_like(a) for a in f32]
        with torch.cuda.stream(stream):
            reps, f32_s = 2, 0.0
            for r in range(reps + 1):  # the first call builds the graph
                for a, b in zip(f32_run, f32):
                    a.copy_(b)
                stream.synchronize()
                t0 = time.perf_counter()
                ltrk.ltrk_track_f32c(*f32_run, T, SPS_RING, integ, moms[0], stream=stream)
                stream.synchronize()
                if r:
                    f32_s += (time.perf_counter() - t0) / reps
        v32 = n * T / f32_s
        del f32, f32_run
        m32 = mom.cpu().numpy()
        rel = np.abs(m32 - m64) / np.abs(m64)
        rel[:, 0] = np.abs(m32[:, 0] - m64[:, 0]) / m64[:, 1]   # means over their rms
        rel[:, 2] = np.abs(m32[:, 2] - m64[:, 2]) / m64[:, 3]
        extras["f32c"] = {"value": v32, "unit": "particle-turns/s", "ms_per_step": f32_s * 1e3,
                          "ratio_to_f64": v32 / value,
                          "moments_vs_f64_max_rel": dict(zip(
                              ["mean_z", "rms_z", "mean_dp", "rms_dp", "emit"],
                              rel.max(axis=0).tolist())),
                          "note": "max over the 1e4 turns; means relative to their rms"}
        log("f32c: %.4e particle-turns/s" % v32)
        # one launch per turn (HBM-bound form) on the same workload, 1e3 turns
        Tu = min(T, 1000)
        saved = ltrk.ltrk_get_plan(integ, "f64", n)
        ltrk.ltrk_set_plan(1, 256, 4, 1)   # HBM-bound form: 4 particles per lane
        z1, d1 = zt.to(dev), dt.to(dev)
        mu = torch.empty((Tu, 5), dtype=torch.float64, device=dev)
        with torch.cuda.stream(stream):
            ltrk.ltrk_track_f64(z1, d1, Tu, SPS_RING, integ, mu, stream=stream)
            stream.synchronize()
            t0 = time.perf_counter()
            ltrk.ltrk_track_f64(z1, d1, Tu, SPS_RING, integ, mu, stream=stream)
            stream.synchronize()
            du = time.perf_counter() - t0
        ltrk.ltrk_set_plan()
        extras["unfused"] = {"value": n * Tu / du, "unit": "particle-turns/s",
                             "hbm_GBps_algorithmic": STATE_BYTES_PER_PARTICLE * 2 * n * Tu / du / 1e9,
                             "turns": Tu, "note": "16 MB state is cache resident at 1e6 "
                             "particles; the HBM roofline sweep is --workload unfused"}
        log("unfused: %.4e particle-turns/s" % (n * Tu / du))
        del saved, z1, d1, mu
        extras["unfused_hbm"] = unfused_hbm_leg(ltrk, torch, stream, dev)

    # The same round trip from warm pinned host buffers (the stages above time
    # a process's first copies, from pageable memory): the initial state in,
    # one call, the final state and the moment rows out; median of 3.
    z_pin = torch.empty(n, dtype=torch.float64, pin_memory=True)
    d_pin = torch.empty(n, dtype=torch.float64, pin_memory=True)
    m_pin = torch.empty((T, 5), dtype=torch.float64, pin_memory=True)
    z_pin.copy_(zt)
    d_pin.copy_(dt)
    round_ms = []
    with torch.cuda.stream(stream):
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            z_run.copy_(z_pin, non_blocking=True)
            d_run.copy_(d_pin, non_blocking=True)
            ltrk.ltrk_track_f64(z_run, d_run, T, SPS_RING, integ, mom, stream=stream)
            z_pin.copy_(z_run, non_blocking=True)
            d_pin.copy_(d_run, non_blocking=True)
            m_pin.copy_(mom, non_blocking=True)
            stream.synchronize()
            round_ms.append((time.perf_counter() - t0) * 1e3)
            z_pin.copy_(zt)
            d_pin.copy_(dt)
    pinned_round_ms = percentile(round_ms, 50)
    del z_pin, d_pin, m_pin

    # final state and moment rows to the host, then free the device memory
    t0 = time.perf_counter()
    host_out = (z_run.cpu(), d_run.cpu(), mom.cpu())
    torch.cuda.synchronize()
    stages["d2h"] = (time.perf_counter() - t0) * 1e3
    del host_out
    t0 = time.perf_counter()
    del z_init, d_init, z_run, d_run, mom, moms
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    torch.cuda.synchronize()
    stages["free"] = (time.perf_counter() - t0) * 1e3
    stages["track"] = percentile(step_ms, 50)
    pcie = stages["h2d"] + stages["track"] + stages["d2h"]

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-turns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "leap-frog FP64, 1e6 particles x 1e4 turns, moments every turn",
                   "particles": n, "turns": T, "integrator": integ, "seed": seed,
                   "ring": "C=6911 m, h=4620, V=2 MV, p0c=26 GeV, m=0.938 GeV, gamma_t=22.77",
                   "plan": plan},
        "latency_ms": {"p50": percentile(step_ms, 50), "p99": percentile(step_ms, 99),
                       "unit": "ms per step (1e10 particle-turns)"},
        "roofline": roofline,
        "stages_ms": dict(stages, note="host timers around device-synchronised stages; "
                          "track = median step; first_call = the first call's scratch "
                          "allocation, graph build and run"),
        "pcie_inclusive": {"value": n * T / (pcie * 1e-3), "unit": "particle-turns/s",
                           "note": "one step with the initial state copied in and the final "
                                   "state and moments copied out (h2d + track + d2h, the "
                                   "process's first copies, pageable host memory)",
                           "warm_pinned": {"value": n * T / (pinned_round_ms * 1e-3),
                                           "ms": pinned_round_ms,
                                           "note": "the same round trip from warm pinned "
                                                   "host buffers, median of 3"}},
    }
    out.update(extras)
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        cb = cpu_baseline(n, T, SPS_RING, seed, budget_s=args.cpu_seconds)
        cb["gpu_speedup"] = {"all_cores": out["value"] / cb["value"],
                             "single_core": out["value"] / cb["single_core"]["value"]}
        out["cpu_baseline"] = cb
        log("cpu: %.4e particle-turns/s on %d threads, %.4e on one" % (
            cb["value"], cb["cores"], cb["single_core"]["value"]))
    print(json.dumps(out), flush=True)


# The HBM-bound form at a size far beyond the 256 MB last-level cache:
# one launch per turn, 2 particles per lane in 64-thread blocks (the fastest
# shape of the --workload unfused sweep at 1e8 particles).
UNFUSED_HBM_N, UNFUSED_HBM_TURNS = 100_000_000, 30


def unfused_hbm_leg(ltrk, torch, stream, dev):
    """One launch per turn at 1e8 particles (1.6 GB of state): kernel time per
    launch from HIP events, algorithmic bytes 32 per particle-turn."""
    n, turns = UNFUSED_HBM_N, UNFUSED_HBM_TURNS
    g = torch.Generator(device=dev).manual_seed(7)
    z = torch.randn(n, dtype=torch.float64, device=dev, generator=g) * 0.23
    dp = torch.randn(n, dtype=torch.float64, device=dev, generator=g) * 1e-3
    mom = torch.empty((turns, 5), dtype=torch.float64, device=dev)
    ltrk.ltrk_set_plan(1, 64, 2, 1)
    reps = 3
    try:
        dt, tm = _timed_track(ltrk, torch, stream, n, turns, "leapfrog", "f64", (z, dp), mom,
                              reps=reps)
    finally:
        ltrk.ltrk_set_plan()
    kern_ms = tm["track_ms"] / max(tm["track_launches"], 1)
    achieved = STATE_BYTES_PER_PARTICLE * 2 * n / (kern_ms * 1e-3) / 1e9
    del z, dp, mom
    torch.cuda.empty_cache()
    leg = {"bound": "hbm", "particles": n, "turns": turns, "plan": {"turns_per_launch": 1,
           "block": 64, "ppl": 2}, "avg_launch_ms": kern_ms, "achieved": achieved,
           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
           "bytes_per_particle_turn": 2 * STATE_BYTES_PER_PARTICLE,
           "particle_turns_per_s": n * turns / dt,
           "finalize_ms_per_turn": tm["finalize_ms"] / (reps * turns)}
    log("unfused at 1e8: %.0f GB/s (%.3f of HBM peak)" % (achieved, achieved / HBM_PEAK_GBS))
    return leg


def _timed_track(ltrk, torch, stream, n, turns, integ, dtype, arrays, mom, reps=1):
    """Run reps calls with launch timing on, after one warm-up call that builds
    their (timed) launch graph; returns (wall seconds per call, timing dict)."""
    from synth import SPS_RING
    fn = ltrk.ltrk_track_f64 if dtype == "f64" else ltrk.ltrk_track_f32c
    with torch.cuda.stream(stream):
        ltrk.ltrk_timing_enable(True)
        fn(*arrays, turns, SPS_RING, integ, mom, stream=stream)
        stream.synchronize()
        ltrk.ltrk_timing_take()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn(*arrays, turns, SPS_RING, integ, mom, stream=stream)
        stream.synchronize()
        dt = (time.perf_counter() - t0) / reps
        tm = ltrk.ltrk_timing_take()
        ltrk.ltrk_timing_enable(False)
    return dt, tm


# Launch shapes tried for the one-launch-per-turn form: (particles per lane,
# block). At 1e8 particles (2, 64) streamed 6.31 TB/s against 6.08 for (4, 256).
UNFUSED_PLANS = ((2, 64), (4, 256), (8, 256))


def bench_unfused(args):
    """One launch per turn (K = 1): the HBM-bound form, swept in n up to far
    beyond the 256 MB last-level cache; each row reports the fastest of the
    UNFUSED_PLANS launch shapes (all of them listed)."""
    import torch
    import paper_1610_05801_amd as ltrk
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    rows = []
    for n in (1_000_000, 10_000_000, 100_000_000, 250_000_000):
        turns = 200 if n <= 10_000_000 else 30
        g = torch.Generator(device=dev).manual_seed(7)
        z = torch.randn(n, dtype=torch.float64, device=dev, generator=g) * 0.23
        dp = torch.randn(n, dtype=torch.float64, device=dev, generator=g) * 1e-3
        mom = torch.empty((turns, 5), dtype=torch.float64, device=dev)
        per_plan = {}
        best = None
        for ppl, block in UNFUSED_PLANS:
            ltrk.ltrk_set_plan(1, block, ppl, 1)
            dt_p, tm_p = _timed_track(ltrk, torch, stream, n, turns, "leapfrog", "f64", (z, dp),
                                      mom)
            ms_p = tm_p["track_ms"] / max(tm_p["track_launches"], 1)
            per_plan["P%d/b%d" % (ppl, block)] = ms_p
            if best is None or ms_p < best[0]:
                best = (ms_p, dt_p, tm_p, (ppl, block))
        kern_ms, dt, tm, (ppl, block) = best
        alg_bytes = STATE_BYTES_PER_PARTICLE * 2 * n
        # Practical ceiling for the same traffic: a device copy of z and dp
        # (read 16 B, write 16 B per particle) with torch's copy kernel.
        zc, dc = torch.empty_like(z), torch.empty_like(dp)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            zc.copy_(z)
            dc.copy_(dp)
            e0.record(stream)
            for _ in range(10):
                zc.copy_(z)
                dc.copy_(dp)
            e1.record(stream)
        stream.synchronize()
        copy_ms = e0.elapsed_time(e1) / 10
        del zc, dc
        achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
        row = {"particles": n, "turns": turns, "particle_turns_per_s": n * turns / dt,
               "plan": {"ppl": ppl, "block": block}, "kernel_ms_by_plan": per_plan,
               "avg_kernel_ms": kern_ms, "achieved_GBps": achieved,
               "frac_hbm": achieved / HBM_PEAK_GBS,
               "copy_GBps": alg_bytes / (copy_ms * 1e-3) / 1e9,
               "frac_of_copy": copy_ms / kern_ms,
               "finalize_ms_per_turn": tm["finalize_ms"] / turns}
        rows.append(row)
        log(json.dumps(row))
        del z, dp, mom
        torch.cuda.empty_cache()
    ltrk.ltrk_set_plan()
    print(json.dumps({"workload": "unfused leap-frog FP64, one launch per turn", "rows": rows,
                      "bytes_per_particle_turn": 32, "peak_GBps": HBM_PEAK_GBS}), flush=True)


NSWEEP_N = tuple(2 ** k for k in range(14)) + (10_000, 100_000, 1_000_000)


def bench_nsweep(args):
    """The paper's small-n table (Table 2: leap-frog, 1e6 turns, 1 ... 8192
    macro-particles, sequential C against the GPU, S and S_pure), extended to
    1e6 particles. Per n: the GPU call's kernel time (HIP events over its
    tracking launches) and its total (host copy in, the call, copy out; warm
    process), the single-core oracle's time (measured on the first turns and
    scaled to all turns: its cost per turn is constant), S = oracle / GPU
    total, S_pure = oracle / GPU kernel (the oracle reads no files, so its
    total and kernel times are one number), the break-even n and the
    single-particle per-turn latency. No moments, as in the paper's kernels."""
    import torch
    import oracle
    import paper_1610_05801_amd as ltrk
    from synth import SIGMA_DP, SIGMA_Z, SPS_RING, SEEDS, gaussian_bunch
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    T = args.sweep_turns
    rows = []
    oracle_budget_pt = 2.5e7   # about 0.3 s of single-core oracle work per row
    for n in NSWEEP_N:
        z0, dp0 = gaussian_bunch(n, SIGMA_Z, SIGMA_DP, SEEDS["paper_scale"])
        z, dp = torch.as_tensor(z0).to(dev), torch.as_tensor(dp0).to(dev)
        with torch.cuda.stream(stream):
            ltrk.ltrk_timing_enable(True)
            ltrk.ltrk_track_f64(z, dp, T, SPS_RING, "leapfrog", None, stream=stream)
            stream.synchronize()          # the first call builds the launch graph
            ltrk.ltrk_timing_take()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            z, dp = torch.as_tensor(z0).to(dev), torch.as_tensor(dp0).to(dev)
            ltrk.ltrk_track_f64(z, dp, T, SPS_RING, "leapfrog", None, stream=stream)
            out = (z.cpu(), dp.cpu())
            torch.cuda.synchronize()
            total_ms = (time.perf_counter() - t0) * 1e3
            tm = ltrk.ltrk_timing_take()
            ltrk.ltrk_timing_enable(False)
        del out
        kern_ms = tm["track_ms"]
        t_or = int(min(T, max(100, oracle_budget_pt / n)))
        t0 = time.perf_counter()
        oracle.track(z0, dp0, t_or, SPS_RING, "leapfrog", with_moments=False, threads=1)
        or_ms = (time.perf_counter() - t0) * 1e3 * T / t_or
        row = {"particles": n, "turns": T, "gpu_kernel_ms": kern_ms, "gpu_total_ms": total_ms,
               "launches": tm["track_launches"], "oracle_1core_ms": or_ms,
               "oracle_turns_measured": t_or, "S": or_ms / total_ms, "S_pure": or_ms / kern_ms,
               "gpu_particle_turns_per_s": n * T / (kern_ms * 1e-3)}
        rows.append(row)
        log(json.dumps(row))
        del z, dp
    even = [r["particles"] for r in rows if r["S"] >= 1.0]
    out = {"workload": "nsweep: leap-frog FP64, %d turns, no moments, 1 ... 1e6 particles" % T,
           "rows": rows, "break_even_particles": even[0] if even else None,
           "break_even_particles_pure": next((r["particles"] for r in rows if r["S_pure"] >= 1.0),
                                             None),
           "single_particle_ns_per_turn": rows[0]["gpu_kernel_ms"] * 1e6 / T,
           "oracle_cpu": host_cpu_model(),
           "note": "GPU totals are warm-process calls (device init excluded: see the default "
                   "run's stages_ms); oracle times scaled from oracle_turns_measured turns"}
    print(json.dumps(out), flush=True)


def bench_ksweep(args):
    import torch
    import paper_1610_05801_amd as ltrk
    from synth import SIGMA_DP, SIGMA_Z, SEEDS, gaussian_bunch
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    n, T = args.particles, min(args.turns, 4096)
    z0, dp0 = gaussian_bunch(n, SIGMA_Z, SIGMA_DP, SEEDS["paper_scale"])
    rows = []
    base = ltrk.ltrk_get_plan("leapfrog", "f64", n)
    for ppl in args.ppls:
        for K in args.ks:
            for graph in args.graphs:
                ltrk.ltrk_set_plan(K, base["block"], ppl, graph)
                z, dp = torch.as_tensor(z0).to(dev), torch.as_tensor(dp0).to(dev)
                mom = torch.empty((T, 5), dtype=torch.float64, device=dev)
                from synth import SPS_RING
                with torch.cuda.stream(stream):
                    ltrk.ltrk_track_f64(z, dp, T, SPS_RING, "leapfrog", mom, stream=stream)
                    stream.synchronize()
                    t0 = time.perf_counter()
                    ltrk.ltrk_track_f64(z, dp, T, SPS_RING, "leapfrog", mom, stream=stream)
                    stream.synchronize()
                    dt = time.perf_counter() - t0
                row = {"K": K, "ppl": ppl, "graph": graph, "block": base["block"],
                       "particle_turns_per_s": n * T / dt}
                del z, dp, mom
                rows.append(row)
                log(json.dumps(row))
    ltrk.ltrk_set_plan()
    print(json.dumps({"workload": "K sweep, leap-frog FP64, %d particles x %d turns" % (n, T),
                      "rows": rows}), flush=True)


def bench_precision(args):
    """FP32 + Kahan vs FP64 at 1e7 particles x 1e5 turns (LF, EC, Ruth4), with
    the oracle on a strided 1e4-particle subset."""
    import torch
    import oracle
    import paper_1610_05801_amd as ltrk
    from synth import (SIGMA_DP, SIGMA_Z, SPS_RING, SEEDS, gaussian_bunch, join_f32c,
                       split_f32c)
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    n = args.particles if args.particles != 1_000_000 else 10_000_000
    T = args.turns if args.turns != 10_000 else 100_000
    z_in, dp_in = gaussian_bunch(n, SIGMA_Z, SIGMA_DP, SEEDS["precision"])
    zh, zc = split_f32c(z_in)
    dh, dc = split_f32c(dp_in)
    z0, dp0 = join_f32c(zh, zc), join_f32c(dh, dc)     # identical start for both paths
    idx = np.arange(0, n, max(1, n // 10_000))
    c = oracle.derive(SPS_RING)
    zb, db = c["bucket_half_length"], c["bucket_height"]
    h0 = oracle.hamiltonian(z0[idx], dp0[idx], SPS_RING)
    core = np.abs(h0 - c["H_sep"]) / abs(c["H_sep"]) > 0.01
    inside = h0 > c["H_sep"]
    results = []
    for integ in ("leapfrog", "euler_cromer", "ruth4"):
        t0 = time.perf_counter()
        zr, dr, mr = oracle.track(z0[idx], dp0[idx], T, SPS_RING, integ,
                                  threads=len(os.sched_getaffinity(0)))
        oracle_s = time.perf_counter() - t0
        out = {"integrator": integ}
        finals = {}
        for dtype in ("f64", "f32c"):
            if dtype == "f64":
                arrays = (torch.as_tensor(z0).to(dev), torch.as_tensor(dp0).to(dev))
            else:
                arrays = tuple(torch.as_tensor(a).to(dev) for a in (zh, dh, zc, dc))
            mom = torch.empty((T, 5), dtype=torch.float64, device=dev)
            fn = ltrk.ltrk_track_f64 if dtype == "f64" else ltrk.ltrk_track_f32c
            with torch.cuda.stream(stream):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                fn(*arrays, T, SPS_RING, integ, mom, stream=stream)
                stream.synchronize()
                dt = time.perf_counter() - t0
            a = [x.cpu().numpy() for x in arrays]
            zf, df = (a[0], a[1]) if dtype == "f64" else (join_f32c(a[0], a[2]), join_f32c(a[1], a[3]))
            finals[dtype] = (zf, df, mom.cpu().numpy())
            e = np.hypot((zf[idx] - zr) / zb, (df[idx] - dr) / db) / np.hypot(zr / zb, dr / db)
            hn = oracle.hamiltonian(zf[idx], df[idx], SPS_RING)
            hr = oracle.hamiltonian(zr, dr, SPS_RING)
            dh_gpu = np.abs(hn - h0)[inside & core] / abs(c["H_sep"])
            dh_ref = np.abs(hr - h0)[inside & core] / abs(c["H_sep"])
            out[dtype] = {"particle_turns_per_s": n * T / dt, "seconds": dt,
                          "subset_e_core_max": float(e[core].max()),
                          "subset_e_core_p50": float(np.median(e[core])),
                          "subset_e_core_p99": float(np.percentile(e[core], 99)),
                          "dH_over_Hsep_max_inside": float(dh_gpu.max()),
                          "dH_over_Hsep_max_inside_oracle": float(dh_ref.max())}
        # full-population moments: F32C against FP64 (both GPU, same start)
        m64, m32 = finals["f64"][2], finals["f32c"][2]
        rel = np.abs(m32 - m64) / np.abs(m64)
        rel[:, 0] = np.abs(m32[:, 0] - m64[:, 0]) / m64[:, 1]
        rel[:, 2] = np.abs(m32[:, 2] - m64[:, 2]) / m64[:, 3]
        out["f32c_vs_f64_moments_max_rel"] = dict(zip(
            ["mean_z", "rms_z", "mean_dp", "rms_dp", "emit"], rel.max(axis=0).tolist()))
        out["f32c_vs_f64_moments_final_rel"] = dict(zip(
            ["mean_z", "rms_z", "mean_dp", "rms_dp", "emit"], rel[-1].tolist()))
        out["oracle_subset_seconds"] = oracle_s
        results.append(out)
        log(json.dumps(out))
    print(json.dumps({"workload": "precision: %d particles x %d turns, F32C vs FP64" % (n, T),
                      "subset": int(idx.size), "results": results}), flush=True)


def bench_schemes(args):
    """Every scheme in FP64 and F32C at 1e6 particles x 2048 turns, moments
    every turn, default plans; kernel time from HIP events."""
    import torch
    import paper_1610_05801_amd as ltrk
    from synth import SIGMA_DP, SIGMA_Z, SPS_RING, SEEDS, gaussian_bunch, split_f32c
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    n, T = args.particles, 2048
    z0, dp0 = gaussian_bunch(n, SIGMA_Z, SIGMA_DP, SEEDS["paper_scale"])
    zh, zc = split_f32c(z0)
    dh, dc = split_f32c(dp0)
    mom = torch.empty((T, 5), dtype=torch.float64, device=dev)
    rows = []
    for integ in ("euler_cromer", "leapfrog", "ruth4", "rk4"):
        for dtype in ("f64", "f32c"):
            if dtype == "f64":
                arrays = (torch.as_tensor(z0).to(dev), torch.as_tensor(dp0).to(dev))
            else:
                arrays = tuple(torch.as_tensor(a).to(dev) for a in (zh, dh, zc, dc))
            dt, tm = _timed_track(ltrk, torch, stream, n, T, integ, dtype, arrays, mom)
            kern = tm["track_ms"] / max(tm["track_launches"], 1)
            per_launch = n * T / max(tm["track_launches"], 1)
            row = {"integrator": integ, "dtype": dtype, "particle_turns_per_s": n * T / dt,
                   "kernel_particle_turns_per_s": per_launch / (kern * 1e-3),
                   "flops_per_particle_turn": FLOPS_PER_PT[integ],
                   "kernel_tflops": FLOPS_PER_PT[integ] * per_launch / (kern * 1e-3) / 1e12,
                   "plan": ltrk.ltrk_get_plan(integ, dtype, n)}
            rows.append(row)
            log(json.dumps(row))
    print(json.dumps({"workload": "schemes: %d particles x %d turns" % (n, T), "rows": rows}),
          flush=True)


def bench_rf2(args):
    """Extended map (double-harmonic RF, phase offsets, slip factor quadratic
    in dp), FP64, every scheme at 1e6 particles x 1e4 turns with moments
    every turn; leap-frog also through the single-harmonic kernel for the
    cost of the second harmonic. Kernel time from HIP events."""
    import torch
    import paper_1610_05801_amd as ltrk
    from synth import SIGMA_DP, SIGMA_Z, SPS_DOUBLE_RF, SPS_RING, SEEDS, gaussian_bunch
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    n, T = args.particles, args.turns
    z0, dp0 = gaussian_bunch(n, SIGMA_Z, SIGMA_DP, SEEDS["paper_scale"])
    mom = torch.empty((T, 5), dtype=torch.float64, device=dev)
    rows = []
    cases = [(i, "rf2") for i in ("euler_cromer", "leapfrog", "ruth4", "rk4")]
    cases.append(("leapfrog", "single"))
    for integ, kind in cases:
        z, dp = torch.as_tensor(z0).to(dev), torch.as_tensor(dp0).to(dev)
        if kind == "rf2":
            call = lambda: ltrk.ltrk_track_rf2_f64(z, dp, T, SPS_DOUBLE_RF, integ, mom,
                                                   stream=stream)
            flops = RF2_FLOPS_PER_PT[integ]
        else:
            call = lambda: ltrk.ltrk_track_f64(z, dp, T, SPS_RING, integ, mom, stream=stream)
            flops = FLOPS_PER_PT[integ]
        with torch.cuda.stream(stream):
            call()
            stream.synchronize()
            t0 = time.perf_counter()
            call()
            stream.synchronize()
            dt = time.perf_counter() - t0
            ltrk.ltrk_timing_enable(True)
            call()
            stream.synchronize()
            ltrk.ltrk_timing_take()
            call()
            stream.synchronize()
            tm = ltrk.ltrk_timing_take()
            ltrk.ltrk_timing_enable(False)
        launches = max(tm["track_launches"], 1)
        kern = tm["track_ms"] / launches
        per_launch = n * T / launches
        row = {"map": kind, "integrator": integ, "particle_turns_per_s": n * T / dt,
               "kernel_particle_turns_per_s": per_launch / (kern * 1e-3),
               "flops_per_particle_turn": flops,
               "kernel_tflops": flops * per_launch / (kern * 1e-3) / 1e12,
               "frac_fp64_peak": flops * per_launch / (kern * 1e-3) / 1e12
               / FP64_VECTOR_PEAK_TFLOPS,
               "avg_launch_ms": kern, "finalize_ms": tm["finalize_ms"]}
        rows.append(row)
        log(json.dumps(row))
    print(json.dumps({"workload": "extended map: %d particles x %d turns, double RF "
                      "(h2 = 2h, V2 = V/4, counter-phase), eta(dp) to second order"
                      % (n, T), "rows": rows}), flush=True)


def _ramp_programme(turns, p0, v1, m, rel_per_turn=2e-6):
    """Synchronous-phase momentum ramp with a modulated RF voltage and a
    second harmonic in counter-phase: every record changes every turn."""
    n = np.arange(turns)
    p_after = p0 * (1 + rel_per_turn * (n + 1))
    p_before = np.concatenate([[p0], p_after[:-1]])
    volts = v1 * (1 + 0.2 * np.sin(n / 300.0))
    beta = p_before / np.sqrt(p_before ** 2 + m * m)
    phi = np.arcsin(beta * (p_after - p_before) / volts)
    return dict(voltage_V=volts, phi1_rad=phi, voltage2_V=0.25 * volts,
                phi2_rad=np.full(turns, math.pi), p0c_eV=p_after)


def bench_program(args):
    """RF programme: 1e6 particles x 1e4 turns through a 2% momentum ramp
    (records change every turn), FP64, moments every turn, every scheme that
    supports a ramp, plus RK4 and leap-frog on a constant-momentum programme.
    Kernel time from HIP events; wall time includes building and uploading
    the per-turn records."""
    import torch
    import paper_1610_05801_amd as ltrk
    from synth import SIGMA_DP, SIGMA_Z, SPS_DOUBLE_RF, SEEDS, gaussian_bunch
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    n, T = args.particles, args.turns
    z0, dp0 = gaussian_bunch(n, SIGMA_Z, SIGMA_DP, SEEDS["paper_scale"])
    mom = torch.empty((T, 5), dtype=torch.float64, device=dev)
    ramp = _ramp_programme(T, SPS_DOUBLE_RF["p0c_eV"], SPS_DOUBLE_RF["voltage_V"],
                           SPS_DOUBLE_RF["mass_eV"])
    flat = dict(ramp, p0c_eV=np.full(T, SPS_DOUBLE_RF["p0c_eV"]),
                phi1_rad=np.zeros(T))
    rows = []
    cases = [(i, "ramp", ramp) for i in ("euler_cromer", "leapfrog", "ruth4")]
    cases += [("leapfrog", "flat", flat), ("rk4", "flat", flat)]
    for integ, kind, prog in cases:
        z, dp = torch.as_tensor(z0).to(dev), torch.as_tensor(dp0).to(dev)
        recs = ltrk.RfTurn.array(prog, T)
        call = lambda: ltrk.ltrk_track_program_f64(z, dp, T, SPS_DOUBLE_RF, recs, integ, mom,
                                                   stream=stream)
        flops = RF2_FLOPS_PER_PT[integ] + (RF2_REF_STEP[integ] if kind == "ramp" else 0)
        with torch.cuda.stream(stream):
            call()
            stream.synchronize()
            t0 = time.perf_counter()
            call()
            stream.synchronize()
            dt = time.perf_counter() - t0
            ltrk.ltrk_timing_enable(True)
            call()
            stream.synchronize()
            ltrk.ltrk_timing_take()
            call()
            stream.synchronize()
            tm = ltrk.ltrk_timing_take()
            ltrk.ltrk_timing_enable(False)
        launches = max(tm["track_launches"], 1)
        kern = tm["track_ms"] / launches
        per_launch = n * T / launches
        row = {"programme": kind, "integrator": integ, "particle_turns_per_s": n * T / dt,
               "kernel_particle_turns_per_s": per_launch / (kern * 1e-3),
               "flops_per_particle_turn": flops,
               "kernel_tflops": flops * per_launch / (kern * 1e-3) / 1e12,
               "frac_fp64_peak": flops * per_launch / (kern * 1e-3) / 1e12
               / FP64_VECTOR_PEAK_TFLOPS,
               "avg_launch_ms": kern, "finalize_ms": tm["finalize_ms"]}
        rows.append(row)
        log(json.dumps(row))
    print(json.dumps({"workload": "RF programme: %d particles x %d turns, 2%% momentum ramp "
                      "at the synchronous phase, V modulated, double RF" % (n, T),
                      "rows": rows}), flush=True)

def bench_6d(args):
    """6-D map: 1e6 particles x 1e4 turns (leap-frog and Ruth4), transverse
    Twiss rotation with chromaticity then the double-RF longitudinal step,
    moments of the three planes every turn. Kernel time from HIP events."""
    import torch
    import paper_1610_05801_amd as ltrk
    from synth import SIGMA_DP, SIGMA_Z, SPS_DOUBLE_RF, SPS_TWISS, SEEDS, gaussian_bunch
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    n, T = args.particles, args.turns
    z0, dp0 = gaussian_bunch(n, SIGMA_Z, SIGMA_DP, SEEDS["paper_scale"])
    rng = np.random.default_rng(SEEDS["paper_scale"] + 1)
    ex = 2e-8  # geometric emittance (m rad) of the transverse Gaussian
    x0 = np.sqrt(ex * SPS_TWISS["beta_x"]) * rng.standard_normal(n)
    xp0 = np.sqrt(ex / SPS_TWISS["beta_x"]) * rng.standard_normal(n)
    y0 = np.sqrt(ex * SPS_TWISS["beta_y"]) * rng.standard_normal(n)
    yp0 = np.sqrt(ex / SPS_TWISS["beta_y"]) * rng.standard_normal(n)
    mom = torch.empty((T, 3, 5), dtype=torch.float64, device=dev)
    rows = []
    for integ in ("leapfrog", "ruth4"):
        arrs = [torch.as_tensor(a).to(dev) for a in (z0, dp0, x0, xp0, y0, yp0)]
        call = lambda: ltrk.ltrk_track_6d_f64(*arrs, T, SPS_DOUBLE_RF, SPS_TWISS, integ, mom,
                                              stream=stream)
        flops = SIXD_FLOPS_PER_PT[integ]
        with torch.cuda.stream(stream):
            call()
            stream.synchronize()
            t0 = time.perf_counter()
            call()
            stream.synchronize()
            dt = time.perf_counter() - t0
            ltrk.ltrk_timing_enable(True)
            call()
            stream.synchronize()
            ltrk.ltrk_timing_take()
            call()
            stream.synchronize()
            tm = ltrk.ltrk_timing_take()
            ltrk.ltrk_timing_enable(False)
        launches = max(tm["track_launches"], 1)
        kern = tm["track_ms"] / launches
        per_launch = n * T / launches
        row = {"map": "6d", "integrator": integ, "particle_turns_per_s": n * T / dt,
               "kernel_particle_turns_per_s": per_launch / (kern * 1e-3),
               "flops_per_particle_turn": flops,
               "kernel_tflops": flops * per_launch / (kern * 1e-3) / 1e12,
               "frac_fp64_peak": flops * per_launch / (kern * 1e-3) / 1e12
               / FP64_VECTOR_PEAK_TFLOPS,
               "avg_launch_ms": kern, "finalize_ms": tm["finalize_ms"]}
        rows.append(row)
        log(json.dumps(row))
    print(json.dumps({"workload": "6-D map: %d particles x %d turns, double RF, chromatic "
                      "transverse rotation, moments of 3 planes every turn" % (n, T),
                      "rows": rows}), flush=True)


def bench_wake(args):
    """Wake kick: 10^6, 10^7 and 10^8 particles (--wake-sizes) x 1000 turns
    (leap-frog, resonator, 256 slices), two launches per turn. The turn kernel
    streams the state once per turn (32 B per particle-turn: the HBM
    roofline); the potential kernel runs blocks of 32 slices. The rate is that of an untimed replay of the call's launch
    graph; kernel times come from HIP events in a replay of its timed graph
    (each graph built by a warm-up call first)."""
    import torch
    import paper_1610_05801_amd as ltrk
    from synth import SIGMA_DP, SIGMA_Z, SPS_RING, SPS_WAKE, SEEDS, gaussian_bunch
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    T = 1000
    rf = dict(SPS_RING, phi1_rad=0.0, harmonic2=0.0, voltage2_V=0.0, phi2_rad=0.0, eta1=0.0,
              eta2=0.0)
    mom = torch.empty((T, 5), dtype=torch.float64, device=dev)
    rows = []
    for n in args.wake_sizes:
        z0, dp0 = gaussian_bunch(n, SIGMA_Z, SIGMA_DP, SEEDS["paper_scale"])
        z, dp = torch.as_tensor(z0).to(dev), torch.as_tensor(dp0).to(dev)
        del z0, dp0
        call = lambda: ltrk.ltrk_track_wake_f64(z, dp, T, rf, SPS_WAKE, "leapfrog", mom,
                                                stream=stream)
        with torch.cuda.stream(stream):
            call()
            stream.synchronize()
            t0 = time.perf_counter()
            call()
            stream.synchronize()
            dt = time.perf_counter() - t0
            ltrk.ltrk_timing_enable(True)
            call()
            stream.synchronize()
            ltrk.ltrk_timing_take()
            call()
            stream.synchronize()
            tm = ltrk.ltrk_timing_take()
            ltrk.ltrk_timing_enable(False)
        turn_ms = tm["track_ms"] / max(tm["track_launches"], 1)
        other_ms = tm["finalize_ms"] / max(tm["finalize_launches"], 1)
        gbs = STATE_BYTES_PER_PARTICLE * 2 * n / (turn_ms * 1e-3) / 1e9
        row = {"particles": n, "turns": T, "particle_turns_per_s": n * T / dt,
               "turn_kernel_ms": turn_ms, "potential_and_finalize_ms": other_ms,
               "hbm_GBps_algorithmic": gbs, "frac_hbm": gbs / HBM_PEAK_GBS,
               "bytes_per_particle_turn": 2 * STATE_BYTES_PER_PARTICLE}
        rows.append(row)
        log(json.dumps(row))
        del z, dp
        torch.cuda.empty_cache()
    print(json.dumps({"workload": "wake kick: leap-frog, resonator (%g ohm, %g Hz, Q %g), "
                      "%d slices, 1000 turns" % (SPS_WAKE["shunt"], SPS_WAKE["freq_hz"],
                                                 SPS_WAKE["quality"], SPS_WAKE["n_slices"]),
                      "rows": rows}), flush=True)


def _event_seconds(torch, stream, call):
    """Device time of call() from events recorded on `stream` around it."""
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    call()
    end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) / 1e3


def _latency_row(label, work, times):
    t = np.asarray(times)
    return {"config": label, "repeats": int(t.size), "p50_ms": float(np.percentile(t, 50)) * 1e3,
            "p99_ms": float(np.percentile(t, 99)) * 1e3, "min_ms": float(t.min()) * 1e3,
            "max_ms": float(t.max()) * 1e3,
            "particle_turns_per_s_at_p50": work / float(np.percentile(t, 50))}


def bench_latency(args):
    """Whole-run latency percentiles, device time from events around each call
    (every launch and the moment finalize included), inputs restored from
    device-resident copies between repeats (outside the timed region):
    config 1 (1000 x 1e3, leap-frog FP64, 50 repeats), config 3 (1e7 x 1e5,
    leap-frog FP64 and F32C, 5 repeats) and config 4 (256 uneven bunches x 1e4
    turns, FP64 and F32C, 5 repeats). With 5 repeats p99 is the maximum."""
    import torch
    import paper_1610_05801_amd as ltrk
    from synth import (SIGMA_DP, SIGMA_Z, SPS_RING, SEEDS, batched_specs, gaussian_bunch,
                       ring_for, split_f32c)
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    rows = []

    def single(label, n, T, seed, dtype, repeats):
        z0, dp0 = gaussian_bunch(n, SIGMA_Z, SIGMA_DP, seed)
        if dtype == "f64":
            master = [torch.as_tensor(a).to(dev) for a in (z0, dp0)]
        else:
            zh, zc = split_f32c(z0)
            dh, dc = split_f32c(dp0)
            master = [torch.as_tensor(a).to(dev) for a in (zh, dh, zc, dc)]
        work = [torch.empty_like(m) for m in master]
        mom = torch.empty((T, 5), dtype=torch.float64, device=dev)
        fn = ltrk.ltrk_track_f64 if dtype == "f64" else ltrk.ltrk_track_f32c
        times = []
        with torch.cuda.stream(stream):
            for r in range(repeats + 1):  # the first call warms up
                for w, m in zip(work, master):
                    w.copy_(m)
                t = _event_seconds(torch, stream, lambda: fn(*work, T, SPS_RING, "leapfrog", mom,
                                                               stream=stream))
                if r:
                    times.append(t)
        row = _latency_row(label, n * T, times)
        rows.append(row)
        log(json.dumps(row))

    single("1: 1000 x 1e3, leap-frog FP64", 1000, 1000, SEEDS["small"], "f64", 50)
    single("3: 1e7 x 1e5, leap-frog FP64", 10_000_000, 100_000, SEEDS["precision"], "f64", 5)
    single("3: 1e7 x 1e5, leap-frog F32C", 10_000_000, 100_000, SEEDS["precision"], "f32c", 5)
    T = 10_000
    specs = batched_specs()
    total = sum(sp.n for sp in specs)
    for dtype in ("f64", "f32c"):
        bunches, masters = [], []
        for sp in specs:
            r = ring_for(sp)
            z0, dp0 = gaussian_bunch(sp.n, _matched_sigma_z(ltrk, r, sp.sigma_dp), sp.sigma_dp,
                                     sp.seed)
            if dtype == "f64":
                m = [torch.as_tensor(a).to(dev) for a in (z0, dp0)]
                keys = ("z", "dp")
            else:
                zh, zc = split_f32c(z0)
                dh, dc = split_f32c(dp0)
                m = [torch.as_tensor(a).to(dev) for a in (zh, dh, zc, dc)]
                keys = ("z", "dp", "z_comp", "dp_comp")
            b = {"ring": r, "moments": torch.empty((T, 5), dtype=torch.float64, device=dev)}
            for k, a in zip(keys, m):
                b[k] = torch.empty_like(a)
            bunches.append(b)
            masters.append(list(zip(keys, m)))
        times = []
        with torch.cuda.stream(stream):
            for rep in range(6):
                for b, m in zip(bunches, masters):
                    for k, a in m:
                        b[k].copy_(a)
                t = _event_seconds(torch, stream, lambda: ltrk.ltrk_track_batched(
                    bunches, T, "leapfrog", dtype, stream=stream))
                if rep:
                    times.append(t)
        row = _latency_row("4: 256 bunches (%d particles) x 1e4, leap-frog %s" % (total, dtype.upper()),
                           total * T, times)
        rows.append(row)
        log(json.dumps(row))
        del bunches, masters
        torch.cuda.empty_cache()
    print(json.dumps({"workload": "latency percentiles, configs 1, 3, 4", "rows": rows}),
          flush=True)


def bench_counters_f32c(args):
    """The fused F32C leap-frog kernel at 1e6 particles in the benchmark's plan
    (4 launches), for FP32 / FP64 VALU counter passes."""
    import torch
    import paper_1610_05801_amd as ltrk
    from synth import SIGMA_DP, SIGMA_Z, SPS_RING, SEEDS, gaussian_bunch, split_f32c
    dev = torch.device("cuda:0")
    n = 1_000_000
    z0, dp0 = gaussian_bunch(n, SIGMA_Z, SIGMA_DP, SEEDS["paper_scale"])
    zh, zc = split_f32c(z0)
    dh, dc = split_f32c(dp0)
    arrs = [torch.as_tensor(a).to(dev) for a in (zh, dh, zc, dc)]
    plan = ltrk.ltrk_get_plan("leapfrog", "f32c", n)
    K = plan["turns_per_launch"]
    ltrk.ltrk_set_plan(K, plan["block"], plan["ppl"], 0)
    mom = torch.empty((4 * K, 5), dtype=torch.float64, device=dev)
    ltrk.ltrk_track_f32c(*arrs, 4 * K, SPS_RING, "leapfrog", mom)
    torch.cuda.synchronize()
    ltrk.ltrk_set_plan()
    print(json.dumps({"workload": "counters_f32c", "plan": plan}), flush=True)


def _matched_sigma_z(ltrk, ring, sigma_dp):
    d = ltrk.ltrk_derive(ring)
    return sigma_dp * d["slip_length"] / d["omega_s"]


def _moment_rel_error(m, ref):
    """Per-row errors of moment rows against reference rows: means over the
    reference rms, rms and emittance relative."""
    m, ref = np.asarray(m), np.asarray(ref)
    err = np.empty_like(ref)
    err[:, 0] = np.abs(m[:, 0] - ref[:, 0]) / ref[:, 1]
    err[:, 2] = np.abs(m[:, 2] - ref[:, 2]) / ref[:, 3]
    for j in (1, 3, 4):
        err[:, j] = np.abs(m[:, j] - ref[:, j]) / np.abs(ref[:, j])
    return err


def bench_batched(args):
    import torch
    import paper_1610_05801_amd as ltrk
    from synth import batched_specs, gaussian_bunch, ring_for, split_f32c
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    T = args.turns
    specs = batched_specs()
    total = sum(s.n for s in specs)
    log("batched: %d bunches, %d particles, %d turns" % (len(specs), total, T))
    res = {"workload": "batched: %d bunches (log-uniform 1e3-1e6), %d turns" % (len(specs), T),
           "particles": total}
    for dtype in ("f64", "f32c"):
        bunches = []
        for s in specs:
            r = ring_for(s)
            z0, dp0 = gaussian_bunch(s.n, _matched_sigma_z(ltrk, r, s.sigma_dp), s.sigma_dp, s.seed)
            b = {"ring": r, "moments": torch.empty((T, 5), dtype=torch.float64, device=dev)}
            if dtype == "f64":
                b["z"], b["dp"] = torch.as_tensor(z0).to(dev), torch.as_tensor(dp0).to(dev)
            else:
                zh, zc = split_f32c(z0)
                dh, dc = split_f32c(dp0)
                b["z"], b["dp"], b["z_comp"], b["dp_comp"] = [torch.as_tensor(a).to(dev)
                                                              for a in (zh, dh, zc, dc)]
            bunches.append(b)

        def timed():
            with torch.cuda.stream(stream):
                warm = [dict(b, moments=None) for b in bunches]
                ltrk.ltrk_track_batched(warm, 64, "leapfrog", dtype, stream=stream)   # warm-up
                stream.synchronize()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ltrk.ltrk_track_batched(bunches, T, "leapfrog", dtype, stream=stream)
                stream.synchronize()
                return time.perf_counter() - t0

        plan = ltrk.ltrk_get_plan_batched("leapfrog", dtype, total)
        dt = timed()
        res[dtype] = {"particle_turns_per_s": total * T / dt, "seconds": dt, "plan": plan}
        moms = [b["moments"].cpu().numpy() for b in bunches]
        if dtype == "f64":
            f64_moms = moms
        else:
            # F32C against FP64, per bunch and over all turns: means scaled by
            # their rms, rms and emittance relative
            worst = np.zeros(5)
            for a, b in zip(moms, f64_moms):
                worst = np.maximum(worst, _moment_rel_error(a, b).max(axis=0))
            res[dtype]["error_vs_f64"] = dict(zip(
                ("mean_z_over_rms", "rms_z", "mean_dp_over_rms", "rms_dp", "emit_rms"),
                worst.tolist()), note="max over bunches and turns of the F32C moments against "
                "the FP64 run of the same bunches")
        if args.tune:
            # the batched launch tuned on its own tile table (probe bunches of
            # these sizes and rings), then the same run with the tuned plan
            t0 = time.perf_counter()
            tuned = ltrk.ltrk_autotune_batched(bunches, "leapfrog", dtype, stream=stream)
            tune_s = time.perf_counter() - t0
            dt_t = timed()
            res[dtype]["tuned"] = {"plan": tuned, "particle_turns_per_s": total * T / dt_t,
                                   "seconds": dt_t, "tuning_seconds": tune_s,
                                   "vs_default": dt / dt_t}
        log(dtype, json.dumps(res[dtype]))
        del bunches
        torch.cuda.empty_cache()
    print(json.dumps(res), flush=True)


def bench_serving(args):
    """Poisson request stream through the continuous-batching engine: capacity
    from a saturating run (all requests at t = 0), then open-loop Poisson
    arrivals at fractions of that capacity; p50/p99 arrival-to-result latency
    and aggregate particle-turns/s per load."""
    import torch
    import paper_1610_05801_amd as ltrk
    from paper_1610_05801_amd.serve import Request, run_stream
    from synth import gaussian_bunch, request_stream, split_f32c, SPS_RING
    count = args.requests
    budget = int(args.budget_gb * (1 << 30))
    specs = request_stream(1.0, count)
    log("serving: generating %d requests" % count)
    states = {}
    rings = {}
    for sp in specs:
        r = dict(SPS_RING, voltage_V=sp.voltage_V, harmonic=sp.harmonic)
        z0, dp0 = gaussian_bunch(sp.n, _matched_sigma_z(ltrk, r, sp.sigma_dp), sp.sigma_dp,
                                 sp.seed)
        if sp.dtype == "f32c":
            zh, zc = split_f32c(z0)
            dh, dc = split_f32c(dp0)
            states[sp.rid] = (zh, dh, zc, dc)
        else:
            states[sp.rid] = (z0, dp0)
        rings[sp.rid] = r
    work = np.array([sp.n * sp.turns for sp in specs], dtype=np.float64)

    def requests_at(arrivals):
        return [Request(sp.rid, float(t), sp.n, sp.turns, rings[sp.rid], sp.integrator,
                        sp.dtype, states[sp.rid]) for sp, t in zip(specs, arrivals)]

    def run(arrivals):
        eng = ltrk.Engine(budget, max_slots=args.slots)
        recs, wall = run_stream(eng, requests_at(arrivals), k=args.k)
        st = eng.stats()
        eng.close()
        lat = np.array([x.latency_s for x in recs])
        return {"p50_latency_s": float(np.percentile(lat, 50)),
                "p99_latency_s": float(np.percentile(lat, 99)),
                "mean_latency_s": float(lat.mean()), "wall_s": wall,
                "particle_turns_per_s": float(sum(x.n * x.turns for x in recs)) / wall,
                "completed": len(recs), "engine_steps": st["steps"]}

    sat = run(np.zeros(count))
    capacity = sat["particle_turns_per_s"] / work.mean()
    log("saturated: %s; capacity %.2f req/s" % (json.dumps(sat), capacity))
    out = {"workload": "serving: Poisson requests, n log-uniform 1e3-1e7, turns log-uniform "
                       "1e3-1e5, EC/LF/Ruth4 x F64/F32C, matched bunches",
           "requests": count, "budget_bytes": budget, "slots": args.slots, "k": args.k,
           "mean_particle_turns_per_request": float(work.mean()),
           "saturated": sat, "capacity_req_per_s": capacity, "rows": []}
    for frac in args.load:
        lam = frac * capacity
        arrivals = np.array([sp.arrival_s for sp in request_stream(lam, count)])
        row = dict(run(arrivals), load=frac, rate_req_per_s=lam)
        out["rows"].append(row)
        log(json.dumps(row))
    out["f32c_error_vs_f64"] = _serving_f32c_error(ltrk, torch, specs, states, rings)
    print(json.dumps(out), flush=True)


def _serving_f32c_error(ltrk, torch, specs, states, rings, max_work=2e10, max_jobs=24):
    """F32C accuracy on the serving mix: F32C requests (the first max_jobs of
    at most max_work particle-turns, so the check stays short; a job's result
    in the engine equals its standalone run) tracked alone in F32C and in
    FP64 from the same initial state; max over turns of the moment errors."""
    from synth import join_f32c
    dev = torch.device("cuda:0")
    per = {}
    picked = [sp for sp in specs if sp.dtype == "f32c" and sp.n * sp.turns <= max_work][:max_jobs]
    for sp in picked:
        zh, dh, zc, dc = states[sp.rid]
        t32 = [torch.as_tensor(a).to(dev) for a in (zh, dh, zc, dc)]
        t64 = [torch.as_tensor(join_f32c(zh, zc)).to(dev), torch.as_tensor(join_f32c(dh, dc)).to(dev)]
        m32 = torch.empty((sp.turns, 5), dtype=torch.float64, device=dev)
        m64 = torch.empty_like(m32)
        ltrk.ltrk_track_f32c(*t32, sp.turns, rings[sp.rid], sp.integrator, m32)
        ltrk.ltrk_track_f64(*t64, sp.turns, rings[sp.rid], sp.integrator, m64)
        torch.cuda.synchronize()
        err = _moment_rel_error(m32.cpu().numpy(), m64.cpu().numpy()).max(axis=0)
        per.setdefault(sp.integrator, []).append(err)
    out = {"jobs": len(picked), "max_work_particle_turns": max_work,
           "note": "max over turns; means over the rms; per integrator: max and median over jobs"}
    for integ, errs in per.items():
        e = np.array(errs)
        out[integ] = {"jobs": len(errs), "max": dict(zip(
            ("mean_z_over_rms", "rms_z", "mean_dp_over_rms", "rms_dp", "emit_rms"),
            e.max(axis=0).tolist())), "median_rms_z": float(np.median(e[:, 1])),
            "median_rms_dp": float(np.median(e[:, 3]))}
    return out


COUNTER_CAL_BYTES = 1 << 29   # 512 MiB read + 512 MiB written by the calibration kernel


def bench_counters(args):
    """Kernels for rocprofv3 counter passes (FETCH_SIZE, WRITE_SIZE, SQ_*): a
    calibration multiply-by-one of known size, the fused leap-frog kernel at
    1e6 particles with the benchmark's plan (4 launches) and the
    one-launch-per-turn kernel at 1e8 particles (5 turns)."""
    import torch
    import paper_1610_05801_amd as ltrk
    from synth import SIGMA_DP, SIGMA_Z, SPS_RING, SEEDS, gaussian_bunch
    dev = torch.device("cuda:0")
    src = torch.ones(COUNTER_CAL_BYTES // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    del src, dst
    n = 1_000_000
    z0, dp0 = gaussian_bunch(n, SIGMA_Z, SIGMA_DP, SEEDS["paper_scale"])
    z, dp = torch.as_tensor(z0).to(dev), torch.as_tensor(dp0).to(dev)
    plan = ltrk.ltrk_get_plan("leapfrog", "f64", n)   # the benchmark's plan
    K = plan["turns_per_launch"]
    ltrk.ltrk_set_plan(K, plan["block"], plan["ppl"], 0)
    mom = torch.empty((4 * K, 5), dtype=torch.float64, device=dev)
    ltrk.ltrk_track_f64(z, dp, 4 * K, SPS_RING, "leapfrog", mom)
    torch.cuda.synchronize()
    n2 = 100_000_000
    g = torch.Generator(device=dev).manual_seed(7)
    z2 = torch.randn(n2, dtype=torch.float64, device=dev, generator=g) * 0.23
    d2 = torch.randn(n2, dtype=torch.float64, device=dev, generator=g) * 1e-3
    ltrk.ltrk_set_plan(1, 256, 4, 0)
    mom2 = torch.empty((5, 5), dtype=torch.float64, device=dev)
    ltrk.ltrk_track_f64(z2, d2, 5, SPS_RING, "leapfrog", mom2)
    torch.cuda.synchronize()
    ltrk.ltrk_set_plan()
    print(json.dumps({"workload": "counters", "fused_plan": plan,
                      "calibration_bytes": COUNTER_CAL_BYTES}), flush=True)


def summarize_valu(csv_path, out_path, turns_per_launch):
    """Condense a rocprofv3 --pmc CSV of the SQ_INSTS_VALU* counters of
    --workload counters into a per-launch table (instructions per
    particle-turn, executed FP64 flops, clock, issue utilisation)."""
    import csv
    rows = {}
    with open(csv_path) as f:
        for r in csv.DictReader(f):
            if "k_track_single" not in r["Kernel_Name"]:
                continue
            d = rows.setdefault(int(r["Dispatch_Id"]), {
                "kernel": r["Kernel_Name"], "grid": int(r["Grid_Size"]),
                "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
            d[r["Counter_Name"]] = float(r["Counter_Value"])
    out = ["| Launch | Kernel | Duration [us] | VALU instr / pt | FP64 FMA / pt | FP64 ADD / pt | "
           "FP64 MUL / pt | executed FP64 flop / pt | clock [GHz] | VALU issue util |",
           "|---|---|---|---|---|---|---|---|---|---|"]
    for i, (_, d) in enumerate(sorted(rows.items())):
        fused = "<1, 0, 8>" in d["kernel"]
        # fused: 1e6 particles x K turns; unfused: 1e8 particles x 1 turn
        pt = 1_000_000 * turns_per_launch if fused else 100_000_000
        per = {k: d.get(k, 0.0) * 64 / pt for k in ("SQ_INSTS_VALU", "SQ_INSTS_VALU_FMA_F64",
                                                      "SQ_INSTS_VALU_ADD_F64",
                                                      "SQ_INSTS_VALU_MUL_F64")}
        cycles = d.get("GRBM_GUI_ACTIVE", 0.0) / 8
        secs = d["ns"] * 1e-9
        out.append("| %d | %s | %.1f | %.2f | %.2f | %.2f | %.2f | %.2f | %.2f | %.2f |" % (
            i, "fused" if fused else "unfused", d["ns"] / 1e3, per["SQ_INSTS_VALU"],
            per["SQ_INSTS_VALU_FMA_F64"], per["SQ_INSTS_VALU_ADD_F64"],
            per["SQ_INSTS_VALU_MUL_F64"],
            2 * per["SQ_INSTS_VALU_FMA_F64"] + per["SQ_INSTS_VALU_ADD_F64"] +
            per["SQ_INSTS_VALU_MUL_F64"], cycles / secs / 1e9 if secs else 0.0,
            d.get("SQ_INSTS_VALU", 0.0) / (256 * cycles) if cycles else 0.0))
    with open(out_path, "w") as f:
        f.write("\n".join(out) + "\n")
    print("\n".join(out))


def summarize_valu_f32c(valu_csv, out_path, turns_per_launch):
    """Condense a rocprofv3 --pmc CSV of --workload counters_f32c (SQ_INSTS_VALU
    and its FP32 / FP64 FMA, ADD, MUL parts, GRBM_GUI_ACTIVE) into a per-launch
    markdown table: instructions per particle-turn, executed FP32 and FP64
    TFLOP/s, clock and issue utilisation at 4 cycles per wave instruction."""
    import csv
    rows = {}
    with open(valu_csv) as f:
        for r in csv.DictReader(f):
            if "k_track_single" not in r["Kernel_Name"]:
                continue
            d = rows.setdefault(int(r["Dispatch_Id"]), {
                "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
            d[r["Counter_Name"]] = float(r["Counter_Value"])
    pt = 1_000_000 * turns_per_launch
    out = ["| Launch | Duration [us] | VALU instr / pt | FP32 FMA / ADD / MUL per pt | "
           "FP64 FMA / ADD / MUL per pt | FP32 TFLOP/s | FP64 TFLOP/s | clock [GHz] | "
           "VALU issue util |", "|---|---|---|---|---|---|---|---|---|"]
    for i, (_, d) in enumerate(sorted(rows.items())):
        per = {k: d.get(k, 0.0) * 64 / pt for k in (
            "SQ_INSTS_VALU", "SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_ADD_F32",
            "SQ_INSTS_VALU_MUL_F32", "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_ADD_F64",
            "SQ_INSTS_VALU_MUL_F64")}
        secs = d["ns"] * 1e-9
        cycles = d.get("GRBM_GUI_ACTIVE", 0.0) / 8
        f32 = 2 * per["SQ_INSTS_VALU_FMA_F32"] + per["SQ_INSTS_VALU_ADD_F32"] + per["SQ_INSTS_VALU_MUL_F32"]
        f64 = 2 * per["SQ_INSTS_VALU_FMA_F64"] + per["SQ_INSTS_VALU_ADD_F64"] + per["SQ_INSTS_VALU_MUL_F64"]
        out.append("| %d | %.1f | %.2f | %.2f / %.2f / %.2f | %.2f / %.2f / %.2f | %.2f | %.2f | "
                   "%.2f | %.2f |" % (
                       i, d["ns"] / 1e3, per["SQ_INSTS_VALU"], per["SQ_INSTS_VALU_FMA_F32"],
                       per["SQ_INSTS_VALU_ADD_F32"], per["SQ_INSTS_VALU_MUL_F32"],
                       per["SQ_INSTS_VALU_FMA_F64"], per["SQ_INSTS_VALU_ADD_F64"],
                       per["SQ_INSTS_VALU_MUL_F64"], f32 * pt / secs / 1e12,
                       f64 * pt / secs / 1e12, cycles / secs / 1e9 if secs else 0.0,
                       d.get("SQ_INSTS_VALU", 0.0) / (256 * cycles) if cycles else 0.0))
    with open(out_path, "w") as f:
        f.write("\n".join(out) + "\n")
    print("\n".join(out))


def summarize_counters(fetch_csv, write_csv, out_path, turns_per_launch):
    """Condense two rocprofv3 --pmc CSVs (FETCH_SIZE run, WRITE_SIZE run) into
    HBM bytes per particle-turn for the fused and unfused kernels, scaled by
    what the same counters read for the calibration kernel."""
    import csv

    def per_kernel(path, counter):
        rows = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name") != counter:
                    continue
                rows.setdefault(r["Kernel_Name"], []).append(
                    (int(r.get("Dispatch_Id", 0)), float(r["Counter_Value"])))
        return rows

    fetch = per_kernel(fetch_csv, "FETCH_SIZE")
    write = per_kernel(write_csv, "WRITE_SIZE")

    def pick(d, key):
        return [v for k, vs in d.items() if key(k) for _, v in sorted(vs)]

    cal_f = pick(fetch, lambda k: "MulFunctor" in k)
    cal_w = pick(write, lambda k: "MulFunctor" in k)
    fus_f = pick(fetch, lambda k: "k_track_single" in k)
    fus_w = pick(write, lambda k: "k_track_single" in k)
    kib = COUNTER_CAL_BYTES / 1024.0
    f_scale = kib / np.median(cal_f)
    w_scale = kib / np.median(cal_w)
    # k_track_single dispatches: 4 fused (1e6 x K turns) then 5 unfused (1e8 x 1 turn)
    K = float(turns_per_launch)
    fused = {"fetch_bytes": float(np.median(fus_f[:4])) * 1024 * f_scale,
             "write_bytes": float(np.median(fus_w[:4])) * 1024 * w_scale,
             "particle_turns": 1e6 * K, "turns_per_launch": K}
    unfused = {"fetch_bytes": float(np.median(fus_f[4:])) * 1024 * f_scale,
               "write_bytes": float(np.median(fus_w[4:])) * 1024 * w_scale, "particle_turns": 1e8}
    out = {"kernel_hash": kernel_source_hash(),
           "calibration": {"bytes_each_way": COUNTER_CAL_BYTES, "fetch_scale": f_scale,
                           "write_scale": w_scale},
           "fused_leapfrog_1e6": fused, "unfused_leapfrog_1e8": unfused,
           "hbm_bytes_per_particle_turn": (fused["fetch_bytes"] + fused["write_bytes"]) / fused["particle_turns"],
           "unfused_hbm_bytes_per_particle_turn":
               (unfused["fetch_bytes"] + unfused["write_bytes"]) / unfused["particle_turns"]}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="paper",
                    choices=["paper", "unfused", "precision", "batched", "serving", "ksweep",
                             "counters", "counters_f32c", "schemes", "rf2", "program", "6d",
                             "wake", "latency", "nsweep"])
    ap.add_argument("--particles", type=int, default=1_000_000)
    ap.add_argument("--turns", type=int, default=10_000)
    ap.add_argument("--wake-sizes", type=int, nargs="+",
                    default=[1_000_000, 10_000_000, 100_000_000],
                    help="particles of the rows of --workload wake")
    ap.add_argument("--sweep-turns", type=int, default=1_000_000,
                    help="turns of every row of --workload nsweep (the paper's table: 1e6)")
    ap.add_argument("--tune", action="store_true", help="autotune the plan before timing")
    ap.add_argument("--ks", type=int, nargs="+", default=[1, 8, 16, 32, 64, 128, 256, 512],
                    help="turns per launch of --workload ksweep")
    ap.add_argument("--ppls", type=int, nargs="+", default=[2, 4, 8],
                    help="particles per lane of --workload ksweep")
    ap.add_argument("--graphs", type=int, nargs="+", default=[0, 1],
                    help="graph replay off/on of --workload ksweep")
    ap.add_argument("--quick", action="store_true", help="skip the FP32 and unfused legs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--requests", type=int, default=500)
    ap.add_argument("--budget-gb", type=float, default=2.0)
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--k", type=int, default=256)
    ap.add_argument("--load", type=float, nargs="+", default=[0.5, 0.8, 1.0])
    ap.add_argument("--summarize", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "OUT", "K"),
                    help="condense rocprofv3 counter CSVs into a profiles/ JSON summary")
    ap.add_argument("--summarize-valu", nargs=3, metavar=("VALU_CSV", "OUT", "K"),
                    help="condense a rocprofv3 SQ_INSTS_VALU* CSV into a markdown table")
    ap.add_argument("--summarize-valu-f32c", nargs=3, metavar=("VALU_CSV", "OUT", "K"),
                    help="the same for the FP32 and FP64 counters of --workload counters_f32c")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: libltrk has no multi-GPU path "
              "(particles would shard by range with one final moment-sum reduction)",
              file=sys.stderr)
        sys.exit(2)
    if args.summarize:
        summarize_counters(args.summarize[0], args.summarize[1], args.summarize[2],
                           int(args.summarize[3]))
        return
    if args.summarize_valu:
        summarize_valu(args.summarize_valu[0], args.summarize_valu[1], int(args.summarize_valu[2]))
        return
    if args.summarize_valu_f32c:
        summarize_valu_f32c(args.summarize_valu_f32c[0], args.summarize_valu_f32c[1],
                            int(args.summarize_valu_f32c[2]))
        return
    {"paper": bench_default, "unfused": bench_unfused, "ksweep": bench_ksweep,
     "precision": bench_precision, "batched": bench_batched, "serving": bench_serving,
     "counters": bench_counters, "schemes": bench_schemes,
     "rf2": bench_rf2, "program": bench_program, "6d": bench_6d, "wake": bench_wake,
     "latency": bench_latency, "counters_f32c": bench_counters_f32c,
     "nsweep": bench_nsweep}[args.workload](args)


if __name__ == "__main__":
    main()
