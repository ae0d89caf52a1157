"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances (FP64): after 1e3 turns, e <= 1e-12 for particles away from the
separatrix and e <= 1e-10 near it (norm in tests/_parity.py); moments to
1e-10 relative. The GPU evaluates sin(k z) with its own revolution-reduced
polynomial and fused multiply-adds, the oracle with libm sin and separate
roundings, so the two differ by a few ulp per turn. Most orbits amplify such
differences by ~3 in 1e3 turns, which the fixed bounds cover many times; the
few orbits just outside the 1% band amplify them by up to a few hundred, and
a particle over the fixed bound is held to 8 ulp per turn times its own
orbit's measured amplification instead, capped at 1e-10 after 1e3 turns, with
at most 0.5% of the bunch over the fixed 1e-12 (tests/_parity.py).
"""
import numpy as np
import pytest

import oracle
from synth import SPS_RING, SIGMA_DP, SIGMA_Z, SEEDS, gaussian_bunch
from tests._parity import (amplification, bucket_error, check_particles, moment_error,
                           near_separatrix)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

INTEGS = ["euler_cromer", "leapfrog", "ruth4", "rk4"]


@pytest.fixture(scope="module")
def ltrk():
    import paper_1610_05801_amd as m
    yield m
    m.ltrk_set_plan()


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def run_f64(ltrk, z0, dp0, turns, integ, ring=SPS_RING, moments=True, stream=None):
    z, dp = dev(z0), dev(dp0)
    mom = torch.empty((turns, 5), dtype=torch.float64, device="cuda") if moments else None
    ltrk.ltrk_track_f64(z, dp, turns, ring, integ, mom, stream=stream)
    torch.cuda.synchronize()
    return z.cpu().numpy(), dp.cpu().numpy(), (mom.cpu().numpy() if moments else None)


def check_against_oracle(z, dp, mom, z0, dp0, turns, integ, ring=SPS_RING, mom_tol=1e-10,
                         label=""):
    """Particle errors e (bucket norm) within the fixed bounds, or for the few
    particles over them within the capped rounding bound of their own orbit
    (tests/_parity.py: check_particles); moments within mom_tol."""
    zr, dr, mr = oracle.track(z0, dp0, turns, ring, integ)
    e = bucket_error(z, dp, zr, dr, ring)
    near = near_separatrix(z0, dp0, ring)
    # plain per-coordinate relative errors, reported (undefined at zero crossings,
    # so not bounded): p50 / p99 / max
    for name, a, ref in (("z", z, zr), ("dp", dp, dr)):
        nz = ref != 0.0
        if np.any(nz):
            rel = np.abs(np.asarray(a)[nz] - ref[nz]) / np.abs(ref[nz])
            print("%s %s n=%d: per-coordinate relative error of %s p50 %.1e p99 %.1e max %.1e"
                  % (label, integ, z0.size, name, np.median(rel), np.percentile(rel, 99),
                     rel.max()))
    check_particles(e, near, turns,
                    lambda m: amplification(oracle.track, z0[m], dp0[m], turns, ring, integ),
                    label="%s %s n=%d" % (label, integ, z0.size))
    if mom is not None and z0.size > 1:
        merr = moment_error(mom, mr).max()
        print("%s %s moments: max rel error %.2e" % (label, integ, merr))
        assert merr <= mom_tol
    return e, near


@pytest.mark.parametrize("integ", INTEGS)
def test_small_workload_all_schemes(ltrk, integ):
    """1e3 particles, 1e3 turns, the small seeded Gaussian bunch."""
    z0, dp0 = gaussian_bunch(1000, SIGMA_Z, SIGMA_DP, SEEDS["small"])
    z, dp, mom = run_f64(ltrk, z0, dp0, 1000, integ)
    check_against_oracle(z, dp, mom, z0, dp0, 1000, integ)


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 255, 257, 4097, 100_003])
@pytest.mark.parametrize("ppl", [1, 2, 4, 8, 16])
def test_sizes_and_tiles(ltrk, n, ppl):
    """Ragged tails and several tiles for every particles-per-lane value."""
    z0, dp0 = gaussian_bunch(n, SIGMA_Z, SIGMA_DP, 7000 + n)
    ltrk.ltrk_set_plan(7, 128, ppl, 0)
    try:
        z, dp, mom = run_f64(ltrk, z0, dp0, 100, "leapfrog")
    finally:
        ltrk.ltrk_set_plan()
    check_against_oracle(z, dp, mom, z0, dp0, 100, "leapfrog")
    if n == 1:
        assert np.all(mom[:, 1] == 0.0) and np.all(mom[:, 4] == 0.0)
        assert np.array_equal(mom[-1, [0, 2]], [z[0], dp[0]])


def test_invariance_across_k_block_graph_and_split(ltrk):
    """Same particles-per-lane: bitwise-identical state and moments for any
    turns-per-launch (1 = one launch per turn), block size, graph replay, and
    for T turns run as T1 + T2."""
    z0, dp0 = gaussian_bunch(50_000, SIGMA_Z, SIGMA_DP, 11)
    T = 97
    ref = None
    stream = torch.cuda.Stream()
    for K, block, graph in [(1, 256, 0), (5, 64, 0), (64, 128, 1), (128, 256, 1), (97, 256, 1)]:
        ltrk.ltrk_set_plan(K, block, 4, graph)
        with torch.cuda.stream(stream):
            out = run_f64(ltrk, z0, dp0, T, "ruth4", stream=stream)
        if ref is None:
            ref = out
            # the one-launch-per-turn run (the unfused form) against the oracle
            check_against_oracle(*out, z0, dp0, T, "ruth4", label="K=1")
        else:
            for a, b in zip(out, ref):
                assert np.array_equal(a, b), (K, block, graph)
    # graph replay a second time (cached graph)
    ltrk.ltrk_set_plan(64, 128, 4, 1)
    with torch.cuda.stream(stream):
        again = run_f64(ltrk, z0, dp0, T, "ruth4", stream=stream)
    for a, b in zip(again, ref):
        assert np.array_equal(a, b)
    # checkpoint / resume: 40 + 57 turns
    z, dp = dev(z0), dev(dp0)
    m1 = torch.empty((40, 5), dtype=torch.float64, device="cuda")
    m2 = torch.empty((57, 5), dtype=torch.float64, device="cuda")
    ltrk.ltrk_track_f64(z, dp, 40, SPS_RING, "ruth4", m1)
    ltrk.ltrk_track_f64(z, dp, 57, SPS_RING, "ruth4", m2)
    torch.cuda.synchronize()
    ltrk.ltrk_set_plan()
    assert np.array_equal(z.cpu().numpy(), ref[0])
    assert np.array_equal(dp.cpu().numpy(), ref[1])
    assert np.array_equal(np.vstack([m1.cpu().numpy(), m2.cpu().numpy()]), ref[2])


@pytest.mark.parametrize("integ", INTEGS)
def test_sixteen_per_lane_invariance_and_clamps(ltrk, integ):
    """16 particles per lane (single-bunch FP64): bit-identical across turns
    per launch, block and graph replay, and against the oracle; the extended
    map under a forced 16 runs with 8 (bit-identical to a forced 8), as the
    header states. F32C at 16: the same states as at 8 bit for bit (the
    per-particle arithmetic does not depend on the lane count), moment rows
    equal to rounding (their sums run in another order), and bit-identical
    across turns per launch, block and graph replay."""
    z0, dp0 = gaussian_bunch(70_001, SIGMA_Z, SIGMA_DP, 16)
    ref = None
    try:
        for K, block, graph in [(1, 256, 0), (37, 64, 1), (200, 128, 0), (300, 256, 1)]:
            ltrk.ltrk_set_plan(K, block, 16, graph)
            out = run_f64(ltrk, z0, dp0, 300, integ)
            if ref is None:
                ref = out
                check_against_oracle(*out, z0, dp0, 300, integ, label="P=16")
            else:
                for a, b in zip(out, ref):
                    assert np.array_equal(a, b), (K, block, graph)
        rf = dict(SPS_RING, phi1_rad=0.0, harmonic2=0.0, voltage2_V=0.0, phi2_rad=0.0,
                  eta1=0.0, eta2=0.0)
        outs = []
        for ppl in (16, 8):
            ltrk.ltrk_set_plan(64, 256, ppl, 0)
            z, dp = dev(z0), dev(dp0)
            mom = torch.empty((50, 5), dtype=torch.float64, device="cuda")
            ltrk.ltrk_track_rf2_f64(z, dp, 50, rf, integ, mom)
            torch.cuda.synchronize()
            outs.append((z.cpu().numpy(), dp.cpu().numpy(), mom.cpu().numpy()))
        for a, b in zip(*outs):
            assert np.array_equal(a, b)
        from synth import split_f32c
        zh, zc = split_f32c(z0)
        dh, dc = split_f32c(dp0)
        outs = []
        side = torch.cuda.Stream()
        for ppl, K, block, graph in [(8, 64, 256, 0), (16, 64, 256, 0), (16, 17, 128, 1),
                                     (16, 50, 64, 1)]:
            ltrk.ltrk_set_plan(K, block, ppl, graph)
            t = [torch.as_tensor(a).cuda() for a in (zh, dh, zc, dc)]
            mom = torch.empty((50, 5), dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            with torch.cuda.stream(side):
                ltrk.ltrk_track_f32c(t[0], t[1], t[2], t[3], 50, SPS_RING, integ, mom,
                                     stream=side)
            torch.cuda.synchronize()
            outs.append([a.cpu().numpy() for a in t] + [mom.cpu().numpy()])
        for a, b in zip(outs[0][:4], outs[1][:4]):
            assert np.array_equal(a, b)
        assert moment_error(outs[1][4], outs[0][4]).max() <= 1e-12
        for o in outs[2:]:
            for a, b in zip(outs[1], o):
                assert np.array_equal(a, b)
    finally:
        ltrk.ltrk_set_plan()


def test_moments_only_entry_point(ltrk):
    z0, dp0 = gaussian_bunch(123_457, SIGMA_Z, SIGMA_DP, 5)
    dp0 = dp0 + 0.2e-3 * z0 / SIGMA_Z
    out = torch.empty((1, 5), dtype=torch.float64, device="cuda")
    ltrk.ltrk_moments_f64(dev(z0), dev(dp0), out)
    got = out.cpu().numpy()[0]
    ref = oracle.moments(z0, dp0)
    assert abs(got[0] - ref[0]) <= 1e-13 * ref[1]
    assert abs(got[2] - ref[2]) <= 1e-13 * ref[3]
    for j in (1, 3, 4):
        assert abs(got[j] - ref[j]) <= 1e-12 * ref[j]


def test_empty_and_zero_turn_calls(ltrk):
    z = torch.empty(0, dtype=torch.float64, device="cuda")
    mom = torch.zeros((3, 5), dtype=torch.float64, device="cuda")
    ltrk.ltrk_track_f64(z, z, 3, SPS_RING, "leapfrog", mom)
    torch.cuda.synchronize()
    assert torch.isnan(mom).all()
    z0, dp0 = gaussian_bunch(10, SIGMA_Z, SIGMA_DP, 1)
    zt, dt = dev(z0), dev(dp0)
    ltrk.ltrk_track_f64(zt, dt, 0, SPS_RING, "leapfrog", None)
    torch.cuda.synchronize()
    assert np.array_equal(zt.cpu().numpy(), z0)


def test_rejects_short_buffers(ltrk):
    """The library itself (not the binding) refuses arrays that run past the
    end of their device allocation: called through the raw C entry point on
    one exact 6 MiB hipMalloc allocation with n or turns too large, it returns
    EINVAL before enqueueing anything. (Tensors from a caching allocator are
    checked against the allocator's underlying segment instead.)"""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so.7")     # the runtime torch already loaded
    lib = ltrk._binding._lib
    ring = ltrk.Ring.of(SPS_RING)
    base = ctypes.c_void_p()
    assert hip.hipMalloc(ctypes.byref(base), ctypes.c_size_t(6 << 20)) == 0
    try:
        mib = 1 << 20
        z = ctypes.c_void_p(base.value)
        dp = ctypes.c_void_p(base.value + 2 * mib)
        mom = ctypes.c_void_p(base.value + 4 * mib)
        s = ctypes.c_void_p(None)
        n = (2 * mib) // 8
        assert hip.hipMemset(base, 0, ctypes.c_size_t(6 << 20)) == 0
        assert lib.ltrk_track_f64(z, dp, n, 1, ctypes.byref(ring), 1, mom, s) == 0
        rows_fit = (2 * mib) // 40
        assert lib.ltrk_track_f64(z, dp, n, rows_fit + 1, ctypes.byref(ring), 1, mom,
                                  s) == ltrk.LTRK_EINVAL
        assert lib.ltrk_track_f64(z, dp, 2 * n + 1, 1, ctypes.byref(ring), 1, None,
                                  s) == ltrk.LTRK_EINVAL
        assert hip.hipDeviceSynchronize() == 0
    finally:
        hip.hipFree(base)


def test_paper_scale_against_oracle(ltrk):
    """1e6 particles, 1e4 turns (the benchmark workload and launch plan): a
    strided sample of 1000 particles against the oracle run on exactly those
    particles (particles are independent; bounds scaled to 1e4 turns), and
    every moment row against the oracle's two-pass moments of the whole bunch
    tracked on all host cores."""
    n, T = 1_000_000, 10_000
    z0, dp0 = gaussian_bunch(n, SIGMA_Z, SIGMA_DP, SEEDS["paper_scale"])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        z, dp, mom = run_f64(ltrk, z0, dp0, T, "leapfrog", stream=stream)
    idx = np.arange(0, n, n // 1000)
    zr, dr, _ = oracle.track(z0[idx], dp0[idx], T, SPS_RING, "leapfrog", with_moments=False)
    e = bucket_error(z[idx], dp[idx], zr, dr, SPS_RING)
    near = near_separatrix(z0[idx], dp0[idx], SPS_RING)
    check_particles(e, near, T,
                    lambda m: amplification(oracle.track, z0[idx][m], dp0[idx][m], T, SPS_RING,
                                            "leapfrog", with_moments=False),
                    label="1e6 x 1e4 sample")
    _, _, mr = oracle.track(z0, dp0, T, SPS_RING, "leapfrog")
    merr = moment_error(mom, mr)
    print("1e6 x 1e4 moments, every row: max rel error %.2e (worst row %d)"
          % (merr.max(), int(np.argmax(merr.max(axis=1)))))
    assert merr.max() <= 1e-10
    last = oracle.moments(z, dp)
    assert moment_error(mom[-1:], last[None, :]).max() <= 1e-12


@pytest.mark.parametrize("integ", INTEGS)
def test_unfused_small_workload(ltrk, integ):
    """One launch per turn (the HBM-bound form) on the small workload against
    the oracle, every scheme."""
    z0, dp0 = gaussian_bunch(1000, SIGMA_Z, SIGMA_DP, SEEDS["small"])
    ltrk.ltrk_set_plan(1, 64, 2, 1)
    try:
        z, dp, mom = run_f64(ltrk, z0, dp0, 1000, integ)
    finally:
        ltrk.ltrk_set_plan()
    check_against_oracle(z, dp, mom, z0, dp0, 1000, integ, label="unfused")


def test_moments_finalized_in_chunks(ltrk):
    """A call whose moment partials exceed the scratch cap (LTRK_SCRATCH_MB)
    is finalized in chunks of whole launches: every row still matches the
    oracle, and the particles and every moment row equal a run in one chunk
    bit for bit (each row is reduced in the same fixed order)."""
    import os
    # at 1e5 particles the default plan has 1 particle per lane: 1563 wave
    # tiles, 62.5 KB of partials per turn, so 16 MiB hold 268 rows: 19 chunks
    # of launches of 268 turns, against one chunk of 1024-turn launches under
    # a 1 GiB cap
    n, T = 100_000, 5000
    z0, dp0 = gaussian_bunch(n, SIGMA_Z, SIGMA_DP, 4242)
    s = torch.cuda.Stream()
    os.environ["LTRK_SCRATCH_MB"] = "1024"
    try:
        whole = run_f64(ltrk, z0, dp0, T, "leapfrog", stream=s)
    finally:
        del os.environ["LTRK_SCRATCH_MB"]
    os.environ["LTRK_SCRATCH_MB"] = "16"
    try:
        chunked = run_f64(ltrk, z0, dp0, T, "leapfrog", stream=s)
    finally:
        del os.environ["LTRK_SCRATCH_MB"]
    for a, b in zip(whole, chunked):
        assert np.array_equal(a, b)
    zr, dr, mr = oracle.track(z0, dp0, T, SPS_RING, "leapfrog")
    assert moment_error(chunked[2], mr).max() <= 1e-10
