"""Moments of bunches far from the origin, against the oracle's two-pass
moments. Moments formed from raw sums (sum z, sum z^2, ...) lose about
(|mean| / rms)^2 ulp of the variance to cancellation: 1e-8 at a mean of 1e4
rms. The library takes each call's sums about a centre fixed for the call
(the mean of a strided sample of the initial state, where it lies more than
4 sample rms from zero), so the moment bound of 1e-10 holds for offsets of
1e2, 1e3 and 1e4 rms:
  - z: bunches in the bucket 15, 154 and 1538 bucket lengths from z = 0
    (the map is periodic in z, so the bunch stays there);
  - dp: a coasting beam (no RF) with a momentum offset of 1e2 ... 1e4 times
    its spread (the offset is then constant);
both for the single-bunch, batched and engine paths and the extended map;
results stay bit-identical across launch plans. The transverse planes of the
6-D map take no centre (the centroid turns with the betatron phase): an
offset of 1e2 rms is within the bound."""
import numpy as np
import pytest

import oracle
from synth import SPS_RING, SIGMA_DP, SIGMA_Z, gaussian_bunch, split_f32c, join_f32c
from tests._parity import moment_error

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RATIOS = [1e2, 1e3, 1e4]
BUCKET = SPS_RING["circumference_m"] / SPS_RING["harmonic"]
COASTING = dict(SPS_RING, voltage_V=0.0)


@pytest.fixture(scope="module")
def ltrk():
    import paper_1610_05801_amd as m
    m.ltrk_set_plan()
    yield m
    m.ltrk_set_plan()


def far_bunch(n, ratio, seed):
    """A Gaussian bunch in the bucket nearest ratio * sigma_z from z = 0."""
    j = round(ratio * SIGMA_Z / BUCKET)
    z0, dp0 = gaussian_bunch(n, SIGMA_Z, SIGMA_DP, seed)
    return z0 + j * BUCKET, dp0


def coasting_bunch(n, ratio, seed):
    sd = 1e-7
    z0, dp0 = gaussian_bunch(n, SIGMA_Z, sd, seed)
    return z0, dp0 + ratio * sd


def run(ltrk, z0, dp0, turns, ring, integ, fn="ltrk_track_f64"):
    z, dp = torch.as_tensor(z0).cuda(), torch.as_tensor(dp0).cuda()
    mom = torch.empty((turns, 5), dtype=torch.float64, device="cuda")
    getattr(ltrk, fn)(z, dp, turns, ring, integ, mom)
    torch.cuda.synchronize()
    return z.cpu().numpy(), dp.cpu().numpy(), mom.cpu().numpy()


def check_moments(mom, mr, label, tol=1e-10):
    err = moment_error(mom, mr).max(axis=0)
    print("%s: moment errors (mean_z, rms_z, mean_dp, rms_dp, emit^2) %s"
          % (label, " ".join("%.1e" % x for x in err)))
    assert err.max() <= tol, (label, err)


@pytest.mark.parametrize("ratio", RATIOS)
def test_bunch_in_a_far_bucket(ltrk, ratio):
    n, T = 100_000, 1000
    z0, dp0 = far_bunch(n, ratio, 900)
    z, dp, mom = run(ltrk, z0, dp0, T, SPS_RING, "leapfrog")
    _, _, mr = oracle.track(z0, dp0, T, SPS_RING, "leapfrog")
    assert abs(mr[0, 0]) / mr[0, 1] > 0.9 * ratio
    check_moments(mom, mr, "far bucket %.0e" % ratio)
    # the same run in other launch plans with the same particles per lane:
    # bit for bit
    ppl = ltrk.ltrk_get_plan("leapfrog", "f64", n)["ppl"]
    for plan in ((7, 64, ppl, 0), (100, 256, ppl, 1)):
        ltrk.ltrk_set_plan(*plan)
        try:
            again = run(ltrk, z0, dp0, T, SPS_RING, "leapfrog")
        finally:
            ltrk.ltrk_set_plan()
        for a, b in zip(again, (z, dp, mom)):
            assert np.array_equal(a, b), plan
    # the allocation-free entry point computes the same
    na = run(ltrk, z0, dp0, T, SPS_RING, "leapfrog", fn="ltrk_track_f64_noalloc")
    for a, b in zip(na, (z, dp, mom)):
        assert np.array_equal(a, b)
    # moments of a state alone
    out = torch.empty((1, 5), dtype=torch.float64, device="cuda")
    ltrk.ltrk_moments_f64(torch.as_tensor(z0).cuda(), torch.as_tensor(dp0).cuda(), out)
    torch.cuda.synchronize()
    check_moments(out.cpu().numpy(), oracle.moments(z0, dp0)[None, :],
                  "state moments %.0e" % ratio, tol=1e-12)


@pytest.mark.parametrize("ratio", RATIOS)
def test_coasting_beam_momentum_offset(ltrk, ratio):
    n, T = 100_000, 1000
    z0, dp0 = coasting_bunch(n, ratio, 901)
    z, dp, mom = run(ltrk, z0, dp0, T, COASTING, "euler_cromer")
    zr, dr, mr = oracle.track(z0, dp0, T, COASTING, "euler_cromer")
    assert np.array_equal(dp, dr)  # no RF: dp is untouched
    assert np.max(np.abs(z - zr) / (np.abs(zr) + SIGMA_Z)) <= 1e-12
    check_moments(mom, mr, "coasting dp offset %.0e" % ratio)


@pytest.mark.parametrize("ratio", RATIOS)
def test_f32c_far_bucket(ltrk, ratio):
    """FP32 + Kahan state in a far bucket: the moment rows against the
    oracle's two-pass moments of the GPU's own final state (the last row) and
    the FP64 run's moments within the F32C accuracy."""
    n, T = 100_000, 300
    z_in, dp_in = far_bunch(n, ratio, 902)
    zh, zc = split_f32c(z_in)
    dh, dc = split_f32c(dp_in)
    t = [torch.as_tensor(a).cuda() for a in (zh, dh, zc, dc)]
    mom = torch.empty((T, 5), dtype=torch.float64, device="cuda")
    ltrk.ltrk_track_f32c(*t, T, SPS_RING, "leapfrog", mom)
    torch.cuda.synchronize()
    a = [x.cpu().numpy() for x in t]
    zf, df = join_f32c(a[0], a[2]), join_f32c(a[1], a[3])
    check_moments(mom.cpu().numpy()[-1:], oracle.moments(zf, df)[None, :],
                  "f32c last row %.0e" % ratio)


def test_batched_bunches_in_far_buckets(ltrk):
    """Four bunches at 1e2 ... 1e4 rms from z = 0 and one centred, in one
    batched call: every bunch's moments against the oracle."""
    T = 500
    inits = [far_bunch(20_000 + 777 * k, r, 910 + k) for k, r in enumerate([0.0] + RATIOS)]
    bunches = [dict(z=torch.as_tensor(z0).cuda(), dp=torch.as_tensor(dp0).cuda(), ring=SPS_RING,
                    moments=torch.empty((T, 5), dtype=torch.float64, device="cuda"))
               for z0, dp0 in inits]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ltrk.ltrk_track_batched(bunches, T, "ruth4", "f64", stream=s)
    torch.cuda.synchronize()
    for k, ((z0, dp0), b) in enumerate(zip(inits, bunches)):
        _, _, mr = oracle.track(z0, dp0, T, SPS_RING, "ruth4")
        check_moments(b["moments"].cpu().numpy(), mr, "batched bunch %d" % k)


def test_engine_job_in_a_far_bucket(ltrk):
    """An engine job 1e4 rms from z = 0: its moments against the oracle and
    bit for bit against the same job tracked alone (8 particles per lane)."""
    n, T = 30_000, 400
    z0, dp0 = far_bunch(n, 1e4, 920)
    eng = ltrk.Engine(hbm_budget_bytes=64 << 20, max_slots=4)
    try:
        slot = eng.admit(n, T, SPS_RING, "leapfrog", "f64", z0, dp0)
        for _ in range(20):
            eng.step(64)
            if eng.poll(slot):
                break
        z, dp, mom = eng.result(slot)
        eng.retire(slot)
    finally:
        eng.close()
    _, _, mr = oracle.track(z0, dp0, T, SPS_RING, "leapfrog")
    check_moments(mom, mr, "engine far bucket")
    ltrk.ltrk_set_plan(128, 256, 8, 0)
    try:
        alone = run(ltrk, z0, dp0, T, SPS_RING, "leapfrog")
    finally:
        ltrk.ltrk_set_plan()
    for a, b in zip(alone, (z, dp, mom)):
        assert np.array_equal(a, b)


def test_extended_map_far_bucket(ltrk):
    """The extended map (second harmonic at 2h, so the map keeps the period
    C/h) in a bucket 1e4 rms from z = 0."""
    rf = dict(SPS_RING, phi1_rad=0.0, harmonic2=2 * SPS_RING["harmonic"],
              voltage2_V=SPS_RING["voltage_V"] / 4, phi2_rad=np.pi, eta1=0.0, eta2=0.0)
    n, T = 50_000, 500
    z0, dp0 = far_bunch(n, 1e4, 930)
    z, dp = torch.as_tensor(z0).cuda(), torch.as_tensor(dp0).cuda()
    mom = torch.empty((T, 5), dtype=torch.float64, device="cuda")
    ltrk.ltrk_track_rf2_f64(z, dp, T, rf, "leapfrog", mom)
    torch.cuda.synchronize()
    _, _, mr = oracle.track_rf2(z0, dp0, T, rf, "leapfrog")
    check_moments(mom.cpu().numpy(), mr, "extended map far bucket")


def test_6d_transverse_offset_1e2(ltrk):
    """6-D map with a 1e2-rms transverse offset in x (no centre for the
    transverse planes) and the bunch in a far bucket (centred (z, dp))."""
    import math
    rf = dict(SPS_RING, phi1_rad=0.0, harmonic2=2 * SPS_RING["harmonic"], voltage2_V=0.0,
              phi2_rad=0.0, eta1=0.0, eta2=0.0)
    tw = dict(q_x=20.13, qp_x=1.5, alpha_x=0.7, beta_x=42.0, q_y=20.18, qp_y=-2.5,
              alpha_y=-1.1, beta_y=87.0)
    n, T = 50_000, 300
    rng = np.random.default_rng(940)
    z0, dp0 = far_bunch(n, 1e3, 940)
    st = dict(z=z0, dp=dp0, x=1e-3 * rng.standard_normal(n) + 0.1,
              xp=2.5e-5 * rng.standard_normal(n), y=1e-3 * rng.standard_normal(n),
              yp=1.2e-5 * rng.standard_normal(n))
    keys = ("z", "dp", "x", "xp", "y", "yp")
    dev = [torch.as_tensor(st[k]).cuda() for k in keys]
    mom = torch.empty((T, 3, 5), dtype=torch.float64, device="cuda")
    ltrk.ltrk_track_6d_f64(*dev, T, rf, tw, "leapfrog", mom)
    torch.cuda.synchronize()
    otw = dict(Qx=tw["q_x"], Qpx=tw["qp_x"], alpha_x=tw["alpha_x"], beta_x=tw["beta_x"],
               Qy=tw["q_y"], Qpy=tw["qp_y"], alpha_y=tw["alpha_y"], beta_y=tw["beta_y"])
    _, mr = oracle.track_6d(st, T, rf, otw, "leapfrog")
    mr = mr.reshape(T, 3, 5)
    m = mom.cpu().numpy()
    assert math.isclose(np.mean(st["x"]) / np.std(st["x"]), 100.0, rel_tol=0.05)
    for p in range(3):
        check_moments(m[:, p], mr[:, p], "6-D plane %d" % p)
