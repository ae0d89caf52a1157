"""FP32 + Kahan-compensated state (LTRK_F32C) against the FP64 oracle.

The state is FP32 (hi, comp) with every increment an FP32 value added with
Kahan compensation; the RF phase is reduced in FP64, the sine of the reduced
phase is an FP32 polynomial (the kick increment's relative error is at most
1.7e-7, median 3e-8, against at most 2^-24 = 6e-8 for an FP64 sine rounded
once to FP32), and the moments are accumulated in FP64. Error model: each
increment carries a relative error of a few 2^-24 (the drifts one rounding,
the kicks up to 3 FP32 ulp), the compensated sums add no further error at
leading order, so after T turns a particle's coordinates differ from FP64 by
roughly sqrt(T) * 2^-24 * |increment| times a small factor (random walk), and
the resulting amplitude error turns into a phase error growing ~T through the
amplitude dependence of the synchrotron tune. The bounds below are that
estimate with a safety factor, checked at 1e3 turns on the small seeded bunch.
"""
import numpy as np
import pytest

import oracle
from synth import SPS_RING, SIGMA_DP, SIGMA_Z, SEEDS, gaussian_bunch, join_f32c, split_f32c
from tests._parity import bucket_error, moment_error, near_separatrix

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# core particles after 1e3 turns; moments after 1e3 turns
F32C_CORE_TOL = {"euler_cromer": 2e-5, "leapfrog": 2e-5, "ruth4": 2e-5, "rk4": 2e-5}
F32C_MOM_TOL = 2e-6


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


@pytest.fixture(scope="module")
def ltrk():
    import paper_1610_05801_amd as m
    yield m
    m.ltrk_set_plan()


def run_f32c(ltrk, z0, dp0, turns, integ):
    zh, zc = split_f32c(z0)
    dh, dc = split_f32c(dp0)
    t = [dev(a, torch.float32) for a in (zh, dh, zc, dc)]
    mom = torch.empty((turns, 5), dtype=torch.float64, device="cuda")
    ltrk.ltrk_track_f32c(t[0], t[1], t[2], t[3], turns, SPS_RING, integ, mom)
    torch.cuda.synchronize()
    zh, dh, zc, dc = [x.cpu().numpy() for x in t]
    return join_f32c(zh, zc), join_f32c(dh, dc), mom.cpu().numpy(), (zh, zc, dh, dc)


@pytest.mark.parametrize("integ", ["euler_cromer", "leapfrog", "ruth4", "rk4"])
def test_f32c_against_fp64_oracle(ltrk, integ):
    z_in, dp_in = gaussian_bunch(1000, SIGMA_Z, SIGMA_DP, SEEDS["small"])
    # the oracle starts from exactly the values the FP32 pairs encode
    z0 = join_f32c(*split_f32c(z_in))
    dp0 = join_f32c(*split_f32c(dp_in))
    z, dp, mom, _ = run_f32c(ltrk, z0, dp0, 1000, integ)
    zr, dr, mr = oracle.track(z0, dp0, 1000, SPS_RING, integ)
    e = bucket_error(z, dp, zr, dr, SPS_RING)
    near = near_separatrix(z0, dp0, SPS_RING, width=0.05)
    print("\n%s F32C: core max e %.3e, p50 %.3e; moments max rel %.3e"
          % (integ, e[~near].max(), np.median(e[~near]), moment_error(mom, mr).max()))
    assert e[~near].max() <= F32C_CORE_TOL[integ]
    assert moment_error(mom, mr).max() <= F32C_MOM_TOL


def plain_fp32_leapfrog(z0, dp0, turns, ring):
    """Leap-frog with the state simply stored in FP32 (no compensation): the
    FP32 rounding of z and dp every turn, with increments computed in FP64."""
    c = oracle.derive(ring)
    z = z0.astype(np.float32)
    d = dp0.astype(np.float32)
    for _ in range(turns):
        z = (z.astype(np.float64) - 0.5 * c["D"] * d.astype(np.float64)).astype(np.float32)
        d = (d.astype(np.float64) + c["A"] * np.sin(c["k"] * z.astype(np.float64))).astype(np.float32)
        z = (z.astype(np.float64) - 0.5 * c["D"] * d.astype(np.float64)).astype(np.float32)
    return z.astype(np.float64), d.astype(np.float64)


def test_f32c_compensation_beats_plain_fp32(ltrk):
    """After 2000 turns the compensated FP32 state stays an order of magnitude
    closer to the FP64 oracle than a state rounded to FP32 every turn."""
    z0, dp0 = gaussian_bunch(2000, 0.1, 5e-4, 17)
    z0 = join_f32c(*split_f32c(z0))
    dp0 = join_f32c(*split_f32c(dp0))
    z, dp, _, (zh, zc, dh, dc) = run_f32c(ltrk, z0, dp0, 2000, "leapfrog")
    zr, dr, _ = oracle.track(z0, dp0, 2000, SPS_RING, "leapfrog", with_moments=False)
    assert np.any(zc != 0) and np.any(dc != 0)
    zp, dpl = plain_fp32_leapfrog(z0, dp0, 2000, SPS_RING)
    e_kahan = np.median(bucket_error(z, dp, zr, dr, SPS_RING))
    e_plain = np.median(bucket_error(zp, dpl, zr, dr, SPS_RING))
    print("\nF32C median e %.3e, plain FP32 median e %.3e" % (e_kahan, e_plain))
    assert e_kahan < 0.1 * e_plain


def test_f32c_moments_entry_point(ltrk):
    z_in, dp_in = gaussian_bunch(10_001, SIGMA_Z, SIGMA_DP, 3)
    zh, zc = split_f32c(z_in)
    dh, dc = split_f32c(dp_in)
    out = torch.empty((1, 5), dtype=torch.float64, device="cuda")
    ltrk.ltrk_moments_f32c(*[dev(a, torch.float32) for a in (zh, dh, zc, dc)], out)
    ref = oracle.moments(join_f32c(zh, zc), join_f32c(dh, dc))
    got = out.cpu().numpy()[0]
    for j in (1, 3, 4):
        assert abs(got[j] - ref[j]) <= 1e-12 * ref[j]
