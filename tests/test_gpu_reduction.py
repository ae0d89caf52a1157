"""The RF kick's range reduction on the GPU, against sin of the exact phase.

One Euler-Cromer turn from delta = 0 leaves z unchanged (the drift adds
-D * 0) and sets delta to A sin(k z), which the kernels evaluate as
A sin(pi u) with u = s z, s = 2h/C in FP64. A wave whose positions stay
below 2^50 / s for the launch reduces the product s z without rounding it
first, so its kicks must match A sin(pi s z) computed in 40-digit arithmetic
from the same FP64 s and z (here up to z = 1e14 m, u ~ 1.3e14, where reducing
the rounded product would be off by ~1e-2 of the amplitude). Other waves
round u = fl(s z) first and reduce that exactly: their kicks must match
A sin(pi fl(s z)), which is 0 once fl(s z) is an integer (|u| >= 2^52).
Non-finite positions give NaN momenta, as sin does.

Error budget of a kick, relative to A: reduction 2^-54 pi (1.7e-16), the
polynomial's relative error (1.8e-16), coefficients scaled by A on the host
(2.2e-16), Horner evaluation (3.3e-16) and the last rounding (1.1e-16):
1e-15 in all.
"""
import mpmath as mp
import numpy as np
import pytest

import oracle
from synth import SPS_RING

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

A = oracle.derive(SPS_RING)["A"]
S = 2.0 * SPS_RING["harmonic"] / SPS_RING["circumference_m"]


@pytest.fixture(scope="module")
def ltrk():
    import paper_1610_05801_amd as m
    yield m


def exact_kick(z):
    """A sin(pi s z) of the exact product."""
    mp.mp.dps = 40
    return np.array([float(A * mp.sin(mp.pi * mp.mpf(S) * mp.mpf(float(v)))) for v in z])


def rounded_kick(z):
    """A sin(pi u) of the rounded product u = fl(s z), reduced exactly:
    u - round(u) is exact for a double u (0 once u is an integer), and
    sin(pi u) = (-1)^round(u) sin(pi (u - round(u)))."""
    mp.mp.dps = 40
    out = []
    for v in z:
        u = float(S * float(v))
        n = round(u)
        r = u - n
        out.append(float(A * (-1) ** (n % 2) * mp.sin(mp.pi * mp.mpf(r))))
    return np.array(out)


Z_EXACT = 2.0 ** 50 / S


def positions(seed, n, lo, hi):
    rng = np.random.default_rng(seed)
    mag = 10.0 ** rng.uniform(lo, hi, n)
    return np.where(rng.random(n) < 0.5, -mag, mag)


def one_turn_f64(ltrk, z0):
    z = torch.as_tensor(z0, dtype=torch.float64).cuda()
    dp = torch.zeros_like(z)
    ltrk.ltrk_track_f64(z, dp, 1, SPS_RING, "euler_cromer")
    torch.cuda.synchronize()
    return z.cpu().numpy(), dp.cpu().numpy()


def test_kick_matches_sin_of_the_exact_product(ltrk):
    z0 = positions(81, 3000, -3.0, 14.0)
    z, dp = one_turn_f64(ltrk, z0)
    assert np.array_equal(z, z0)
    err = np.abs(dp - exact_kick(z0)) / A
    assert err.max() <= 1e-15, (err.max(), z0[np.argmax(err)])
    # the rounded product would not do: it is off by far more at these phases
    assert np.abs(rounded_kick(z0) - exact_kick(z0)).max() > 1e-6 * A


def test_far_positions_reduce_the_rounded_product_exactly(ltrk):
    z0 = positions(82, 2000, 15.0, 300.0)
    assert np.abs(z0).min() > Z_EXACT
    z, dp = one_turn_f64(ltrk, z0)
    assert np.array_equal(z, z0)
    want = rounded_kick(z0)
    assert np.abs(dp - want).max() <= 1e-15 * A
    big = np.abs(S * z0) >= 2.0 ** 52
    assert big.sum() > 1000 and np.all(dp[big] == 0.0)


def test_one_far_particle_switches_only_its_own_wave(ltrk):
    """Each kick matches one of the two reductions, and only wave tiles that
    hold a far particle (tiles of 64 x 8 particles, the plan set here) use the
    rounded product."""
    ltrk.ltrk_set_plan(turns_per_launch=64, block=256, ppl=8)
    try:
        z0 = positions(84, 4096, 0.0, 6.0)
        far = np.array([5, 1500, 1501, 4000])
        z0[far] = [3e15, -7e15, 2e16, 1e300]
        _, dp = one_turn_f64(ltrk, z0)
    finally:
        ltrk.ltrk_set_plan()
    tiles_far = set(far // 512)
    slow = np.isin(np.arange(z0.size) // 512, list(tiles_far))
    assert np.abs(dp[~slow] - exact_kick(z0[~slow])).max() <= 1e-15 * A
    assert np.abs(dp[slow] - rounded_kick(z0[slow])).max() <= 1e-15 * A


def test_non_finite_positions_give_nan_momenta(ltrk):
    z0 = np.array([np.inf, -np.inf, np.nan, 0.1])
    _, dp = one_turn_f64(ltrk, z0)
    assert np.all(np.isnan(dp[:3])) and np.isfinite(dp[3])


def test_f32c_kick_is_within_three_fp32_ulp_of_the_exact_kick(ltrk):
    """F32C: the phase is reduced in FP64 from hi - comp and the sine of the
    reduced phase evaluated in FP32 (rounding of r, r^2, four FMA, r * p, the
    two-part amplitude), so the kick is within 3 FP32 ulp (3 * 2^-24 relative)
    of the exact kick plus the FP64 budget, and within one ulp on median."""
    z0 = positions(83, 3000, -3.0, 14.0).astype(np.float32)
    z = torch.as_tensor(z0).cuda()
    dp, zc, dc = torch.zeros_like(z), torch.zeros_like(z), torch.zeros_like(z)
    ltrk.ltrk_track_f32c(z, dp, zc, dc, 1, SPS_RING, "euler_cromer")
    torch.cuda.synchronize()
    assert np.array_equal(z.cpu().numpy(), z0)
    got = dp.cpu().numpy().astype(np.float64) - dc.cpu().numpy().astype(np.float64)
    want = exact_kick(z0.astype(np.float64))
    assert np.all(np.abs(got - want) <= 3 * 2.0 ** -24 * np.abs(want) + 1e-15 * A)
    nz = want != 0
    assert np.median(np.abs(got - want)[nz] / np.abs(want[nz])) <= 2.0 ** -24
