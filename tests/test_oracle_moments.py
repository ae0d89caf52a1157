"""Pins of the oracle's per-turn moments: against NumPy's mean/std(ddof=0) and
math.fsum, exact rational arithmetic on small sets, and closed-form special
cases (n = 0, 1, 2 and a rank-1 phase-space set)."""
import math
from fractions import Fraction

import numpy as np

import oracle
from synth import gaussian_bunch


def exact_moments(z, dp):
    """Population moments computed in exact rational arithmetic."""
    zs = [Fraction(float(v)) for v in z]
    ds = [Fraction(float(v)) for v in dp]
    n = len(zs)
    mz = sum(zs) / n
    md = sum(ds) / n
    vz = sum((a - mz) ** 2 for a in zs) / n
    vd = sum((b - md) ** 2 for b in ds) / n
    cov = sum((a - mz) * (b - md) for a, b in zip(zs, ds)) / n
    e2 = vz * vd - cov * cov
    return [float(mz), math.sqrt(vz), float(md), math.sqrt(vd), math.sqrt(max(e2, 0))]


def test_against_numpy_and_fsum():
    z, dp = gaussian_bunch(100_003, 0.23, 1e-3, 3)
    dp = dp + 0.3 * z * 1e-3          # correlated, so the emittance term matters
    m = oracle.moments(z, dp)
    assert abs(m[0] - math.fsum(z) / z.size) <= 1e-15 * 0.23
    assert abs(m[2] - math.fsum(dp) / dp.size) <= 1e-15 * 1e-3
    assert abs(m[1] - np.std(z)) / np.std(z) < 1e-13
    assert abs(m[3] - np.std(dp)) / np.std(dp) < 1e-13
    cov = np.mean((z - z.mean()) * (dp - dp.mean()))
    e = math.sqrt(np.var(z) * np.var(dp) - cov * cov)
    assert abs(m[4] - e) / e < 1e-12


def test_exact_rational_small_sets():
    for seed in range(5):
        z, dp = gaussian_bunch(37, 0.5, 2e-3, 100 + seed)
        z = z + 3.0                     # offset mean: the two-pass form must not cancel
        got = oracle.moments(z, dp)
        want = exact_moments(z, dp)
        for g, w in zip(got, want):
            assert abs(g - w) <= 1e-15 * max(abs(w), 1e-300) + 1e-300


def test_special_cases():
    assert np.all(np.isnan(oracle.moments([], [])))
    m1 = oracle.moments([0.7], [-2e-3])
    assert m1.tolist() == [0.7, 0.0, -2e-3, 0.0, 0.0]
    m2 = oracle.moments([0.1, 0.5], [1e-3, -3e-3])
    assert abs(m2[1] - 0.2) < 1e-16 and abs(m2[3] - 2e-3) < 1e-18
    # two points span a rank-1 covariance: emit^2 = vz vd - cov^2 cancels to
    # rounding level, so emit is at most ~sqrt(eps) rms_z rms_dp
    assert m2[4] <= 3e-8 * m2[1] * m2[3]


def test_rank_one_set_has_zero_emittance():
    z = np.linspace(-1, 1, 1001)
    m = oracle.moments(z, -2e-3 * z)
    assert m[4] <= 3e-8 * m[1] * m[3]


def test_moments_rows_follow_tracking():
    """Row t of the tracking output equals the moments of the state after turn t+1."""
    from synth import SPS_RING
    z, dp = gaussian_bunch(500, 0.23, 1e-3, 5)
    _, _, mom = oracle.track(z, dp, 3, SPS_RING, "leapfrog")
    z3, dp3, _ = oracle.track(z, dp, 3, SPS_RING, "leapfrog", with_moments=False)
    assert np.array_equal(mom[2], oracle.moments(z3, dp3))


def test_thread_count_does_not_change_results():
    from synth import SPS_RING
    z, dp = gaussian_bunch(20_000, 0.23, 1e-3, 9)
    a = oracle.track(z, dp, 20, SPS_RING, "ruth4", threads=1)
    b = oracle.track(z, dp, 20, SPS_RING, "ruth4", threads=4)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
