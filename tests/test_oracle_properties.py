"""Property pins of the oracle over generated inputs (hypothesis, derandomized,
so every run draws the same cases): the moments against exact rational
arithmetic for sets of any size, offset and scale; time reversibility of the
symmetric schemes and a unit Jacobian determinant of every scheme on the
seeded random rings (tests/_rings.py), not only the SPS-like ring."""
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from tests._rings import random_ring
from tests.test_oracle_moments import exact_moments

PROFILE = settings(max_examples=40, deadline=None, derandomize=True)


@PROFILE
@given(n=st.integers(1, 60), offset=st.floats(-1e4, 1e4), scale=st.floats(1e-6, 1e3),
       corr=st.floats(-1.0, 1.0), seed=st.integers(0, 2 ** 31))
def test_moments_exact_for_any_set(n, offset, scale, corr, seed):
    rng = np.random.default_rng(seed)
    z = offset + scale * rng.standard_normal(n)
    dp = 1e-3 * (corr * (z - offset) / scale + rng.standard_normal(n))
    got = oracle.moments(z, dp)
    want = exact_moments(z, dp)
    # means to an ulp of the offset, rms to an ulp of themselves; the emittance
    # through its radicand (rms_z rms_dp)^2 - cov^2, relative to (rms_z rms_dp)^2
    assert abs(got[0] - want[0]) <= 2.3e-16 * (abs(offset) + 8 * scale)
    assert abs(got[2] - want[2]) <= 2.3e-16 * abs(want[2]) + 1e-18 + 2.3e-16 * 8e-3
    for j in (1, 3):
        assert abs(got[j] - want[j]) <= 4.5e-16 * want[j] + 1e-300
    if n > 2 and want[1] > 0 and want[3] > 0:
        r = (want[1] * want[3]) ** 2
        assert abs(got[4] ** 2 - want[4] ** 2) <= 1e-14 * r


def inside_state(ring, rng, fill):
    d = oracle.derive(ring)
    # small amplitude: a fraction of the bucket, well inside the separatrix
    return (fill * d["bucket_half_length"] * rng.uniform(-1, 1, 4),
            fill * d["bucket_height"] * rng.uniform(-1, 1, 4), d)


@PROFILE
@given(ring_seed=st.integers(0, 11), integ=st.sampled_from(["leapfrog", "ruth4"]),
       turns=st.integers(1, 400), fill=st.floats(0.01, 0.5), seed=st.integers(0, 2 ** 31))
def test_time_reversibility_on_random_rings(ring_seed, integ, turns, fill, seed):
    """R M R = M^-1 for the symmetric compositions, R: dp -> -dp."""
    ring = random_ring(ring_seed)
    z0, dp0, d = inside_state(ring, np.random.default_rng(seed), fill)
    z, dp, _ = oracle.track(z0, dp0, turns, ring, integ, with_moments=False)
    z, dp, _ = oracle.track(z, -dp, turns, ring, integ, with_moments=False)
    e = np.hypot((z - z0) / d["bucket_half_length"], (-dp - dp0) / d["bucket_height"])
    assert np.max(e) < 1e-12 * max(1.0, turns / 100.0)


@PROFILE
@given(ring_seed=st.integers(0, 11),
       integ=st.sampled_from(["euler_cromer", "leapfrog", "ruth4"]),
       fill=st.floats(0.01, 0.8), seed=st.integers(0, 2 ** 31))
def test_unit_jacobian_on_random_rings(ring_seed, integ, fill, seed):
    """The symplectic schemes preserve phase-space area: det of the one-turn
    Jacobian (central differences) is 1."""
    ring = random_ring(ring_seed)
    rng = np.random.default_rng(seed)
    d = oracle.derive(ring)
    zb, db = d["bucket_half_length"], d["bucket_height"]
    z0, d0 = fill * zb * rng.uniform(-1, 1), fill * db * rng.uniform(-1, 1)
    hz, hd = 1e-6 * zb, 1e-6 * db
    zs = np.array([z0 + hz, z0 - hz, z0, z0])
    ds = np.array([d0, d0, d0 + hd, d0 - hd])
    z, dp, _ = oracle.track(zs, ds, 1, ring, integ, with_moments=False)
    j = np.array([[(z[0] - z[1]) / (2 * hz), (z[2] - z[3]) / (2 * hd)],
                  [(dp[0] - dp[1]) / (2 * hz), (dp[2] - dp[3]) / (2 * hd)]])
    assert abs(np.linalg.det(j) - 1.0) < 1e-7
