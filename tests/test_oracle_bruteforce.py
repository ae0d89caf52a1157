"""Brute-force pin: the same maps evaluated in 50-digit mpmath on a few
particles. The FP64 oracle must stay within 1e-12 (bucket-normalised) of the
high-precision trajectories; a dropped term or a wrong weight would show as
an O(1) difference."""
import mpmath as mp
import numpy as np
import pytest

import oracle
from synth import SPS_RING, gaussian_bunch

mp.mp.dps = 50
C = oracle.derive(SPS_RING)


def mp_constants(r):
    Cc = mp.mpf(r["circumference_m"])
    h = mp.mpf(r["harmonic"])
    p = mp.mpf(r["p0c_eV"])
    m = mp.mpf(r["mass_eV"])
    E = mp.sqrt(p * p + m * m)
    eta = 1 / mp.mpf(r["gamma_t"]) ** 2 - (m / E) ** 2
    A = mp.mpf(r["charge_e"]) * mp.mpf(r["voltage_V"]) / (p / E * p)
    return A, 2 * mp.pi * h / Cc, eta * Cc


A, K, D = mp_constants(SPS_RING)
TH = 1 / (2 - mp.cbrt(2))


def f(z, d):
    return -D * d, A * mp.sin(K * z)


def mp_turn(z, d, integ):
    if integ == "euler_cromer":
        z = z - D * d
        d = d + A * mp.sin(K * z)
    elif integ == "leapfrog":
        z = z - D * d / 2
        d = d + A * mp.sin(K * z)
        z = z - D * d / 2
    elif integ == "ruth4":
        for dw, kw in ((TH / 2, TH), ((1 - TH) / 2, 1 - 2 * TH), ((1 - TH) / 2, TH)):
            z = z - dw * D * d
            d = d + kw * A * mp.sin(K * z)
        z = z - TH / 2 * D * d
    else:
        a1 = f(z, d)
        a2 = f(z + a1[0] / 2, d + a1[1] / 2)
        a3 = f(z + a2[0] / 2, d + a2[1] / 2)
        a4 = f(z + a3[0], d + a3[1])
        z = z + (a1[0] + 2 * a2[0] + 2 * a3[0] + a4[0]) / 6
        d = d + (a1[1] + 2 * a2[1] + 2 * a3[1] + a4[1]) / 6
    return z, d


@pytest.mark.parametrize("integ,npart,turns", [("leapfrog", 10, 1000), ("euler_cromer", 4, 300),
                                               ("ruth4", 4, 300), ("rk4", 4, 300)])
def test_fp64_oracle_matches_50_digit_brute_force(integ, npart, turns):
    z0, d0 = gaussian_bunch(npart, 0.23, 1e-3, 21)
    z, dp, _ = oracle.track(z0, d0, turns, SPS_RING, integ, with_moments=False)
    zb, db = C["bucket_half_length"], C["bucket_height"]
    for i in range(npart):
        zm, dm = mp.mpf(float(z0[i])), mp.mpf(float(d0[i]))
        for _ in range(turns):
            zm, dm = mp_turn(zm, dm, integ)
        err = np.hypot((z[i] - float(zm)) / zb, (dp[i] - float(dm)) / db)
        norm = np.hypot(float(zm) / zb, float(dm) / db)
        assert err / norm < 1e-12, (i, err / norm)
