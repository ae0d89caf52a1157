"""Pins of the oracle's extended map (double-harmonic RF with phase offsets,
slip factor eta0 + eta1 dp + eta2 dp^2) against what does not depend on it:
the base single-harmonic map it must reduce to, the exact pure-drift solution,
the linearised double-harmonic tune, bounded Hamiltonian error of the
symplectic schemes, reversibility, unit Jacobian, convergence orders and a
50-digit brute force."""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from synth import SPS_RING, gaussian_bunch

mp.mp.dps = 50
C0 = oracle.derive(SPS_RING)
H1 = SPS_RING["harmonic"]

# bunch-lengthening double RF (second harmonic at 2h, a quarter of V1, opposite
# phase), slip factor with both higher orders
BLM = dict(SPS_RING, phi1_rad=0.0, harmonic2=2 * H1, voltage2_V=SPS_RING["voltage_V"] / 4,
           phi2_rad=math.pi, eta1=0.4 * C0["eta"], eta2=-30.0 * C0["eta"])
PLAIN = dict(SPS_RING, phi1_rad=0.0, harmonic2=2 * H1, voltage2_V=0.0, phi2_rad=0.0,
             eta1=0.0, eta2=0.0)
INTEGS = ["euler_cromer", "leapfrog", "ruth4", "rk4"]


def err(z, dp, zr, dr):
    zb, db = C0["bucket_half_length"], C0["bucket_height"]
    return np.hypot((z - zr) / zb, (dp - dr) / db) / np.hypot(zr / zb, dr / db)


@pytest.mark.parametrize("integ", INTEGS)
def test_reduces_to_single_harmonic_map(integ):
    z0, dp0 = gaussian_bunch(200, 0.2, 1e-3, 31)
    z, dp, m = oracle.track_rf2(z0, dp0, 500, PLAIN, integ)
    zr, dr, mr = oracle.track(z0, dp0, 500, SPS_RING, integ)
    assert np.max(err(z, dp, zr, dr)) < 1e-12
    assert np.max(np.abs(m - mr) / np.abs(mr).max(axis=0)) < 1e-12


@pytest.mark.parametrize("integ", ["euler_cromer", "leapfrog", "ruth4"])
def test_pure_drift_closed_form(integ):
    """With no RF, dp is constant and z_n = z0 - n C eta(dp0) dp0 exactly."""
    rf = dict(BLM, voltage_V=0.0, voltage2_V=0.0)
    dp0 = np.array([-2e-3, -5e-4, 1e-4, 7e-4, 2.5e-3])
    z0 = np.full(5, 0.1)
    n = 300
    z, dp, _ = oracle.track_rf2(z0, dp0, n, rf, integ, with_moments=False)
    C = SPS_RING["circumference_m"]
    eta = C0["eta"] + rf["eta1"] * dp0 + rf["eta2"] * dp0 ** 2
    want = z0 - n * C * eta * dp0
    assert np.array_equal(dp, dp0)
    assert np.max(np.abs(z - want) / np.abs(n * C * eta * dp0)) < 1e-13


def tune_recurrence(z):
    zc = z[1:-1]
    return math.acos(np.dot(zc, z[2:] + z[:-2]) / (2.0 * np.dot(zc, zc))) / (2 * math.pi)


@pytest.mark.parametrize("phi2,sign", [(math.pi, -1.0), (0.0, +1.0)])
def test_double_harmonic_small_amplitude_tune(phi2, sign):
    """Linearised force: (A1 k1 + A2 k2 cos phi2) z = A1 k1 (1 + sign 2 V2/V1) z, so
    cos(2 pi Q) = 1 - omega^2 / 2 with omega^2 = C eta0 A1 k1 (1 + sign/2)."""
    rf = dict(BLM, phi2_rad=phi2, eta1=0.0, eta2=0.0)
    _, _, mom = oracle.track_rf2([1e-5], [0.0], 100_000, rf, "leapfrog")
    z = np.concatenate([[1e-5], mom[:, 0]])
    w2 = SPS_RING["circumference_m"] * C0["eta"] * C0["A"] * C0["k"] * (1.0 + sign * 0.5)
    q_expect = 2.0 * math.asin(math.sqrt(w2) / 2.0) / (2 * math.pi)
    assert abs(tune_recurrence(z) - q_expect) / q_expect < 1e-7


def _inside(rf, n=150, seed=8):
    z, dp = gaussian_bunch(4 * n, 0.15, 6e-4, seed)
    h = oracle.hamiltonian_rf2(z, dp, rf)
    hsep = oracle.hamiltonian_rf2([C0["bucket_half_length"]], [0.0], rf)[0]
    keep = (h > hsep + 0.2 * abs(hsep)) & (np.abs(z) < 0.5)
    return z[keep][:n], dp[keep][:n]


def _max_dh(rf, integ, turns=10_000, every=10):
    z, dp = _inside(rf)
    h0 = oracle.hamiltonian_rf2(z, dp, rf)
    scale = np.max(np.abs(h0))
    early = late = 0.0
    for t in range(every, turns + 1, every):
        z, dp, _ = oracle.track_rf2(z, dp, every, rf, integ, with_moments=False)
        dh = np.max(np.abs(oracle.hamiltonian_rf2(z, dp, rf) - h0)) / scale
        if t <= turns // 10:
            early = max(early, dh)
        else:
            late = max(late, dh)
    return early, late


@pytest.mark.parametrize("integ,bound", [("leapfrog", 1e-3), ("ruth4", 1e-6)])
def test_bounded_hamiltonian_error(integ, bound):
    early, late = _max_dh(BLM, integ)
    assert early < bound and late < bound and late < 2.0 * early


def test_rk4_energy_drifts():
    early, late = _max_dh(BLM, "rk4")
    assert late > 2.0 * early


@pytest.mark.parametrize("integ", ["leapfrog", "ruth4"])
def test_time_reversibility_with_even_slip(integ):
    """R: dp -> -dp reverses the symmetric schemes when eta(dp) is even (eta1 = 0)."""
    rf = dict(BLM, eta1=0.0)
    z0, dp0 = _inside(rf, 60, 12)
    z, dp, _ = oracle.track_rf2(z0, dp0, 1000, rf, integ, with_moments=False)
    z, dp, _ = oracle.track_rf2(z, -dp, 1000, rf, integ, with_moments=False)
    assert np.max(err(z, -dp, z0, dp0)) < 1e-10


@pytest.mark.parametrize("integ", INTEGS)
def test_unit_jacobian(integ):
    hz, hd = 1e-6, 1e-8
    for z0, d0 in [(0.05, 3e-4), (-0.2, -6e-4), (0.3, 9e-4)]:
        zs = np.array([z0 + hz, z0 - hz, z0, z0])
        ds = np.array([d0, d0, d0 + hd, d0 - hd])
        z, dp, _ = oracle.track_rf2(zs, ds, 1, BLM, integ, with_moments=False)
        j = np.array([[(z[0] - z[1]) / (2 * hz), (z[2] - z[3]) / (2 * hd)],
                      [(dp[0] - dp[1]) / (2 * hz), (dp[2] - dp[3]) / (2 * hd)]])
        assert abs(np.linalg.det(j) - 1.0) < 1e-9


@pytest.mark.parametrize("integ,order", [("euler_cromer", 1), ("leapfrog", 2), ("ruth4", 4),
                                         ("rk4", 4)])
def test_convergence_order(integ, order):
    z0, d0, turns = 0.25, 4e-4, 50
    zr, dr, _ = oracle.track_rf2([z0], [d0], turns, BLM, "ruth4", substeps=512,
                                 with_moments=False)
    errs = []
    for m in (1, 2, 4, 8):
        z, dp, _ = oracle.track_rf2([z0], [d0], turns, BLM, integ, substeps=m, with_moments=False)
        errs.append(float(err(z, dp, zr, dr)[0]))
    for i in range(3):
        assert abs(math.log2(errs[i] / errs[i + 1]) - order) < 0.2, errs


def test_fp64_matches_50_digit_brute_force():
    C = mp.mpf(SPS_RING["circumference_m"])
    p = mp.mpf(SPS_RING["p0c_eV"])
    m = mp.mpf(SPS_RING["mass_eV"])
    E = mp.sqrt(p * p + m * m)
    eta0 = 1 / mp.mpf(SPS_RING["gamma_t"]) ** 2 - (m / E) ** 2
    A1 = mp.mpf(SPS_RING["voltage_V"]) / (p / E * p)
    A2 = mp.mpf(BLM["voltage2_V"]) / (p / E * p)
    k1 = 2 * mp.pi * mp.mpf(H1) / C
    k2 = 2 * mp.pi * mp.mpf(BLM["harmonic2"]) / C
    e1, e2 = mp.mpf(BLM["eta1"]), mp.mpf(BLM["eta2"])
    ph2 = mp.mpf(BLM["phi2_rad"])
    z0, d0 = gaussian_bunch(5, 0.15, 6e-4, 41)
    z, dp, _ = oracle.track_rf2(z0, d0, 300, BLM, "leapfrog", with_moments=False)
    for i in range(5):
        zm, dm = mp.mpf(float(z0[i])), mp.mpf(float(d0[i]))
        for _ in range(300):
            zm = zm - C * (eta0 + e1 * dm + e2 * dm * dm) * dm / 2
            dm = dm + A1 * mp.sin(k1 * zm) + A2 * mp.sin(k2 * zm + ph2)
            zm = zm - C * (eta0 + e1 * dm + e2 * dm * dm) * dm / 2
        e = err(np.array([z[i]]), np.array([dp[i]]), np.array([float(zm)]),
                np.array([float(dm)]))[0]
        assert e < 1e-12, (i, e)


def test_invalid_second_harmonic_rejected():
    with pytest.raises(ValueError):
        oracle.track_rf2([0.1], [0.0], 1, dict(BLM, harmonic2=0.0), "leapfrog")
