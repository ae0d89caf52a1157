"""Pins of the oracle's 6-D map (transverse linear one-turn map with chromatic
phase advance, then the extended longitudinal map) against what does not
depend on it: exact matrix powers of the Twiss rotation, the chromatic phase
for constant momentum, the Courant-Snyder invariants, the closed form of
chromatic decoherence, recoherence after one synchrotron period, volume
preservation and a 50-digit brute force."""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from synth import SPS_RING, gaussian_bunch

mp.mp.dps = 50
C0 = oracle.derive(SPS_RING)
RF = dict(SPS_RING, phi1_rad=0.0, harmonic2=2 * SPS_RING["harmonic"], voltage2_V=0.0,
          phi2_rad=0.0, eta1=0.0, eta2=0.0)
TW = dict(Qx=20.13, Qpx=1.5, alpha_x=0.7, beta_x=42.0, Qy=20.18, Qpy=-2.5, alpha_y=-1.1,
          beta_y=87.0)


def state(n, seed, sz=0.15, sd=6e-4, sx=1e-3):
    rng = np.random.default_rng(seed)
    z, dp = gaussian_bunch(n, sz, sd, seed)
    return dict(z=z, dp=dp, x=sx * rng.standard_normal(n), xp=sx / 40 * rng.standard_normal(n),
                y=sx * rng.standard_normal(n), yp=sx / 80 * rng.standard_normal(n))


def exact_power(u0, v0, mu, turns, alpha, beta):
    """M^n = cos(n mu) I + sin(n mu) J, J = [[alpha, beta], [-gamma, -alpha]], in
    50 digits with the FP64 phase mu of the oracle's turn."""
    g = (1 + mp.mpf(alpha) ** 2) / mp.mpf(beta)
    c, s = mp.cos(turns * mp.mpf(mu)), mp.sin(turns * mp.mpf(mu))
    u0, v0 = mp.mpf(u0), mp.mpf(v0)
    return (float((c + alpha * s) * u0 + beta * s * v0),
            float(-g * s * u0 + (c - alpha * s) * v0))


@pytest.mark.parametrize("qp_x,qp_y", [(0.0, 0.0), (1.5, -2.5)])
def test_matrix_powers_with_constant_momentum(qp_x, qp_y):
    """No RF: dp stays constant, so n turns are the n-th power of one rotation
    by mu = 2 pi (frac(Q) + Q' dp) (FP64 as the oracle forms it)."""
    tw = dict(TW, Qpx=qp_x, Qpy=qp_y)
    rf = dict(RF, voltage_V=0.0)
    st = state(20, 61)
    turns = 777
    out, _ = oracle.track_6d(st, turns, rf, tw, "leapfrog", with_moments=False)
    assert np.array_equal(out["dp"], st["dp"])
    for plane, (u, v) in (("x", ("x", "xp")), ("y", ("y", "yp"))):
        a, b = tw["alpha_" + plane], tw["beta_" + plane]
        for i in range(20):
            q = tw["Q" + plane]
            mu = 2.0 * math.pi * ((q - math.floor(q)) + tw["Qp" + plane] * st["dp"][i])
            eu, ev = exact_power(st[u][i], st[v][i], mu, turns, a, b)
            norm = math.sqrt(oracle.courant_snyder(eu, ev, a, b) * b)
            assert abs(out[u][i] - eu) < 1e-12 * norm
            assert abs(out[v][i] - ev) * b < 1e-12 * norm


@pytest.mark.parametrize("integ", ["euler_cromer", "leapfrog", "ruth4", "rk4"])
def test_longitudinal_part_is_the_extended_map(integ):
    rf = dict(RF, voltage2_V=0.5e6, phi2_rad=math.pi, eta1=1e-4, eta2=-1e-2)
    st = state(300, 62)
    out, mom = oracle.track_6d(st, 200, rf, TW, integ)
    z, dp, m = oracle.track_rf2(st["z"], st["dp"], 200, rf, integ)
    assert np.array_equal(out["z"], z) and np.array_equal(out["dp"], dp)
    assert np.array_equal(mom[:, :5], m)


def test_total_phase_is_the_sum_of_start_of_turn_phases():
    """Rotations with the same Twiss parameters commute, so n turns are one
    rotation by the sum of the turn phases 2 pi (frac(Q) + Q' dp_t), dp_t the
    momentum at the start of turn t, taken from the longitudinal map alone."""
    rf = dict(RF, voltage2_V=0.5e6, phi2_rad=math.pi)
    tw = dict(TW, Qpx=30.0, Qpy=-20.0)
    st = state(6, 67)
    turns = 300
    out, _ = oracle.track_6d(st, turns, rf, tw, "leapfrog", with_moments=False)
    dps = [st["dp"].copy()]
    z, dp = st["z"], st["dp"]
    for _ in range(turns - 1):
        z, dp, _m = oracle.track_rf2(z, dp, 1, rf, "leapfrog", with_moments=False)
        dps.append(dp.copy())
    dps = np.array(dps)  # [turn, particle]
    for plane, (u, v) in (("x", ("x", "xp")), ("y", ("y", "yp"))):
        a, b = tw["alpha_" + plane], tw["beta_" + plane]
        q = tw["Q" + plane]
        for i in range(6):
            phases = [2.0 * math.pi * ((q - math.floor(q)) + tw["Qp" + plane] * d)
                      for d in dps[:, i]]
            total = mp.fsum([mp.mpf(x) for x in phases])
            eu, ev = exact_power(st[u][i], st[v][i], total, 1, a, b)
            norm = math.sqrt(oracle.courant_snyder(eu, ev, a, b) * b)
            assert abs(out[u][i] - eu) < 1e-12 * norm, (plane, i)
            assert abs(out[v][i] - ev) * b < 1e-12 * norm, (plane, i)


def test_courant_snyder_invariants_with_synchrotron_motion():
    st = state(500, 63)
    out, _ = oracle.track_6d(st, 2000, RF, TW, "leapfrog", with_moments=False)
    for u, v, p in (("x", "xp", "x"), ("y", "yp", "y")):
        a, b = TW["alpha_" + p], TW["beta_" + p]
        j0 = oracle.courant_snyder(st[u], st[v], a, b)
        j1 = oracle.courant_snyder(out[u], out[v], a, b)
        assert np.max(np.abs(j1 / j0 - 1.0)) < 1e-12


def _quantile_dp(n, sigma):
    from scipy.stats import norm
    return sigma * norm.ppf((np.arange(n) + 0.5) / n)


def test_chromatic_decoherence_closed_form():
    """No RF, Gaussian dp (a grid of 2e4 quantiles), all particles displaced by
    x0: the centroid is x0 cos(2 pi n Q) exp(-(2 pi n Q' sigma)^2 / 2)."""
    n, sigma, x0 = 20000, 1e-3, 1e-3
    tw = dict(TW, alpha_x=0.0, Qpx=2.0)
    dp = _quantile_dp(n, sigma)
    st = dict(z=np.zeros(n), dp=dp, x=np.full(n, x0), xp=np.zeros(n), y=np.zeros(n),
              yp=np.zeros(n))
    _, mom = oracle.track_6d(st, 600, dict(RF, voltage_V=0.0), tw, "leapfrog")
    t = np.arange(1, 601)
    want = x0 * np.cos(2 * np.pi * t * tw["Qx"]) * np.exp(-(2 * np.pi * t * 2.0 * sigma) ** 2 / 2)
    # quadrature error of the quantile grid: ~4e-5 x0 at the last turns
    assert np.max(np.abs(mom[:, 5] - want)) < 1e-4 * x0
    assert abs(mom[-1, 5]) < 1e-3 * x0  # fully decohered


def test_recoherence_after_one_synchrotron_period():
    """Linear synchrotron motion: the chromatic phase a particle collects over
    one synchrotron period is zero, so a decohered centroid comes back."""
    n = 4000
    ts = 1.0 / C0["Q_lf"]
    sd = 2e-4
    sz = sd * C0["D"] / C0["omega"]
    z, dp = gaussian_bunch(n, sz, sd, 64)
    x0 = 1e-3
    tw = dict(TW, alpha_x=0.0, Qpx=30.0)
    st = dict(z=z, dp=dp, x=np.full(n, x0), xp=np.zeros(n), y=np.zeros(n), yp=np.zeros(n))
    turns = int(round(ts))
    _, mom = oracle.track_6d(st, turns, RF, tw, "leapfrog")
    b = tw["beta_x"]
    amp = np.hypot(mom[:, 5], b * mom[:, 7])  # centroid amplitude (alpha = 0)
    assert amp[turns // 2 - 1] < 0.3 * x0
    assert amp[turns - 1] > 0.98 * x0


@pytest.mark.parametrize("integ", ["euler_cromer", "leapfrog", "ruth4"])
def test_one_turn_map_preserves_volume(integ):
    rf = dict(RF, voltage2_V=0.5e6, phi2_rad=math.pi, eta1=1e-4, eta2=-1e-2)
    keys = ("z", "dp", "x", "xp", "y", "yp")
    x0 = np.array([0.1, 3e-4, 1e-3, -2e-5, -5e-4, 1e-5])
    h = np.array([1e-6, 1e-8, 1e-7, 1e-9, 1e-7, 1e-9])
    cols = []
    for k in range(6):
        pts = np.tile(x0, (2, 1))
        pts[0, k] += h[k]
        pts[1, k] -= h[k]
        out, _ = oracle.track_6d({key: pts[:, i] for i, key in enumerate(keys)}, 1, rf, TW, integ,
                                 with_moments=False)
        col = np.array([(out[key][0] - out[key][1]) / (2 * h[k]) for key in keys])
        cols.append(col)
    assert abs(np.linalg.det(np.array(cols).T) - 1.0) < 1e-7


def test_fp64_matches_50_digit_brute_force():
    rf = dict(RF, voltage2_V=0.5e6, phi2_rad=math.pi, eta1=1e-4, eta2=-1e-2)
    st = state(4, 65)
    turns = 300
    out, _ = oracle.track_6d(st, turns, rf, TW, "leapfrog", with_moments=False)
    C = mp.mpf(SPS_RING["circumference_m"])
    p = mp.mpf(SPS_RING["p0c_eV"])
    m = mp.mpf(SPS_RING["mass_eV"])
    E = mp.sqrt(p * p + m * m)
    eta0 = 1 / mp.mpf(SPS_RING["gamma_t"]) ** 2 - (m / E) ** 2
    A1 = mp.mpf(SPS_RING["voltage_V"]) / (p / E * p)
    A2 = mp.mpf(rf["voltage2_V"]) / (p / E * p)
    k1 = 2 * mp.pi * mp.mpf(SPS_RING["harmonic"]) / C
    k2 = 2 * mp.pi * mp.mpf(rf["harmonic2"]) / C
    e1, e2, ph2 = mp.mpf(rf["eta1"]), mp.mpf(rf["eta2"]), mp.mpf(rf["phi2_rad"])

    def rot(u, v, d, plane):
        a, b = mp.mpf(TW["alpha_" + plane]), mp.mpf(TW["beta_" + plane])
        g = (1 + a * a) / b
        phi = 2 * mp.pi * (mp.mpf(TW["Q" + plane]) + mp.mpf(TW["Qp" + plane]) * d)
        c, s = mp.cos(phi), mp.sin(phi)
        return (c + a * s) * u + b * s * v, -g * s * u + (c - a * s) * v

    for i in range(4):
        zm, dm = mp.mpf(float(st["z"][i])), mp.mpf(float(st["dp"][i]))
        xm, xpm = mp.mpf(float(st["x"][i])), mp.mpf(float(st["xp"][i]))
        ym, ypm = mp.mpf(float(st["y"][i])), mp.mpf(float(st["yp"][i]))
        for _ in range(turns):
            xm, xpm = rot(xm, xpm, dm, "x")
            ym, ypm = rot(ym, ypm, dm, "y")
            zm = zm - C * (eta0 + e1 * dm + e2 * dm * dm) * dm / 2
            dm = dm + A1 * mp.sin(k1 * zm) + A2 * mp.sin(k2 * zm + ph2)
            zm = zm - C * (eta0 + e1 * dm + e2 * dm * dm) * dm / 2
        for key, ref, plane in (("x", xm, "x"), ("y", ym, "y")):
            pk = "xp" if key == "x" else "yp"
            refp = xpm if key == "x" else ypm
            a, b = TW["alpha_" + plane], TW["beta_" + plane]
            norm = math.sqrt(b * oracle.courant_snyder(float(ref), float(refp), a, b))
            assert abs(out[key][i] - float(ref)) < 1e-12 * norm, (i, key)
            assert abs(out[pk][i] - float(refp)) * b < 1e-12 * norm, (i, pk)
        zb, db = C0["bucket_half_length"], C0["bucket_height"]
        e = math.hypot((out["z"][i] - float(zm)) / zb, (out["dp"][i] - float(dm)) / db)
        assert e < 1e-12 * math.hypot(float(zm) / zb, float(dm) / db)


def test_invalid_twiss_rejected():
    st = state(4, 66)
    with pytest.raises(ValueError):
        oracle.track_6d(st, 1, RF, dict(TW, beta_x=0.0), "leapfrog")
    with pytest.raises(ValueError):
        oracle.track_6d(st, 1, RF, dict(TW, Qpy=float("nan")), "leapfrog")
