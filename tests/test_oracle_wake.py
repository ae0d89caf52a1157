"""Pins of the oracle's wake kick against what does not depend on it: the
resonator wake as the cosine transform of its impedance (read back from the
kick of two particles), the potential of a constant wake as the charge ahead,
the energy loss of a Gaussian bunch from the resonator's loss factor,
causality, the slicing range, and reduction to the extended map at zero
intensity."""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.stats import norm

import oracle
from synth import SPS_RING

C0 = oracle.derive(SPS_RING)
BETA = C0["beta"]
P0C = SPS_RING["p0c_eV"]
Q = SPS_RING["charge_e"]
NO_RF = dict(SPS_RING, voltage_V=0.0, phi1_rad=0.0, harmonic2=0.0, voltage2_V=0.0, phi2_rad=0.0,
             eta1=0.0, eta2=0.0)
RES = dict(model=0, R_s=1e4, f_r=1.0e9, Q=1.0, intensity=1e11, n_slices=400, z_lo=-0.6,
           z_hi=0.6)


def kappa(wake, n):
    """delta kick per volt of potential per count: q Q_mp / (beta p0 c)."""
    return Q * (Q * oracle.E_CHARGE * wake["intensity"] / n) / (BETA * P0C)


def impedance_re(omega, R_s, f_r, Qf):
    w_r = 2 * np.pi * f_r
    x = Qf * (omega / w_r - w_r / omega)
    return R_s / (1 + x * x)


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
def test_resonator_wake_is_the_cosine_transform_of_its_impedance():
    """Two particles at slice centres, no RF and dp = 0 (the map does not move
    them): the trailing one's kick is -kappa (W(0) + W(lag)), so the oracle's
    wake at each lag is read back and compared with
    W(tau) = (2/pi) int_0^inf Re Z(omega) cos(omega tau) d omega."""
    w = dict(RES, n_slices=200)
    dz = (w["z_hi"] - w["z_lo"]) / w["n_slices"]
    centre = lambda k: w["z_lo"] + (k + 0.5) * dz
    k_trail = 20
    w0 = None
    for lag in (0, 1, 3, 10, 40):
        if lag == 0:
            z = np.array([centre(k_trail)])
        else:
            z = np.array([centre(k_trail), centre(k_trail + lag)])
        _, dp, _ = oracle.track_wake(z, np.zeros_like(z), 1, NO_RF, w, "euler_cromer")
        pot = -dp[0] / kappa(w, z.size)
        if lag == 0:
            w0 = pot
            wr = 2 * np.pi * w["f_r"]
            assert abs(w0 - wr / (2 * w["Q"]) * w["R_s"]) < 1e-12 * w0  # W(0) = alpha R_s
            continue
        tau = lag * dz / (BETA * oracle.C_LIGHT)
        got = pot - w0
        f = lambda om: impedance_re(om, w["R_s"], w["f_r"], w["Q"])
        want = 2 / np.pi * integrate.quad(f, 0.0, np.inf, weight="cos", wvar=tau, limlst=200)[0]
        # the Fourier integral of the slowly decaying Re Z converges to ~1e-5 of
        # W(0+) = 2 W(0); a wrong sign, factor or frequency is off by > 1e-1
        assert abs(got - want) < 1e-5 * 2 * w0, (lag, got, want)


def test_constant_wake_potential_is_the_charge_ahead():
    """model 1: W = R_s behind the source, R_s / 2 at zero lag, so the potential
    at centre k is R_s Q_mp (count ahead + count_k / 2); particles then get it
    interpolated between centres. The momenta start non-zero, so the map step
    (a drift of ~1 slice; no RF) moves the particles before they are sliced:
    the kick follows the positions after the step."""
    rng = np.random.default_rng(71)
    w = dict(RES, model=1, R_s=3e12, n_slices=50)
    n = 3000
    z0 = rng.uniform(-0.55, 0.55, n)
    dp0 = 5e-3 * rng.standard_normal(n)
    z, dp, _ = oracle.track_wake(z0, dp0, 1, NO_RF, w, "euler_cromer")
    assert np.max(np.abs(z - z0)) > 2 * (w["z_hi"] - w["z_lo"]) / w["n_slices"]
    edges = np.linspace(w["z_lo"], w["z_hi"], w["n_slices"] + 1)
    counts = np.histogram(z, bins=edges)[0].astype(np.float64)
    ahead = np.concatenate([np.cumsum(counts[::-1])[::-1][1:], [0.0]])
    pot = w["R_s"] * (ahead + 0.5 * counts)
    centres = 0.5 * (edges[1:] + edges[:-1])
    inside = (z >= w["z_lo"]) & (z < w["z_hi"])
    want = np.where(inside, -kappa(w, n) * np.interp(z, centres, pot), 0.0)
    assert np.max(np.abs((dp - dp0) - want)) < 1e-12 * np.max(np.abs(want))


def test_gaussian_bunch_energy_loss_is_the_loss_factor():
    """A Gaussian bunch (quantile grid) loses, per particle, the energy
    k q Q_b with the loss factor k = (1/pi) int_0^inf Re Z exp(-(omega sigma_t)^2)."""
    n, sigma = 200_000, 0.1
    z = sigma * norm.ppf((np.arange(n) + 0.5) / n)
    w = dict(RES, n_slices=2000, z_lo=-0.7, z_hi=0.7)
    _, dp, _ = oracle.track_wake(z, np.zeros(n), 1, NO_RF, w, "euler_cromer")
    sig_t = sigma / (BETA * oracle.C_LIGHT)
    k_loss = integrate.quad(lambda om: impedance_re(om, w["R_s"], w["f_r"], w["Q"]) *
                            np.exp(-(om * sig_t) ** 2), 0, 50 / sig_t, limit=500)[0] / np.pi
    q_b = Q * oracle.E_CHARGE * w["intensity"]
    want = -k_loss * Q * q_b / (BETA * P0C)
    assert abs(dp.mean() / want - 1) < 2e-3, (dp.mean(), want)


def test_head_particle_feels_only_its_own_slice():
    """The leading particle, alone in the upper half of its slice: the centre
    ahead has no charge at or ahead of it, so the particle gets (1 - f) times
    its own half wake W(0) = alpha R_s."""
    rng = np.random.default_rng(72)
    w = dict(RES)
    dz = (w["z_hi"] - w["z_lo"]) / w["n_slices"]
    zh = w["z_lo"] + 350.75 * dz
    z = np.concatenate([rng.uniform(-0.5, 0.3, 500), [zh]])
    _, dp, _ = oracle.track_wake(z, np.zeros(z.size), 1, NO_RF, w, "euler_cromer")
    s = (zh - w["z_lo"]) / dz - 0.5
    f = s - math.floor(s)
    wr = 2 * np.pi * w["f_r"]
    v_own = wr / (2 * w["Q"]) * w["R_s"]  # one count at zero lag; the centre ahead is empty
    want = -kappa(w, z.size) * (1 - f) * v_own
    assert abs(dp[-1] - want) < 1e-13 * abs(want)


def test_particles_outside_the_slices_are_neither_counted_nor_kicked():
    rng = np.random.default_rng(73)
    z_in = rng.uniform(-0.6, 0.6, 1000)  # every slice, the last and first included
    z = np.concatenate([z_in, [0.61, 0.8, -0.7]])
    w = dict(RES)
    _, dp, _ = oracle.track_wake(z, np.zeros(z.size), 1, NO_RF, w, "euler_cromer")
    assert np.all(dp[-3:] == 0.0)
    # the inside particles feel the same potential as without the outsiders
    # (kappa scales with the number of macro-particles, so keep Q_mp fixed)
    w_in = dict(w, intensity=w["intensity"] * 1000 / 1003)
    _, dp_in, _ = oracle.track_wake(z_in, np.zeros(1000), 1, NO_RF, w_in, "euler_cromer")
    assert np.max(np.abs(dp[:1000] - dp_in)) < 1e-14 * np.max(np.abs(dp_in))


@pytest.mark.parametrize("integ", ["euler_cromer", "leapfrog", "ruth4", "rk4"])
def test_zero_intensity_is_the_extended_map(integ):
    rf = dict(SPS_RING, phi1_rad=0.1, harmonic2=9240.0, voltage2_V=0.5e6, phi2_rad=math.pi,
              eta1=1e-4, eta2=-1e-2)
    rng = np.random.default_rng(74)
    z, dp = 0.1 * rng.standard_normal(300), 5e-4 * rng.standard_normal(300)
    a = oracle.track_wake(z, dp, 200, rf, dict(RES, intensity=0.0), integ)
    b = oracle.track_rf2(z, dp, 200, rf, integ)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])


def test_invalid_wake_rejected():
    for bad in (dict(Q=0.5), dict(n_slices=0), dict(z_hi=-0.6), dict(f_r=0.0), dict(model=2),
                dict(n_slices=10.5)):
        with pytest.raises(ValueError):
            oracle.track_wake([0.1], [0.0], 1, NO_RF, dict(RES, **bad), "leapfrog")
