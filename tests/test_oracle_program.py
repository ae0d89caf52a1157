"""Pins of the oracle's RF-programme map (per-turn RF voltages and phases and
a per-turn reference momentum) against what does not depend on it: the
extended map it must reduce to turn by turn, the closed form of a first turn
under a momentum step, the synchronous particle as a fixed point, the one-turn
Jacobian p_a / p_b (adiabatic damping), the adiabatic invariants of slow
voltage and momentum ramps, and a 50-digit brute force in absolute momentum."""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from synth import SPS_RING, gaussian_bunch

mp.mp.dps = 50
C0 = oracle.derive(SPS_RING)
H1 = SPS_RING["harmonic"]
P0 = SPS_RING["p0c_eV"]
V1 = SPS_RING["voltage_V"]
RF = dict(SPS_RING, phi1_rad=0.0, harmonic2=2 * H1, voltage2_V=V1 / 4, phi2_rad=math.pi,
          eta1=0.4 * C0["eta"], eta2=-30.0 * C0["eta"])
SYMPLECTIC = ["euler_cromer", "leapfrog", "ruth4"]


def constant_programme(turns, rf=RF, **over):
    vals = dict(voltage_V=rf["voltage_V"], phi1_rad=rf["phi1_rad"], voltage2_V=rf["voltage2_V"],
                phi2_rad=rf["phi2_rad"], p0c_eV=rf["p0c_eV"])
    vals.update(over)
    return {k: np.full(turns, float(v)) for k, v in vals.items()}


def beta_of(p):
    m = SPS_RING["mass_eV"]
    return p / np.sqrt(p * p + m * m)


def synchronous_programme(turns, dp_per_turn, v1=V1, v2=0.0):
    """Linear momentum ramp with the synchronous phase of every turn."""
    p_after = P0 + dp_per_turn * np.arange(1, turns + 1)
    p_before = np.concatenate([[P0], p_after[:-1]])
    phi = np.arcsin(beta_of(p_before) * (p_after - p_before) / (SPS_RING["charge_e"] * v1))
    return dict(voltage_V=np.full(turns, v1), phi1_rad=phi, voltage2_V=np.full(turns, v2),
                phi2_rad=np.full(turns, math.pi), p0c_eV=p_after)


def err(z, dp, zr, dr):
    zb, db = C0["bucket_half_length"], C0["bucket_height"]
    return np.hypot((z - zr) / zb, (dp - dr) / db) / np.hypot(zr / zb, dr / db)


@pytest.mark.parametrize("integ", ["euler_cromer", "leapfrog", "ruth4", "rk4"])
def test_constant_programme_is_extended_map(integ):
    z0, dp0 = gaussian_bunch(200, 0.2, 1e-3, 51)
    z, dp, m = oracle.track_program(z0, dp0, 400, RF, constant_programme(400), integ)
    zr, dr, mr = oracle.track_rf2(z0, dp0, 400, RF, integ)
    assert np.max(err(z, dp, zr, dr)) < 1e-12
    assert np.max(np.abs(m - mr) / np.abs(mr).max(axis=0)) < 1e-12


@pytest.mark.parametrize("integ", ["euler_cromer", "leapfrog", "ruth4", "rk4"])
def test_entry_t_applies_to_turn_t(integ):
    """Settings that change after turn 150: the programme equals 150 turns of
    the extended map with the first settings followed by 250 with the second."""
    a = dict(RF)
    b = dict(RF, voltage_V=3.1e6, phi1_rad=0.05, voltage2_V=-0.2e6, phi2_rad=2.0)
    prog = constant_programme(400)
    for k, key in [("voltage_V", "voltage_V"), ("phi1_rad", "phi1_rad"),
                   ("voltage2_V", "voltage2_V"), ("phi2_rad", "phi2_rad")]:
        prog[k][150:] = b[key]
    z0, dp0 = gaussian_bunch(100, 0.15, 6e-4, 52)
    z, dp, _ = oracle.track_program(z0, dp0, 400, RF, prog, integ, with_moments=False)
    z1, d1, _ = oracle.track_rf2(z0, dp0, 150, a, integ, with_moments=False)
    zr, dr, _ = oracle.track_rf2(z1, d1, 250, b, integ, with_moments=False)
    assert np.max(err(z, dp, zr, dr)) < 1e-12


def test_first_turn_under_a_momentum_step_closed_form():
    """From z = delta = 0 with no RF force at z = 0, one turn moves the
    reference from p_a to p_b, so delta = (p_a - p_b)/p_b, and leap-frog's
    second half drift uses eta at p_b."""
    pb = P0 * (1 + 1e-4)
    prog = constant_programme(1, phi1_rad=0.0, voltage2_V=0.0, p0c_eV=pb)
    want_d = (P0 - pb) / pb
    z, dp, _ = oracle.track_program([0.0], [0.0], 1, RF, prog, "euler_cromer")
    assert z[0] == 0.0 and abs(dp[0] - want_d) <= 2e-16 * abs(want_d)
    z, dp, _ = oracle.track_program([0.0], [0.0], 1, RF, prog, "leapfrog")
    m = SPS_RING["mass_eV"]
    eta_b = 1 / SPS_RING["gamma_t"] ** 2 - m * m / (pb * pb + m * m)
    eta = eta_b + RF["eta1"] * want_d + RF["eta2"] * want_d ** 2
    want_z = -0.5 * SPS_RING["circumference_m"] * eta * want_d
    assert abs(dp[0] - want_d) <= 2e-16 * abs(want_d)
    assert abs(z[0] - want_z) <= 1e-14 * abs(want_z)


@pytest.mark.parametrize("integ", SYMPLECTIC)
@pytest.mark.parametrize("v2", [0.0, V1 / 4])
def test_synchronous_particle_is_a_fixed_point(integ, v2):
    """Ramp of 1e-5 p0 per turn with the synchronous phase: the particle at
    the origin stays there, while an off-phase programme moves it."""
    turns = 2000
    prog = synchronous_programme(turns, 1e-5 * P0, v2=v2)
    z, dp, _ = oracle.track_program([0.0], [0.0], turns, RF, prog, integ)
    assert abs(z[0]) < 1e-13 and abs(dp[0]) < 1e-16
    prog["phi1_rad"][:] = 0.0
    z, dp, _ = oracle.track_program([0.0], [0.0], turns, RF, prog, integ)
    assert abs(dp[0]) > 1e-6


@pytest.mark.parametrize("integ", SYMPLECTIC)
def test_one_turn_jacobian_is_momentum_ratio(integ):
    """Adiabatic damping: a turn that raises the reference from p_a to p_b
    scales phase-space area by p_a / p_b (unit for constant momentum)."""
    hz, hd = 1e-6, 1e-8
    for ratio in (1.0, 1.001, 0.998):
        prog = constant_programme(1, p0c_eV=P0 * ratio, phi1_rad=0.02)
        for z0, d0 in [(0.05, 3e-4), (-0.2, -6e-4)]:
            zs = np.array([z0 + hz, z0 - hz, z0, z0])
            ds = np.array([d0, d0, d0 + hd, d0 - hd])
            z, dp, _ = oracle.track_program(zs, ds, 1, RF, prog, integ, with_moments=False)
            j = np.array([[(z[0] - z[1]) / (2 * hz), (z[2] - z[3]) / (2 * hd)],
                          [(dp[0] - dp[1]) / (2 * hz), (dp[2] - dp[3]) / (2 * hd)]])
            assert abs(np.linalg.det(j) - 1.0 / ratio) < 1e-9, (ratio, np.linalg.det(j))


def _matched_ring(amplitude, n=64):
    """n particles at equally spaced phases on one small matched ellipse: for
    linear motion their sample moments do not depend on the rotation angle
    (rms_z = amplitude / sqrt 2), so slow-ramp scalings show without the
    1/sqrt(n) phase noise of a random bunch."""
    psi = 2 * np.pi * (np.arange(n) + 0.25) / n
    return amplitude * np.cos(psi), amplitude * C0["omega"] / C0["D"] * np.sin(psi)


def test_adiabatic_voltage_ramp_bunch_length():
    """Constant momentum, V1 raised 2 -> 8 MV over 2e4 turns (~120 synchrotron
    periods): a small matched bunch keeps its emittance and its length scales
    as V^(-1/4) (linear motion, adiabatic invariant)."""
    turns = 20000
    rf = dict(RF, voltage2_V=0.0, eta1=0.0, eta2=0.0)
    prog = constant_programme(turns, rf, voltage2_V=0.0)
    prog["voltage_V"] = np.linspace(2e6, 8e6, turns)
    z0, dp0 = _matched_ring(0.02)
    m0 = oracle.moments(z0, dp0)
    z, dp, _ = oracle.track_program(z0, dp0, turns, rf, prog, "leapfrog", with_moments=False)
    m1 = oracle.moments(z, dp)
    assert abs(m1[1] / m0[1] - 4 ** -0.25) < 2e-4
    assert abs(m1[3] / m0[3] - 4 ** 0.25) < 2e-4
    assert abs(m1[4] / m0[4] - 1.0) < 2e-4


@pytest.mark.parametrize("integ", SYMPLECTIC)
def test_adiabatic_momentum_ramp_damps_emittance(integ):
    """Momentum raised by 10% over 2e4 turns at the synchronous phase: the
    longitudinal emittance in (z, delta) shrinks as 1/p0 (p0 * emittance is
    the adiabatic invariant), i.e. by 9.1%."""
    turns = 20000
    rf = dict(RF, voltage2_V=0.0, eta1=0.0, eta2=0.0)
    prog = synchronous_programme(turns, 0.1 * P0 / turns)
    z0, dp0 = _matched_ring(0.02)
    e0 = oracle.moments(z0, dp0)[4]
    z, dp, _ = oracle.track_program(z0, dp0, turns, rf, prog, integ, with_moments=False)
    e1 = oracle.moments(z, dp)[4]
    ratio = prog["p0c_eV"][-1] / P0
    assert abs(e1 * ratio / e0 - 1.0) < 2e-4
    assert abs(e1 / e0 - 1.0) > 0.08


@pytest.mark.parametrize("integ,order", [("euler_cromer", 1), ("leapfrog", 2), ("ruth4", 4)])
def test_convergence_order_under_a_ramp(integ, order):
    """Splitting each turn's momentum step over the kicks in proportion to
    their weights keeps each scheme's order (strong ramp: 2e-4 p0 per turn
    at 12 MV)."""
    turns = 50
    prog = synchronous_programme(turns, 2e-4 * P0, v1=12e6)
    zr, dr, _ = oracle.track_program([0.25], [4e-4], turns, RF, prog, "ruth4", substeps=512,
                                     with_moments=False)
    errs = []
    for m in (1, 2, 4, 8):
        z, dp, _ = oracle.track_program([0.25], [4e-4], turns, RF, prog, integ, substeps=m,
                                        with_moments=False)
        errs.append(float(err(z, dp, zr, dr)[0]))
    for i in range(3):
        assert abs(math.log2(errs[i] / errs[i + 1]) - order) < 0.2, errs


def test_fp64_matches_50_digit_brute_force_in_absolute_momentum():
    """Leap-frog through a programme with a momentum ramp, changing voltages
    and phases, a second harmonic and slip factor orders, against 50-digit
    arithmetic in the absolute momentum P = p0 (1 + delta)."""
    turns = 150
    rng = np.random.default_rng(55)
    prog = synchronous_programme(turns, 2e-6 * P0, v2=V1 / 5)
    prog["voltage_V"] = prog["voltage_V"] * (1 + 0.1 * np.sin(np.arange(turns) / 20))
    prog["phi1_rad"] = prog["phi1_rad"] + 0.01 * rng.standard_normal(turns)
    prog["phi2_rad"] = prog["phi2_rad"] + 0.3 * np.cos(np.arange(turns) / 7)
    z0, d0 = gaussian_bunch(4, 0.15, 6e-4, 56)
    z, dp, _ = oracle.track_program(z0, d0, turns, RF, prog, "leapfrog", with_moments=False)
    C = mp.mpf(SPS_RING["circumference_m"])
    m = mp.mpf(SPS_RING["mass_eV"])
    q = mp.mpf(SPS_RING["charge_e"])
    gt2 = mp.mpf(SPS_RING["gamma_t"]) ** 2
    k1 = 2 * mp.pi * mp.mpf(H1) / C
    k2 = 2 * mp.pi * mp.mpf(RF["harmonic2"]) / C
    e1, e2 = mp.mpf(RF["eta1"]), mp.mpf(RF["eta2"])

    def eta(p, d):
        return 1 / gt2 - m * m / (p * p + m * m) + e1 * d + e2 * d * d

    for i in range(4):
        zm, dm = mp.mpf(float(z0[i])), mp.mpf(float(d0[i]))
        pa = mp.mpf(P0)
        for t in range(turns):
            pb = mp.mpf(float(prog["p0c_eV"][t]))
            beta = pa / mp.sqrt(pa * pa + m * m)
            zm = zm - C * eta(pa, dm) * dm / 2
            gain = q * (mp.mpf(float(prog["voltage_V"][t])) *
                        mp.sin(k1 * zm + mp.mpf(float(prog["phi1_rad"][t]))) +
                        mp.mpf(float(prog["voltage2_V"][t])) *
                        mp.sin(k2 * zm + mp.mpf(float(prog["phi2_rad"][t]))))
            P = pa * (1 + dm) + gain / beta
            dm = P / pb - 1
            zm = zm - C * eta(pb, dm) * dm / 2
            pa = pb
        e = err(np.array([z[i]]), np.array([dp[i]]), np.array([float(zm)]),
                np.array([float(dm)]))[0]
        assert e < 1e-12, (i, e)


def test_rk4_with_a_momentum_ramp_is_rejected():
    prog = synchronous_programme(10, 1e-5 * P0)
    with pytest.raises(ValueError):
        oracle.track_program([0.1], [0.0], 10, RF, prog, "rk4")
    oracle.track_program([0.1], [0.0], 10, RF, constant_programme(10), "rk4")


def test_invalid_programme_rejected():
    prog = constant_programme(5)
    prog["p0c_eV"][2] = -1.0
    with pytest.raises(ValueError):
        oracle.track_program([0.1], [0.0], 5, RF, prog, "leapfrog")
    prog = constant_programme(5)
    prog["voltage_V"][4] = float("nan")
    with pytest.raises(ValueError):
        oracle.track_program([0.1], [0.0], 5, RF, prog, "leapfrog")
