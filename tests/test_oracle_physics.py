"""Pins of the oracle's nonlinear tracking against what the physics fixes:
synchrotron tunes (small amplitude and the pendulum's elliptic-integral law),
bounded Hamiltonian error of the symplectic schemes, time reversibility of the
symmetric schemes, unit Jacobian determinant, the convergence order of each
scheme, and the stability sign convention."""
import math

import numpy as np
import pytest
from scipy.special import ellipk

import oracle
from synth import SPS_RING, gaussian_bunch

C = oracle.derive(SPS_RING)


def trajectory(z0, dp0, turns, integrator, ring=SPS_RING):
    """z after every turn of a single particle (mean of a one-particle bunch)."""
    _, _, mom = oracle.track([z0], [dp0], turns, ring, integrator)
    return np.concatenate([[z0], mom[:, 0]])


def tune_recurrence(z):
    """Least-squares cos(mu) from z[n+1] + z[n-1] = 2 cos(mu) z[n], exact for any
    linear unimodular map."""
    zc = z[1:-1]
    cosmu = np.dot(zc, z[2:] + z[:-2]) / (2.0 * np.dot(zc, zc))
    return math.acos(cosmu) / (2 * math.pi)


def tune_crossings(z):
    """Mean frequency from upward zero crossings (linear interpolation)."""
    idx = np.nonzero((z[:-1] < 0) & (z[1:] >= 0))[0]
    t = idx + (-z[idx]) / (z[idx + 1] - z[idx])
    return (len(t) - 1) / (t[-1] - t[0])


def test_small_amplitude_tune_matches_leapfrog_closed_form():
    z = trajectory(1.0e-4, 0.0, 200_000, "leapfrog")
    q = tune_recurrence(z)
    # pendulum detuning at phi_hat = k z0 is phi_hat^2/16 relative (~1.1e-8)
    assert abs(q - C["Q_lf"]) / C["Q_lf"] < 1e-7
    # the analytic smooth tune differs from the leap-frog one by ~omega^2/24
    w2 = C["omega"] ** 2
    assert abs(q - C["Qs"]) / C["Qs"] < w2 / 24 + 1e-6


def test_small_amplitude_tune_euler_cromer_equals_leapfrog():
    q_ec = tune_recurrence(trajectory(1.0e-4, 0.0, 50_000, "euler_cromer"))
    assert abs(q_ec - C["Q_lf"]) / C["Q_lf"] < 1e-7


@pytest.mark.parametrize("z0", [0.2, 0.4, 0.6])
def test_ruth4_nonlinear_tune_matches_pendulum(z0):
    """phi = k z obeys phi'' = -omega^2 sin(phi): a pendulum whose tune at
    amplitude phi_hat is Q_s pi / (2 K(m)), m = sin^2(phi_hat/2)."""
    phi = C["k"] * z0
    q_expect = C["Qs"] * math.pi / (2.0 * ellipk(math.sin(phi / 2) ** 2))
    q = tune_crossings(trajectory(z0, 0.0, 100_000, "ruth4"))
    assert abs(q - q_expect) / q_expect < 1e-6


def test_leapfrog_nonlinear_tune_error_is_second_order():
    z0 = 0.4
    phi = C["k"] * z0
    q_expect = C["Qs"] * math.pi / (2.0 * ellipk(math.sin(phi / 2) ** 2))
    q = tune_crossings(trajectory(z0, 0.0, 100_000, "leapfrog"))
    err = abs(q - q_expect) / q_expect
    assert 1e-6 < err < 1e-4     # O(omega^2) = O(1.4e-3) scheme error, small prefactor


def _inside_bunch(n=200, seed=7):
    z, dp = gaussian_bunch(4 * n, 0.23, 1.0e-3, seed)
    h = oracle.hamiltonian(z, dp, SPS_RING)
    keep = (h > 0.9 * C["H_sep"]) & (np.abs(z) < C["bucket_half_length"])
    return z[keep][:n], dp[keep][:n]


def _max_dh(integrator, turns, every=10):
    z, dp = _inside_bunch()
    h0 = oracle.hamiltonian(z, dp, SPS_RING)
    worst_early = worst_late = 0.0
    t = 0
    while t < turns:
        z, dp, _ = oracle.track(z, dp, every, SPS_RING, integrator, with_moments=False)
        t += every
        dh = np.max(np.abs(oracle.hamiltonian(z, dp, SPS_RING) - h0)) / abs(C["H_sep"])
        if t <= turns // 10:
            worst_early = max(worst_early, dh)
        else:
            worst_late = max(worst_late, dh)
    return worst_early, worst_late


@pytest.mark.parametrize("integrator,bound", [("leapfrog", 4e-4), ("euler_cromer", 5e-2),
                                              ("ruth4", 3e-7)])
def test_symplectic_hamiltonian_error_is_bounded(integrator, bound):
    early, late = _max_dh(integrator, 20_000)
    assert early < bound and late < bound
    # no secular growth: the late window is not much worse than the early one
    assert late < 2.0 * early


def test_rk4_hamiltonian_error_grows():
    early, late = _max_dh("rk4", 20_000)
    assert late > 2.0 * early      # non-symplectic drift of the energy


@pytest.mark.parametrize("integrator", ["leapfrog", "ruth4"])
def test_time_reversibility(integrator):
    """Symmetric compositions satisfy R M R = M^-1 with R: dp -> -dp."""
    z0, dp0 = _inside_bunch(100, seed=11)
    z, dp, _ = oracle.track(z0, dp0, 1000, SPS_RING, integrator, with_moments=False)
    z, dp, _ = oracle.track(z, -dp, 1000, SPS_RING, integrator, with_moments=False)
    dp = -dp
    e = np.hypot((z - z0) / C["bucket_half_length"], (dp - dp0) / C["bucket_height"])
    assert np.max(e) < 1e-10


def test_euler_cromer_is_not_time_symmetric():
    z0, dp0 = _inside_bunch(20, seed=12)
    z, dp, _ = oracle.track(z0, dp0, 100, SPS_RING, "euler_cromer", with_moments=False)
    z, dp, _ = oracle.track(z, -dp, 100, SPS_RING, "euler_cromer", with_moments=False)
    e = np.hypot((z - z0) / C["bucket_half_length"], (-dp - dp0) / C["bucket_height"])
    assert np.max(e) > 1e-6


@pytest.mark.parametrize("integrator", ["euler_cromer", "leapfrog", "ruth4", "rk4"])
def test_unit_jacobian_determinant(integrator):
    pts = [(0.1, 2e-4), (-0.3, -1e-3), (0.5, 1.5e-3)]
    hz, hd = 1e-6, 1e-8
    for z0, d0 in pts:
        zs = np.array([z0 + hz, z0 - hz, z0, z0])
        ds = np.array([d0, d0, d0 + hd, d0 - hd])
        z, dp, _ = oracle.track(zs, ds, 1, SPS_RING, integrator, with_moments=False)
        j = np.array([[(z[0] - z[1]) / (2 * hz), (z[2] - z[3]) / (2 * hd)],
                      [(dp[0] - dp[1]) / (2 * hz), (dp[2] - dp[3]) / (2 * hd)]])
        assert abs(np.linalg.det(j) - 1.0) < 1e-9


@pytest.mark.parametrize("integrator,order", [("euler_cromer", 1), ("leapfrog", 2),
                                              ("ruth4", 4), ("rk4", 4)])
def test_convergence_order(integrator, order):
    z0, d0, turns = 0.3, 5e-4, 50
    zr, dr, _ = oracle.track([z0], [d0], turns, SPS_RING, "ruth4", substeps=512,
                             with_moments=False)
    errs = []
    for m in (1, 2, 4, 8):
        z, dp, _ = oracle.track([z0], [d0], turns, SPS_RING, integrator, substeps=m,
                                with_moments=False)
        errs.append(math.hypot((z[0] - zr[0]) / C["bucket_half_length"],
                               (dp[0] - dr[0]) / C["bucket_height"]))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    for o in orders:
        assert abs(o - order) < 0.15, orders


def test_stability_sign_convention():
    """Above transition (eta > 0) with V > 0 the bucket centre z = 0 is stable;
    below transition it is stable only with the voltage negated."""
    z = trajectory(1e-3, 0.0, 2000, "leapfrog")
    assert np.max(np.abs(z)) <= 1.00001e-3
    below = dict(SPS_RING, gamma_t=40.0)            # gamma = 27.7 < gamma_t
    assert oracle.derive(below)["eta"] < 0
    z = trajectory(1e-3, 0.0, 2000, "leapfrog", ring=below)
    assert np.max(np.abs(z)) > 1.0
    below_neg = dict(below, voltage_V=-SPS_RING["voltage_V"])
    z = trajectory(1e-3, 0.0, 2000, "leapfrog", ring=below_neg)
    assert np.max(np.abs(z)) <= 1.00001e-3
