"""Pins of the oracle's derived ring constants against relativistic identities
and textbook RF-bucket formulas (written here in their textbook form, with the
total energy E, evaluated in 50-digit mpmath) rather than against the oracle's
own expressions."""
import math

import mpmath as mp
import pytest

import oracle
from synth import SPS_RING

mp.mp.dps = 50


def _mp_ring(r):
    C = mp.mpf(r["circumference_m"])
    h = mp.mpf(r["harmonic"])
    V = mp.mpf(r["voltage_V"])
    p = mp.mpf(r["p0c_eV"])
    m = mp.mpf(r["mass_eV"])
    gt = mp.mpf(r["gamma_t"])
    q = mp.mpf(r["charge_e"])
    return C, h, V, p, m, gt, q


def rel(a, b):
    return abs(float(a) - float(b)) / abs(float(b))


def test_relativistic_identities():
    c = oracle.derive(SPS_RING)
    m, p = SPS_RING["mass_eV"], SPS_RING["p0c_eV"]
    # gamma^2 - (beta gamma)^2 = 1 and beta gamma = p / m
    assert abs(c["gamma"] ** 2 - (c["beta"] * c["gamma"]) ** 2 - 1.0) < 1e-12
    assert rel(c["beta"] * c["gamma"], p / m) < 2e-15
    assert 0.0 < c["beta"] < 1.0


def test_synchrotron_tune_textbook():
    """Q_s = sqrt(h q V |eta| / (2 pi beta^2 E)) for a stationary bucket
    (e.g. S.Y. Lee, Accelerator Physics, ch. 3), E the total energy."""
    C, h, V, p, m, gt, q = _mp_ring(SPS_RING)
    E = mp.sqrt(p ** 2 + m ** 2)
    gamma = E / m
    beta = p / E
    eta = 1 / gt ** 2 - 1 / gamma ** 2
    qs = mp.sqrt(h * q * V * abs(eta) / (2 * mp.pi * beta ** 2 * E))
    c = oracle.derive(SPS_RING)
    assert rel(c["Qs"], qs) < 1e-14
    assert rel(c["eta"], eta) < 1e-13
    # the discrete leap-frog tune solves cos(2 pi Q) = 1 - omega^2/2
    w = 2 * mp.pi * qs
    q_lf = mp.acos(1 - w ** 2 / 2) / (2 * mp.pi)
    assert rel(c["Q_lf"], q_lf) < 1e-13
    assert c["Q_lf"] > c["Qs"]


def test_bucket_height_textbook():
    """Stationary bucket half-height (dp/p)_max = sqrt(2 q V / (pi h |eta| beta^2 E))."""
    C, h, V, p, m, gt, q = _mp_ring(SPS_RING)
    E = mp.sqrt(p ** 2 + m ** 2)
    beta = p / E
    eta = 1 / gt ** 2 - (m / E) ** 2
    height = mp.sqrt(2 * q * V / (mp.pi * h * abs(eta) * beta ** 2 * E))
    c = oracle.derive(SPS_RING)
    assert rel(c["bucket_height"], height) < 1e-13
    assert rel(c["bucket_half_length"], C / (2 * h)) < 1e-15
    # on the separatrix at z = 0 the Hamiltonian -(D/2) dp^2 equals H_sep
    h0 = oracle.hamiltonian([0.0], [c["bucket_height"]], SPS_RING)[0]
    assert rel(h0, c["H_sep"]) < 1e-13
    # and the unstable fixed point z = C/(2h), dp = 0 sits on it too
    hz = oracle.hamiltonian([c["bucket_half_length"]], [0.0], SPS_RING)[0]
    assert rel(hz, c["H_sep"]) < 1e-12


def test_transition_energy_has_zero_slip():
    r = dict(SPS_RING)
    m = r["mass_eV"]
    gt = r["gamma_t"]
    r["p0c_eV"] = m * math.sqrt(gt * gt - 1.0)
    c = oracle.derive(r)
    assert abs(c["eta"]) < 1e-15 / gt ** 2 * 10


def test_massless_limit():
    r = dict(SPS_RING, mass_eV=0.0)
    c = oracle.derive(r)
    assert c["beta"] == 1.0
    assert math.isinf(c["gamma"])
    assert c["eta"] == 1.0 / r["gamma_t"] ** 2
    assert c["A"] == r["voltage_V"] / r["p0c_eV"]


@pytest.mark.parametrize("key,val", [("circumference_m", 0.0), ("harmonic", -1.0),
                                     ("p0c_eV", 0.0), ("mass_eV", -1.0),
                                     ("gamma_t", 0.0), ("voltage_V", float("nan"))])
def test_invalid_rings_rejected(key, val):
    with pytest.raises(ValueError):
        oracle.derive(dict(SPS_RING, **{key: val}))
