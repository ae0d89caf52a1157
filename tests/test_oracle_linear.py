"""Pins of the oracle's one-turn maps in the linear regime.

For |k z| <= 1e-7 the kick sin(k z) equals k z to ~2e-15 relative, so each
integrator reduces to a 2x2 matrix acting on (z, dp):
  drift Dr(w) = [[1, -w D], [0, 1]],  kick Ki(w) = [[1, 0], [w A k, 1]].
Leap-frog is checked against the closed form of the n-th power of a
unimodular 2x2 matrix, M^n = cos(n mu) I + sin(n mu) (M - cos(mu) I)/sin(mu),
with cos(mu) = 1 - omega^2/2 (omega^2 = A k D); the others against
numpy.linalg.matrix_power of their own compositions (RK4: the 4th-order
Taylor polynomial of exp(L) with L = [[0, -D], [A k, 0]], which RK4
reproduces exactly on a linear system).
"""
import math

import numpy as np
import pytest

import oracle
from synth import SPS_RING

C = oracle.derive(SPS_RING)
D, A, K = C["D"], C["A"], C["k"]
THETA = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))


def Dr(w):
    return np.array([[1.0, -w * D], [0.0, 1.0]])


def Ki(w):
    return np.array([[1.0, 0.0], [w * A * K, 1.0]])


def m_leapfrog():
    return Dr(0.5) @ Ki(1.0) @ Dr(0.5)


def m_euler_cromer():
    return Ki(1.0) @ Dr(1.0)          # drift first, then kick


def m_ruth4():
    seq = [Dr(THETA / 2), Ki(THETA), Dr((1 - THETA) / 2), Ki(1 - 2 * THETA),
           Dr((1 - THETA) / 2), Ki(THETA), Dr(THETA / 2)]
    m = np.eye(2)
    for s in seq:                      # applied left to right in time
        m = s @ m
    return m


def m_rk4():
    L = np.array([[0.0, -D], [A * K, 0.0]])
    return np.eye(2) + L + L @ L / 2 + L @ L @ L / 6 + L @ L @ L @ L / 24


def _bucket_err(x, ref):
    zb, db = C["bucket_half_length"], C["bucket_height"]
    num = np.hypot((x[0] - ref[0]) / zb, (x[1] - ref[1]) / db)
    den = np.hypot(ref[0] / zb, ref[1] / db)
    return num / den


X0 = np.array([[1.0e-9, 2.0e-9, -1.5e-9, 0.0],
               [0.0, 1.0e-11, 3.0e-12, -2.0e-11]])


def test_leapfrog_closed_form():
    w2 = A * K * D
    mu = 2.0 * math.asin(math.sqrt(w2) / 2.0)   # = acos(1 - w^2/2), no cancellation
    M = m_leapfrog()
    assert abs(np.trace(M) - (2.0 - w2)) < 1e-15
    n = 1000
    Mn = math.cos(n * mu) * np.eye(2) + math.sin(n * mu) * (M - math.cos(mu) * np.eye(2)) / math.sin(mu)
    z, dp, _ = oracle.track(X0[0], X0[1], n, SPS_RING, "leapfrog", with_moments=False)
    ref = Mn @ X0
    assert np.max(_bucket_err(np.vstack([z, dp]), ref)) < 1e-12


@pytest.mark.parametrize("name,mat", [("euler_cromer", m_euler_cromer),
                                      ("leapfrog", m_leapfrog),
                                      ("ruth4", m_ruth4), ("rk4", m_rk4)])
def test_linear_map_matrix_power(name, mat):
    n = 1000
    ref = np.linalg.matrix_power(mat(), n) @ X0
    z, dp, _ = oracle.track(X0[0], X0[1], n, SPS_RING, name, with_moments=False)
    assert np.max(_bucket_err(np.vstack([z, dp]), ref)) < 1e-12


def test_euler_cromer_shares_leapfrog_trace():
    assert abs(np.trace(m_euler_cromer()) - np.trace(m_leapfrog())) < 1e-15


def test_ruth4_weights_sum_to_one_turn():
    # a transposed drift/kick order or a wrong weight changes the tune at O(w^2)
    q_ruth = math.acos(np.trace(m_ruth4()) / 2.0) / (2 * math.pi)
    assert abs(q_ruth - C["Qs"]) / C["Qs"] < 1e-6
