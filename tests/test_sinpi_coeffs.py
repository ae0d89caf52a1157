"""The kernels' sin polynomial (csrc/sinpi_coeffs.h, fitted by gen_sinpi.py)
against 50-digit mpmath: r * p(r^2) approximates sin(pi r) on |r| <= 1/2 to
the error the header states, and the half-revolution reduction with the
(-1)^n sign reproduces sin(pi u) for large u."""
import os
import re

import mpmath as mp
import numpy as np

mp.mp.dps = 50
HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_1610_05801_amd", "csrc", "sinpi_coeffs.h")


def coeffs():
    text = open(HDR).read()
    return [float.fromhex(h) for h in re.findall(r"(-?0x[0-9a-fA-Fp.+-]+),", text)]


def eval_mp(c, r):
    s = r * r
    p = mp.mpf(0)
    for cc in reversed(c):
        p = p * s + mp.mpf(cc)
    return r * p


def test_polynomial_accuracy_in_exact_arithmetic():
    c = coeffs()
    assert 8 <= len(c) <= 12
    worst = mp.mpf(0)
    for i in range(1, 2001):
        r = mp.mpf(i) / 4000            # (0, 1/2]; odd function
        ref = mp.sin(mp.pi * r)
        worst = max(worst, abs(eval_mp(c, r) - ref) / abs(ref))
    assert worst < 2.0e-16, float(worst)


def test_fp64_horner_within_a_few_ulp():
    c = coeffs()
    r = np.linspace(-0.5, 0.5, 20001)
    s = r * r
    p = np.full_like(r, c[-1])
    for cc in reversed(c[:-1]):
        p = p * s + cc
    y = r * p
    ref = np.array([float(mp.sin(mp.pi * mp.mpf(float(x)))) for x in r[::25]])
    got = y[::25]
    nz = ref != 0
    rel = np.abs(got[nz] - ref[nz]) / np.abs(ref[nz])
    assert rel.max() < 8 * 2.0 ** -53


def test_half_revolution_reduction_and_sign():
    c = coeffs()
    for u in (0.3, 1.7, -2.25, 123.456, -98765.4321, 2.0 ** 40 + 0.25):
        n = round(u)
        r = u - n
        val = eval_mp(c, mp.mpf(r)) * (-1 if int(n) % 2 else 1)
        ref = mp.sin(mp.pi * mp.mpf(u))
        assert abs(val - ref) < 1e-15 * max(1.0, abs(float(ref))), u
