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


# The F32C kick's FP32 polynomial (csrc/sinpi32_coeffs.h, gen_sinpi.py --fp32):
# sin(pi r) = pi r * h(r^2) with h(0) = 1, the factor pi carried by the kick
# amplitude as an FP32 hi + lo pair.
HDR32 = os.path.join(os.path.dirname(HDR), "sinpi32_coeffs.h")


def coeffs32():
    text = open(HDR32).read()
    return [float.fromhex(h) for h in re.findall(r"(-?0x[0-9a-fA-Fp.+-]+)f,", text)]


def test_fp32_polynomial_in_exact_arithmetic():
    c = coeffs32()
    assert len(c) == 5 and c[0] == 1.0
    assert all(float(np.float32(x)) == x for x in c)      # FP32 values
    worst = mp.mpf(0)
    for i in range(1, 2001):
        r = mp.mpf(i) / 4000
        s = r * r
        p = mp.mpf(0)
        for cc in reversed(c):
            p = p * s + mp.mpf(cc)
        ref = mp.sin(mp.pi * r)
        worst = max(worst, abs(mp.pi * r * p - ref) / abs(ref))
    assert worst < 7e-9, float(worst)


def _fma32(a, b, c):
    # FP32 fused multiply-add: the product of two FP32 values is exact in
    # FP64, so one FP64 add and the rounding to FP32 stand in for it
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def test_fp32_kick_evaluation_error():
    """The kernels' FP32 steps (r rounded to FP32, r^2, Horner by FMA, r * p,
    the amplitude pi as hi + lo) stay within 3 FP32 ulp of sin(pi r), with r
    the FP64-reduced phase before rounding."""
    c = coeffs32()
    r64 = np.linspace(-0.5, 0.5, 200001)
    r = r64.astype(np.float32)
    r2 = r * r
    p = np.full_like(r, np.float32(c[-1]))
    for cc in reversed(c[:-1]):
        p = _fma32(p, r2, np.full_like(r, np.float32(cc)))
    v = r * p
    ah = np.float32(np.pi)
    al = np.float32(np.pi - float(ah))
    out = _fma32(np.full_like(v, ah), v, np.full_like(v, al) * v).astype(np.float64)
    ref = np.sin(np.pi * r64)
    nz = ref != 0
    rel = np.abs(out[nz] - ref[nz]) / np.abs(ref[nz])
    assert rel.max() < 3 * 2.0 ** -24, rel.max()
    assert np.median(rel) < 2.0 ** -24
