"""Shared helpers for GPU-vs-oracle comparisons.

Per-particle error norm (the per-coordinate relative error is undefined at
zero crossings): coordinates are scaled by the bucket half-length z_b = C/(2h)
and half-height dp_b, and
    e = |(dz/z_b, ddp/dp_b)| / |(z/z_b, dp/dp_b)|.
Particles whose initial Hamiltonian lies within 1% of the separatrix value are
"near-separatrix": there the map is chaotic and last-bit differences grow, so
they get a looser bound and are counted separately.

Two correct FP64 evaluations of the map round differently (the kernels'
sine polynomial, fused multiply-adds and phase reduction against libm sin and
separate roundings), so they differ by about one unit in the last place per
turn; a particle's own orbit then amplifies that by the factor measured here
(the oracle's response to a relative perturbation of 1e-13 of its initial z
or delta). The per-particle bound is 8 ulp per turn times that factor
(at least 1), the bound the extended-map tests use.
"""
import numpy as np

import oracle


def bucket_error(z, dp, z_ref, dp_ref, ring):
    c = oracle.derive(ring)
    zb, db = c["bucket_half_length"], c["bucket_height"]
    num = np.hypot((np.asarray(z) - z_ref) / zb, (np.asarray(dp) - dp_ref) / db)
    den = np.hypot(z_ref / zb, dp_ref / db)
    return num / np.maximum(den, 1e-300)


def near_separatrix(z0, dp0, ring, width=0.01):
    c = oracle.derive(ring)
    h = oracle.hamiltonian(z0, dp0, ring)
    return np.abs(h - c["H_sep"]) / abs(c["H_sep"]) <= width


def moment_error(m_gpu, m_ref):
    """Per-row relative error of the 5 moments. Means are scaled by their rms.
    The emittance is compared through its square, the well-conditioned
    radicand rms_z^2 rms_dp^2 - cov^2, scaled by rms_z^2 rms_dp^2: for a nearly
    rank-1 bunch (e.g. two particles) the emittance itself is the square root
    of rounding noise and differs at ~sqrt(eps) between any two evaluations."""
    m_gpu = np.asarray(m_gpu)
    m_ref = np.asarray(m_ref)
    err = np.empty_like(m_ref)
    err[:, 0] = np.abs(m_gpu[:, 0] - m_ref[:, 0]) / m_ref[:, 1]
    err[:, 2] = np.abs(m_gpu[:, 2] - m_ref[:, 2]) / m_ref[:, 3]
    for j in (1, 3):
        err[:, j] = np.abs(m_gpu[:, j] - m_ref[:, j]) / np.abs(m_ref[:, j])
    err[:, 4] = np.abs(m_gpu[:, 4] ** 2 - m_ref[:, 4] ** 2) / (m_ref[:, 1] * m_ref[:, 3]) ** 2
    return err


def amplification(track, z0, dp0, turns, ring_like, integ, eps=1e-13, **kw):
    """Oracle response, in the bucket norm, to perturbing z0 or dp0 by eps
    (relative), divided by eps. `track` is the oracle function (track,
    track_rf2, ...) called as track(z, dp, turns, ring_like, integ, **kw)."""
    za, da = track(z0, dp0, turns, ring_like, integ, **kw)[:2]
    zb, db = track(np.asarray(z0) * (1 + eps), dp0, turns, ring_like, integ, **kw)[:2]
    zc, dc = track(z0, np.asarray(dp0) * (1 + eps), turns, ring_like, integ, **kw)[:2]
    ring = ring_like
    return np.maximum(bucket_error(zb, db, za, da, ring), bucket_error(zc, dc, za, da, ring)) / eps


def rounding_tolerance(amp, turns):
    """8 ulp (2^-53 each) per turn, amplified by the orbit (at least 1)."""
    return 8 * 2.0 ** -53 * turns * np.maximum(amp, 1.0)
