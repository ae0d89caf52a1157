"""Shared helpers for GPU-vs-oracle comparisons.

Per-particle error norm (the per-coordinate relative error is undefined at
zero crossings): coordinates are scaled by the bucket half-length z_b = C/(2h)
and half-height dp_b, and
    e = |(dz/z_b, ddp/dp_b)| / |(z/z_b, dp/dp_b)|.
Particles whose initial Hamiltonian lies within 1% of the separatrix value are
"near-separatrix": there the map is chaotic and last-bit differences grow, so
they get a looser fixed bound and are counted separately.

Fixed bounds after 1e3 turns: e <= 1e-12 away from the separatrix, 1e-10
near it (longer runs: in proportion to the turns). Two correct FP64 evaluations of the map round differently (the
kernels' sine polynomial, fused multiply-adds and phase reduction against libm
sin and separate roundings), so they differ by about one unit in the last
place per turn, and a particle's own orbit amplifies that by the factor
measured here (the oracle's response to a relative perturbation of 1e-13 of
its initial z or delta). A particle over its fixed bound is held instead to 8
ulp per turn times that factor, but never to more than the ceiling
amplified_cap(turns) (1e-10 at 1e3 turns, 1e-9 at 1e4), and at most
MAX_OVER_FIXED of the bunch may be over the fixed core bound at all.
"""
import math

import numpy as np

import oracle

FIXED_CORE = 1e-12
FIXED_SEP = 1e-10
MAX_OVER_FIXED = 0.005


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


def amplification(track, z0, dp0, turns, ring_like, integ, eps=1e-13, err=None, **kw):
    """Oracle response, in the bucket norm, to perturbing z0 or dp0 by eps
    (relative), divided by eps. `track` is the oracle function (track,
    track_rf2, ...) called as track(z, dp, turns, ring_like, integ, **kw);
    `err(z, dp, z_ref, dp_ref)` is the norm (default: bucket_error on
    ring_like)."""
    if err is None:
        def err(a, b, c, d):
            return bucket_error(a, b, c, d, ring_like)
    z0 = np.asarray(z0, dtype=np.float64)
    dp0 = np.asarray(dp0, dtype=np.float64)
    za, da = track(z0, dp0, turns, ring_like, integ, **kw)[:2]
    zb, db = track(z0 * (1 + eps), dp0, turns, ring_like, integ, **kw)[:2]
    zc, dc = track(z0, dp0 * (1 + eps), turns, ring_like, integ, **kw)[:2]
    return np.maximum(err(zb, db, za, da), err(zc, dc, za, da)) / eps


def rounding_tolerance(amp, turns):
    """8 ulp (2^-53 each) per turn, amplified by the orbit (at least 1)."""
    return 8 * 2.0 ** -53 * turns * np.maximum(amp, 1.0)


def _per_kturn(turns):
    return max(1.0, turns / 1000.0)


def fixed_bounds(turns):
    """(core, near-separatrix) fixed bounds after `turns` turns."""
    return FIXED_CORE * _per_kturn(turns), FIXED_SEP * _per_kturn(turns)


def amplified_cap(turns):
    """Ceiling of every per-particle bound: 1e-10 up to 1e3 turns, then
    growing in proportion to the turns (1e-9 at 1e4)."""
    return 1e-10 * _per_kturn(turns)


def check_particles(e, near, turns, amp_of, label="", max_over=MAX_OVER_FIXED):
    """Assert the per-particle bounds above. `e`: errors in the bucket norm;
    `near`: near-separatrix mask; `amp_of(mask)`: the amplification of the
    particles selected by mask (called only for particles over their fixed
    bound). Returns (tol, number over the fixed core bound)."""
    e = np.asarray(e)
    assert np.all(np.isfinite(e)), label
    core, sep = fixed_bounds(turns)
    tol = np.where(near, sep, core)
    over = e > tol
    if np.any(over):
        amp = amp_of(over)
        tol[over] = np.minimum(np.maximum(tol[over], rounding_tolerance(amp, turns)),
                               amplified_cap(turns))
    worst = int(np.argmax(e / tol))
    n_over = int(np.count_nonzero(e > core))
    allowed = int(math.floor(max_over * e.size))
    print("%s: e p50 %.2e max %.2e; %d of %d over %.0e (allowed %d), %d near the separatrix"
          % (label, np.median(e), e.max(), n_over, e.size, core, allowed,
             int(np.count_nonzero(near))))
    assert np.all(e <= tol), (label, e[worst], tol[worst], bool(near[worst]))
    assert n_over <= allowed, (label, n_over, allowed)
    return tol, n_over
