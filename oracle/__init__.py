"""Independent FP64 CPU oracle for longitudinal macro-particle tracking.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product package. It shares no code
with the HIP path; the tracking arithmetic lives in ``ltrk_oracle.c`` (plain C,
FP64, ``-O2 -ffp-contract=off``), this module only marshals NumPy arrays.

The method (paper, section 1.1.2): each macro-particle's (z, delta) is
integrated turn by turn by Euler-Cromer, leap-frog, fourth-order Ruth or
Runge-Kutta; particles are independent (section 2.3). The single-harmonic
map and its constants are documented in ``ltrk_oracle.c``.

Every function here is pinned by tests against physics closed forms,
textbook formulas, library routines or high-precision brute force; none is
"parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

INTEGRATORS = {"euler_cromer": 0, "leapfrog": 1, "ruth4": 2, "rk4": 3}

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ltrk_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "liboracle.so")
_lock = threading.Lock()
_lib = None

RING_FIELDS = ("circumference_m", "harmonic", "voltage_V", "p0c_eV", "mass_eV",
               "gamma_t", "charge_e")


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc into ``oracle/_build/liboracle.so``."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
            "-shared", "-fPIC", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            d = ctypes.c_double
            p = ctypes.POINTER(ctypes.c_double)
            lib.oracle_derive.argtypes = [d] * 7 + [p]
            lib.oracle_derive.restype = ctypes.c_int
            lib.oracle_track.argtypes = [p, p, ctypes.c_int64, ctypes.c_int64] + [d] * 7 + \
                [ctypes.c_int, ctypes.c_int, p, ctypes.c_int]
            lib.oracle_track.restype = ctypes.c_int
            lib.oracle_moments.argtypes = [p, p, ctypes.c_int64, p]
            lib.oracle_moments.restype = None
            lib.oracle_track_rf2.argtypes = [p, p, ctypes.c_int64, ctypes.c_int64] + [d] * 13 + \
                [ctypes.c_int, ctypes.c_int, p, ctypes.c_int]
            lib.oracle_track_rf2.restype = ctypes.c_int
            lib.oracle_track_program.argtypes = [p, p, ctypes.c_int64, ctypes.c_int64] + \
                [d] * 9 + [p] * 5 + [ctypes.c_int, ctypes.c_int, p, ctypes.c_int]
            lib.oracle_track_program.restype = ctypes.c_int
            lib.oracle_track_6d.argtypes = [p] * 6 + [ctypes.c_int64, ctypes.c_int64] + \
                [d] * 13 + [p, ctypes.c_int, p, ctypes.c_int]
            lib.oracle_track_6d.restype = ctypes.c_int
            lib.oracle_track_wake.argtypes = [p, p, ctypes.c_int64, ctypes.c_int64] + [d] * 13 + \
                [p, ctypes.c_int, p, ctypes.c_int]
            lib.oracle_track_wake.restype = ctypes.c_int
            lib.oracle_max_threads.argtypes = []
            lib.oracle_max_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def _ring_values(ring) -> list:
    if isinstance(ring, dict):
        return [float(ring[k]) for k in RING_FIELDS]
    return [float(getattr(ring, k)) for k in RING_FIELDS]


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


DERIVED_FIELDS = ("gamma", "beta", "eta", "A", "k", "D", "omega", "Qs", "Q_lf",
                  "bucket_half_length", "bucket_height", "H_sep")


def derive(ring) -> dict:
    """Derived ring constants (FP64), keyed by ``DERIVED_FIELDS``."""
    out = np.zeros(12)
    rc = _load().oracle_derive(*_ring_values(ring), _ptr(out))
    if rc != 0:
        raise ValueError("invalid ring parameters")
    return dict(zip(DERIVED_FIELDS, out.tolist()))


def track(z, dp, turns: int, ring, integrator="leapfrog", substeps: int = 1,
          with_moments: bool = True, threads: int = 0):
    """Track copies of (z, dp) for ``turns`` turns.

    Returns ``(z, dp, moments)`` with ``moments`` of shape ``[turns, 5]``
    (mean_z, rms_z, mean_dp, rms_dp, emit_rms after each turn) or None.
    ``substeps`` > 1 splits each turn into that many steps of length
    1/substeps (used only by the convergence-order check).
    """
    integ = INTEGRATORS[integrator] if isinstance(integrator, str) else int(integrator)
    z = np.array(z, dtype=np.float64, copy=True, order="C").ravel()
    dp = np.array(dp, dtype=np.float64, copy=True, order="C").ravel()
    if z.shape != dp.shape:
        raise ValueError("z and dp differ in length")
    mom = np.empty((max(turns, 0), 5)) if with_moments else None
    rc = _load().oracle_track(_ptr(z), _ptr(dp), z.size, int(turns), *_ring_values(ring),
                              integ, int(substeps), _ptr(mom) if mom is not None else None,
                              int(threads))
    if rc != 0:
        raise ValueError("invalid arguments to oracle_track")
    return z, dp, mom


def moments(z, dp) -> np.ndarray:
    """Two-pass compensated population moments of one bunch (5 values)."""
    z = np.ascontiguousarray(z, dtype=np.float64).ravel()
    dp = np.ascontiguousarray(dp, dtype=np.float64).ravel()
    out = np.zeros(5)
    _load().oracle_moments(_ptr(z), _ptr(dp), z.size, _ptr(out))
    return out


def hamiltonian(z, dp, ring) -> np.ndarray:
    """Smooth single-harmonic Hamiltonian with one turn as the time unit,
    H = -(D/2) dp^2 + (A/k)(cos(k z) - 1); H_sep = -2A/k on the separatrix."""
    c = derive(ring)
    z = np.asarray(z, dtype=np.float64)
    dp = np.asarray(dp, dtype=np.float64)
    return -0.5 * c["D"] * dp * dp + (c["A"] / c["k"]) * (np.cos(c["k"] * z) - 1.0)


RF2_FIELDS = ("phi1_rad", "harmonic2", "voltage2_V", "phi2_rad", "eta1", "eta2")


def _rf2_values(rf2) -> list:
    get = (lambda k: rf2[k]) if isinstance(rf2, dict) else (lambda k: getattr(rf2, k))
    return [float(get(k)) for k in RF2_FIELDS]


def track_rf2(z, dp, turns: int, rf2, integrator="leapfrog", substeps: int = 1,
              with_moments: bool = True, threads: int = 0):
    """Track copies of (z, dp) through the extended map (double-harmonic RF
    with phase offsets, slip factor eta0 + eta1 dp + eta2 dp^2). `rf2` holds
    the ring fields plus phi1_rad, harmonic2, voltage2_V, phi2_rad, eta1, eta2."""
    integ = INTEGRATORS[integrator] if isinstance(integrator, str) else int(integrator)
    z = np.array(z, dtype=np.float64, copy=True, order="C").ravel()
    dp = np.array(dp, dtype=np.float64, copy=True, order="C").ravel()
    if z.shape != dp.shape:
        raise ValueError("z and dp differ in length")
    mom = np.empty((max(turns, 0), 5)) if with_moments else None
    rc = _load().oracle_track_rf2(_ptr(z), _ptr(dp), z.size, int(turns), *_ring_values(rf2),
                                  *_rf2_values(rf2), integ, int(substeps),
                                  _ptr(mom) if mom is not None else None, int(threads))
    if rc != 0:
        raise ValueError("invalid arguments to oracle_track_rf2")
    return z, dp, mom


def hamiltonian_rf2(z, dp, rf2) -> np.ndarray:
    """H = -C (eta0 dp^2/2 + eta1 dp^3/3 + eta2 dp^4/4) + sum_i (A_i/k_i) cos(k_i z + phi_i),
    whose flow is the extended map's vector field."""
    c = derive(rf2)
    get = (lambda k: rf2[k]) if isinstance(rf2, dict) else (lambda k: getattr(rf2, k))
    C = float(get("circumference_m"))
    eta1, eta2 = float(get("eta1")), float(get("eta2"))
    A2 = float(get("charge_e")) * float(get("voltage2_V")) / (c["beta"] * float(get("p0c_eV")))
    k2 = 2.0 * np.pi * float(get("harmonic2")) / C
    z = np.asarray(z, dtype=np.float64)
    dp = np.asarray(dp, dtype=np.float64)
    h = -C * (c["eta"] * dp ** 2 / 2 + eta1 * dp ** 3 / 3 + eta2 * dp ** 4 / 4)
    h = h + (c["A"] / c["k"]) * np.cos(c["k"] * z + float(get("phi1_rad")))
    if A2 != 0.0:
        h = h + (A2 / k2) * np.cos(k2 * z + float(get("phi2_rad")))
    return h


PROGRAM_FIELDS = ("voltage_V", "phi1_rad", "voltage2_V", "phi2_rad", "p0c_eV")


def track_program(z, dp, turns: int, rf2, program, integrator="leapfrog", substeps: int = 1,
                  with_moments: bool = True, threads: int = 0):
    """Track copies of (z, dp) through the extended map with per-turn settings.

    `rf2` gives the fixed parameters (ring fields, harmonic2, eta1, eta2; its
    p0c_eV is the momentum before the first turn; its voltages and phases are
    not used). `program` maps each of PROGRAM_FIELDS to an array with one
    entry per turn: the RF voltages and phases of turn t and the reference
    momentum after turn t.
    """
    integ = INTEGRATORS[integrator] if isinstance(integrator, str) else int(integrator)
    z = np.array(z, dtype=np.float64, copy=True, order="C").ravel()
    dp = np.array(dp, dtype=np.float64, copy=True, order="C").ravel()
    if z.shape != dp.shape:
        raise ValueError("z and dp differ in length")
    cols = []
    for k in PROGRAM_FIELDS:
        a = np.ascontiguousarray(program[k], dtype=np.float64).ravel()
        if a.size < turns:
            raise ValueError("programme field %s has %d < %d entries" % (k, a.size, turns))
        cols.append(a)
    get = (lambda k: rf2[k]) if isinstance(rf2, dict) else (lambda k: getattr(rf2, k))
    fixed = [float(get(k)) for k in ("circumference_m", "harmonic", "p0c_eV", "mass_eV",
                                     "gamma_t", "charge_e", "harmonic2", "eta1", "eta2")]
    mom = np.empty((max(turns, 0), 5)) if with_moments else None
    rc = _load().oracle_track_program(_ptr(z), _ptr(dp), z.size, int(turns), *fixed,
                                      *[_ptr(a) for a in cols], integ, int(substeps),
                                      _ptr(mom) if mom is not None else None, int(threads))
    if rc != 0:
        raise ValueError("invalid arguments to oracle_track_program")
    return z, dp, mom


TWISS_FIELDS = ("Qx", "Qpx", "alpha_x", "beta_x", "Qy", "Qpy", "alpha_y", "beta_y")


def track_6d(state, turns: int, rf2, twiss, integrator="leapfrog", with_moments: bool = True,
             threads: int = 0):
    """Track copies of a 6-D state through the transverse linear one-turn map
    with chromatic phase advance, then the extended longitudinal map, per
    turn. `state` maps z, dp, x, xp, y, yp to arrays; `twiss` maps
    TWISS_FIELDS to numbers (tunes, chromaticities Q' per unit dp, alpha,
    beta in metres). Returns (state dict, moments [turns, 15] or None): the
    five moments of (z, dp), (x, xp) and (y, yp) after each turn."""
    integ = INTEGRATORS[integrator] if isinstance(integrator, str) else int(integrator)
    keys = ("z", "dp", "x", "xp", "y", "yp")
    arrs = [np.array(state[k], dtype=np.float64, copy=True, order="C").ravel() for k in keys]
    if len({a.size for a in arrs}) != 1:
        raise ValueError("state arrays differ in length")
    tw = np.array([float(twiss[k]) for k in TWISS_FIELDS])
    mom = np.empty((max(turns, 0), 15)) if with_moments else None
    rc = _load().oracle_track_6d(*[_ptr(a) for a in arrs], arrs[0].size, int(turns),
                                 *_ring_values(rf2), *_rf2_values(rf2), _ptr(tw), integ,
                                 _ptr(mom) if mom is not None else None, int(threads))
    if rc != 0:
        raise ValueError("invalid arguments to oracle_track_6d")
    return dict(zip(keys, arrs)), mom


def courant_snyder(u, up, alpha, beta) -> np.ndarray:
    """Courant-Snyder invariant gamma u^2 + 2 alpha u u' + beta u'^2."""
    u = np.asarray(u, dtype=np.float64)
    up = np.asarray(up, dtype=np.float64)
    return (1.0 + alpha * alpha) / beta * u * u + 2.0 * alpha * u * up + beta * up * up


WAKE_FIELDS = ("model", "R_s", "f_r", "Q", "intensity", "n_slices", "z_lo", "z_hi")
E_CHARGE = 1.602176634e-19
C_LIGHT = 299792458.0


def track_wake(z, dp, turns: int, rf2, wake, integrator="leapfrog", with_moments: bool = True,
               threads: int = 0):
    """Track copies of (z, dp) through the extended map with a longitudinal
    wake kick after every turn. `wake` maps WAKE_FIELDS to numbers: model (0
    resonator, 1 constant wake R_s V/C), R_s (ohm), f_r (Hz), Q, intensity
    (particles in the bunch), n_slices, z_lo, z_hi (m)."""
    integ = INTEGRATORS[integrator] if isinstance(integrator, str) else int(integrator)
    z = np.array(z, dtype=np.float64, copy=True, order="C").ravel()
    dp = np.array(dp, dtype=np.float64, copy=True, order="C").ravel()
    if z.shape != dp.shape:
        raise ValueError("z and dp differ in length")
    wk = np.array([float(wake.get(k, 0.0)) for k in WAKE_FIELDS])
    mom = np.empty((max(turns, 0), 5)) if with_moments else None
    rc = _load().oracle_track_wake(_ptr(z), _ptr(dp), z.size, int(turns), *_ring_values(rf2),
                                   *_rf2_values(rf2), _ptr(wk), integ,
                                   _ptr(mom) if mom is not None else None, int(threads))
    if rc != 0:
        raise ValueError("invalid arguments to oracle_track_wake")
    return z, dp, mom


def resonator_wake(tau, R_s, f_r, Q):
    """Resonator wake function W(tau) in V/C (tau in s; W(0) is half the limit)."""
    tau = np.asarray(tau, dtype=np.float64)
    w_r = 2 * np.pi * f_r
    a = w_r / (2 * Q)
    wb = np.sqrt(w_r * w_r - a * a)
    w = 2 * a * R_s * np.exp(-a * tau) * (np.cos(wb * tau) - a / wb * np.sin(wb * tau))
    return np.where(tau == 0.0, a * R_s, np.where(tau > 0.0, w, 0.0))


def max_threads() -> int:
    """OpenMP threads the C oracle uses by default on this host."""
    return int(_load().oracle_max_threads())
