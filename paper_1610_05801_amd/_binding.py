"""ctypes binding of libltrk (include/ltrk.h): argument marshalling only.

Every computation runs in the HIP library; this module checks tensor
dtypes/devices/sizes, passes raw device pointers and the stream handle, and
turns negative return codes into exceptions. PyTorch provides the device
memory and the streams. There is no CPU fallback: if libltrk.so is missing the
import fails.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# LTRK_LIBRARY may name another build of this same library to load instead of
# the in-tree one (a development and testing override, e.g. to time a kernel
# change against the committed build in one process); unset, the in-tree
# build is the one that runs.
LIB_PATH = os.environ.get("LTRK_LIBRARY") or os.path.join(HERE, "libltrk.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libltrk.so is not built: run `python -m paper_1610_05801_amd.build` "
                      "(or __graft_entry__.build())")

# PyTorch ships its own HIP runtime (same SONAME as the system one). Loading
# torch first makes libltrk bind to that already-loaded runtime, so device
# pointers and streams from torch are valid inside the library; loading
# libltrk first would pull in a second HIP runtime that sees no device.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)


def _hip_runtimes():
    try:
        with open("/proc/self/maps") as f:
            return sorted({line.split()[-1] for line in f if "libamdhip64" in line})
    except OSError:
        return []


if len(_hip_runtimes()) > 1:
    raise ImportError("two HIP runtimes are loaded in this process (%s); import torch before "
                      "anything that loads libamdhip64" % ", ".join(_hip_runtimes()))

LTRK_OK = 0
LTRK_EINVAL = -1
LTRK_ENOMEM = -2
LTRK_EDEVICE = -3
LTRK_EAGAIN = -4
LTRK_EUNSUPPORTED = -5

INTEGRATORS = {"euler_cromer": 0, "leapfrog": 1, "ruth4": 2, "rk4": 3}
DTYPES = {"f64": 0, "f32c": 1}

c_d = ctypes.c_double
c_i64 = ctypes.c_int64
c_i32 = ctypes.c_int32
c_vp = ctypes.c_void_p


class Ring(ctypes.Structure):
    _fields_ = [("circumference_m", c_d), ("harmonic", c_d), ("voltage_V", c_d),
                ("p0c_eV", c_d), ("mass_eV", c_d), ("gamma_t", c_d), ("charge_e", c_d)]

    @classmethod
    def of(cls, r) -> "Ring":
        if isinstance(r, Ring):
            return r
        if isinstance(r, dict):
            return cls(**{k: float(r[k]) for k, _ in cls._fields_})
        return cls(**{k: float(getattr(r, k)) for k, _ in cls._fields_})


class Rf2(ctypes.Structure):
    _fields_ = [("ring", Ring), ("phi1_rad", c_d), ("harmonic2", c_d), ("voltage2_V", c_d),
                ("phi2_rad", c_d), ("eta1", c_d), ("eta2", c_d)]

    @classmethod
    def of(cls, r) -> "Rf2":
        if isinstance(r, Rf2):
            return r
        get = (lambda k: r[k]) if isinstance(r, dict) else (lambda k: getattr(r, k))
        return cls(Ring.of(r), *[float(get(k)) for k in ("phi1_rad", "harmonic2", "voltage2_V",
                                                        "phi2_rad", "eta1", "eta2")])


class RfTurn(ctypes.Structure):
    _fields_ = [("voltage_V", c_d), ("phi1_rad", c_d), ("voltage2_V", c_d), ("phi2_rad", c_d),
                ("p0c_eV", c_d)]

    FIELDS = ("voltage_V", "phi1_rad", "voltage2_V", "phi2_rad", "p0c_eV")

    @classmethod
    def array(cls, program, turns: int):
        """A ctypes array of `turns` entries from a dict of per-turn arrays
        (keys FIELDS) or a sequence of RfTurn."""
        if isinstance(program, ctypes.Array) and len(program) >= turns:
            return program
        arr = (cls * max(int(turns), 1))()
        if isinstance(program, dict):
            import numpy as np
            cols = [np.ascontiguousarray(program[k], dtype=np.float64).ravel() for k in cls.FIELDS]
            for c in cols:
                if c.size < turns:
                    raise ValueError("programme has %d < %d entries" % (c.size, turns))
            flat = np.stack([c[:turns] for c in cols], axis=1)
            ctypes.memmove(arr, flat.ctypes.data, flat.nbytes)
        else:
            for i in range(int(turns)):
                arr[i] = program[i]
        return arr


class Twiss(ctypes.Structure):
    _fields_ = [("q_x", c_d), ("qp_x", c_d), ("alpha_x", c_d), ("beta_x", c_d),
                ("q_y", c_d), ("qp_y", c_d), ("alpha_y", c_d), ("beta_y", c_d)]

    @classmethod
    def of(cls, t) -> "Twiss":
        if isinstance(t, Twiss):
            return t
        get = (lambda k: t[k]) if isinstance(t, dict) else (lambda k: getattr(t, k))
        return cls(*[float(get(k)) for k, _ in cls._fields_])


class Wake(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("n_slices", ctypes.c_int32), ("shunt", c_d),
                ("freq_hz", c_d), ("quality", c_d), ("intensity", c_d), ("z_lo", c_d),
                ("z_hi", c_d)]
    MODELS = {"resonator": 0, "constant": 1}

    @classmethod
    def of(cls, w) -> "Wake":
        if isinstance(w, Wake):
            return w
        get = (lambda k, dflt=None: w.get(k, dflt)) if isinstance(w, dict) else \
            (lambda k, dflt=None: getattr(w, k, dflt))
        model = get("model", 0)
        model = cls.MODELS[model] if isinstance(model, str) else int(model)
        return cls(model, int(get("n_slices")), float(get("shunt")), float(get("freq_hz", 0.0)),
                   float(get("quality", 0.0)), float(get("intensity")), float(get("z_lo")),
                   float(get("z_hi")))


class Moments(ctypes.Structure):
    _fields_ = [("mean_z", c_d), ("rms_z", c_d), ("mean_dp", c_d), ("rms_dp", c_d),
                ("emit_rms", c_d)]


class Derived(ctypes.Structure):
    _fields_ = [("gamma", c_d), ("beta", c_d), ("eta", c_d), ("kick_amplitude", c_d),
                ("wavenumber", c_d), ("slip_length", c_d), ("omega_s", c_d), ("q_s", c_d),
                ("q_leapfrog", c_d), ("bucket_half_length", c_d), ("bucket_height", c_d),
                ("h_separatrix", c_d)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Bunch(ctypes.Structure):
    _fields_ = [("z", c_vp), ("dp", c_vp), ("z_comp", c_vp), ("dp_comp", c_vp), ("n", c_i64),
                ("ring", Ring), ("moments", c_vp)]


class Plan(ctypes.Structure):
    _fields_ = [("turns_per_launch", c_i32), ("block", c_i32), ("ppl", c_i32),
                ("use_graph", c_i32)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class Timing(ctypes.Structure):
    _fields_ = [("track_launches", c_i64), ("track_ms", c_d), ("finalize_launches", c_i64),
                ("finalize_ms", c_d)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Job(ctypes.Structure):
    _fields_ = [("n", c_i64), ("turns", c_i64), ("ring", Ring), ("integrator", c_i32),
                ("dtype", c_i32), ("z0", c_vp), ("dp0", c_vp), ("z0_comp", c_vp),
                ("dp0_comp", c_vp)]


class EngineStats(ctypes.Structure):
    _fields_ = [("active_slots", c_i32), ("max_slots", c_i32), ("arena_bytes", c_i64),
                ("arena_free_bytes", c_i64), ("largest_free_block", c_i64), ("steps", c_i64),
                ("particle_turns", c_i64)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


P = ctypes.POINTER
_SIGS = {
    "ltrk_abi_version": ([], ctypes.c_int),
    "ltrk_derive": ([P(Ring), P(Derived)], ctypes.c_int),
    "ltrk_track_f64": ([c_vp, c_vp, c_i64, c_i64, P(Ring), ctypes.c_int, c_vp, c_vp], ctypes.c_int),
    "ltrk_track_f64_noalloc": ([c_vp, c_vp, c_i64, c_i64, P(Ring), ctypes.c_int, c_vp, c_vp],
                               ctypes.c_int),
    "ltrk_track_f32c": ([c_vp, c_vp, c_vp, c_vp, c_i64, c_i64, P(Ring), ctypes.c_int, c_vp, c_vp],
                        ctypes.c_int),
    "ltrk_track_rf2_f64": ([c_vp, c_vp, c_i64, c_i64, P(Rf2), ctypes.c_int, c_vp, c_vp],
                           ctypes.c_int),
    "ltrk_track_program_f64": ([c_vp, c_vp, c_i64, c_i64, P(Rf2), P(RfTurn), ctypes.c_int, c_vp,
                                c_vp], ctypes.c_int),
    "ltrk_track_6d_f64": ([c_vp] * 6 + [c_i64, c_i64, P(Rf2), P(Twiss), ctypes.c_int, c_vp, c_vp],
                          ctypes.c_int),
    "ltrk_track_wake_f64": ([c_vp, c_vp, c_i64, c_i64, P(Rf2), P(Wake), ctypes.c_int, c_vp, c_vp],
                            ctypes.c_int),
    "ltrk_moments_f64": ([c_vp, c_vp, c_i64, c_vp, c_vp], ctypes.c_int),
    "ltrk_moments_f32c": ([c_vp, c_vp, c_vp, c_vp, c_i64, c_vp, c_vp], ctypes.c_int),
    "ltrk_track_batched": ([P(Bunch), ctypes.c_int, c_i64, ctypes.c_int, ctypes.c_int, c_vp],
                           ctypes.c_int),
    "ltrk_set_plan": ([P(Plan)], ctypes.c_int),
    "ltrk_get_plan": ([ctypes.c_int, ctypes.c_int, c_i64, P(Plan)], ctypes.c_int),
    "ltrk_autotune": ([ctypes.c_int, ctypes.c_int, c_i64, c_vp, P(Plan)], ctypes.c_int),
    "ltrk_get_plan_batched": ([ctypes.c_int, ctypes.c_int, c_i64, P(Plan)], ctypes.c_int),
    "ltrk_autotune_batched": ([P(Bunch), ctypes.c_int, ctypes.c_int, ctypes.c_int, c_vp, P(Plan)],
                              ctypes.c_int),
    "ltrk_tune_cache_save": ([ctypes.c_char_p], ctypes.c_int),
    "ltrk_tune_cache_load": ([ctypes.c_char_p], ctypes.c_int),
    "ltrk_timing_enable": ([ctypes.c_int], ctypes.c_int),
    "ltrk_timing_take": ([P(Timing)], ctypes.c_int),
    "ltrk_engine_create": ([ctypes.c_int, c_i64, ctypes.c_int, P(c_vp)], ctypes.c_int),
    "ltrk_engine_footprint": ([P(Job), P(c_i64)], ctypes.c_int),
    "ltrk_engine_admit": ([c_vp, P(Job), P(ctypes.c_int)], ctypes.c_int),
    "ltrk_engine_step": ([c_vp, ctypes.c_int, c_vp, P(c_i64)], ctypes.c_int),
    "ltrk_engine_poll": ([c_vp, ctypes.c_int, P(ctypes.c_int)], ctypes.c_int),
    "ltrk_engine_result": ([c_vp, ctypes.c_int, c_vp, c_vp, c_vp, c_vp, c_vp], ctypes.c_int),
    "ltrk_engine_retire": ([c_vp, ctypes.c_int], ctypes.c_int),
    "ltrk_engine_cancel": ([c_vp, ctypes.c_int], ctypes.c_int),
    "ltrk_engine_stats_get": ([c_vp, P(EngineStats)], ctypes.c_int),
    "ltrk_engine_destroy": ([c_vp], ctypes.c_int),
    "ltrk_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "ltrk_last_error": ([ctypes.c_char_p, ctypes.c_size_t], ctypes.c_int),
    "ltrk_shutdown": ([], ctypes.c_int),
}
for _name, (_args, _res) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res

EXPORTED = tuple(_SIGS)


class LtrkError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("%s (%d): %s" % (_lib.ltrk_strerror(code).decode(), code, message))
        self.code = code


def _check(rc: int):
    if rc != LTRK_OK:
        buf = ctypes.create_string_buffer(512)
        _lib.ltrk_last_error(buf, len(buf))
        raise LtrkError(rc, buf.value.decode(errors="replace"))


def _integ(i) -> int:
    return INTEGRATORS[i] if isinstance(i, str) else int(i)


def _dtype(d) -> int:
    return DTYPES[d] if isinstance(d, str) else int(d)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_vp(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _dev_ptr(t, dtype, n=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if t.device.type != "cuda":
        raise ValueError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must be %s" % (name, dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if n is not None and t.numel() != n:
        raise ValueError("%s must hold %d elements" % (name, n))
    return c_vp(t.data_ptr())


def _mom_ptr(moments, rows):
    import torch
    if moments is None:
        return c_vp(None)
    if moments.dtype != torch.float64 or moments.device.type != "cuda" or \
            not moments.is_contiguous() or moments.numel() != rows * 5:
        raise ValueError("moments must be a contiguous float64 device tensor of shape [turns, 5]")
    return c_vp(moments.data_ptr())


# ---- entry points (same names as the C ABI) ----

def ltrk_abi_version() -> int:
    return int(_lib.ltrk_abi_version())


def ltrk_derive(ring) -> dict:
    out = Derived()
    _check(_lib.ltrk_derive(ctypes.byref(Ring.of(ring)), ctypes.byref(out)))
    return out.as_dict()


def ltrk_track_f64(z, dp, turns: int, ring, integrator="leapfrog", moments=None, stream=None):
    """Track float64 device tensors z, dp in place; moments: [turns, 5] float64 or None."""
    import torch
    n = z.numel()
    _check(_lib.ltrk_track_f64(_dev_ptr(z, torch.float64, None, "z"),
                               _dev_ptr(dp, torch.float64, n, "dp"), n, int(turns),
                               ctypes.byref(Ring.of(ring)), _integ(integrator),
                               _mom_ptr(moments, int(turns)), _stream(stream)))


def ltrk_track_f64_noalloc(z, dp, turns: int, ring, integrator="leapfrog", moments=None,
                           stream=None):
    """ltrk_track_f64 without any allocation (moment partials in the library's
    fixed per-device array); same arguments and results."""
    import torch
    n = z.numel()
    _check(_lib.ltrk_track_f64_noalloc(_dev_ptr(z, torch.float64, None, "z"),
                                       _dev_ptr(dp, torch.float64, n, "dp"), n, int(turns),
                                       ctypes.byref(Ring.of(ring)), _integ(integrator),
                                       _mom_ptr(moments, int(turns)), _stream(stream)))


def ltrk_track_f32c(z, dp, z_comp, dp_comp, turns: int, ring, integrator="leapfrog",
                    moments=None, stream=None):
    """Track the FP32 + Kahan state (four float32 device tensors) in place."""
    import torch
    n = z.numel()
    f = torch.float32
    _check(_lib.ltrk_track_f32c(_dev_ptr(z, f, None, "z"), _dev_ptr(dp, f, n, "dp"),
                                _dev_ptr(z_comp, f, n, "z_comp"), _dev_ptr(dp_comp, f, n, "dp_comp"),
                                n, int(turns), ctypes.byref(Ring.of(ring)), _integ(integrator),
                                _mom_ptr(moments, int(turns)), _stream(stream)))


def ltrk_track_rf2_f64(z, dp, turns: int, rf2, integrator="leapfrog", moments=None,
                       stream=None):
    """Track through the extended map (double-harmonic RF, phase offsets, slip
    factor expanded in dp). rf2: ring fields plus phi1_rad, harmonic2,
    voltage2_V, phi2_rad, eta1, eta2."""
    import torch
    n = z.numel()
    _check(_lib.ltrk_track_rf2_f64(_dev_ptr(z, torch.float64, None, "z"),
                                   _dev_ptr(dp, torch.float64, n, "dp"), n, int(turns),
                                   ctypes.byref(Rf2.of(rf2)), _integ(integrator),
                                   _mom_ptr(moments, int(turns)), _stream(stream)))


def ltrk_track_program_f64(z, dp, turns: int, rf2, program, integrator="leapfrog",
                           moments=None, stream=None):
    """Track through the extended map with per-turn RF settings and reference
    momentum. rf2: fixed parameters (its p0c_eV is the momentum before the
    first turn); program: dict of per-turn arrays (RfTurn.FIELDS, entry t for
    turn t, p0c_eV the momentum after it) or an RfTurn array."""
    import torch
    n = z.numel()
    prog = RfTurn.array(program, int(turns))
    _check(_lib.ltrk_track_program_f64(_dev_ptr(z, torch.float64, None, "z"),
                                       _dev_ptr(dp, torch.float64, n, "dp"), n, int(turns),
                                       ctypes.byref(Rf2.of(rf2)), prog, _integ(integrator),
                                       _mom_ptr(moments, int(turns)), _stream(stream)))


def ltrk_track_6d_f64(z, dp, x, xp, y, yp, turns: int, rf2, twiss, integrator="leapfrog",
                      moments=None, stream=None):
    """Track a 6-D state (transverse Twiss rotation with chromatic phase, then
    the extended longitudinal step, per turn). twiss: q_x, qp_x, alpha_x,
    beta_x, q_y, qp_y, alpha_y, beta_y. moments: [turns, 3, 5] float64 or
    None (rows of (z, dp), (x, xp), (y, yp) after each turn)."""
    import torch
    n = z.numel()
    f = torch.float64
    mom = _mom_ptr(moments, 3 * int(turns))
    _check(_lib.ltrk_track_6d_f64(_dev_ptr(z, f, None, "z"), _dev_ptr(dp, f, n, "dp"),
                                  _dev_ptr(x, f, n, "x"), _dev_ptr(xp, f, n, "xp"),
                                  _dev_ptr(y, f, n, "y"), _dev_ptr(yp, f, n, "yp"), n,
                                  int(turns), ctypes.byref(Rf2.of(rf2)),
                                  ctypes.byref(Twiss.of(twiss)), _integ(integrator), mom,
                                  _stream(stream)))


def ltrk_track_wake_f64(z, dp, turns: int, rf2, wake, integrator="leapfrog", moments=None,
                        stream=None):
    """Track through the extended map with a longitudinal wake kick after
    every turn. wake: model ("resonator" or "constant"), n_slices, shunt,
    freq_hz, quality, intensity, z_lo, z_hi."""
    import torch
    n = z.numel()
    _check(_lib.ltrk_track_wake_f64(_dev_ptr(z, torch.float64, None, "z"),
                                    _dev_ptr(dp, torch.float64, n, "dp"), n, int(turns),
                                    ctypes.byref(Rf2.of(rf2)), ctypes.byref(Wake.of(wake)),
                                    _integ(integrator), _mom_ptr(moments, int(turns)),
                                    _stream(stream)))


def ltrk_moments_f64(z, dp, out, stream=None):
    import torch
    n = z.numel()
    _check(_lib.ltrk_moments_f64(_dev_ptr(z, torch.float64, None, "z"),
                                 _dev_ptr(dp, torch.float64, n, "dp"), n, _mom_ptr(out, 1),
                                 _stream(stream)))


def ltrk_moments_f32c(z, dp, z_comp, dp_comp, out, stream=None):
    import torch
    n = z.numel()
    f = torch.float32
    _check(_lib.ltrk_moments_f32c(_dev_ptr(z, f, None, "z"), _dev_ptr(dp, f, n, "dp"),
                                  _dev_ptr(z_comp, f, n, "z_comp"),
                                  _dev_ptr(dp_comp, f, n, "dp_comp"), n, _mom_ptr(out, 1),
                                  _stream(stream)))


def ltrk_track_batched(bunches, turns: int, integrator="leapfrog", dtype="f64", stream=None):
    """bunches: list of dicts with keys z, dp, (z_comp, dp_comp for f32c), ring, moments."""
    import torch
    dt = _dtype(dtype)
    tdt = torch.float64 if dt == 0 else torch.float32
    arr = (Bunch * max(len(bunches), 1))()
    for i, b in enumerate(bunches):
        n = b["z"].numel()
        arr[i].z = _dev_ptr(b["z"], tdt, None, "z")
        arr[i].dp = _dev_ptr(b["dp"], tdt, n, "dp")
        if dt == 1:
            arr[i].z_comp = _dev_ptr(b["z_comp"], tdt, n, "z_comp")
            arr[i].dp_comp = _dev_ptr(b["dp_comp"], tdt, n, "dp_comp")
        arr[i].n = n
        arr[i].ring = Ring.of(b["ring"])
        arr[i].moments = _mom_ptr(b.get("moments"), int(turns))
    _check(_lib.ltrk_track_batched(arr, len(bunches), int(turns), _integ(integrator), dt,
                                   _stream(stream)))


def ltrk_set_plan(turns_per_launch=None, block=None, ppl=None, use_graph=1):
    """Force a plan (all four values) or, with no arguments, return to automatic plans."""
    if turns_per_launch is None:
        _check(_lib.ltrk_set_plan(None))
        return
    p = Plan(int(turns_per_launch), int(block), int(ppl), int(use_graph))
    _check(_lib.ltrk_set_plan(ctypes.byref(p)))


def ltrk_get_plan(integrator="leapfrog", dtype="f64", n=1) -> dict:
    p = Plan()
    _check(_lib.ltrk_get_plan(_integ(integrator), _dtype(dtype), int(n), ctypes.byref(p)))
    return p.as_dict()


def ltrk_get_plan_batched(integrator="leapfrog", dtype="f64", total_n=1) -> dict:
    p = Plan()
    _check(_lib.ltrk_get_plan_batched(_integ(integrator), _dtype(dtype), int(total_n),
                                      ctypes.byref(p)))
    return p.as_dict()


def ltrk_autotune_batched(bunches, integrator="leapfrog", dtype="f64", stream=None) -> dict:
    """Tune the batched launch for a table like `bunches` (dicts with n or z,
    ring and optionally moments; only sizes, rings and whether moments are
    asked for are used) and cache the plan for batched calls."""
    arr = (Bunch * max(len(bunches), 1))()
    for i, b in enumerate(bunches):
        arr[i].n = int(b["n"]) if "n" in b else b["z"].numel()
        arr[i].ring = Ring.of(b["ring"])
        arr[i].moments = 1 if b.get("moments") is not None else None
    p = Plan()
    _check(_lib.ltrk_autotune_batched(arr, len(bunches), _integ(integrator), _dtype(dtype),
                                      _stream(stream), ctypes.byref(p)))
    return p.as_dict()


def ltrk_autotune(integrator="leapfrog", dtype="f64", n=1_000_000, stream=None) -> dict:
    p = Plan()
    _check(_lib.ltrk_autotune(_integ(integrator), _dtype(dtype), int(n), _stream(stream),
                              ctypes.byref(p)))
    return p.as_dict()


def ltrk_tune_cache_save(path: str):
    _check(_lib.ltrk_tune_cache_save(path.encode()))


def ltrk_tune_cache_load(path: str):
    _check(_lib.ltrk_tune_cache_load(path.encode()))


def ltrk_timing_enable(on: bool = True):
    _check(_lib.ltrk_timing_enable(1 if on else 0))


def ltrk_timing_take() -> dict:
    t = Timing()
    _check(_lib.ltrk_timing_take(ctypes.byref(t)))
    return t.as_dict()


def ltrk_last_error() -> tuple:
    buf = ctypes.create_string_buffer(512)
    code = _lib.ltrk_last_error(buf, len(buf))
    return int(code), buf.value.decode(errors="replace")


def ltrk_strerror(code: int) -> str:
    return _lib.ltrk_strerror(int(code)).decode()


def ltrk_shutdown():
    _check(_lib.ltrk_shutdown())


# ---- serving engine ----

class EngineBusy(LtrkError):
    """Admission refused for now (no slot or no arena block): retry later."""


def ltrk_engine_footprint(n: int, turns: int) -> int:
    j = Job()
    j.n, j.turns = int(n), int(turns)
    out = c_i64()
    _check(_lib.ltrk_engine_footprint(ctypes.byref(j), ctypes.byref(out)))
    return int(out.value)


class Engine:
    """Owner of an ltrk_engine handle (ltrk_engine_create ... ltrk_engine_destroy)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 64, device: int = 0):
        h = c_vp()
        _check(_lib.ltrk_engine_create(int(device), int(hbm_budget_bytes), int(max_slots),
                                       ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def admit(self, n, turns, ring, integrator, dtype, z0, dp0, z0_comp=None, dp0_comp=None):
        """Admit a job from host numpy arrays (float64 for f64, float32 for f32c).
        Returns the slot, or raises EngineBusy when it does not fit right now."""
        import numpy as np
        dt = _dtype(dtype)
        want = np.float64 if dt == 0 else np.float32
        arrs = [np.ascontiguousarray(a, dtype=want) for a in
                ((z0, dp0) if dt == 0 else (z0, dp0, z0_comp, dp0_comp))]
        for a in arrs:
            if a.size != n:
                raise ValueError("initial state arrays must hold n elements")
        j = Job()
        j.n, j.turns = int(n), int(turns)
        j.ring = Ring.of(ring)
        j.integrator, j.dtype = _integ(integrator), dt
        j.z0, j.dp0 = arrs[0].ctypes.data, arrs[1].ctypes.data
        if dt == 1:
            j.z0_comp, j.dp0_comp = arrs[2].ctypes.data, arrs[3].ctypes.data
        slot = ctypes.c_int(-1)
        rc = _lib.ltrk_engine_admit(self._h, ctypes.byref(j), ctypes.byref(slot))
        if rc == LTRK_EAGAIN:
            buf = ctypes.create_string_buffer(512)
            _lib.ltrk_last_error(buf, len(buf))
            raise EngineBusy(rc, buf.value.decode())
        _check(rc)
        self._keep[slot.value] = (int(n), int(turns), dt)
        return slot.value

    def step(self, k: int, stream=None) -> int:
        adv = c_i64(0)
        s = c_vp(None) if stream is None else _stream(stream)
        _check(_lib.ltrk_engine_step(self._h, int(k), s, ctypes.byref(adv)))
        return int(adv.value)

    def poll(self, slot: int) -> bool:
        d = ctypes.c_int(0)
        _check(_lib.ltrk_engine_poll(self._h, int(slot), ctypes.byref(d)))
        return bool(d.value)

    def result(self, slot: int):
        """(z, dp[, z_comp, dp_comp], moments[turns, 5]) as numpy arrays (host)."""
        import numpy as np
        n, turns, dt = self._keep[slot]
        t = np.float64 if dt == 0 else np.float32
        z, dp = np.empty(n, t), np.empty(n, t)
        zc = np.empty(n, t) if dt == 1 else None
        dc = np.empty(n, t) if dt == 1 else None
        mom = np.full((turns, 5), np.nan)   # rows a cancelled job never reached stay NaN
        _check(_lib.ltrk_engine_result(self._h, int(slot), z.ctypes.data, dp.ctypes.data,
                                       zc.ctypes.data if zc is not None else None,
                                       dc.ctypes.data if dc is not None else None,
                                       mom.ctypes.data))
        return (z, dp, mom) if dt == 0 else (z, dp, zc, dc, mom)

    def retire(self, slot: int):
        _check(_lib.ltrk_engine_retire(self._h, int(slot)))
        self._keep.pop(slot, None)

    def cancel(self, slot: int):
        _check(_lib.ltrk_engine_cancel(self._h, int(slot)))

    def stats(self) -> dict:
        s = EngineStats()
        _check(_lib.ltrk_engine_stats_get(self._h, ctypes.byref(s)))
        return s.as_dict()

    def close(self):
        if self._h:
            _check(_lib.ltrk_engine_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
