"""CPU-side checks of the C-ABI library: it loads, exports every entry point
that include/ltrk.h declares, and its host-only logic (constant derivation,
argument validation, error strings, plans) behaves as documented. No kernel
is launched here."""
import ctypes
import math
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ltrk.h")

ltrk = pytest.importorskip("paper_1610_05801_amd")

import oracle  # noqa: E402
from synth import SPS_RING  # noqa: E402


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(ltrk_\w+)\s*\(", text, re.M)))


def test_header_declarations_are_exported():
    names = declared_functions()
    assert len(names) >= 25
    out = subprocess.run(["nm", "-D", "--defined-only", ltrk.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (ltrk_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(ltrk.LIB_PATH)
    for n in names:
        assert getattr(lib, n) is not None


def test_binding_covers_header():
    assert set(declared_functions()) == set(ltrk.EXPORTED)


def test_abi_version():
    assert ltrk.ltrk_abi_version() == 1


def test_derive_matches_oracle():
    d = ltrk.ltrk_derive(SPS_RING)
    o = oracle.derive(SPS_RING)
    pairs = [("gamma", "gamma"), ("beta", "beta"), ("eta", "eta"), ("kick_amplitude", "A"),
             ("wavenumber", "k"), ("slip_length", "D"), ("omega_s", "omega"), ("q_s", "Qs"),
             ("q_leapfrog", "Q_lf"), ("bucket_half_length", "bucket_half_length"),
             ("bucket_height", "bucket_height"), ("h_separatrix", "H_sep")]
    for a, b in pairs:
        assert abs(d[a] - o[b]) <= 1e-14 * abs(o[b]), (a, d[a], o[b])


@pytest.mark.parametrize("seed", range(12))
def test_derive_matches_oracle_on_random_rings(seed):
    from tests._rings import random_ring
    ring = random_ring(seed)
    d = ltrk.ltrk_derive(ring)
    o = oracle.derive(ring)
    pairs = [("gamma", "gamma"), ("beta", "beta"), ("eta", "eta"), ("kick_amplitude", "A"),
             ("wavenumber", "k"), ("slip_length", "D"), ("omega_s", "omega"), ("q_s", "Qs"),
             ("q_leapfrog", "Q_lf"), ("bucket_half_length", "bucket_half_length"),
             ("bucket_height", "bucket_height"), ("h_separatrix", "H_sep")]
    for a, b in pairs:
        assert abs(d[a] - o[b]) <= 1e-13 * abs(o[b]), (seed, a, d[a], o[b])


def test_derive_unstable_ring_has_nan_tune():
    d = ltrk.ltrk_derive(dict(SPS_RING, gamma_t=40.0))
    assert d["eta"] < 0 and math.isnan(d["q_s"]) and math.isnan(d["bucket_height"])


@pytest.mark.parametrize("key,val", [("circumference_m", 0.0), ("harmonic", 0.0),
                                     ("harmonic", 4620.5), ("p0c_eV", -1.0),
                                     ("mass_eV", -1.0), ("gamma_t", 0.0),
                                     ("voltage_V", float("inf"))])
def test_invalid_ring_rejected(key, val):
    with pytest.raises(ltrk.LtrkError) as e:
        ltrk.ltrk_derive(dict(SPS_RING, **{key: val}))
    assert e.value.code == ltrk.LTRK_EINVAL


def _raw():
    return ctypes.CDLL(ltrk.LIB_PATH)


def test_track_rejects_invalid_arguments_before_any_launch():
    lib = _raw()
    r = ltrk.Ring.of(SPS_RING)
    f = lib.ltrk_track_f64
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                  ctypes.POINTER(ltrk.Ring), ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    # negative sizes, unknown scheme, NULL arrays with n > 0, host memory
    assert f(None, None, -1, 10, ctypes.byref(r), 1, None, None) == ltrk.LTRK_EINVAL
    assert f(None, None, 10, -1, ctypes.byref(r), 1, None, None) == ltrk.LTRK_EINVAL
    assert f(None, None, 10, 10, ctypes.byref(r), 9, None, None) == ltrk.LTRK_EINVAL
    assert f(None, None, 10, 10, None, 1, None, None) == ltrk.LTRK_EINVAL
    host = (ctypes.c_double * 10)()
    rc = f(host, host, 10, 10, ctypes.byref(r), 1, None, None)
    assert rc == ltrk.LTRK_EINVAL
    code, msg = ltrk.ltrk_last_error()
    assert code == ltrk.LTRK_EINVAL and "device memory" in msg
    # n = 0 or turns = 0 without moments: success, nothing enqueued
    assert f(None, None, 0, 10, ctypes.byref(r), 1, None, None) == 0
    assert f(None, None, 10, 0, ctypes.byref(r), 1, None, None) == 0


def test_batched_rejects_bad_tables():
    lib = _raw()
    f = lib.ltrk_track_batched
    f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                  ctypes.c_void_p]
    assert f(None, 3, 10, 1, 0, None) == ltrk.LTRK_EINVAL
    arr = (ltrk._binding.Bunch * 1)()
    arr[0].n = -5
    arr[0].ring = ltrk.Ring.of(SPS_RING)
    assert f(ctypes.cast(arr, ctypes.c_void_p), 1, 10, 1, 0, None) == ltrk.LTRK_EINVAL
    arr[0].n = 4
    assert f(ctypes.cast(arr, ctypes.c_void_p), 1, 10, 1, 7, None) == ltrk.LTRK_EINVAL


def test_strerror_and_plans():
    assert ltrk.ltrk_strerror(0) == "success"
    assert "invalid" in ltrk.ltrk_strerror(-1)
    p = ltrk.ltrk_get_plan("leapfrog", "f64", 1_000_000)
    assert p["ppl"] in (1, 2, 4, 8) and p["block"] in (64, 128, 256)
    ltrk.ltrk_set_plan(64, 128, 2, 0)
    assert ltrk.ltrk_get_plan("ruth4", "f32c", 10) == {"turns_per_launch": 64, "block": 128,
                                                       "ppl": 2, "use_graph": 0}
    with pytest.raises(ltrk.LtrkError):
        ltrk.ltrk_set_plan(64, 96, 2, 0)
    ltrk.ltrk_set_plan()
    assert ltrk.ltrk_get_plan("leapfrog", "f64", 1_000_000) == p


def test_tune_cache_file_roundtrip(tmp_path):
    """Loading a tuning-cache file merges its valid entries (written here for
    this host's architecture name, gfx950 or "unknown" without a GPU) and
    skips comments, malformed lines and invalid plans; saving writes the
    entries back; a missing file is an error."""
    ltrk.ltrk_set_plan()
    src = tmp_path / "in.txt"
    src.write_text("# arch integrator dtype log2n batched K block ppl graph\n"
                   "not a plan line\n"
                   "unknown 3 1 1 0 48 64 2 0\n"
                   "gfx950 3 1 1 0 48 64 2 0\n"
                   "gfx950 3 1 1 0 48 96 2 0\n")      # block 96: invalid, skipped
    ltrk.ltrk_tune_cache_load(str(src))
    assert ltrk.ltrk_get_plan("rk4", "f32c", 3) == {"turns_per_launch": 48, "block": 64,
                                                    "ppl": 2, "use_graph": 0}
    out = tmp_path / "out.txt"
    ltrk.ltrk_tune_cache_save(str(out))
    assert "3 1 1 0 48 64 2 0" in out.read_text()
    with pytest.raises(ltrk.LtrkError):
        ltrk.ltrk_tune_cache_load(str(tmp_path / "missing.txt"))


def test_engine_footprint():
    # state and moment rows rounded up to 256 B, plus 256 B for the centre of
    # the moment sums
    assert ltrk.ltrk_engine_footprint(1000, 100) == 16128 + 4096 + 256
    assert ltrk.ltrk_engine_footprint(10_000_000, 100_000) == 160_000_000 + 4_000_000 + 256


def test_rf2_validation_before_any_launch():
    lib = _raw()
    f = lib.ltrk_track_rf2_f64
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                  ctypes.POINTER(ltrk.Rf2), ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    good = dict(SPS_RING, phi1_rad=0.1, harmonic2=9240.0, voltage2_V=1e6, phi2_rad=3.1,
                eta1=1e-4, eta2=-1e-2)
    assert f(None, None, 0, 0, ctypes.byref(ltrk.Rf2.of(good)), 1, None, None) == 0
    for key, val in [("harmonic2", 9240.5), ("harmonic2", 0.0), ("phi2_rad", float("nan")),
                     ("eta1", float("inf")), ("harmonic", -3.0)]:
        bad = ltrk.Rf2.of(dict(good, **{key: val}))
        assert f(None, None, 0, 0, ctypes.byref(bad), 1, None, None) == ltrk.LTRK_EINVAL, key
    # no second harmonic: its harmonic number is not used
    ok = ltrk.Rf2.of(dict(good, voltage2_V=0.0, harmonic2=0.0))
    assert f(None, None, 0, 0, ctypes.byref(ok), 1, None, None) == 0
    assert f(None, None, 0, 0, None, 1, None, None) == ltrk.LTRK_EINVAL


def _programme(turns, **over):
    arr = (ltrk.RfTurn * turns)()
    for i in range(turns):
        vals = dict(voltage_V=2e6, phi1_rad=0.0, voltage2_V=0.0, phi2_rad=0.0,
                    p0c_eV=SPS_RING["p0c_eV"])
        vals.update(over)
        arr[i] = ltrk.RfTurn(**vals)
    return arr


def test_programme_validation_before_any_launch():
    lib = _raw()
    f = lib.ltrk_track_program_f64
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                  ctypes.POINTER(ltrk.Rf2), ctypes.POINTER(ltrk.RfTurn), ctypes.c_int,
                  ctypes.c_void_p, ctypes.c_void_p]
    rf = ltrk.Rf2.of(dict(SPS_RING, phi1_rad=0.0, harmonic2=9240.0, voltage2_V=0.0,
                          phi2_rad=0.0, eta1=0.0, eta2=0.0))
    ok = _programme(4)
    assert f(None, None, 0, 4, ctypes.byref(rf), ok, 1, None, None) == 0
    for over in (dict(p0c_eV=0.0), dict(voltage_V=float("nan")), dict(phi2_rad=float("inf"))):
        assert f(None, None, 0, 4, ctypes.byref(rf), _programme(4, **over), 1, None,
                 None) == ltrk.LTRK_EINVAL, over
    assert f(None, None, 0, 4, ctypes.byref(rf), None, 1, None, None) == ltrk.LTRK_EINVAL
    # a second harmonic needs an integer harmonic2
    bad_h2 = ltrk.Rf2.of(dict(SPS_RING, phi1_rad=0.0, harmonic2=0.5, voltage2_V=0.0,
                              phi2_rad=0.0, eta1=0.0, eta2=0.0))
    assert f(None, None, 0, 4, ctypes.byref(bad_h2), _programme(4, voltage2_V=1e5), 1, None,
             None) == ltrk.LTRK_EINVAL
    assert f(None, None, 0, 4, ctypes.byref(bad_h2), ok, 1, None, None) == 0
    # RK4 supports constant momentum only
    ramp = _programme(4)
    ramp[2].p0c_eV = SPS_RING["p0c_eV"] * 1.001
    assert f(None, None, 0, 4, ctypes.byref(rf), ramp, 3, None, None) == ltrk.LTRK_EUNSUPPORTED
    assert f(None, None, 0, 4, ctypes.byref(rf), ok, 3, None, None) == 0
    assert f(None, None, 0, 4, ctypes.byref(rf), ramp, 2, None, None) == 0


def test_6d_validation_before_any_launch():
    lib = _raw()
    f = lib.ltrk_track_6d_f64
    f.argtypes = [ctypes.c_void_p] * 6 + [ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ltrk.Rf2),
                                          ctypes.POINTER(ltrk.Twiss), ctypes.c_int,
                                          ctypes.c_void_p, ctypes.c_void_p]
    rf = ltrk.Rf2.of(dict(SPS_RING, phi1_rad=0.0, harmonic2=9240.0, voltage2_V=0.0,
                          phi2_rad=0.0, eta1=0.0, eta2=0.0))
    tw = dict(q_x=20.13, qp_x=1.0, alpha_x=0.5, beta_x=40.0, q_y=20.18, qp_y=-1.0,
              alpha_y=-0.5, beta_y=60.0)
    nul = [None] * 6
    assert f(*nul, 0, 0, ctypes.byref(rf), ctypes.byref(ltrk.Twiss.of(tw)), 1, None, None) == 0
    for key, val in [("beta_x", 0.0), ("beta_y", -1.0), ("qp_x", float("nan")),
                     ("alpha_y", float("inf"))]:
        bad = ltrk.Twiss.of(dict(tw, **{key: val}))
        assert f(*nul, 0, 0, ctypes.byref(rf), ctypes.byref(bad), 1, None,
                 None) == ltrk.LTRK_EINVAL, key
    assert f(*nul, 0, 0, ctypes.byref(rf), None, 1, None, None) == ltrk.LTRK_EINVAL
    assert f(*nul, 10, 5, ctypes.byref(rf), ctypes.byref(ltrk.Twiss.of(tw)), 1, None,
             None) == ltrk.LTRK_EINVAL  # NULL state arrays


def test_wake_validation_before_any_launch():
    lib = _raw()
    f = lib.ltrk_track_wake_f64
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                  ctypes.POINTER(ltrk.Rf2), ctypes.POINTER(ltrk.Wake), ctypes.c_int,
                  ctypes.c_void_p, ctypes.c_void_p]
    rf = ltrk.Rf2.of(dict(SPS_RING, phi1_rad=0.0, harmonic2=9240.0, voltage2_V=0.0,
                          phi2_rad=0.0, eta1=0.0, eta2=0.0))
    good = dict(model="resonator", n_slices=64, shunt=1e4, freq_hz=1e9, quality=1.0,
                intensity=1e11, z_lo=-1.0, z_hi=1.0)
    assert f(None, None, 0, 0, ctypes.byref(rf), ctypes.byref(ltrk.Wake.of(good)), 1, None,
             None) == 0
    for key, val in [("n_slices", 0), ("n_slices", 4097), ("quality", 0.5), ("freq_hz", 0.0),
                     ("z_hi", -1.0), ("intensity", -1.0), ("model", 2),
                     ("shunt", float("nan"))]:
        bad = ltrk.Wake.of(dict(good, **{key: val}))
        assert f(None, None, 0, 0, ctypes.byref(rf), ctypes.byref(bad), 1, None,
                 None) == ltrk.LTRK_EINVAL, key
    # a constant wake needs no frequency or quality
    const = ltrk.Wake.of(dict(good, model="constant", freq_hz=0.0, quality=0.0))
    assert f(None, None, 0, 0, ctypes.byref(rf), ctypes.byref(const), 1, None, None) == 0
    assert f(None, None, 0, 0, ctypes.byref(rf), None, 1, None, None) == ltrk.LTRK_EINVAL
    assert f(None, None, 10, 5, ctypes.byref(rf), ctypes.byref(ltrk.Wake.of(good)), 1, None,
             None) == ltrk.LTRK_EINVAL  # NULL state arrays
