"""Longitudinal wake kick on the GPU through the C ABI, against the oracle's
wake map (map step, slicing, causal potential, interpolated kick, every
turn).

Per-particle bounds as for the single-harmonic map (tests/_parity.py:
check_particles): e <= 1e-12 after 1e3 turns; a particle over it is held to
8 ulp per turn times its sensitivity amp_i, capped at 1e-10, with at most
0.5% of the bunch over 1e-12. amp_i is measured with the oracle's wake map on
the whole bunch (it includes the collective coupling: a perturbation of every
particle also moves the potential). Slice
counts are integers on both sides; a particle that sits within rounding of
a slice edge could fall on different sides, which these bunches do not
have (checked: the tolerance is met with a wide margin)."""
import math

import numpy as np
import pytest

import oracle
from synth import SPS_RING, gaussian_bunch
from tests._parity import amplification, check_particles, moment_error

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

C0 = oracle.derive(SPS_RING)
RF = dict(SPS_RING, phi1_rad=0.0, harmonic2=2 * SPS_RING["harmonic"], voltage2_V=0.0,
          phi2_rad=0.0, eta1=0.0, eta2=0.0)
RES = dict(model="resonator", n_slices=256, shunt=1e4, freq_hz=1.0e9, quality=1.0,
           intensity=1e11, z_lo=-0.8, z_hi=0.8)


def oracle_wake(w):
    return dict(model={"resonator": 0, "constant": 1}[w["model"]], R_s=w["shunt"],
                f_r=w["freq_hz"], Q=w["quality"], intensity=w["intensity"],
                n_slices=w["n_slices"], z_lo=w["z_lo"], z_hi=w["z_hi"])


@pytest.fixture(scope="module")
def ltrk():
    import paper_1610_05801_amd as m
    m.ltrk_set_plan()
    yield m
    m.ltrk_set_plan()


def run(ltrk, z0, dp0, turns, w, integ, rf=RF, moments=True):
    z, dp = torch.as_tensor(z0).cuda(), torch.as_tensor(dp0).cuda()
    mom = torch.empty((turns, 5), dtype=torch.float64, device="cuda") if moments else None
    ltrk.ltrk_track_wake_f64(z, dp, turns, rf, w, integ, mom)
    torch.cuda.synchronize()
    return z.cpu().numpy(), dp.cpu().numpy(), (mom.cpu().numpy() if moments else None)


def err(z, dp, zr, dr):
    zb, db = C0["bucket_half_length"], C0["bucket_height"]
    return np.hypot((z - zr) / zb, (dp - dr) / db) / np.hypot(zr / zb, dr / db)


def check(e, z0, dp0, turns, w, integ, label, rf=RF):
    """check_particles with the amplification of the whole bunch (the wake
    couples the particles, so a subset would see another potential)."""
    ow = oracle_wake(w)

    def track(z, dp, t, r, ig, **k):
        return oracle.track_wake(z, dp, t, r, ow, ig, with_moments=False)
    amp = {}

    def amp_of(m):
        if "all" not in amp:
            amp["all"] = amplification(track, z0, dp0, turns, rf, integ, err=err)
        return amp["all"][m]
    return check_particles(e, np.zeros(e.size, dtype=bool), turns, amp_of, label=label)


@pytest.mark.parametrize("integ", ["euler_cromer", "leapfrog", "ruth4", "rk4"])
@pytest.mark.parametrize("model", ["resonator", "constant"])
def test_wake_against_oracle(ltrk, integ, model):
    w = dict(RES) if model == "resonator" else dict(RES, model="constant", shunt=2e13)
    z0, dp0 = gaussian_bunch(2000, 0.15, 6e-4, 101)
    z, dp, mom = run(ltrk, z0, dp0, 300, w, integ)
    zr, dr, mr = oracle.track_wake(z0, dp0, 300, RF, oracle_wake(w), integ)
    e = err(z, dp, zr, dr)
    check(e, z0, dp0, 300, w, integ, "%s %s wake" % (model, integ))
    assert moment_error(mom, mr).max() <= 1e-10
    # the wake did something: against the map without it
    z2, d2, _ = oracle.track_rf2(z0, dp0, 300, RF, integ, with_moments=False)
    assert np.median(err(z, dp, z2, d2)) > 1e-6


def test_zero_intensity_is_the_extended_map(ltrk):
    z0, dp0 = gaussian_bunch(10000, 0.2, 8e-4, 102)
    z, dp, mom = run(ltrk, z0, dp0, 200, dict(RES, intensity=0.0), "leapfrog")
    zs, ds = torch.as_tensor(z0).cuda(), torch.as_tensor(dp0).cuda()
    ms = torch.empty((200, 5), dtype=torch.float64, device="cuda")
    ltrk.ltrk_track_rf2_f64(zs, ds, 200, RF, "leapfrog", ms)
    torch.cuda.synchronize()
    assert np.array_equal(z, zs.cpu().numpy()) and np.array_equal(dp, ds.cpu().numpy())
    assert moment_error(mom, ms.cpu().numpy()).max() <= 1e-13


def test_split_calls_bitwise(ltrk):
    z0, dp0 = gaussian_bunch(50000, 0.15, 6e-4, 103)
    z, dp, mom = run(ltrk, z0, dp0, 150, RES, "leapfrog")
    z1, d1, m1 = run(ltrk, z0, dp0, 60, RES, "leapfrog")
    z2, d2, m2 = run(ltrk, z1, d1, 90, RES, "leapfrog")
    assert np.array_equal(z, z2) and np.array_equal(dp, d2)
    assert np.array_equal(mom, np.concatenate([m1, m2]))


@pytest.mark.parametrize("n,slices", [(1, 1), (7, 1), (333, 3), (4097, 4096)])
def test_small_and_edge_cases(ltrk, n, slices):
    rng = np.random.default_rng(104 + n)
    z0 = rng.uniform(-1.0, 1.0, n)  # some outside [z_lo, z_hi)
    dp0 = 4e-4 * rng.standard_normal(n)
    w = dict(RES, n_slices=slices)
    z, dp, mom = run(ltrk, z0, dp0, 20, w, "ruth4")
    zr, dr, mr = oracle.track_wake(z0, dp0, 20, RF, oracle_wake(w), "ruth4")
    assert np.max(err(z, dp, zr, dr)) <= 1e-12
    assert moment_error(mom, mr).max() <= 1e-10 if n > 2 else np.allclose(mom[:, [0, 2]], mr[:, [0, 2]], rtol=1e-12, atol=0)


def test_empty_bunch_moments_are_nan(ltrk):
    z = torch.empty(0, dtype=torch.float64, device="cuda")
    mom = torch.zeros((5, 5), dtype=torch.float64, device="cuda")
    ltrk.ltrk_track_wake_f64(z, z, 5, RF, RES, "leapfrog", mom)
    torch.cuda.synchronize()
    assert torch.isnan(mom).all()


def test_wake_1e6_against_full_oracle(ltrk):
    """10^6 particles x 200 turns in the default plan against the oracle on
    the whole bunch (the potential couples every particle)."""
    n, T = 1_000_000, 200
    z0, dp0 = gaussian_bunch(n, 0.15, 6e-4, 1002)
    z, dp, mom = run(ltrk, z0, dp0, T, RES, "leapfrog")
    zr, dr, mr = oracle.track_wake(z0, dp0, T, RF, oracle_wake(RES), "leapfrog")
    e = err(z, dp, zr, dr)
    check(e, z0, dp0, T, RES, "leapfrog", "wake 1e6")
    assert moment_error(mom, mr).max() <= 1e-10
