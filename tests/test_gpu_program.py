"""RF programme on the GPU (per-turn RF voltages and phases, momentum ramp)
through the C ABI, against the oracle's programme map; a constant programme
against the extended-map kernel bit for bit; launch-plan and call-split
invariance.

Per-particle bounds as for the single-harmonic map (tests/_parity.py:
check_particles): e <= 1e-12 after 1e3 turns (in proportion beyond); a
particle over it is held to 8 ulp per turn times its sensitivity measured
with the oracle (relative perturbations of 1e-13 in z and in dp), capped at
1e-10 after 1e3 turns, and at most 0.5% of the bunch may be over 1e-12. The
bunches stay inside their buckets, so none is counted as near the
separatrix."""
import math

import numpy as np
import pytest

import oracle
from synth import SPS_RING, gaussian_bunch
from tests._parity import amplification, check_particles, moment_error

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

C0 = oracle.derive(SPS_RING)
H1 = SPS_RING["harmonic"]
P0 = SPS_RING["p0c_eV"]
V1 = SPS_RING["voltage_V"]
RF = dict(SPS_RING, phi1_rad=0.0, harmonic2=2 * H1, voltage2_V=V1 / 4, phi2_rad=math.pi,
          eta1=0.4 * C0["eta"], eta2=-30.0 * C0["eta"])
FIELDS = ("voltage_V", "phi1_rad", "voltage2_V", "phi2_rad", "p0c_eV")


def beta_of(p):
    m = SPS_RING["mass_eV"]
    return p / np.sqrt(p * p + m * m)


def ramp_programme(turns, rel_per_turn=2e-6, p_start=P0, t0=0):
    """Momentum ramp at the synchronous phase, V1 and V2 modulated, phases
    jittered: every coefficient of every record changes from turn to turn."""
    n = np.arange(t0, t0 + turns)
    p_after = p_start * (1 + rel_per_turn * (n - t0 + 1))
    p_before = np.concatenate([[p_start], p_after[:-1]])
    v1 = V1 * (1 + 0.2 * np.sin(n / 300.0))
    phi = np.arcsin(beta_of(p_before) * (p_after - p_before) / v1)
    return dict(voltage_V=v1, phi1_rad=phi + 0.002 * np.sin(n / 7.0),
                voltage2_V=0.25 * v1 * (1 + 0.1 * np.cos(n / 50.0)),
                phi2_rad=math.pi + 0.05 * np.sin(n / 90.0), p0c_eV=p_after)


def constant_programme(turns, **over):
    vals = dict(voltage_V=V1, phi1_rad=0.0, voltage2_V=RF["voltage2_V"], phi2_rad=math.pi,
                p0c_eV=P0)
    vals.update(over)
    return {k: np.full(turns, float(v)) for k, v in vals.items()}


def err(z, dp, zr, dr):
    zb, db = C0["bucket_half_length"], C0["bucket_height"]
    return np.hypot((z - zr) / zb, (dp - dr) / db) / np.hypot(zr / zb, dr / db)


def check(e, z0, dp0, turns, prog, integ, label):
    kw = dict(with_moments=False, threads=1 if len(z0) < 2000 else 0)

    def track(z, dp, t, rf, ig, **k):
        return oracle.track_program(z, dp, t, rf, prog, ig, **k)
    return check_particles(
        e, np.zeros(e.size, dtype=bool), turns,
        lambda m: amplification(track, z0[m], dp0[m], turns, RF, integ, err=err, **kw),
        label=label)


@pytest.fixture(scope="module")
def ltrk():
    import paper_1610_05801_amd as m
    m.ltrk_set_plan()
    yield m
    m.ltrk_set_plan()


def run(ltrk, z0, dp0, turns, prog, integ, rf=RF):
    z, dp = torch.as_tensor(z0).cuda(), torch.as_tensor(dp0).cuda()
    mom = torch.empty((turns, 5), dtype=torch.float64, device="cuda")
    ltrk.ltrk_track_program_f64(z, dp, turns, rf, prog, integ, mom)
    torch.cuda.synchronize()
    return z.cpu().numpy(), dp.cpu().numpy(), mom.cpu().numpy()


@pytest.mark.parametrize("integ", ["euler_cromer", "leapfrog", "ruth4", "rk4"])
def test_programme_against_oracle(ltrk, integ):
    turns = 1000
    prog = ramp_programme(turns)
    if integ == "rk4":  # constant momentum only
        prog["p0c_eV"][:] = P0
        prog["phi1_rad"] = 0.002 * np.sin(np.arange(turns) / 7.0)
    z0, dp0 = gaussian_bunch(1000, 0.15, 6e-4, 81)
    z, dp, mom = run(ltrk, z0, dp0, turns, prog, integ)
    zr, dr, mr = oracle.track_program(z0, dp0, turns, RF, prog, integ)
    e = err(z, dp, zr, dr)
    check(e, z0, dp0, turns, prog, integ, "programme %s" % integ)
    assert moment_error(mom, mr).max() <= 1e-10


@pytest.mark.parametrize("integ", ["euler_cromer", "leapfrog", "ruth4", "rk4"])
def test_constant_programme_is_extended_map_bitwise(ltrk, integ):
    z0, dp0 = gaussian_bunch(5000, 0.23, 1e-3, 82)
    rf = dict(RF, phi1_rad=0.1)
    z, dp, mom = run(ltrk, z0, dp0, 300, constant_programme(300, phi1_rad=0.1), integ, rf)
    zs, ds = torch.as_tensor(z0).cuda(), torch.as_tensor(dp0).cuda()
    ms = torch.empty((300, 5), dtype=torch.float64, device="cuda")
    ltrk.ltrk_track_rf2_f64(zs, ds, 300, rf, integ, ms)
    torch.cuda.synchronize()
    assert np.array_equal(z, zs.cpu().numpy()) and np.array_equal(dp, ds.cpu().numpy())
    assert np.array_equal(mom, ms.cpu().numpy())


def test_split_calls_and_launch_plans_bitwise(ltrk):
    """1000 turns in one call equal 400 + 600 turns in two calls (the second
    starting from the momentum reached), and a plan of 64 turns per launch."""
    turns = 1000
    prog = ramp_programme(turns)
    z0, dp0 = gaussian_bunch(20000, 0.15, 6e-4, 83)
    z, dp, mom = run(ltrk, z0, dp0, turns, prog, "ruth4")
    first = {k: v[:400] for k, v in prog.items()}
    second = {k: v[400:] for k, v in prog.items()}
    z1, d1, m1 = run(ltrk, z0, dp0, 400, first, "ruth4")
    rf_b = dict(RF, p0c_eV=float(prog["p0c_eV"][399]))
    z2, d2, m2 = run(ltrk, z1, d1, 600, second, "ruth4", rf_b)
    assert np.array_equal(z, z2) and np.array_equal(dp, d2)
    assert np.array_equal(mom, np.concatenate([m1, m2]))
    plan = ltrk.ltrk_get_plan("ruth4", "f64", z0.size)
    try:
        ltrk.ltrk_set_plan(64, plan["block"], plan["ppl"], 0)
        z3, d3, m3 = run(ltrk, z0, dp0, turns, prog, "ruth4")
    finally:
        ltrk.ltrk_set_plan()
    assert np.array_equal(z, z3) and np.array_equal(dp, d3) and np.array_equal(mom, m3)


def test_programme_reuse_across_calls_and_streams(ltrk):
    """Back-to-back calls with different programmes on two streams: each
    result equals its own run alone (the staged upload is not overwritten
    under a pending copy)."""
    z0, dp0 = gaussian_bunch(4096, 0.15, 6e-4, 84)
    progs = [ramp_programme(200, r) for r in (1e-6, -2e-6, 3e-6, 0.0)]
    want = [run(ltrk, z0, dp0, 200, p, "leapfrog") for p in progs]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = []
    for i, p in enumerate(progs):
        s = streams[i % 2]
        z, dp = torch.as_tensor(z0).cuda(), torch.as_tensor(dp0).cuda()
        mom = torch.empty((200, 5), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            ltrk.ltrk_track_program_f64(z, dp, 200, RF, p, "leapfrog", mom, stream=s)
        outs.append((z, dp, mom))
    torch.cuda.synchronize()
    for (z, dp, mom), (zw, dw, mw) in zip(outs, want):
        assert np.array_equal(z.cpu().numpy(), zw) and np.array_equal(dp.cpu().numpy(), dw)
        assert np.array_equal(mom.cpu().numpy(), mw)


def test_rk4_ramp_unsupported(ltrk):
    z, dp = torch.zeros(64, dtype=torch.float64, device="cuda"), torch.zeros(
        64, dtype=torch.float64, device="cuda")
    with pytest.raises(ltrk.LtrkError) as e:
        ltrk.ltrk_track_program_f64(z, dp, 10, RF, ramp_programme(10), "rk4")
    assert e.value.code == ltrk.LTRK_EUNSUPPORTED


def test_programme_paper_scale_sampled(ltrk):
    """1e6 particles x 1e4 turns through a 2% momentum ramp in the default
    launch plan, 500 particles sampled."""
    n, T = 1_000_000, 10_000
    prog = ramp_programme(T)
    z0, dp0 = gaussian_bunch(n, 0.15, 6e-4, 1002)
    z, dp, mom = run(ltrk, z0, dp0, T, prog, "leapfrog")
    idx = np.arange(0, n, n // 500)
    zr, dr, _ = oracle.track_program(z0[idx], dp0[idx], T, RF, prog, "leapfrog",
                                     with_moments=False, threads=1)
    e = err(z[idx], dp[idx], zr, dr)
    check(e, z0[idx], dp0[idx], T, prog, "leapfrog", "programme 1e6 x 1e4 sample")
    assert moment_error(mom[-1:], oracle.moments(z, dp)[None, :]).max() <= 1e-12
