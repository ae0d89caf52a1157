"""6-D map on the GPU (transverse Twiss rotation with chromatic phase, then
the extended longitudinal step) through the C ABI, against the oracle's 6-D
map and against exact matrix powers.

Longitudinal per-particle bounds as for the single-harmonic map
(tests/_parity.py: check_particles: 1e-12 after 1e3 turns, in proportion
beyond; a particle over it held to 8 ulp per turn times its oracle-measured
sensitivity, capped at 1e-10 after 1e3 turns; at most 0.5% over 1e-12; the
(z, dp) part of the 6-D map is the extended map alone). Transverse: the error in the
Courant-Snyder amplitude sqrt(beta J) stays below 1e-12 after 1e3 turns (it
comes from the phase of each turn, ~1e-16 per turn; chromaticity carries the
longitudinal differences in over 2 pi Q' delta, below that)."""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from synth import SPS_RING, gaussian_bunch
from tests._parity import amplification, check_particles, moment_error

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

C0 = oracle.derive(SPS_RING)
H1 = SPS_RING["harmonic"]
RF = dict(SPS_RING, phi1_rad=0.0, harmonic2=2 * H1, voltage2_V=SPS_RING["voltage_V"] / 4,
          phi2_rad=math.pi, eta1=0.4 * C0["eta"], eta2=-30.0 * C0["eta"])
TW = dict(Qx=20.13, Qpx=1.5, alpha_x=0.7, beta_x=42.0, Qy=20.18, Qpy=-2.5, alpha_y=-1.1,
          beta_y=87.0)
KEYS = ("z", "dp", "x", "xp", "y", "yp")


def twiss_abi(tw):
    return dict(q_x=tw["Qx"], qp_x=tw["Qpx"], alpha_x=tw["alpha_x"], beta_x=tw["beta_x"],
                q_y=tw["Qy"], qp_y=tw["Qpy"], alpha_y=tw["alpha_y"], beta_y=tw["beta_y"])


def state(n, seed):
    rng = np.random.default_rng(seed)
    z, dp = gaussian_bunch(n, 0.15, 6e-4, seed)
    return dict(z=z, dp=dp, x=1e-3 * rng.standard_normal(n), xp=2.5e-5 * rng.standard_normal(n),
                y=1e-3 * rng.standard_normal(n), yp=1.2e-5 * rng.standard_normal(n))


@pytest.fixture(scope="module")
def ltrk():
    import paper_1610_05801_amd as m
    m.ltrk_set_plan()
    yield m
    m.ltrk_set_plan()


def run(ltrk, st, turns, integ, rf=RF, tw=TW, moments=True):
    dev = [torch.as_tensor(st[k]).cuda() for k in KEYS]
    mom = torch.empty((turns, 3, 5), dtype=torch.float64, device="cuda") if moments else None
    ltrk.ltrk_track_6d_f64(*dev, turns, rf, twiss_abi(tw), integ, mom)
    torch.cuda.synchronize()
    out = {k: d.cpu().numpy() for k, d in zip(KEYS, dev)}
    return out, (mom.cpu().numpy() if moments else None)


def long_err(z, dp, zr, dr):
    zb, db = C0["bucket_half_length"], C0["bucket_height"]
    return np.hypot((z - zr) / zb, (dp - dr) / db) / np.hypot(zr / zb, dr / db)


def trans_err(out, ref, plane):
    u, v = ("x", "xp") if plane == "x" else ("y", "yp")
    a, b = TW["alpha_" + plane], TW["beta_" + plane]
    amp = np.sqrt(b * oracle.courant_snyder(ref[u], ref[v], a, b))
    return np.hypot(out[u] - ref[u], b * (out[v] - ref[v])) / amp


def long_check(el, st, turns, integ, label):
    kw = dict(with_moments=False, threads=1 if len(st["z"]) < 2000 else 0)
    return check_particles(
        el, np.zeros(el.size, dtype=bool), turns,
        lambda m: amplification(oracle.track_rf2, st["z"][m], st["dp"][m], turns, RF, integ,
                                err=long_err, **kw),
        label=label)


@pytest.mark.parametrize("integ", ["euler_cromer", "leapfrog", "ruth4", "rk4"])
def test_6d_against_oracle(ltrk, integ):
    st = state(1000, 91)
    out, mom = run(ltrk, st, 1000, integ)
    ref, mr = oracle.track_6d(st, 1000, RF, TW, integ)
    el = long_err(out["z"], out["dp"], ref["z"], ref["dp"])
    long_check(el, st, 1000, integ, "6-D longitudinal %s" % integ)
    ex, ey = trans_err(out, ref, "x"), trans_err(out, ref, "y")
    print("%s 6-D: long e max %.2e, x e max %.2e, y e max %.2e" % (integ, el.max(), ex.max(),
                                                                   ey.max()))
    assert ex.max() <= 1e-12 and ey.max() <= 1e-12
    mr = mr.reshape(1000, 3, 5)
    for p in range(3):
        assert moment_error(mom[:, p], mr[:, p]).max() <= 1e-10, p


def test_transverse_matrix_powers_exact(ltrk):
    """No RF: delta is constant and n turns are the n-th power of one rotation
    by 2 pi (frac(Q) + Q' delta), evaluated here in 50 digits."""
    st = state(5000, 92)
    rf = dict(RF, voltage_V=0.0, voltage2_V=0.0)
    turns = 2000
    out, _ = run(ltrk, st, turns, "leapfrog", rf=rf, moments=False)
    assert np.array_equal(out["dp"], st["dp"])
    mp.mp.dps = 40
    for plane, (u, v) in (("x", ("x", "xp")), ("y", ("y", "yp"))):
        a, b = TW["alpha_" + plane], TW["beta_" + plane]
        g = (1 + mp.mpf(a) ** 2) / b
        q = mp.mpf(TW["Q" + plane]) - math.floor(TW["Q" + plane])
        for i in range(0, 5000, 250):
            mu = 2 * mp.pi * (q + mp.mpf(TW["Qp" + plane]) * mp.mpf(float(st["dp"][i])))
            c, s = mp.cos(turns * mu), mp.sin(turns * mu)
            u0, v0 = mp.mpf(float(st[u][i])), mp.mpf(float(st[v][i]))
            eu = float((c + a * s) * u0 + b * s * v0)
            ev = float(-g * s * u0 + (c - a * s) * v0)
            amp = math.sqrt(b * oracle.courant_snyder(eu, ev, a, b))
            err = math.hypot(out[u][i] - eu, b * (out[v][i] - ev)) / amp
            assert err <= 2e-12, (plane, i, err)


def test_longitudinal_part_equals_extended_map_kernel(ltrk):
    st = state(7000, 93)
    out, mom = run(ltrk, st, 300, "ruth4")
    z, dp = torch.as_tensor(st["z"]).cuda(), torch.as_tensor(st["dp"]).cuda()
    m2 = torch.empty((300, 5), dtype=torch.float64, device="cuda")
    ltrk.ltrk_track_rf2_f64(z, dp, 300, RF, "ruth4", m2)
    torch.cuda.synchronize()
    assert np.array_equal(out["z"], z.cpu().numpy()) and np.array_equal(out["dp"], dp.cpu().numpy())
    assert moment_error(mom[:, 0], m2.cpu().numpy()).max() <= 1e-13


def test_split_calls_bitwise(ltrk):
    st = state(30000, 94)
    out, mom = run(ltrk, st, 700, "leapfrog")
    a, ma = run(ltrk, st, 300, "leapfrog")
    b, mb = run(ltrk, a, 400, "leapfrog")
    for k in KEYS:
        assert np.array_equal(out[k], b[k]), k
    assert np.array_equal(mom, np.concatenate([ma, mb]))


def test_6d_paper_scale_sampled(ltrk):
    """1e6 particles x 1e4 turns, leap-frog, default plan: 200 sampled
    particles against the oracle, last moment rows against two-pass moments
    of the final state."""
    n, T = 1_000_000, 10_000
    st = state(n, 1002)
    out, mom = run(ltrk, st, T, "leapfrog")
    idx = np.arange(0, n, n // 200)
    sub = {k: st[k][idx] for k in KEYS}
    ref, _ = oracle.track_6d(sub, T, RF, TW, "leapfrog", with_moments=False, threads=1)
    got = {k: out[k][idx] for k in KEYS}
    el = long_err(got["z"], got["dp"], ref["z"], ref["dp"])
    long_check(el, sub, T, "leapfrog", "6-D longitudinal 1e6 x 1e4 sample")
    ex, ey = trans_err(got, ref, "x"), trans_err(got, ref, "y")
    print("6-D paper scale: long e max %.2e, x e max %.2e, y e max %.2e" % (el.max(), ex.max(),
                                                                          ey.max()))
    assert ex.max() <= 1e-11 and ey.max() <= 1e-11
    for p, (u, v) in enumerate((("z", "dp"), ("x", "xp"), ("y", "yp"))):
        assert moment_error(mom[-1:, p], oracle.moments(out[u], out[v])[None, :]).max() <= 1e-12
