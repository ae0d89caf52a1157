"""Edge cases of the extended entry points on the GPU: an empty bunch (moment
rows are NaN), zero turns (no-op), one particle, and bunch sizes that leave
a ragged last wave tile, each against the oracle."""
import math

import numpy as np
import pytest

import oracle
from synth import SPS_RING, gaussian_bunch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

C0 = oracle.derive(SPS_RING)
RF = dict(SPS_RING, phi1_rad=0.2, harmonic2=2 * SPS_RING["harmonic"],
          voltage2_V=SPS_RING["voltage_V"] / 4, phi2_rad=math.pi, eta1=0.4 * C0["eta"],
          eta2=-30.0 * C0["eta"])
TW = dict(q_x=20.13, qp_x=1.5, alpha_x=0.7, beta_x=42.0, q_y=20.18, qp_y=-2.5, alpha_y=-1.1,
          beta_y=87.0)
TW_ORACLE = dict(Qx=20.13, Qpx=1.5, alpha_x=0.7, beta_x=42.0, Qy=20.18, Qpy=-2.5, alpha_y=-1.1,
                 beta_y=87.0)


@pytest.fixture(scope="module")
def ltrk():
    import paper_1610_05801_amd as m
    m.ltrk_set_plan()
    yield m


def programme(turns):
    n = np.arange(turns)
    p = SPS_RING["p0c_eV"] * (1 + 1e-6 * (n + 1))
    return dict(voltage_V=np.full(turns, 2e6), phi1_rad=np.full(turns, 0.2),
                voltage2_V=np.full(turns, 0.5e6), phi2_rad=np.full(turns, math.pi), p0c_eV=p)


def err(z, dp, zr, dr):
    zb, db = C0["bucket_half_length"], C0["bucket_height"]
    return np.hypot((z - zr) / zb, (dp - dr) / db) / np.hypot(zr / zb, dr / db)


def call(ltrk, kind, z, dp, turns, mom, extra=None):
    if kind == "rf2":
        ltrk.ltrk_track_rf2_f64(z, dp, turns, RF, "ruth4", mom)
    elif kind == "program":
        ltrk.ltrk_track_program_f64(z, dp, turns, RF, programme(max(turns, 1)), "ruth4", mom)
    else:
        x, xp, y, yp = extra
        ltrk.ltrk_track_6d_f64(z, dp, x, xp, y, yp, turns, RF, TW, "ruth4", mom)


@pytest.mark.parametrize("kind", ["rf2", "program", "6d"])
def test_empty_bunch_gives_nan_moments(ltrk, kind):
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    rows = 3 if kind == "6d" else 1
    mom = torch.zeros((7 * rows, 5), dtype=torch.float64, device="cuda")
    call(ltrk, kind, e, e, 7, mom.view(7, rows, 5) if kind == "6d" else mom, (e, e, e, e))
    torch.cuda.synchronize()
    assert torch.isnan(mom).all()


@pytest.mark.parametrize("kind", ["rf2", "program", "6d"])
def test_zero_turns_is_a_no_op(ltrk, kind):
    z0, dp0 = gaussian_bunch(100, 0.1, 5e-4, 201)
    z, dp = torch.as_tensor(z0).cuda(), torch.as_tensor(dp0).cuda()
    ex = tuple(torch.full((100,), 1e-3, dtype=torch.float64, device="cuda") for _ in range(4))
    call(ltrk, kind, z, dp, 0, None, ex)
    torch.cuda.synchronize()
    assert np.array_equal(z.cpu().numpy(), z0) and np.array_equal(dp.cpu().numpy(), dp0)


@pytest.mark.parametrize("n", [1, 63, 65, 257, 1025, 4097])
@pytest.mark.parametrize("kind", ["rf2", "program", "6d"])
def test_ragged_sizes_against_oracle(ltrk, kind, n):
    turns = 100
    z0, dp0 = gaussian_bunch(n, 0.12, 5e-4, 300 + n)
    rng = np.random.default_rng(400 + n)
    xs = [1e-3 * rng.standard_normal(n), 2e-5 * rng.standard_normal(n),
          1e-3 * rng.standard_normal(n), 1e-5 * rng.standard_normal(n)]
    z, dp = torch.as_tensor(z0).cuda(), torch.as_tensor(dp0).cuda()
    ex = tuple(torch.as_tensor(a).cuda() for a in xs)
    mom = torch.empty((turns, 3, 5) if kind == "6d" else (turns, 5), dtype=torch.float64,
                      device="cuda")
    call(ltrk, kind, z, dp, turns, mom, ex)
    torch.cuda.synchronize()
    if kind == "rf2":
        zr, dr, mr = oracle.track_rf2(z0, dp0, turns, RF, "ruth4")
    elif kind == "program":
        zr, dr, mr = oracle.track_program(z0, dp0, turns, RF, programme(turns), "ruth4")
    else:
        st, mr = oracle.track_6d(dict(z=z0, dp=dp0, x=xs[0], xp=xs[1], y=xs[2], yp=xs[3]),
                                 turns, RF, TW_ORACLE, "ruth4")
        zr, dr = st["z"], st["dp"]
        mr = mr.reshape(turns, 3, 5)
        for k, key in zip(ex, ("x", "xp", "y", "yp")):
            scale = np.abs(st[key]).max()
            assert np.max(np.abs(k.cpu().numpy() - st[key])) <= 1e-12 * scale
    assert np.max(err(z.cpu().numpy(), dp.cpu().numpy(), zr, dr)) <= 1e-12
    m = mom.cpu().numpy()
    if n >= 3:
        means, rmses = (m[..., [0, 2]], mr[..., [0, 2]]), (m[..., [1, 3]], mr[..., [1, 3]])
        assert np.max(np.abs(rmses[0] - rmses[1]) / np.abs(rmses[1])) <= 1e-10
        assert np.max(np.abs(means[0] - means[1]) / np.abs(rmses[1])) <= 1e-10
    else:
        # one or two particles: the means are the coordinates themselves, compared on
        # the scale of their own oscillation (a relative error is undefined at zero
        # crossings)
        got, want = m[..., [0, 2]], mr[..., [0, 2]]
        scale = np.abs(want).max(axis=0, keepdims=True)
        assert np.max(np.abs(got - want) / scale) <= 1e-12
