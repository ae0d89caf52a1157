"""Batched tracking of uneven bunches (own V and h each) in one tiled launch
sequence: every bunch against the oracle, and bitwise against tracking the
same bunch alone with the same particles-per-lane."""
import numpy as np
import pytest

import oracle
from synth import BunchSpec, SPS_RING, gaussian_bunch, join_f32c, ring_for, split_f32c
from tests._parity import bucket_error, moment_error, near_separatrix

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ltrk():
    import paper_1610_05801_amd as m
    yield m
    m.ltrk_set_plan()


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def matched_sigma_z(ring, sigma_dp):
    c = oracle.derive(ring)
    return sigma_dp * c["D"] / c["omega"]


SPECS = [BunchSpec(1000, 2e6, 4620.0, 1e-3, 1), BunchSpec(1, 5e6, 9240.0, 1e-3, 2),
         BunchSpec(0, 3e6, 4620.0, 1e-3, 3), BunchSpec(65, 7.5e6, 9240.0, 2e-3, 4),
         BunchSpec(20_000, 1.2e6, 4620.0, 6e-4, 5), BunchSpec(3333, 8e6, 9240.0, 1.5e-3, 6)]


def make(spec):
    r = ring_for(spec)
    return gaussian_bunch(spec.n, matched_sigma_z(r, spec.sigma_dp), spec.sigma_dp, spec.seed)


@pytest.mark.parametrize("ppl", [4, 16])
@pytest.mark.parametrize("integ", ["leapfrog", "ruth4"])
def test_batched_f64_matches_oracle_and_alone(ltrk, integ, ppl):
    T = 300
    ltrk.ltrk_set_plan(64, 256, ppl, 1)
    stream = torch.cuda.Stream()
    bunches, inits = [], []
    for s in SPECS:
        z0, dp0 = make(s)
        inits.append((z0, dp0))
        bunches.append(dict(z=dev(z0), dp=dev(dp0), ring=ring_for(s),
                            moments=torch.empty((T, 5), dtype=torch.float64, device="cuda")))
    with torch.cuda.stream(stream):
        ltrk.ltrk_track_batched(bunches, T, integ, "f64", stream=stream)
    torch.cuda.synchronize()
    for s, b, (z0, dp0) in zip(SPECS, bunches, inits):
        z, dp, mom = b["z"].cpu().numpy(), b["dp"].cpu().numpy(), b["moments"].cpu().numpy()
        if s.n == 0:
            assert np.isnan(mom).all()
            continue
        r = ring_for(s)
        zr, dr, mr = oracle.track(z0, dp0, T, r, integ)
        e = bucket_error(z, dp, zr, dr, r)
        near = near_separatrix(z0, dp0, r)
        if (~near).any():
            assert e[~near].max() <= 1e-12
        if near.any():
            assert e[near].max() <= 1e-10
        if s.n > 1:
            assert moment_error(mom, mr).max() <= 1e-10
        # alone, same plan: bitwise
        za, da = dev(z0), dev(dp0)
        ma = torch.empty((T, 5), dtype=torch.float64, device="cuda")
        ltrk.ltrk_track_f64(za, da, T, r, integ, ma)
        torch.cuda.synchronize()
        assert np.array_equal(za.cpu().numpy(), z)
        assert np.array_equal(da.cpu().numpy(), dp)
        assert np.array_equal(ma.cpu().numpy(), mom)
    ltrk.ltrk_set_plan()


def test_batched_f32c_matches_alone(ltrk):
    T = 200
    ltrk.ltrk_set_plan(32, 128, 2, 0)
    bunches, alone = [], []
    for s in SPECS[:2] + SPECS[3:]:
        z0, dp0 = make(s)
        zh, zc = split_f32c(z0)
        dh, dc = split_f32c(dp0)
        arrs = [dev(a, torch.float32) for a in (zh, dh, zc, dc)]
        bunches.append(dict(z=arrs[0], dp=arrs[1], z_comp=arrs[2], dp_comp=arrs[3],
                            ring=ring_for(s),
                            moments=torch.empty((T, 5), dtype=torch.float64, device="cuda")))
        alone.append([dev(a, torch.float32) for a in (zh, dh, zc, dc)])
    ltrk.ltrk_track_batched(bunches, T, "euler_cromer", "f32c")
    for s, b, a in zip(SPECS[:2] + SPECS[3:], bunches, alone):
        m = torch.empty((T, 5), dtype=torch.float64, device="cuda")
        ltrk.ltrk_track_f32c(a[0], a[1], a[2], a[3], T, ring_for(s), "euler_cromer", m)
        torch.cuda.synchronize()
        for x, y in zip((b["z"], b["dp"], b["z_comp"], b["dp_comp"]), a):
            assert torch.equal(x, y)
        assert torch.equal(b["moments"], m)
    ltrk.ltrk_set_plan()


def test_autotuned_batched_plan_matches_oracle(ltrk):
    """The batched launch tuned on its own tile table: the plan is cached for
    batched calls of that total size (and only for them), and a batched call
    with it matches the oracle on every bunch."""
    specs = [(1_000, 2_000_000.0, 4620), (23_456, 5_000_000.0, 9240), (4_097, 1_000_000.0, 4620),
             (70_001, 8_000_000.0, 9240), (515, 3_000_000.0, 4620)]
    T = 300
    bunches, inits = [], []
    for k, (n, v, h) in enumerate(specs):
        r = dict(SPS_RING, voltage_V=v, harmonic=float(h))
        c = oracle.derive(r)
        z0, dp0 = gaussian_bunch(n, 1e-3 * c["D"] / c["omega"], 1e-3, 300 + k)
        inits.append((z0, dp0, r))
        bunches.append(dict(z=dev(z0), dp=dev(dp0), ring=r,
                            moments=torch.empty((T, 5), dtype=torch.float64, device="cuda")))
    total = sum(n for n, _v, _h in specs)
    stream = torch.cuda.Stream()
    tuned = ltrk.ltrk_autotune_batched(bunches, "ruth4", "f64", stream=stream)
    assert tuned["turns_per_launch"] in (128, 256, 512, 1024)
    assert tuned["block"] in (64, 128, 256) and tuned["ppl"] in (2, 4, 8, 16)
    assert ltrk.ltrk_get_plan_batched("ruth4", "f64", total) == tuned
    # the probe bunches left the caller's arrays alone
    assert np.array_equal(bunches[0]["z"].cpu().numpy(), inits[0][0])
    with torch.cuda.stream(stream):
        ltrk.ltrk_track_batched(bunches, T, "ruth4", "f64", stream=stream)
    torch.cuda.synchronize()
    for (z0, dp0, r), b in zip(inits, bunches):
        zr, dr, mr = oracle.track(z0, dp0, T, r, "ruth4")
        e = bucket_error(b["z"].cpu().numpy(), b["dp"].cpu().numpy(), zr, dr, r)
        near = near_separatrix(z0, dp0, r)
        assert e[~near].max() <= 1e-12
        if near.any():
            assert e[near].max() <= 1e-10
        assert moment_error(b["moments"].cpu().numpy(), mr).max() <= 1e-10
