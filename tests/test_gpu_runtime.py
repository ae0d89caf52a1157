"""Runtime services through the C ABI on the GPU: the autotuner and its cache
file, per-launch event timing, and that a tuned plan still reproduces the
oracle."""
import numpy as np
import pytest

import oracle
from synth import SPS_RING, gaussian_bunch
from tests._parity import bucket_error, near_separatrix

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ltrk():
    import paper_1610_05801_amd as m
    yield m
    m.ltrk_set_plan()


def test_timing_counts_launches(ltrk):
    z0, dp0 = gaussian_bunch(10_000, 0.2, 1e-3, 2)
    z, dp = torch.as_tensor(z0).cuda(), torch.as_tensor(dp0).cuda()
    mom = torch.empty((64, 5), dtype=torch.float64, device="cuda")
    ltrk.ltrk_set_plan(16, 256, 2, 1)
    ltrk.ltrk_timing_enable(True)
    ltrk.ltrk_timing_take()
    ltrk.ltrk_track_f64(z, dp, 64, SPS_RING, "leapfrog", mom)
    t = ltrk.ltrk_timing_take()
    ltrk.ltrk_timing_enable(False)
    ltrk.ltrk_set_plan()
    assert t["track_launches"] == 4 and t["finalize_launches"] == 1
    assert t["track_ms"] > 0 and t["finalize_ms"] > 0


def test_autotune_and_cache_roundtrip(ltrk, tmp_path):
    n = 200_000
    best = ltrk.ltrk_autotune("leapfrog", "f64", n)
    assert best["ppl"] in (1, 2, 4, 8) and best["block"] in (64, 128, 256)
    assert 16 <= best["turns_per_launch"] <= 512
    assert ltrk.ltrk_get_plan("leapfrog", "f64", n) == best
    path = str(tmp_path / "tune.txt")
    ltrk.ltrk_tune_cache_save(path)
    text = open(path).read()
    assert "gfx" in text
    ltrk.ltrk_tune_cache_load(path)
    assert ltrk.ltrk_get_plan("leapfrog", "f64", n) == best
    # the tuned plan still tracks correctly
    z0, dp0 = gaussian_bunch(n, 0.23, 1e-3, 9)
    z, dp = torch.as_tensor(z0).cuda(), torch.as_tensor(dp0).cuda()
    ltrk.ltrk_track_f64(z, dp, 200, SPS_RING, "leapfrog", None)
    torch.cuda.synchronize()
    idx = np.arange(0, n, 97)
    zr, dr, _ = oracle.track(z0[idx], dp0[idx], 200, SPS_RING, "leapfrog", with_moments=False)
    e = bucket_error(z.cpu().numpy()[idx], dp.cpu().numpy()[idx], zr, dr, SPS_RING)
    near = near_separatrix(z0[idx], dp0[idx], SPS_RING)
    assert e[~near].max() <= 1e-12
