"""The allocation-free entry point (ltrk_track_f64_noalloc) against
ltrk_track_f64 through the C ABI: same plan, so the same particles and moment
rows bit for bit. Two calls in a row, the second on a smaller bunch (the
fixed per-device array keeps the first call's contents); a call long enough
to be finalized in several chunks of the array; an empty bunch; and the
refusal of a bunch whose partials of one turn exceed the array."""
import numpy as np
import pytest

from synth import SPS_RING, SIGMA_DP, SIGMA_Z, gaussian_bunch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ltrk():
    import paper_1610_05801_amd as m
    m.ltrk_set_plan()
    yield m
    m.ltrk_set_plan()


def run(fn, z0, dp0, turns, integ, stream):
    z = torch.as_tensor(z0).cuda()
    dp = torch.as_tensor(dp0).cuda()
    mom = torch.empty((turns, 5), dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        fn(z, dp, turns, SPS_RING, integ, mom, stream=stream)
    torch.cuda.synchronize()
    return z.cpu().numpy(), dp.cpu().numpy(), mom.cpu().numpy()


def same(a, b, label):
    for x, y in zip(a, b):
        assert np.array_equal(x, y), label


def test_two_calls_second_smaller(ltrk):
    s = torch.cuda.Stream()
    for n, turns, integ in ((300_001, 700, "leapfrog"), (4_097, 333, "ruth4")):
        z0, dp0 = gaussian_bunch(n, SIGMA_Z, SIGMA_DP, 60_000 + n)
        got = run(ltrk.ltrk_track_f64_noalloc, z0, dp0, turns, integ, s)
        ref = run(ltrk.ltrk_track_f64, z0, dp0, turns, integ, s)
        assert np.isfinite(got[2]).all()
        same(got, ref, (n, turns, integ))


def test_chunked_by_the_fixed_array(ltrk):
    """1e6 particles at 8 per lane: 78 KB of partials per turn, so the 64 MiB
    array holds 858 turns and 2000 turns run in three chunks."""
    s = torch.cuda.Stream()
    z0, dp0 = gaussian_bunch(1_000_000, SIGMA_Z, SIGMA_DP, 61_000)
    got = run(ltrk.ltrk_track_f64_noalloc, z0, dp0, 2000, "euler_cromer", s)
    ref = run(ltrk.ltrk_track_f64, z0, dp0, 2000, "euler_cromer", s)
    same(got, ref, "chunked")


def test_empty_bunch_and_refusal(ltrk):
    z = torch.empty(0, dtype=torch.float64, device="cuda")
    mom = torch.zeros((4, 5), dtype=torch.float64, device="cuda")
    ltrk.ltrk_track_f64_noalloc(z, z, 4, SPS_RING, "leapfrog", mom)
    torch.cuda.synchronize()
    assert torch.isnan(mom).all()
    # one turn of partials for 9e8 particles at 8 per lane (70 MB) exceeds the
    # array (the default plan would take 16 per lane there: 35 MB)
    n = 900_000_000
    big_z = torch.zeros(n, dtype=torch.float64, device="cuda")
    big_d = torch.zeros(n, dtype=torch.float64, device="cuda")
    mom1 = torch.empty((1, 5), dtype=torch.float64, device="cuda")
    ltrk.ltrk_set_plan(1024, 256, 8, 1)
    try:
        with pytest.raises(ltrk.LtrkError) as err:
            ltrk.ltrk_track_f64_noalloc(big_z, big_d, 1, SPS_RING, "leapfrog", mom1)
    finally:
        ltrk.ltrk_set_plan()
    assert err.value.code == ltrk.LTRK_EINVAL
    del big_z, big_d
    torch.cuda.empty_cache()


def test_captured_into_a_graph(ltrk):
    """The allocation-free call captured into a graph of the caller's own
    (after one eager call has set the array's address up on the device):
    every replay, with the state restored between replays, equals the eager
    call bit for bit."""
    z0, dp0 = gaussian_bunch(50_000, SIGMA_Z, SIGMA_DP, 62_000)
    T = 96
    s = torch.cuda.Stream()
    z_init, d_init = torch.as_tensor(z0).cuda(), torch.as_tensor(dp0).cuda()
    z, dp = z_init.clone(), d_init.clone()
    mom = torch.empty((T, 5), dtype=torch.float64, device="cuda")
    with torch.cuda.stream(s):
        ltrk.ltrk_track_f64_noalloc(z, dp, T, SPS_RING, "ruth4", mom, stream=s)
    s.synchronize()
    ref = (z.cpu().numpy(), dp.cpu().numpy(), mom.cpu().numpy())
    z.copy_(z_init)
    dp.copy_(d_init)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s, capture_error_mode="relaxed"):
        ltrk.ltrk_track_f64_noalloc(z, dp, T, SPS_RING, "ruth4", mom, stream=s)
    torch.cuda.synchronize()
    for _ in range(3):
        z.copy_(z_init)
        dp.copy_(d_init)
        mom.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        same((z.cpu().numpy(), dp.cpu().numpy(), mom.cpu().numpy()), ref, "replay")
