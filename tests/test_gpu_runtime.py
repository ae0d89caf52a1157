"""Runtime services through the C ABI on the GPU: the autotuner and its cache
file, per-launch event timing (eager and inside replayed graphs), and that a
tuned plan still reproduces the oracle."""
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
    # finalize-kind launches: the centre of the moment sums and one finalize
    assert t["track_launches"] == 4 and t["finalize_launches"] == 2
    assert t["track_ms"] > 0 and t["finalize_ms"] > 0


def test_default_plan_follows_the_moment_partials(ltrk):
    """The default plan's 1024 turns per launch are lowered for calls with
    moments so that one launch's partial rows stay within 192 MiB: at 1e7
    particles (16 per lane, 9766 wave tiles, 391 KB per row) 512 turns; at
    1e6 (8 per lane, 78 KB per row) the full 1024; without moments nothing
    changes."""
    ltrk.ltrk_set_plan()

    def launches(n, turns, moments):
        z = torch.zeros(n, dtype=torch.float64, device="cuda")
        dp = torch.zeros(n, dtype=torch.float64, device="cuda")
        mom = torch.empty((turns, 5), dtype=torch.float64, device="cuda") if moments else None
        ltrk.ltrk_timing_enable(True)
        ltrk.ltrk_timing_take()
        ltrk.ltrk_track_f64(z, dp, turns, SPS_RING, "leapfrog", mom)
        t = ltrk.ltrk_timing_take()
        ltrk.ltrk_timing_enable(False)
        return t["track_launches"]

    plan = ltrk.ltrk_get_plan("leapfrog", "f64", 10_000_000)
    assert plan["turns_per_launch"] == 1024 and plan["ppl"] == 16
    assert ltrk.ltrk_get_plan("leapfrog", "f64", 1_000_000)["ppl"] == 8
    # F32C: 16 for Euler-Cromer and leap-frog, 8 for Ruth4 and RK4
    assert ltrk.ltrk_get_plan("leapfrog", "f32c", 10_000_000)["ppl"] == 16
    assert ltrk.ltrk_get_plan("ruth4", "f32c", 10_000_000)["ppl"] == 8
    assert ltrk.ltrk_get_plan("rk4", "f32c", 10_000_000)["ppl"] == 8
    assert launches(10_000_000, 1024, True) == 2
    assert launches(10_000_000, 1024, False) == 1
    assert launches(1_000_000, 2048, True) == 2


def test_timing_inside_replayed_graphs(ltrk):
    """Per-launch timing of a hipGraph replay (event-record nodes between the
    launches, fresh events per replay): results equal the eager run bit for
    bit, every replay counts all its launches, and the launches' times add up
    to no more than the whole call; with timing off again the untimed graph
    runs and nothing is counted."""
    z0, dp0 = gaussian_bunch(100_000, 0.2, 1e-3, 3)
    s = torch.cuda.Stream()
    T = 64

    bufs = [torch.empty(z0.size, dtype=torch.float64, device="cuda") for _ in range(2)]
    mom_d = torch.empty((T, 5), dtype=torch.float64, device="cuda")

    def call(use_graph, fresh=False):
        # the same buffers replay one cached graph; fresh ones build another
        ltrk.ltrk_set_plan(16, 256, 4, use_graph)
        if fresh:
            z, dp = torch.as_tensor(z0).cuda(), torch.as_tensor(dp0).cuda()
        else:
            z, dp = bufs
            z.copy_(torch.as_tensor(z0))
            dp.copy_(torch.as_tensor(dp0))
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s)
            ltrk.ltrk_track_f64(z, dp, T, SPS_RING, "leapfrog", mom_d, stream=s)
            b.record(s)
        s.synchronize()
        return z.cpu().numpy(), dp.cpu().numpy(), mom_d.cpu().numpy(), a.elapsed_time(b)

    try:
        ze, de, me, _ = call(0)
        ltrk.ltrk_timing_enable(True)
        ltrk.ltrk_timing_take()
        for i in range(4):
            z, dp, mom, wall_ms = call(1, fresh=(i == 2))
            t = ltrk.ltrk_timing_take()
            assert t["track_launches"] == 4 and t["finalize_launches"] == 2
            assert t["track_ms"] > 0 and t["finalize_ms"] > 0
            assert t["track_ms"] + t["finalize_ms"] <= wall_ms * 1.02 + 0.01
            assert np.array_equal(z, ze) and np.array_equal(dp, de) and np.array_equal(mom, me)
        ltrk.ltrk_timing_enable(False)
        z, dp, mom, _ = call(1)
        assert ltrk.ltrk_timing_take()["track_launches"] == 0
        assert np.array_equal(z, ze) and np.array_equal(dp, de) and np.array_equal(mom, me)
    finally:
        ltrk.ltrk_timing_enable(False)
        ltrk.ltrk_set_plan()


def test_long_sequences_run_eagerly_in_pieces(ltrk, monkeypatch):
    """A call of more launches than LTRK_MAX_GRAPH_LAUNCHES (here 16) is not
    captured into a graph: its launches are enqueued eagerly, in pieces, as
    they are generated. Every tracking entry point then gives the results of
    the same call replayed from a graph bit for bit (single bunch with
    moments, 6-D, wake, batched; 51 to 123 launches per call)."""
    from tests.test_gpu_6d import KEYS, RF as RF6, TW, state, twiss_abi
    from tests.test_gpu_wake import RES, RF as RFW
    from synth import BunchSpec, ring_for
    s = torch.cuda.Stream()
    T, Tw = 200, 60
    z0, dp0 = gaussian_bunch(5000, 0.2, 1e-3, 11)
    st6 = state(3000, 12)
    zw0, dw0 = gaussian_bunch(4000, 0.15, 6e-4, 13)
    specs = [BunchSpec(700, 2e6, 4620.0, 1e-3, 14), BunchSpec(2500, 5e6, 9240.0, 6e-4, 15)]
    wake = dict(RES, n_slices=64)

    def f64(a):
        return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=torch.float64)

    def run_all():
        ltrk.ltrk_set_plan(4, 256, 4, 1)
        out = []
        with torch.cuda.stream(s):
            z, dp = f64(z0), f64(dp0)
            mom = torch.empty((T, 5), dtype=torch.float64, device="cuda")
            ltrk.ltrk_track_f64(z, dp, T, SPS_RING, "leapfrog", mom, stream=s)
            d6 = [f64(st6[k]) for k in KEYS]
            m6 = torch.empty((T, 3, 5), dtype=torch.float64, device="cuda")
            ltrk.ltrk_track_6d_f64(*d6, T, RF6, twiss_abi(TW), "ruth4", m6, stream=s)
            zw, dw = f64(zw0), f64(dw0)
            mw = torch.empty((Tw, 5), dtype=torch.float64, device="cuda")
            ltrk.ltrk_track_wake_f64(zw, dw, Tw, RFW, wake, "leapfrog", mw, stream=s)
            bunches = []
            for sp in specs:
                bz, bd = gaussian_bunch(sp.n, 0.1, sp.sigma_dp, sp.seed)
                bunches.append(dict(z=f64(bz), dp=f64(bd), ring=ring_for(sp),
                                    moments=torch.empty((T, 5), dtype=torch.float64,
                                                        device="cuda")))
            ltrk.ltrk_track_batched(bunches, T, "euler_cromer", "f64", stream=s)
        s.synchronize()
        out = [z, dp, mom, *d6, m6, zw, dw, mw]
        for b in bunches:
            out += [b["z"], b["dp"], b["moments"]]
        return [t.cpu().numpy() for t in out]

    try:
        graph = run_all()
        monkeypatch.setenv("LTRK_MAX_GRAPH_LAUNCHES", "16")
        pieces = run_all()
    finally:
        monkeypatch.delenv("LTRK_MAX_GRAPH_LAUNCHES", raising=False)
        ltrk.ltrk_set_plan()
    assert len(graph) == len(pieces) == 19
    for a, b in zip(graph, pieces):
        assert np.isfinite(a).all() and np.array_equal(a, b)


def test_calls_captured_by_the_caller_replay_exactly(ltrk):
    """A caller may capture a call into a graph of its own (here torch's, on a
    stream that one eager call has already set up, so the captured call
    allocates nothing): the library enqueues its kernels into the capture, and
    every replay, with the state restored by the program between replays,
    equals the eager call bit for bit."""
    z0, dp0 = gaussian_bunch(50_000, 0.2, 1e-3, 21)
    T = 96
    s = torch.cuda.Stream()
    ltrk.ltrk_set_plan(16, 256, 4, 1)
    try:
        z_init, d_init = torch.as_tensor(z0).cuda(), torch.as_tensor(dp0).cuda()
        z, dp = z_init.clone(), d_init.clone()
        mom = torch.empty((T, 5), dtype=torch.float64, device="cuda")
        with torch.cuda.stream(s):
            ltrk.ltrk_track_f64(z, dp, T, SPS_RING, "leapfrog", mom, stream=s)
        s.synchronize()
        ze, de, me = z.cpu().numpy(), dp.cpu().numpy(), mom.cpu().numpy()
        z.copy_(z_init)
        dp.copy_(d_init)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s, capture_error_mode="relaxed"):
            ltrk.ltrk_track_f64(z, dp, T, SPS_RING, "leapfrog", mom, stream=s)
        torch.cuda.synchronize()
        for _ in range(3):
            z.copy_(z_init)
            dp.copy_(d_init)
            mom.fill_(float("nan"))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(z.cpu().numpy(), ze) and np.array_equal(dp.cpu().numpy(), de)
            assert np.array_equal(mom.cpu().numpy(), me)
    finally:
        ltrk.ltrk_set_plan()


def test_capture_refusals_enqueue_nothing(ltrk):
    """Under a caller's stream capture, a batched call (it uploads tables) and
    a call that would have to grow its stream's moment scratch return
    EUNSUPPORTED before enqueueing anything: the captured graph is empty and
    the arrays are untouched."""
    z0, dp0 = gaussian_bunch(4096, 0.2, 1e-3, 22)
    s = torch.cuda.Stream()  # a new stream: no scratch yet
    z, dp = torch.as_tensor(z0).cuda(), torch.as_tensor(dp0).cuda()
    mom = torch.empty((10, 5), dtype=torch.float64, device="cuda")
    bunches = [dict(z=z, dp=dp, ring=SPS_RING, moments=mom)]
    torch.cuda.synchronize()
    codes = []
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s, capture_error_mode="relaxed"):
        for call in (lambda: ltrk.ltrk_track_batched(bunches, 10, "leapfrog", "f64", stream=s),
                     lambda: ltrk.ltrk_track_f64(z, dp, 10, SPS_RING, "leapfrog", mom,
                                                 stream=s)):
            try:
                call()
                codes.append(0)
            except ltrk.LtrkError as err:
                codes.append(err.code)
    torch.cuda.synchronize()
    assert codes == [ltrk.LTRK_EUNSUPPORTED, ltrk.LTRK_EUNSUPPORTED]
    g.replay()
    torch.cuda.synchronize()
    assert np.array_equal(z.cpu().numpy(), z0) and np.array_equal(dp.cpu().numpy(), dp0)


def test_autotune_and_cache_roundtrip(ltrk, tmp_path):
    n = 200_000
    best = ltrk.ltrk_autotune("leapfrog", "f64", n)
    assert best["ppl"] in (1, 2, 4, 8, 16) and best["block"] in (64, 128, 256)
    assert 16 <= best["turns_per_launch"] <= 2048
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
    if near.any():
        assert e[near].max() <= 1e-10
