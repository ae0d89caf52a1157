"""Serving engine: jobs of different sizes, schemes and precisions admitted
while others run, advanced together step by step; each job's result is
bitwise equal to tracking it alone with the same particles-per-lane (8), the
FP64 jobs' results also match the oracle directly (tests/_parity.py bounds),
and admission respects slots and the arena budget."""
import time

import numpy as np
import pytest

import oracle
from synth import SPS_RING, gaussian_bunch, split_f32c
from tests._parity import (amplification, bucket_error, check_particles, moment_error,
                           near_separatrix)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ltrk():
    import paper_1610_05801_amd as m
    yield m
    m.ltrk_set_plan()


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


JOBS = [(1000, 250, "leapfrog", "f64"), (70_001, 90, "ruth4", "f32c"),
        (5, 400, "euler_cromer", "f64"), (30_000, 333, "rk4", "f64"),
        (4097, 120, "leapfrog", "f32c")]


def alone(ltrk, n, turns, integ, dtype, z0, dp0):
    # the engine's tiles hold 8 particles per lane; the same plan alone
    ltrk.ltrk_set_plan(128, 256, 8, 0)
    mom = torch.empty((turns, 5), dtype=torch.float64, device="cuda")
    if dtype == "f64":
        z, dp = dev(z0, torch.float64), dev(dp0, torch.float64)
        ltrk.ltrk_track_f64(z, dp, turns, SPS_RING, integ, mom)
        out = [z, dp]
    else:
        zh, zc = split_f32c(z0)
        dh, dc = split_f32c(dp0)
        t = [dev(a, torch.float32) for a in (zh, dh, zc, dc)]
        ltrk.ltrk_track_f32c(t[0], t[1], t[2], t[3], turns, SPS_RING, integ, mom)
        out = [t[0], t[1], t[2], t[3]]
    torch.cuda.synchronize()
    ltrk.ltrk_set_plan()
    return [x.cpu().numpy() for x in out] + [mom.cpu().numpy()]


def test_engine_mix_equals_alone(ltrk):
    eng = ltrk.Engine(hbm_budget_bytes=64 << 20, max_slots=8)
    inits = [gaussian_bunch(n, 0.2, 1e-3, 500 + i) for i, (n, *_r) in enumerate(JOBS)]
    slots = {}
    # admit the first three, step, then admit the rest while those are running
    for i in range(3):
        n, T, integ, dt = JOBS[i]
        z0, dp0 = inits[i]
        if dt == "f64":
            slots[i] = eng.admit(n, T, SPS_RING, integ, dt, z0, dp0)
        else:
            zh, zc = split_f32c(z0)
            dh, dc = split_f32c(dp0)
            slots[i] = eng.admit(n, T, SPS_RING, integ, dt, zh, dh, zc, dc)
    eng.step(64)
    for i in range(3, len(JOBS)):
        n, T, integ, dt = JOBS[i]
        z0, dp0 = inits[i]
        zh, zc = split_f32c(z0)
        dh, dc = split_f32c(dp0)
        if dt == "f64":
            slots[i] = eng.admit(n, T, SPS_RING, integ, dt, z0, dp0)
        else:
            slots[i] = eng.admit(n, T, SPS_RING, integ, dt, zh, dh, zc, dc)
    results = {}
    for _ in range(100):
        if len(results) == len(JOBS):
            break
        eng.step(50)
        for i, s in slots.items():
            if i not in results and eng.poll(s):
                results[i] = eng.result(s)
                eng.retire(s)
    assert len(results) == len(JOBS)
    for i, (n, T, integ, dt) in enumerate(JOBS):
        z0, dp0 = inits[i]
        ref = alone(ltrk, n, T, integ, dt, z0, dp0)
        got = results[i]
        if dt == "f64":
            pairs = [(got[0], ref[0]), (got[1], ref[1]), (got[2], ref[2])]
        else:
            # engine returns (z, dp, z_comp, dp_comp, mom); alone (z, dp, zc, dc, mom)
            pairs = list(zip(got, ref))
        for a, b in pairs:
            assert np.array_equal(a, b), (i, JOBS[i])
        if dt == "f64":
            # the job's result in the mix against the oracle itself
            zr, dr, mr = oracle.track(z0, dp0, T, SPS_RING, integ)
            e = bucket_error(got[0], got[1], zr, dr, SPS_RING)
            check_particles(e, near_separatrix(z0, dp0, SPS_RING), T,
                            lambda m: amplification(oracle.track, z0[m], dp0[m], T, SPS_RING,
                                                    integ),
                            label="engine job %d %s" % (i, integ))
            assert moment_error(got[2], mr).max() <= 1e-10
    st = eng.stats()
    assert st["active_slots"] == 0 and st["arena_free_bytes"] == st["arena_bytes"]
    eng.close()


def test_engine_admission_limits(ltrk):
    fp = ltrk.ltrk_engine_footprint(10_000, 100)
    eng = ltrk.Engine(hbm_budget_bytes=2 * fp, max_slots=3)
    z0, dp0 = gaussian_bunch(10_000, 0.2, 1e-3, 1)
    a = eng.admit(10_000, 100, SPS_RING, "leapfrog", "f64", z0, dp0)
    b = eng.admit(10_000, 100, SPS_RING, "leapfrog", "f64", z0, dp0)
    with pytest.raises(ltrk.EngineBusy):          # budget exhausted
        eng.admit(10_000, 100, SPS_RING, "leapfrog", "f64", z0, dp0)
    with pytest.raises(ltrk.LtrkError):           # can never fit
        eng.admit(100_000, 100, SPS_RING, "leapfrog", "f64", np.zeros(100_000), np.zeros(100_000))
    eng.cancel(b)
    eng.step(30)
    assert eng.poll(b)                             # cancelled: no further turns
    eng.retire(b)
    c = eng.admit(10_000, 100, SPS_RING, "leapfrog", "f64", z0, dp0)
    with pytest.raises(ltrk.EngineBusy):          # all arena blocks taken again
        eng.admit(10, 10, SPS_RING, "leapfrog", "f64", z0[:10], dp0[:10])
    for _ in range(10):
        eng.step(50)
    torch.cuda.synchronize()
    for _ in range(1000):                         # steps are asynchronous: wait for them
        if eng.poll(a) and eng.poll(c):
            break
        time.sleep(0.001)
    assert eng.poll(a) and eng.poll(c)
    z, dp, mom = eng.result(a)
    z2, dp2, mom2 = eng.result(c)
    assert np.array_equal(z, z2) and np.array_equal(mom, mom2)
    eng.close()


def test_engine_admission_by_partial_scratch(ltrk, monkeypatch):
    """Running jobs share the engine's moment-partial scratch (here 1 MiB:
    26214 columns of 5 doubles, one column per 512 particles): a job that
    needs more than all of it is refused for good, one that does not fit
    beside the running jobs waits (EngineBusy) until they are done, and steps
    never run out of scratch."""
    monkeypatch.setenv("LTRK_ENGINE_PARTIALS_MB", "1")
    try:
        eng = ltrk.Engine(hbm_budget_bytes=512 << 20, max_slots=4)
    finally:
        monkeypatch.delenv("LTRK_ENGINE_PARTIALS_MB", raising=False)
    rng = np.random.default_rng(3)
    na, nb_, nc = 6_000_000, 9_000_000, 15_000_000   # ~11.7k, ~17.6k, ~29.3k columns
    za, da = 0.2 * rng.standard_normal(na), 1e-3 * rng.standard_normal(na)
    with pytest.raises(ltrk.LtrkError) as bad:
        eng.admit(nc, 4, SPS_RING, "leapfrog", "f64", np.zeros(nc), np.zeros(nc))
    assert not isinstance(bad.value, ltrk.EngineBusy)
    a = eng.admit(na, 4, SPS_RING, "leapfrog", "f64", za, da)
    zb = 0.2 * rng.standard_normal(nb_)
    with pytest.raises(ltrk.EngineBusy):
        eng.admit(nb_, 4, SPS_RING, "leapfrog", "f64", zb, np.zeros(nb_))
    while not eng.poll(a):
        eng.step(4)
        torch.cuda.synchronize()
    b = eng.admit(nb_, 4, SPS_RING, "leapfrog", "f64", zb, np.zeros(nb_))
    while not eng.poll(b):
        eng.step(4)
        torch.cuda.synchronize()
    z, dp, mom = eng.result(a)
    assert np.isfinite(z).all() and np.isfinite(mom).all()
    _, _, mom_b = eng.result(b)
    assert np.isfinite(mom_b).all()
    eng.close()

