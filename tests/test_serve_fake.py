"""The request loop (paper_1610_05801_amd/serve.py) against a CPU fake of the
native engine that has the same admit/step/poll/result/retire interface, the
same footprint rule and the oracle as its tracker: first-come first-served
admission, retries after EngineBusy, every request completed with the
oracle's result, latencies consistent with arrivals."""
import numpy as np
import pytest

import oracle
from synth import SPS_RING, gaussian_bunch

serve = pytest.importorskip("paper_1610_05801_amd.serve")
binding = pytest.importorskip("paper_1610_05801_amd._binding")


class FakeEngine:
    def __init__(self, budget, slots):
        self.budget, self.free = budget, budget
        self.slots = [None] * slots
        self.admit_order = []
        self.busy = 0

    @staticmethod
    def footprint(n, turns):
        r = lambda x: (x + 255) // 256 * 256
        return r(16 * n) + r(40 * turns)

    def admit(self, n, turns, ring, integ, dtype, z0, dp0, *comp):
        need = self.footprint(n, turns)
        if need > self.budget:
            raise binding.LtrkError(-1, "never fits")
        idx = next((i for i, s in enumerate(self.slots) if s is None), None)
        if idx is None or need > self.free:
            self.busy += 1
            raise binding.EngineBusy(-4, "busy")
        self.free -= need
        self.slots[idx] = dict(n=n, turns=turns, done=0, need=need, ring=ring, integ=integ,
                               z=np.array(z0, dtype=np.float64), dp=np.array(dp0, dtype=np.float64),
                               mom=[])
        self.admit_order.append(idx)
        return idx

    def step(self, k):
        adv = 0
        for s in self.slots:
            if s is None or s["done"] >= s["turns"]:
                continue
            t = min(k, s["turns"] - s["done"])
            s["z"], s["dp"], m = oracle.track(s["z"], s["dp"], t, s["ring"], s["integ"])
            s["mom"].append(m)
            s["done"] += t
            adv += s["n"] * t
        return adv

    def poll(self, slot):
        s = self.slots[slot]
        return s["done"] >= s["turns"]

    def result(self, slot):
        s = self.slots[slot]
        return s["z"], s["dp"], np.vstack(s["mom"])

    def retire(self, slot):
        self.free += self.slots[slot]["need"]
        self.slots[slot] = None


def make_requests(count=12, seed=3):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        n = int(rng.integers(1, 400))
        turns = int(rng.integers(1, 120))
        z0, dp0 = gaussian_bunch(n, 0.2, 1e-3, 100 + i)
        integ = ["euler_cromer", "leapfrog", "ruth4"][i % 3]
        reqs.append(serve.Request(i, 0.0005 * i, n, turns, SPS_RING, integ, "f64", (z0, dp0)))
    return reqs


def test_all_requests_complete_with_oracle_results():
    reqs = make_requests()
    eng = FakeEngine(budget=3 * FakeEngine.footprint(400, 120), slots=2)
    recs, wall = serve.run_stream(eng, reqs, k=50, keep_results=True)
    assert sorted(r.rid for r in recs) == list(range(len(reqs)))
    assert eng.busy > 0                         # admission actually had to wait
    assert eng.free == eng.budget and all(s is None for s in eng.slots)
    for rec in recs:
        q = reqs[rec.rid]
        z, dp, mom = oracle.track(q.state[0], q.state[1], q.turns, SPS_RING, q.integrator)
        # chunked tracking (steps of k turns) equals one call: the map is per turn
        assert np.array_equal(rec.result[0], z) and np.array_equal(rec.result[1], dp)
        assert np.array_equal(rec.result[2], mom)
        assert rec.arrival_s <= rec.admitted_s <= rec.finished_s
        assert rec.latency_s >= 0


def test_admission_is_first_come_first_served():
    reqs = make_requests(8)
    eng = FakeEngine(budget=10 * FakeEngine.footprint(400, 120), slots=1)
    recs, _ = serve.run_stream(eng, reqs, k=1000)
    assert [r.rid for r in recs] == sorted(r.rid for r in recs)


def test_job_that_never_fits_raises():
    reqs = [serve.Request(0, 0.0, 10_000, 10, SPS_RING, "leapfrog", "f64",
                          gaussian_bunch(10_000, 0.2, 1e-3, 1))]
    eng = FakeEngine(budget=1024, slots=2)
    with pytest.raises(binding.LtrkError):
        serve.run_stream(eng, reqs, k=10)


def test_request_refused_by_an_idle_engine_raises():
    """A slot held outside the loop and no job of the loop running: nothing
    would ever free room for the request, so the loop raises instead of
    waiting forever."""
    eng = FakeEngine(budget=10 * FakeEngine.footprint(400, 120), slots=1)
    z0, dp0 = gaussian_bunch(10, 0.2, 1e-3, 2)
    eng.admit(10, 10, SPS_RING, "leapfrog", "f64", z0, dp0)      # held by someone else
    reqs = [serve.Request(0, 0.0, 10, 10, SPS_RING, "leapfrog", "f64", (z0, dp0))]
    with pytest.raises(RuntimeError):
        serve.run_stream(eng, reqs, k=10)

