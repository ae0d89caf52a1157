"""Continuous-batching request loop over the native serving engine.

Requests arrive on a clock (e.g. a Poisson stream); each one is admitted into
an engine slot as soon as a slot and an arena block large enough for its
footprint are free, its state then stays on the device, and every engine step
advances all admitted jobs together by up to k turns in one launch. Finished
jobs are copied back, retired, and their arrival-to-result latency recorded.
All tracking runs in libltrk; this loop only schedules.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

from ._binding import Engine, EngineBusy


@dataclass
class Request:
    rid: int
    arrival_s: float          # relative to the start of the run
    n: int
    turns: int
    ring: dict
    integrator: str
    dtype: str                # "f64" or "f32c"
    state: tuple = ()         # host arrays: (z, dp) or (z, dp, z_comp, dp_comp)


@dataclass
class Record:
    rid: int
    n: int
    turns: int
    integrator: str
    dtype: str
    arrival_s: float
    admitted_s: float
    finished_s: float
    result: tuple = field(default=(), repr=False)

    @property
    def latency_s(self) -> float:
        return self.finished_s - self.arrival_s


def run_stream(engine: Engine, requests, k: int = 256, keep_results: bool = False,
               clock=time.perf_counter, on_finish=None):
    """Serve `requests` (sorted by arrival) in real time; returns the records
    in completion order and the wall time of the run."""
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival_s))
    waiting = collections.deque()
    active = {}
    records = []
    t0 = clock()
    while pending or waiting or active:
        now = clock() - t0
        while pending and pending[0].arrival_s <= now:
            waiting.append(pending.popleft())
        # first-come first-served admission while slots and arena space last
        while waiting:
            r = waiting[0]
            try:
                slot = engine.admit(r.n, r.turns, r.ring, r.integrator, r.dtype, *r.state)
            except EngineBusy:
                break
            waiting.popleft()
            active[slot] = (r, clock() - t0)
        if waiting and not active:
            # nothing of this loop runs that could free a slot or space
            raise RuntimeError("request %d does not fit into the engine although none of this "
                               "loop's jobs are running (slots or space held elsewhere)"
                               % waiting[0].rid)
        if active:
            advanced = engine.step(k)
            progressed = False
            for slot in list(active):
                if engine.poll(slot):
                    r, adm = active.pop(slot)
                    res = engine.result(slot) if keep_results else ()
                    engine.retire(slot)
                    rec = Record(r.rid, r.n, r.turns, r.integrator, r.dtype, r.arrival_s, adm,
                                 clock() - t0, res)
                    records.append(rec)
                    progressed = True
                    if on_finish:
                        on_finish(rec)
            if advanced == 0 and not progressed:
                time.sleep(0.0002)   # everything enqueued: wait for the device
        elif pending:
            time.sleep(max(0.0, min(pending[0].arrival_s - (clock() - t0), 0.01)))
    return records, clock() - t0
