"""Host logic of the continuous-batching scheduler, against a fake executor
that only records what it is asked to do (no GPU)."""
import numpy as np
import pytest

from paper_2404_15249_amd.serving import Request, Scheduler, summarize


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeExecutor:
    """Each live problem converges after `iters(n)` batched steps; a step costs time."""

    def __init__(self, clock, step_cost=1e-3):
        self.clock = clock
        self.step_cost = step_cost
        self.live = {}
        self.admitted = []
        self.max_live = 0
        self.reserved_log = []

    def estimate(self, r):
        return r.n * r.n * 100

    def prepare(self, r):
        return {"r": r, "steps": 0}

    def admit(self, hd):
        slot = next(s for s in range(10_000) if s not in self.live)
        self.live[slot] = hd
        self.admitted.append(hd["r"].rid)
        self.max_live = max(self.max_live, len(self.live))
        return slot

    def step(self, k):
        self.clock.t += k * self.step_cost
        for hd in self.live.values():
            hd["steps"] += k

    def poll(self):
        out = {}
        for s, hd in self.live.items():
            need = 10 + hd["r"].n // 64
            out[s] = (1 if hd["steps"] >= need else 0, hd["steps"], 1e-11)
        return out

    def finish(self, slot, hd):
        del self.live[slot]
        return hd["steps"]

    def release(self, hd):
        pass


def stream(n_req, qps, seed=0, sizes=(64, 128, 256), p=(0.5, 0.3, 0.2)):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / qps, n_req))
    ns = rng.choice(sizes, size=n_req, p=p)
    return [Request(i, float(t[i]), int(ns[i]), i) for i in range(n_req)]


@pytest.mark.parametrize("budget_factor,slots", [(1.0, 4), (3.0, 16), (100.0, 64)])
def test_scheduler_fifo_budget_and_slots(budget_factor, slots):
    clock = FakeClock()
    ex = FakeExecutor(clock)
    reqs = stream(200, qps=500.0)
    budget = int(budget_factor * 256 * 256 * 100) + 1
    sch = Scheduler(ex, budget, slots, steps_per_poll=4, prepare_workers=0)
    recs, span = sch.run(reqs, clock=clock, sleep=clock.sleep)
    assert len(recs) == len(reqs) and all(r.converged for r in recs)
    assert ex.admitted == sorted(ex.admitted)                 # first in, first out
    assert sch.peak_reserved <= budget
    assert ex.max_live <= slots and sch.peak_live <= slots
    for r in recs:
        assert r.finished >= r.admitted >= r.arrival - 1e-12
        assert r.iters >= 10 + r.n // 64
    s = summarize(recs, span)
    assert s["p99_ms"] >= s["p50_ms"] > 0 and s["solves_per_s"] > 0


def test_scheduler_overlaps_requests():
    """Requests that arrive while others run are admitted into the same batch."""
    clock = FakeClock()
    ex = FakeExecutor(clock, step_cost=1e-2)
    reqs = [Request(i, 0.001 * i, 64, i) for i in range(8)]
    sch = Scheduler(ex, 10 ** 12, 16, steps_per_poll=2, prepare_workers=0)
    recs, _ = sch.run(reqs, clock=clock, sleep=clock.sleep)
    assert ex.max_live >= 4
    assert len(recs) == 8


def test_scheduler_rejects_impossible_request():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    with pytest.raises(ValueError):
        Scheduler(ex, 10, 4, prepare_workers=0).run([Request(0, 0.0, 64, 0)], clock=clock, sleep=clock.sleep)


def test_scheduler_with_thread_pool():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    reqs = stream(50, qps=2000.0, seed=3)
    recs, _ = Scheduler(ex, 10 ** 12, 8, prepare_workers=3).run(reqs, clock=clock, sleep=clock.sleep)
    assert len(recs) == 50


class RefusingExecutor(FakeExecutor):
    """Preparation fails for every third request (as for an unsupported geometry)."""

    class Refused(Exception):
        pass

    request_errors = (Refused,)

    def prepare(self, r):
        if r.rid % 3 == 0:
            raise self.Refused(f"request {r.rid}: edge crossed twice")
        return super().prepare(r)


@pytest.mark.parametrize("workers", [0, 2])
def test_refused_requests_are_recorded_and_release_their_memory(workers):
    clock = FakeClock()
    ex = RefusingExecutor(clock)
    reqs = stream(60, qps=300.0)
    budget = 3 * 256 * 256 * 100 + 1
    sch = Scheduler(ex, budget, 4, steps_per_poll=4, prepare_workers=workers)
    recs, span = sch.run(reqs, clock=clock, sleep=clock.sleep)
    assert len(recs) == len(reqs)
    refused = [r for r in recs if r.rejected]
    assert sorted(r.rid for r in refused) == [r.rid for r in reqs if r.rid % 3 == 0]
    assert sch.reserved == 0                                  # every reservation was returned
    s = summarize(recs, span)
    assert s["rejected"] == len(refused) and s["completed"] == len(reqs) - len(refused)
    assert all(r.converged for r in recs if not r.rejected)
