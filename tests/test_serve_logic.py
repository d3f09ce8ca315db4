"""Serving loop logic on the CPU: a fake backend with a simulated clock."""
import random

from paper_2304_07342_amd.serve import COMPRESS, DECOMPRESS, Request, Scheduler, serve


class FakeBackend:
    """Batches take bytes / rate seconds; at most `slots` run at once (the
    scheduler enforces that); time only advances in idle()."""

    def __init__(self, rate=1e9):
        self.rate = rate
        self.t = 0.0
        self.running = []
        self.max_bytes = 0
        self.max_batches = 0
        self.launch_order = []

    def start(self):
        self.t = 0.0

    def now(self):
        return self.t

    def launch(self, batch):
        done = self.t + sum(r.nbytes for r in batch) / self.rate + 1e-4
        h = [done]
        self.running.append(h)
        self.launch_order += [r.rid for r in batch]
        self.max_batches = max(self.max_batches, len(self.running))
        return h

    def poll(self, h):
        return h[0] if h[0] <= self.t else None

    def release(self, h, batch):
        self.running.remove(h)
        for r in batch:
            r.status = 0

    def idle(self, now, next_arrival, poll_s, busy):
        cands = [h[0] for h in self.running]
        if next_arrival is not None:
            cands.append(next_arrival)
        self.t = max(self.t, min(cands)) if cands else self.t + poll_s


def _trace(n, seed, rate=1000.0):
    rng = random.Random(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.expovariate(rate)
        nb = rng.randrange(1, 50 << 20)
        r = Request(i, rng.choice([COMPRESS, DECOMPRESS]), t, nb, 2)
        r.need = 3 * nb
        out.append(r)
    return out


def test_all_requests_complete_in_fifo_order_within_budget(monkeypatch):
    reqs = _trace(500, 1)
    be = FakeBackend(rate=20e9)
    budget = 1 << 30
    peak = {"bytes": 0}
    orig = Scheduler.next_batch

    def spy_next(self):
        b = orig(self)
        peak["bytes"] = max(peak["bytes"], self.in_flight_bytes)
        return b
    monkeypatch.setattr(Scheduler, "next_batch", spy_next)
    sched = serve(reqs, be, budget, slots=3, max_batch=64)
    assert not sched.rejected
    assert all(r.done is not None and r.done >= r.arrival for r in reqs)
    assert be.launch_order == sorted(be.launch_order)          # FIFO admission
    assert 0 < peak["bytes"] <= budget
    assert be.max_batches <= 3
    assert sched.in_flight_bytes == 0 and sched.in_flight_batches == 0


def test_requests_larger_than_the_budget_are_rejected():
    reqs = _trace(20, 2)
    reqs[5].need = 10 << 30
    sched = serve(reqs, FakeBackend(), 1 << 30, slots=2)
    assert [r.rid for r in sched.rejected] == [5]
    assert reqs[5].done is None
    assert all(r.done is not None for i, r in enumerate(reqs) if i != 5)


def test_new_arrivals_join_while_batches_run():
    # a slow first batch must not block later arrivals from being launched
    # in the other slots
    reqs = [Request(0, COMPRESS, 0.0, 10 << 30, 1), Request(1, COMPRESS, 0.001, 1 << 20, 1),
            Request(2, DECOMPRESS, 0.002, 1 << 20, 1)]
    for r in reqs:
        r.need = r.nbytes
    be = FakeBackend(rate=1e9)
    serve(reqs, be, 64 << 30, slots=3)
    assert reqs[1].done < reqs[0].done and reqs[2].done < reqs[0].done


def test_scheduler_respects_slots_and_budget():
    s = Scheduler(budget_bytes=100, slots=2, max_batch=10)
    for i in range(5):
        r = Request(i, COMPRESS, 0.0, 10)
        r.need = 40
        s.arrive(r)
    b1 = s.next_batch()
    assert [r.rid for r in b1] == [0, 1]          # 80 of 100 bytes
    b2 = s.next_batch()
    assert b2 == []                               # the next needs 40 > 20 left
    s.finish(b1)
    b2 = s.next_batch()
    assert [r.rid for r in b2] == [2, 3]
    s.in_flight_batches = 2
    assert s.next_batch() == []                   # no slot
