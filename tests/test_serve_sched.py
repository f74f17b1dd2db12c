"""Serving policy on the CPU: a fake executor with a virtual clock drives the
same Scheduler the GPU engine uses."""
import numpy as np
import pytest

from paper_2506_20202_amd.serve import Completion, Request, Scheduler


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class Cam:
    def __init__(self, w, h):
        self.width, self.height = w, h


class FakeExecutor:
    """Each request takes `dur(req)` virtual seconds; a request needs
    `pairs(req)` pairs and overflows a slot with less capacity."""

    def __init__(self, clock, resident=1000, dur=lambda r: 1.0, pairs=lambda r: 10, fail=lambda r: False):
        self.clock, self.resident = clock, resident
        self.dur, self.pairs, self.fail = dur, pairs, fail
        self.created, self.destroyed, self.launched = 0, 0, []
        self.live = []

    def resident_bytes(self):
        return self.resident

    def slot_bytes(self, shape, cap):
        _, w, h = shape
        return cap + w * h

    def create_slot(self, shape, cap):
        self.created += 1
        h = dict(shape=shape, cap=cap, req=None, t_end=None)
        self.live.append(h)
        return h

    def destroy_slot(self, h):
        self.destroyed += 1
        self.live.remove(h)

    def launch(self, h, req):
        h["req"], h["t_end"] = req, self.clock() + self.dur(req)
        self.launched.append((self.clock(), req.rid, h["shape"]))

    def poll(self, h):
        if h["req"] is None or self.clock() < h["t_end"]:
            return None
        req, h["req"] = h["req"], None
        if self.fail(req):
            return Completion(ok=False, error="injected")
        need = self.pairs(req)
        if need > h["cap"]:
            return Completion(ok=True, overflow=True, num_pairs=need)
        return Completion(ok=True, result=("img", req.rid))


def _run(s, clock, dt=0.25, limit=1000):
    for _ in range(limit):
        s.step()
        assert s.used_bytes() <= s.budget
        if s.idle():
            return
        clock.t += dt
    raise AssertionError("did not drain")


def _req(scene, w, h, t=0.0):
    return Request(scene, Cam(w, h), None, arrival=t)


def test_fifo_and_slot_reuse():
    clock = Clock()
    ex = FakeExecutor(clock)
    s = Scheduler(ex, hbm_budget=10_000, max_slots=1, clock=clock, capacity_of=lambda sh: 100)
    futs = [s.submit(_req("a", 10, 10, 0.0)) for _ in range(5)]
    _run(s, clock)
    assert [r for _, r, _ in ex.launched] == [0, 1, 2, 3, 4]
    assert ex.created == 1
    assert [f.result()[1] for f in futs] == [0, 1, 2, 3, 4]


def test_concurrency_limited_by_budget():
    clock = Clock()
    ex = FakeExecutor(clock, resident=1000)
    # one slot of shape (20x20, cap 100) costs 500 bytes: 3 fit in 2600
    s = Scheduler(ex, hbm_budget=2600, max_slots=8, clock=clock, capacity_of=lambda sh: 100)
    for _ in range(7):
        s.submit(_req("a", 20, 20))
    _run(s, clock)
    assert s.max_inflight == 3
    assert s.stats()["completed"] == 7


def test_continuous_admission_while_others_run():
    """A request arriving while others run starts as soon as a slot frees,
    not when the whole batch drains."""
    clock = Clock()
    ex = FakeExecutor(clock, dur=lambda r: 4.0 if r.rid == 0 else 1.0)
    s = Scheduler(ex, hbm_budget=10_000, max_slots=2, clock=clock, capacity_of=lambda sh: 100)
    s.submit(_req("a", 10, 10))
    s.submit(_req("a", 10, 10))
    s.step()
    clock.t = 1.5
    s.submit(_req("a", 10, 10, 1.5))   # arrives while request 0 is still running
    _run(s, clock, dt=0.5)
    starts = {rid: t for t, rid, _ in ex.launched}
    assert starts[2] < 4.0             # admitted before request 0 finished


def test_eviction_between_shapes():
    clock = Clock()
    ex = FakeExecutor(clock, resident=0)
    # each slot 100 + w*h; budget fits one slot at a time
    s = Scheduler(ex, hbm_budget=700, max_slots=4, clock=clock, capacity_of=lambda sh: 100)
    for k in range(6):
        s.submit(_req("a" if k % 2 == 0 else "b", 20, 20 + k % 2))
    _run(s, clock)
    assert s.evictions >= 4
    assert s.stats()["completed"] == 6


def test_overflow_retry_grows_capacity():
    clock = Clock()
    ex = FakeExecutor(clock, pairs=lambda r: 5000)
    s = Scheduler(ex, hbm_budget=1 << 30, max_slots=2, clock=clock, capacity_of=lambda sh: 1000)
    f = s.submit(_req("a", 10, 10))
    _run(s, clock)
    assert f.result() == ("img", 0)
    assert s.retries == 1
    assert s.capacity_hint[("a", 10, 10)] >= 5000
    assert all(h["cap"] >= 5000 for h in ex.live)


def test_rejects_request_that_can_never_fit():
    clock = Clock()
    ex = FakeExecutor(clock, resident=900)
    s = Scheduler(ex, hbm_budget=1000, clock=clock, capacity_of=lambda sh: 100)
    f = s.submit(_req("a", 100, 100))
    with pytest.raises(MemoryError):
        f.result(timeout=0)
    assert s.idle()


def test_failed_render_is_isolated():
    clock = Clock()
    ex = FakeExecutor(clock, fail=lambda r: r.rid == 1)
    s = Scheduler(ex, hbm_budget=10_000, max_slots=2, clock=clock, capacity_of=lambda sh: 100)
    fs = [s.submit(_req("a", 10, 10)) for _ in range(3)]
    _run(s, clock)
    assert fs[0].result() and fs[2].result()
    with pytest.raises(RuntimeError):
        fs[1].result(timeout=0)


def test_latency_percentiles():
    clock = Clock()
    ex = FakeExecutor(clock, dur=lambda r: 1.0)
    s = Scheduler(ex, hbm_budget=10_000, max_slots=1, clock=clock, capacity_of=lambda sh: 100)
    for _ in range(4):
        s.submit(_req("a", 10, 10, 0.0))
    _run(s, clock, dt=1.0)
    st = s.stats()
    lat = np.array(s.latencies) * 1e3
    assert sorted(lat.tolist()) == pytest.approx([1000.0, 2000.0, 3000.0, 4000.0])
    assert st["p50_ms"] == pytest.approx(np.percentile(lat, 50))
    assert st["p99_ms"] == pytest.approx(np.percentile(lat, 99))


def test_inflight_cap_keeps_slots_cached():
    """max_inflight bounds the frames running at once; the extra slots stay
    cached, so a shape that comes back reuses its slot (no new capture)."""
    clock = Clock()
    ex = FakeExecutor(clock, resident=0, dur=lambda r: 1.0)
    s = Scheduler(ex, hbm_budget=1 << 30, max_slots=8, clock=clock, capacity_of=lambda sh: 100, max_inflight=2)
    for k in range(12):
        s.submit(_req("a" if k % 3 == 0 else ("b" if k % 3 == 1 else "c"), 10, 10))
    _run(s, clock)
    assert s.max_inflight == 2
    assert s.stats()["completed"] == 12
    assert ex.created <= 4 and ex.destroyed == 0


def test_requests_wait_for_their_arrival_time():
    """A request submitted ahead of its arrival time is admitted only once the
    clock reaches it, and its latency counts from the arrival."""
    clock = Clock()
    ex = FakeExecutor(clock, dur=lambda r: 1.0)
    s = Scheduler(ex, hbm_budget=10_000, max_slots=2, clock=clock, capacity_of=lambda sh: 100)
    s.submit(_req("a", 10, 10, 0.0))
    s.submit(_req("a", 10, 10, 3.0))
    _run(s, clock, dt=0.5)
    starts = {rid: t for t, rid, _ in ex.launched}
    assert starts[0] == 0.0 and starts[1] == 3.0
    assert sorted(np.array(s.latencies).round(6).tolist()) == [1.0, 1.0]
