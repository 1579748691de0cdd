"""Scheduler logic of the serving loop on a simulated executor and clock (CPU)."""
import numpy as np
import pytest

from paper_2510_07625_amd.serve import Request, Scheduler


class FakeClock:
    def __init__(self):
        self.t = 0.0
        self.ex = None

    def now(self):
        return self.t

    def wait_until(self, t):
        self.t = max(self.t, t)

    def idle(self, inflight, pending):
        nxt = [self.ex.done_at[L.handle] for L in inflight]
        if pending:
            nxt.append(pending[-1].arrival)
        if nxt:
            self.t = max(self.t, min(nxt))


class FakeExecutor:
    """Service time a + b * requests; x1 = x_s + 1 per element."""

    def __init__(self, clock, slots=2, capacity=64, a=200e-6, b=2e-6, nbytes=1000):
        self.clock, self.slots, self.capacity = clock, slots, capacity
        self.a, self.b, self.bytes_per_request = a, b, nbytes
        self.done_at, self.batches, self.inflight_instances = {}, {}, {}
        self.log = []

    def launch(self, slot, reqs, xs):
        now = self.clock.now()
        for other, inst in self.inflight_instances.items():
            assert not (inst & {r.instance for r in reqs}), "instance in two launches at once"
        self.done_at[slot] = now + self.a + self.b * len(reqs)
        self.batches[slot] = (reqs, xs.copy())
        self.inflight_instances[slot] = {r.instance for r in reqs}
        self.log.append((now, len(reqs), [r.rid for r in reqs], xs.copy()))
        return slot

    def poll(self, slot):
        return self.clock.now() >= self.done_at[slot]

    def finish(self, slot):
        reqs, xs = self.batches.pop(slot)
        self.inflight_instances.pop(slot)
        return [(0, xs[i] + 1.0, np.zeros(2)) for i in range(len(reqs))]


def _stream(rate, duration, P, seed=0):
    g = np.random.default_rng(seed)
    n = g.poisson(rate * duration)
    t = np.sort(g.uniform(0, duration, n))
    inst = g.integers(0, P, n)
    return [Request(i, int(inst[i]), float(t[i]), np.zeros(2)) for i in range(n)]


def _run(reqs, P=16, slots=2, budget=None, queue_limit=None, nx=4):
    clock = FakeClock()
    ex = FakeExecutor(clock, slots=slots)
    clock.ex = ex
    sch = Scheduler(ex, np.zeros((P, nx)), memory_budget=budget, deadline_s=1e-3, queue_limit=queue_limit,
                    clock=clock)
    return sch.run(reqs), ex


def test_every_request_completes_once_and_after_it_arrived():
    reqs = _stream(20000, 0.05, 16)
    rep, ex = _run(reqs)
    assert sorted(c.rid for c in rep.completions) == [r.rid for r in reqs]
    for c in rep.completions:
        assert c.done >= c.launched >= c.arrival
        assert c.latency >= 200e-6
    s = rep.summary()
    assert s["completed"] == len(reqs) and s["rejected"] == 0


def test_continuous_batching_overlaps_launches():
    # Requests that arrive while a launch is on the device start the next
    # launch at once on the second slot instead of waiting for the first.
    # With both slots busy, later arrivals wait and leave together.
    reqs = [Request(0, 0, 0.0, np.zeros(2)), Request(1, 1, 50e-6, np.zeros(2)), Request(2, 2, 60e-6, np.zeros(2)),
            Request(3, 3, 70e-6, np.zeros(2))]
    rep, ex = _run(reqs, slots=2)
    assert rep.max_inflight == 2
    assert [e[2] for e in ex.log] == [[0], [1], [2, 3]]
    assert ex.log[1][0] == pytest.approx(50e-6)                 # launched while launch 0 is on the device
    assert ex.log[2][0] == pytest.approx(ex.log[0][0] + 202e-6)  # first slot to free up


def test_instance_state_follows_the_plan():
    # Second request of an instance starts from the first result's next knot.
    reqs = [Request(0, 3, 0.0, np.zeros(2)), Request(1, 3, 10e-6, np.zeros(2))]
    rep, ex = _run(reqs, slots=2)
    assert len(ex.log) == 2
    np.testing.assert_array_equal(ex.log[0][3][0], np.zeros(4))
    np.testing.assert_array_equal(ex.log[1][3][0], np.ones(4))
    assert ex.log[1][0] >= ex.log[0][0] + 200e-6      # waited for its own instance


def test_memory_admission_limits_requests_in_flight():
    reqs = _stream(50000, 0.02, 64, seed=1)
    rep, ex = _run(reqs, P=64, slots=4, budget=3 * 1000)
    assert all(n <= 3 for _, n, _, _ in ex.log)
    assert rep.summary()["completed"] == len(reqs)


def test_budget_below_one_request_is_rejected():
    clock = FakeClock()
    ex = FakeExecutor(clock, nbytes=1000)
    with pytest.raises(ValueError):
        Scheduler(ex, np.zeros((4, 4)), memory_budget=999, clock=clock)


def test_queue_limit_rejects_and_deadline_is_accounted():
    reqs = _stream(200000, 0.01, 8, seed=2)
    rep, ex = _run(reqs, P=8, slots=1, queue_limit=4)
    s = rep.summary()
    assert s["rejected"] > 0
    assert s["completed"] + s["rejected"] == len(reqs)
    lat = np.array([c.latency for c in rep.completions])
    assert s["deadline_miss_rate"] == pytest.approx(np.mean(lat > 1e-3))
