"""Continuous-batching request loop for MPC re-solves (the serving pattern).

Requests ``(instance, arrival time, goal)`` arrive over time. Each instance
is one solve slot of a :class:`paper_2510_07625_amd.Batch` whose trajectory
stays resident on the device; a request re-solves its instance from the
previous trajectory shifted by one knot (the warm start of the paper's
experiments, Sec. IV) with the instance's current start state.

The scheduler admits requests as they arrive and launches every eligible
waiting request together as soon as a launch slot is free, while earlier
launches are still on the GPU (continuous batching, not a queue drained one
batch at a time). Admission is limited by device memory (bytes per in-flight
request) and by one request in flight per instance. Latency runs from arrival
to the moment the result is visible on the host.

The executor does the device work; :class:`GpuExecutor` drives the C ABI's
serving launch contexts (``gato_serve_ctx_*``, one HIP stream per launch slot). Any object with the
same methods can stand in for it (the tests use a simulated one).
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass

import numpy as np


@dataclass
class Request:
    rid: int
    instance: int
    arrival: float            # seconds, on the scheduler clock
    goal: np.ndarray          # [n] joint goal


@dataclass
class Completion:
    rid: int
    instance: int
    arrival: float
    launched: float
    done: float
    status: int
    x1: np.ndarray            # the instance's next knot (the plant's next state)
    u0: np.ndarray            # the control to apply

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class ServeReport:
    completions: list
    rejected: list
    deadline_s: float
    launches: int
    mean_batch: float
    max_inflight: int

    def summary(self) -> dict:
        lat = np.array([c.latency for c in self.completions]) if self.completions else np.zeros(1)
        span = (max(c.done for c in self.completions) - min(c.arrival for c in self.completions)
                if self.completions else 1.0)
        return dict(completed=len(self.completions), rejected=len(self.rejected),
                    p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                    solves_per_s=len(self.completions) / max(span, 1e-12),
                    deadline_miss_rate=float(np.mean(lat > self.deadline_s)) if self.completions else 0.0,
                    launches=self.launches, mean_batch=self.mean_batch, max_inflight=self.max_inflight)


class WallClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def wait_until(self, t: float):
        while self.now() < t:
            pass


@dataclass
class _Launch:
    handle: object
    reqs: list
    launched: float
    nbytes: int


class Scheduler:
    """Continuous batching over an executor.

    executor: object with ``slots`` (launch slots, i.e. concurrent launches),
    ``capacity`` (max requests per launch), ``bytes_per_request``,
    ``launch(reqs, xs) -> handle``, ``poll(handle) -> bool`` and
    ``finish(handle) -> list[(status, x1, u0)]``.
    """

    def __init__(self, executor, start_states: np.ndarray, memory_budget: int | None = None,
                 deadline_s: float = 1e-3, queue_limit: int | None = None, clock=None):
        self.ex = executor
        self.state = np.array(start_states, dtype=np.float64, copy=True)   # [P, nx] current start states
        self.budget = memory_budget if memory_budget is not None else 1 << 62
        if self.budget < int(executor.bytes_per_request):
            raise ValueError("memory budget below one request's workspace: nothing could ever launch")
        self.deadline = deadline_s
        self.queue_limit = queue_limit
        self.clock = clock or WallClock()

    def run(self, requests: list) -> ServeReport:
        reqs = sorted(requests, key=lambda r: r.arrival)
        pending = list(reqs)
        pending.reverse()                        # pop() from the end = earliest arrival
        # Waiting requests: a FIFO per instance, and a FIFO of the instances
        # that have a waiting request and nothing in flight (O(1) per request).
        queues: dict = {}
        ready: deque = deque()
        in_ready: set = set()
        n_waiting = 0
        inflight: list = []
        busy = set()
        bytes_inflight = 0
        done, rejected = [], []
        launches, launched_reqs, max_inflight = 0, 0, 0
        free_slots = list(range(self.ex.slots))
        per_req = int(self.ex.bytes_per_request)

        def make_ready(inst):
            if inst not in busy and inst not in in_ready and queues.get(inst):
                ready.append(inst)
                in_ready.add(inst)

        while pending or n_waiting or inflight:
            now = self.clock.now()
            # 1. Admit every request that has arrived.
            while pending and pending[-1].arrival <= now:
                r = pending.pop()
                if self.queue_limit is not None and n_waiting >= self.queue_limit:
                    rejected.append(r)
                else:
                    queues.setdefault(r.instance, deque()).append(r)
                    n_waiting += 1
                    make_ready(r.instance)
            # 2. Retire finished launches (results become host-visible now).
            still = []
            for L in inflight:
                if self.ex.poll(L.handle):
                    t_done = self.clock.now()
                    for r, (status, x1, u0) in zip(L.reqs, self.ex.finish(L.handle)):
                        self.state[r.instance] = x1          # the plant follows the plan
                        done.append(Completion(r.rid, r.instance, r.arrival, L.launched, t_done, int(status),
                                               np.asarray(x1), np.asarray(u0)))
                        busy.discard(r.instance)
                        make_ready(r.instance)
                    bytes_inflight -= L.nbytes
                    free_slots.append(L.handle_slot)
                else:
                    still.append(L)
            inflight = still
            # 3. Launch the oldest request of every ready instance while a slot is free.
            if free_slots and ready:
                room = (self.budget - bytes_inflight) // max(per_req, 1)
                take = min(len(ready), self.ex.capacity, room)
                if take > 0:
                    batch = []
                    for _ in range(take):
                        inst = ready.popleft()
                        in_ready.discard(inst)
                        batch.append(queues[inst].popleft())
                        busy.add(inst)
                    n_waiting -= take
                    slot = free_slots.pop()
                    xs = np.stack([self.state[r.instance] for r in batch])
                    t_l = self.clock.now()
                    h = self.ex.launch(slot, batch, xs)
                    L = _Launch(h, batch, t_l, per_req * take)
                    L.handle_slot = slot
                    inflight.append(L)
                    bytes_inflight += L.nbytes
                    launches += 1
                    launched_reqs += take
                    max_inflight = max(max_inflight, len(inflight))
                    continue
            # 4. Nothing to do right now: wait for the next arrival or completion.
            if not inflight and pending and not (free_slots and ready):
                self.clock.wait_until(pending[-1].arrival)
            elif hasattr(self.clock, "idle"):
                self.clock.idle(inflight, pending)
        return ServeReport(done, rejected, self.deadline, launches, launched_reqs / max(launches, 1), max_inflight)


class NativeScheduler:
    """The same continuous-batching policy run natively (``gato_serve_run``).

    Per-instance FIFOs, the ready queue of idle instances, the queue limit and
    the memory budget behave as in :class:`Scheduler`; the loop, the clock
    (steady clock, seconds from the start of the call) and the launch
    contexts are all in the C library, so the host overhead per launch is a
    few microseconds instead of Python's tens. The start states are updated in
    place as results arrive, exactly as :class:`Scheduler` does.
    """

    def __init__(self, batch, start_states: np.ndarray, slots: int = 4, n_iters: int = 1,
                 memory_budget: int | None = None, deadline_s: float = 1e-3, queue_limit: int | None = None):
        from . import workspace_bytes
        self.b = batch
        self.slots = int(slots)
        self.n_iters = int(n_iters)
        self.budget = int(memory_budget or 0)
        if 0 < self.budget < workspace_bytes(batch.n_max, batch.N_max, batch.params):
            raise ValueError("memory budget below one request's workspace: nothing could ever launch")
        self.deadline = deadline_s
        self.queue_limit = int(queue_limit or 0)
        self.state = np.zeros((batch.M, batch.nx_max), np.float32)
        s = np.asarray(start_states, np.float32)
        self.state[:, :s.shape[1]] = s

    def run(self, requests: list) -> ServeReport:
        import ctypes as C
        from . import ST_ADMIT_REJECT, _check, lib
        reqs = sorted(requests, key=lambda r: r.arrival)
        R, nu = len(reqs), self.b.nu_max
        arrival = np.array([r.arrival for r in reqs], np.float64)
        inst = np.array([r.instance for r in reqs], np.int32)
        goal = np.zeros((R, nu), np.float32)
        for i, r in enumerate(reqs):
            goal[i, :len(r.goal)] = r.goal
        lat = np.zeros(R, np.float64)
        tl = np.zeros(R, np.float64)
        status = np.zeros(R, np.uint32)
        u0 = np.zeros((R, nu), np.float32)
        launches = C.c_int()
        p = lambda a: a.ctypes.data_as(C.c_void_p)
        _check(lib().gato_serve_run(self.b._h, self.slots, self.n_iters, R, p(arrival), p(inst), p(goal),
                                    p(self.state), self.queue_limit, self.budget, p(lat), p(tl), p(status),
                                    p(u0), C.byref(launches)))
        done, rejected = [], []
        for i, r in enumerate(reqs):
            if status[i] & ST_ADMIT_REJECT:
                rejected.append(r)
            else:
                done.append(Completion(r.rid, r.instance, r.arrival, float(tl[i]), r.arrival + float(lat[i]),
                                       int(status[i]), None, u0[i].astype(np.float64)))
        # Launch intervals (requests of one launch share its launch time) give the peak concurrency.
        spans: dict = {}
        for c in done:
            spans[c.launched] = max(spans.get(c.launched, c.done), c.done)
        events = sorted([(t, 1) for t in spans] + [(e, -1) for e in spans.values()], key=lambda x: (x[0], x[1]))
        cur = peak = 0
        for _, d in events:
            cur += d
            peak = max(peak, cur)
        n_l = max(launches.value, 1)
        return ServeReport(done, rejected, self.deadline, launches.value, len(done) / n_l, peak)


class GpuExecutor:
    """Drives the serving launch contexts of the C ABI for a pool of MPC instances.

    One ``gato_serve_ctx`` per launch slot: its own HIP stream (default
    priority), completion event and pinned staging. A launch writes the
    requests into the pinned inputs and makes one native call that enqueues the
    input copy, the fused SQP kernel over the requested instances (warm start
    shifted one knot) and the copy back of each request's next state x1, first
    control u0 and statistics; completion is an event query.
    """

    def __init__(self, batch, slots: int = 4, n_iters: int = 1):
        from . import ServeContext, workspace_bytes
        self.b = batch
        self.slots = slots
        self.capacity = batch.M
        self.n_iters = n_iters
        self.bytes_per_request = workspace_bytes(batch.n_max, batch.N_max, batch.params)
        self.ctx = [ServeContext(batch, batch.M, n_iters) for _ in range(slots)]
        self.nx, self.nu = batch.nx_max, batch.nu_max

    def launch(self, slot: int, reqs: list, xs: np.ndarray):
        c = self.ctx[slot]
        R = len(reqs)
        c.slots[:R] = [r.instance for r in reqs]
        c.xs[:R, :xs.shape[1]] = xs
        for i, r in enumerate(reqs):
            c.goal[i, :len(r.goal)] = r.goal
        c.submit(R, shift=1)
        return slot

    def poll(self, slot: int) -> bool:
        return self.ctx[slot].done()

    def finish(self, slot: int):
        c = self.ctx[slot]
        R = c.n
        status = np.bitwise_or.reduce(c.stats["status"][:R], axis=1)
        x1 = c.x1[:R].astype(np.float64)
        u0 = c.u0[:R].astype(np.float64)
        return [(status[r], x1[r], u0[r]) for r in range(R)]

    def close(self):
        for c in self.ctx:
            c.close()
