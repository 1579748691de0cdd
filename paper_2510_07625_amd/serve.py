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

The executor does the device work; :class:`GpuExecutor` drives the C ABI
(``gato_serve_step`` on one HIP stream per launch slot). Any object with the
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


class GpuExecutor:
    """Drives ``gato_serve_step`` for a pool of MPC instances.

    One HIP stream (default priority) and one set of pinned staging buffers
    per launch slot; a launch is H2D of slots/start states/goals, the fused
    SQP kernel over the requested instances, and D2H of the per-request
    trajectories and statistics, all on the slot's stream.
    """

    def __init__(self, batch, slots: int = 4, n_iters: int = 1, base_goals: np.ndarray | None = None):
        import torch

        from . import STATS_DTYPE, workspace_bytes
        self.torch = torch
        self.b = batch
        self.slots = slots
        self.capacity = batch.M
        self.n_iters = n_iters
        self.bytes_per_request = workspace_bytes(batch.n_max, batch.N_max, batch.params)
        M, N, nx, nu = batch.M, batch.N_max, batch.nx_max, batch.nu_max
        self.nx, self.nu = nx, nu
        mk = lambda shape, dt=torch.float32: torch.zeros(shape, dtype=dt).pin_memory()
        dev = lambda shape, dt=torch.float32: torch.zeros(shape, dtype=dt, device="cuda")
        self.st = []
        for _ in range(slots):
            self.st.append(dict(
                stream=torch.cuda.Stream(), event=torch.cuda.Event(),
                h_slots=mk((M,), torch.int32), h_xs=mk((M, nx)), h_goal=mk((M, nu)),
                d_slots=dev((M,), torch.int32), d_xs=dev((M, nx)), d_goal=dev((M, nu)),
                d_X=dev((M, N, nx)), d_U=dev((M, N - 1, nu)),
                d_stats=dev((M * n_iters * STATS_DTYPE.itemsize,), torch.uint8),
                h_X=mk((M, N, nx)), h_U=mk((M, N - 1, nu)),
                h_stats=mk((M * n_iters * STATS_DTYPE.itemsize,), torch.uint8), n=0))
        self.stats_dtype = STATS_DTYPE

    def launch(self, slot: int, reqs: list, xs: np.ndarray):
        torch = self.torch
        s = self.st[slot]
        R = len(reqs)
        s["n"] = R
        inst = np.array([r.instance for r in reqs], dtype=np.int32)
        s["h_slots"][:R] = torch.from_numpy(inst)
        s["h_xs"][:R, :xs.shape[1]] = torch.from_numpy(xs.astype(np.float32))
        g = np.stack([r.goal for r in reqs]).astype(np.float32)
        s["h_goal"][:R, :g.shape[1]] = torch.from_numpy(g)
        # Every re-solve shifts the instance's previous solution by one knot
        # (harmless for the constant initial guess).
        shift = 1
        with torch.cuda.stream(s["stream"]):
            s["d_slots"][:R].copy_(s["h_slots"][:R], non_blocking=True)
            s["d_xs"][:R].copy_(s["h_xs"][:R], non_blocking=True)
            s["d_goal"][:R].copy_(s["h_goal"][:R], non_blocking=True)
            self.b.serve_step(s["d_slots"][:R], s["d_xs"][:R], s["d_goal"][:R], n_iters=self.n_iters, shift=shift,
                              Xout=s["d_X"][:R], Uout=s["d_U"][:R], d_stats=s["d_stats"], stream=s["stream"])
            s["h_X"][:R].copy_(s["d_X"][:R], non_blocking=True)
            s["h_U"][:R].copy_(s["d_U"][:R], non_blocking=True)
            s["h_stats"].copy_(s["d_stats"], non_blocking=True)
            s["event"].record(s["stream"])
        return slot

    def poll(self, slot: int) -> bool:
        return self.st[slot]["event"].query()

    def finish(self, slot: int):
        s = self.st[slot]
        R = s["n"]
        X = s["h_X"][:R].numpy()
        U = s["h_U"][:R].numpy()
        st = np.frombuffer(s["h_stats"].numpy().tobytes(), dtype=self.stats_dtype)[:R * self.n_iters]
        status = st["status"].reshape(R, self.n_iters).max(axis=1)
        return [(status[r], X[r, 1].astype(np.float64), U[r, 0].astype(np.float64)) for r in range(R)]
