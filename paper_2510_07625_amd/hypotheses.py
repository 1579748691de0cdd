"""Batched hypothesize-and-test over external tip forces (Sec. IV-D).

P MPC instances each carry H force hypotheses, one solve per (instance,
hypothesis) in one batch (slot p H + j): the solves of an instance differ only
in the assumed external force on the tip of the last link. Every control tick:

1. all P H solves re-solve from their instance's plant state, warm-started
   from their previous plans shifted one knot;
2. each instance applies the first control of hypothesis 0 (its current
   estimate) to its plant, which feels the true force;
3. every hypothesis predicts the instance's next state under the applied
   control with its own force (the RK4 plant of that solve); the hypothesis
   closest to the measured next state (Euclidean norm over the state) becomes
   the instance's estimate;
4. the hypotheses are re-centred on the estimate: hypothesis j is the estimate
   plus sigma r_j d_j, with d_j fixed directions uniform on the sphere and r_j
   spread over (0, 1] (hypothesis 0: the estimate itself), so that both the
   direction and the magnitude are explored around it.

Steps 3-4 run in the library (gato_select_hypotheses): the estimates and the
hypotheses' forces stay on the device, and a tick is enqueued without any host
synchronisation.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def offsets(H: int, seed: int = 0) -> np.ndarray:
    """[H, 3] hypothesis offsets of unit scale: row 0 zero, rows j > 0 direction
    uniform on the sphere times a radius spread over (0, 1]."""
    rng = np.random.default_rng([seed, H])
    out = np.zeros((H, 3))
    if H > 1:
        d = rng.normal(size=(H - 1, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        r = np.arange(1, H) / (H - 1)
        out[1:] = d * r[:, None]
    return out


@dataclass
class HypothesisRun:
    states: np.ndarray        # [ticks + 1, P, nx] plant states
    estimates: np.ndarray     # [ticks + 1, P, 3] force estimates (before each tick; last after it)
    selected: np.ndarray      # [ticks, P] selected hypothesis index
    controls: np.ndarray      # [ticks, P, nu] applied controls
    tick_ms: list


def run(batch, P: int, H: int, x0, goal, ticks: int, true_force, sigma: float = 10.0, n_iters: int = 1,
        h: float = 0.01, substeps: int = 10, seed: int = 0, f0=None) -> HypothesisRun:
    """batch holds P H solves (slot p H + j); x0 [P, nx_max] and goal [P, nu_max]
    are device tensors; true_force(tick) returns the plants' true forces [P, 3]
    (numpy); f0 [P, 3] is the initial estimate (default zero)."""
    import torch
    M = P * H
    assert batch.M == M
    dev = x0.device
    nx, nu, N = batch.nx_max, batch.nu_max, batch.N_max
    off_h = offsets(H, seed) * sigma                                 # [H, 3]
    est0 = np.zeros((P, 3)) if f0 is None else np.array(f0, np.float64).reshape(P, 3)
    batch.set_external_force((est0[:, None, :] + off_h[None, :, :]).reshape(M, 3))
    off = torch.from_numpy(off_h).to(dev)
    est = torch.from_numpy(est0.copy()).to(dev)
    slots = torch.arange(M, dtype=torch.int32, device=dev)
    inst_slots = (torch.arange(P, dtype=torch.int32, device=dev) * H).contiguous()
    Xo = torch.empty((M, N, nx), dtype=torch.float32, device=dev)
    Uo = torch.empty((M, N - 1, nu), dtype=torch.float32, device=dev)
    goal_m = goal.repeat_interleave(H, dim=0).contiguous()
    states = torch.empty((ticks + 1, P, nx), dtype=torch.float32, device=dev)
    ests = torch.empty((ticks + 1, P, 3), dtype=torch.float64, device=dev)
    sel = torch.empty((ticks, P), dtype=torch.int32, device=dev)
    ctrl = torch.empty((ticks, P, nu), dtype=torch.float32, device=dev)
    states[0].copy_(x0)
    ests[0].copy_(est)
    f_true = [torch.from_numpy(np.asarray(true_force(t), np.float32).reshape(P, 3)).to(dev) for t in range(ticks)]
    evs = []
    for t in range(ticks):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        x = states[t]
        xs_m = x.repeat_interleave(H, dim=0).contiguous()
        batch.serve_step(slots, xs_m, goal_m, n_iters=n_iters, shift=1, Xout=Xo, Uout=Uo)
        ctrl[t].copy_(Uo[::H, 0])                                      # hypothesis 0 of every instance
        batch.plant_step(x, ctrl[t], h=h, substeps=substeps, slots=inst_slots, fext=f_true[t], xn=states[t + 1])
        pred = batch.plant_step(xs_m, ctrl[t].repeat_interleave(H, dim=0).contiguous(), h=h, substeps=substeps,
                                slots=slots)                           # each solve's own hypothesis
        batch.select_hypotheses(P, H, pred, states[t + 1], off, est, sel=sel[t])
        ests[t + 1].copy_(est)
        e1.record()
        evs.append((e0, e1))
    torch.cuda.synchronize()
    tick_ms = [a.elapsed_time(b) for a, b in evs]
    return HypothesisRun(states.cpu().numpy(), ests.cpu().numpy(), sel.cpu().numpy(), ctrl.cpu().numpy(), tick_ms)


def realized_cost(run: HypothesisRun, solves_per_instance, dt_weighting: bool = False) -> np.ndarray:
    """Closed-loop stage cost actually incurred per instance, summed over the
    ticks: 1/2 (x - x_g)^T Q (x - x_g) + 1/2 u^T R u with the problem's own
    weights (x_g = [q_goal; 0]) -- the quantity each re-solve minimises."""
    P = run.states.shape[1]
    out = np.zeros(P)
    for p, s in enumerate(solves_per_instance):
        n = s.n
        xg = np.concatenate([s.qgoal, np.zeros(n)])
        d = run.states[:-1, p, :2 * n].astype(np.float64) - xg
        u = run.controls[:, p, :n].astype(np.float64)
        out[p] = 0.5 * np.sum(d * d * s.Qd) + 0.5 * np.sum(u * u * s.Rd)
    return out
