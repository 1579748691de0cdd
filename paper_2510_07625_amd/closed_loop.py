"""Closed-loop MPC batch on the device.

Every control tick re-solves every instance from its plant state, warm-started
from the instance's previous plan shifted one knot (the experiments of Sec. IV
warm-start each control step from the previous solution), applies the plan's
first control plus any disturbance torque to the plant, and advances the plant
one control period with RK4 sub-steps (Sec. IV-E simulates the plant at 1 kHz
with RK4). All work is stream-ordered on the device; the host only enqueues.
"""
from __future__ import annotations

from dataclasses import dataclass, field


@dataclass
class ClosedLoopRun:
    states: object            # [ticks + 1, M, nx_max] plant states (device)
    controls: object          # [ticks, M, nu_max] applied controls, disturbance excluded (device)
    tick_ms: list             # device time per tick (HIP events), ms
    records: dict = field(default_factory=dict)   # tick -> dict of host arrays (see run)
    solve_ms: list = field(default_factory=list)  # device time of each tick's serving step (the solver kernel), ms
    pcg_iters: int = 0        # PCG iterations over all solves and ticks (with count_pcg)


def run(batch, x0, goal, ticks: int, n_iters: int = 3, h: float | None = None, substeps: int = 10,
        disturbance=None, record_ticks=(), timing: bool = True, reference=None,
        count_pcg: bool = False) -> ClosedLoopRun:
    """Runs `ticks` control ticks over all M instances of `batch`.

    x0 [M, nx_max] and goal [M, nu_max] are device tensors. disturbance(tick)
    returns a [M, nu_max] device torque added at the plant (or None).
    reference(tick), for batches with a tip tracking term, returns the tick's
    reference tip positions [M, N_max, 3] (device): the horizon moves with the
    clock. For the ticks in record_ticks the run keeps, on the host, the
    instances' plans and PCG multipliers before the tick (X_prev, U_prev,
    lam_prev), the plant state (xs),
    the new plans (X, U), the per-iteration statistics and the reference
    (pref), so that the tick can be replayed. The batch's resident
    trajectories are the warm start of the first tick. With count_pcg the PCG
    iterations of every solve are summed on the device (for FLOP accounting).
    """
    import torch
    from . import STATS_DTYPE, Batch
    M, N, nx, nu = batch.M, batch.N_max, batch.nx_max, batch.nu_max
    h = float(h if h is not None else 0.01)
    dev = x0.device
    slots = torch.arange(M, dtype=torch.int32, device=dev)
    states = torch.empty((ticks + 1, M, nx), dtype=torch.float32, device=dev)
    controls = torch.empty((ticks, M, nu), dtype=torch.float32, device=dev)
    states[0].copy_(x0)
    Xo = torch.empty((M, N, nx), dtype=torch.float32, device=dev)
    Uo = torch.empty((M, N - 1, nu), dtype=torch.float32, device=dev)
    st = torch.zeros(M * n_iters * STATS_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    tau = torch.empty((M, nu), dtype=torch.float32, device=dev)
    rec_set = set(int(t) for t in record_ticks)
    records = {}
    evs = []
    pcg_total = torch.zeros((), dtype=torch.int64, device=dev)
    # pcg_iters is the fourth 32-bit word of each 24-byte statistics record.
    assert STATS_DTYPE.itemsize == 24 and STATS_DTYPE.fields["pcg_iters"][1] == 12
    for t in range(ticks):
        if t in rec_set:
            Xp, Up = batch.get_trajectories()
            Lp = batch.get_multipliers()
        ref = reference(t) if reference is not None else None
        if timing:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
        if ref is not None:
            batch.set_tip_reference(ref)
        batch.serve_step(slots, states[t], goal, n_iters=n_iters, shift=1, Xout=Xo, Uout=Uo, d_stats=st)
        if timing:
            em = torch.cuda.Event(enable_timing=True)
            em.record()
        if count_pcg:
            pcg_total += st.view(torch.int32).view(-1, 6)[:, 3].sum()
        controls[t].copy_(Uo[:, 0])
        tau.copy_(controls[t])
        if disturbance is not None:
            d = disturbance(t)
            if d is not None:
                tau.add_(d)
        batch.plant_step(states[t], tau, h=h, substeps=substeps, xn=states[t + 1])
        if timing:
            e1.record()
            evs.append((e0, em, e1))
        if t in rec_set:
            records[t] = dict(X_prev=Xp.cpu().numpy(), U_prev=Up.cpu().numpy(), lam_prev=Lp.cpu().numpy(),
                              xs=states[t].cpu().numpy(),
                              X=Xo.cpu().numpy(), U=Uo.cpu().numpy(), stats=Batch.decode_stats(st, M, n_iters),
                              pref=None if ref is None else ref.cpu().numpy())
    torch.cuda.synchronize()
    tick_ms = [a.elapsed_time(c) for a, _, c in evs]
    solve_ms = [a.elapsed_time(m) for a, m, _ in evs]
    return ClosedLoopRun(states, controls, tick_ms, records, solve_ms, int(pcg_total.item()))
