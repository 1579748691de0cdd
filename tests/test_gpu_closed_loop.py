"""Closed-loop batch on the GPU: the RK4 plant against the oracle, and ticks
replayed in the oracle from the same plant state and warm start."""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
import workload as w

from . import _parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2510_07625_amd as g  # noqa: E402
from paper_2510_07625_amd import closed_loop  # noqa: E402


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def test_plant_step_matches_the_oracle_rk4():
    _say("plant rk4")
    solves = w.uneven_batch(31, M=6, horizons=(16,))
    b = g.Batch.from_solves(solves, g.Params(sqp_iters=1))
    rng = np.random.default_rng(5)
    nx, nu = b.nx_max, b.nu_max
    x = np.zeros((6, nx), np.float32)
    tau = np.zeros((6, nu), np.float32)
    for i, s in enumerate(solves):
        x[i, :2 * s.n] = rng.uniform(-1, 1, 2 * s.n)
        tau[i, :s.n] = rng.normal(0, 3, s.n)
    order = np.array([5, 2, 0, 4, 1, 3], np.int32)        # instances through a slot map
    xd = torch.from_numpy(x[order]).cuda()
    td = torch.from_numpy(tau[order]).cuda()
    status = torch.full((6,), -1, dtype=torch.int32, device="cuda")
    xn = b.plant_step(xd, td, h=0.01, substeps=10, slots=torch.from_numpy(order).cuda(), status=status)
    xn = xn.cpu().numpy()
    assert (status.cpu().numpy() == 0).all()
    for r, i in enumerate(order):
        s = solves[i]
        ref = oracle.plant_rk4(s, x[i, :2 * s.n].astype(np.float64), tau[i, :s.n].astype(np.float64), 0.01, 10)
        np.testing.assert_allclose(xn[r, :2 * s.n], ref, rtol=2e-6, atol=2e-6)
    b.close()


def test_closed_loop_ticks_replay_in_the_oracle():
    _say("closed loop ticks")
    M, N, iters = 4, 32, 3
    solves = w.chain_batch(32, M, N=N)
    p = g.Params(sqp_iters=iters, pcg_tol=1e-7)
    b = g.Batch.from_solves(solves, p)
    xs, goal, X0, U0 = g.pack_inputs(solves)
    b.set_trajectories(X0, U0)
    rng = np.random.default_rng(9)
    kick = torch.from_numpy(rng.normal(0, 5, (M, 7)).astype(np.float32)).cuda()
    ticks, rec = 12, (0, 4, 5, 11)
    run = closed_loop.run(b, xs, goal, ticks, n_iters=iters, disturbance=lambda t: kick if t == 4 else None,
                          record_ticks=rec)
    states = run.states.cpu().numpy()
    assert np.isfinite(states).all()
    for t in rec:
        R = run.records[t]
        for i, s in enumerate(solves):
            Xp, Up = R["X_prev"][i].astype(np.float64), R["U_prev"][i].astype(np.float64)
            Xw = Xp[np.minimum(np.arange(N) + 1, N - 1)]
            Uw = Up[np.minimum(np.arange(N - 1) + 1, N - 2)]
            st = dataclasses.replace(s, xs=R["xs"][i].astype(np.float64))
            ref = oracle.sqp(st, oracle.Params(sqp_iters=iters, kkt_mode=0), X=Xw, U=Uw,
                             alpha_replay=R["stats"][i]["alpha"].astype(np.float64))
            ex = np.abs(R["X"][i] - ref.X).max() / np.abs(ref.X).max()
            eu = np.abs(R["U"][i] - ref.U).max() / np.abs(ref.U).max()
            assert ex <= 1e-4 and eu <= 1e-4, (t, i, ex, eu)
    # The plant followed the applied controls: replay two ticks of the plant in the oracle.
    ctrl = run.controls.cpu().numpy()
    for t in (3, 4):
        for i, s in enumerate(solves):
            tau = ctrl[t, i].astype(np.float64) + (kick[i].cpu().numpy().astype(np.float64) if t == 4 else 0.0)
            ref = oracle.plant_rk4(s, states[t, i].astype(np.float64), tau, 0.01, 10)
            np.testing.assert_allclose(states[t + 1, i], ref, rtol=2e-6, atol=2e-6)
    b.close()


def test_full_size_closed_loop_sampled_ticks():
    # The closed-loop benchmark's batch: 256 7-DoF N = 64 instances (seed 0),
    # 3 SQP iterations per tick at PCG tolerance 1e-5, torque impulses
    # N(0, 5^2) N m at tick 100 (the benchmark's draw), 102 ticks. At ticks 0,
    # 100 and 101, sixteen instances (evenly spread, plus the slowest and the
    # fastest PCG instance of the tick) are replayed in the same-method FP64
    # oracle from the same plant state, shifted plan and shifted multipliers
    # (bar 1e-4, valid steps); the distance to the exact solve is printed.
    _say("closed loop full size M=256 N=64")
    M, N, iters = 256, 64, 3
    solves = w.chain_batch(0, M, N=N)
    p = g.Params(sqp_iters=iters, pcg_tol=1e-5)
    b = g.Batch.from_solves(solves, p)
    xs, goal, X0, U0 = g.pack_inputs(solves)
    b.set_trajectories(X0, U0)
    rng = np.random.default_rng([0, 5])
    kick = torch.from_numpy(rng.normal(0.0, 5.0, (M, 7)).astype(np.float32)).cuda()
    rec = (0, 100, 101)
    run = closed_loop.run(b, xs, goal, 102, n_iters=iters, disturbance=lambda t: kick if t == 100 else None,
                          record_ticks=rec)
    b.close()
    assert np.isfinite(run.states.cpu().numpy()).all()
    shift_x = np.minimum(np.arange(N) + 1, N - 1)
    shift_u = np.minimum(np.arange(N - 1) + 1, N - 2)
    for t in rec:
        R = run.records[t]
        assert not (R["stats"]["status"] & (g.ST_NONFINITE | g.ST_PCG_MAXITER)).any()
        tot = R["stats"]["pcg_iters"].sum(axis=1)
        cases = []
        for i in _parity.sample_indices(M, tot, count=16):
            s = dataclasses.replace(solves[i], xs=R["xs"][i].astype(np.float64))
            cases.append(dict(s=s, Xg=R["X"][i].astype(np.float64), Ug=R["U"][i].astype(np.float64),
                              st=R["stats"][i], p_gpu=p, X0=R["X_prev"][i].astype(np.float64)[shift_x],
                              U0=R["U_prev"][i].astype(np.float64)[shift_u], lam0=R["lam_prev"][i][shift_x],
                              label=f"tick {t} instance {i}"))
        res = _parity.check_many(cases)
        _parity.report(res, f"closed loop tick {t}")
