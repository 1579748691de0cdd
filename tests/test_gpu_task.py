"""Task-space (tip tracking) variant on the GPU against the FP64 oracle.

The oracle solves the QP with the dense state Hessian blocks exactly as
Eq. (5) is written (dense LU of the KKT matrix, or its Schur + PCG mode); the
GPU rewrites each knot in the variables y = T^-1 x, T^T Q T diagonal. The two
are the same linear algebra, so the bars are those of the joint-space tests:
trajectories within 1e-4 of the exact oracle after the SQP iterations (with
the GPU's accepted steps replayed), and the PCG iteration counts of the
congruent systems equal to those of the oracle's PCG up to rounding.
"""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
import workload as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2510_07625_amd as g  # noqa: E402


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _run(solves, params):
    b = g.Batch.from_solves(solves, params)
    assert b.task
    xs, goal, X, U = g.pack_inputs(solves)
    st = b.solve(xs, goal, X, U)
    out = X.cpu().numpy().astype(np.float64), U.cpu().numpy().astype(np.float64), st
    b.close()
    return out


def _replay(s, Xg, Ug, st, p, kkt_mode=0, pcg_tol=1e-6):
    alphas = st["alpha"].astype(np.float64)
    ref = oracle.sqp(s, oracle.Params(sqp_iters=p.sqp_iters, kkt_mode=kkt_mode, pcg_tol=pcg_tol,
                                      pcg_max_iter=4000), alpha_replay=alphas)
    n, N = s.n, s.N
    ex = np.abs(Xg[:N, :2 * n] - ref.X).max() / np.abs(ref.X).max()
    eu = np.abs(Ug[:N - 1, :n] - ref.U).max() / np.abs(ref.U).max()
    return ex, eu, ref


# (7, 33): two knots per lane group with a single knot in the second pass.
@pytest.mark.parametrize("n,N,M", [(7, 32, 3), (6, 48, 2), (7, 64, 1), (3, 100, 2), (7, 2, 2), (7, 33, 2)])
def test_task_space_trajectory_parity(n, N, M):
    _say(f"task sqp n={n} N={N} M={M}")
    solves = [w.figure8_solve(3, i, n=n, N=N) for i in range(M)]
    p = g.Params(sqp_iters=6, pcg_tol=1e-8, pcg_max_iter=2000)
    Xg, Ug, st = _run(solves, p)
    for i, s in enumerate(solves):
        ex, eu, ref = _replay(s, Xg[i], Ug[i], st[i], p, kkt_mode=0 if N <= 32 else 2)
        print(f"solve {i}: traj err X {ex:.2e} U {eu:.2e}; pcg its {st[i]['pcg_iters'].tolist()}")
        assert ex <= 1e-4 and eu <= 1e-4, (i, ex, eu)
        assert not (st[i]["status"] & g.ST_NONFINITE).any()
        assert st[i]["merit"][-1] < st[i]["merit0"][0]
        # The merit the kernel saw at the start of every iteration is the oracle's (tip term included).
        for it, L in enumerate(ref.logs):
            assert abs(st[i]["merit0"][it] - L["merit0"]) <= 2e-4 * abs(L["merit0"]) + 1e-4, (it, i)


def test_pcg_iterations_of_the_rewritten_system_match_the_dense_one():
    # The stair preconditioner transforms with the Schur complement under the
    # change of variables, so from the same iterate and the same (zero) start
    # PCG needs the same number of iterations as the oracle's PCG on the
    # dense-Q_k system at the same tolerance, up to rounding (the GPU's QP data
    # are FP32). A wrong preconditioner would multiply the count; one rounded
    # to FP32 already adds tens of per cent on these systems.
    _say("task pcg iteration counts")
    solves = [w.figure8_solve(5, i, n=7, N=32) for i in range(4)]
    p = g.Params(sqp_iters=1, pcg_tol=1e-5, pcg_max_iter=2000)
    Xg, Ug, st = _run(solves, p)
    for i, s in enumerate(solves):
        _, _, ref = _replay(s, Xg[i], Ug[i], st[i], p, kkt_mode=1, pcg_tol=1e-5)
        a, b_ = int(st[i]["pcg_iters"][0]), int(ref.logs[0]["pcg_iters"])
        print(f"solve {i}: gpu {a}, oracle {b_}")
        assert abs(a - b_) <= max(2, 0.02 * b_), (i, a, b_)


def test_zero_tip_weights_match_the_joint_space_kernel():
    _say("task kernel with zero tip weights vs joint-space kernel")
    solves = [w.figure8_solve(6, i, n=7, N=32) for i in range(3)]
    for s in solves:
        s.Wee = np.zeros(3)
        s.WeeN = np.zeros(3)
    plain = [w.figure8_solve(6, i, n=7, N=32) for i in range(3)]
    for s in plain:
        s.Wee = s.WeeN = s.pref = None
    p = g.Params(sqp_iters=4, pcg_tol=1e-8)
    Xa, Ua, sa = _run(solves, p)
    b = g.Batch.from_solves(plain, p)
    assert not b.task
    xs, goal, X, U = g.pack_inputs(plain)
    sb = b.solve(xs, goal, X, U)
    Xb, Ub = X.cpu().numpy().astype(np.float64), U.cpu().numpy().astype(np.float64)
    b.close()
    np.testing.assert_array_equal(sa["alpha"], sb["alpha"])
    assert np.abs(Xa - Xb).max() <= 1e-5 * np.abs(Xb).max()
    assert np.abs(Ua - Ub).max() <= 1e-5 * np.abs(Ub).max()


def test_full_size_figure8_batch_step_by_step():
    # The task-space launch of the benchmark: M = 256 7-DoF chains tracking
    # figure-8s, N = 32, PCG tolerance 1e-5, 10 SQP iterations, here taken one
    # iteration per call so that every iterate can be checked. Each GPU step,
    # from the GPU's own iterate, must match the exact (FP64 Riccati) step of
    # that iterate within max(1e-4, 3 e_m), e_m the error of the oracle's own
    # PCG at the same tolerance from the same (zero) start: how far a PCG
    # solve stopped at a given residual is from the solution depends on where
    # it started, so both sides start from zero here. (Whole trajectories
    # after many iterations at this tolerance measure the SQP's sensitivity
    # to the PCG error, which the FP64 method shares: trajectories are checked
    # at tight tolerance above.)
    _say("task full size M=256, step by step")
    M, iters = 256, 10
    solves = w.figure8_batch(0, M)
    p = g.Params(sqp_iters=iters, pcg_tol=1e-5, pcg_max_iter=1000, warm_lambda=0)
    b = g.Batch.from_solves(solves, p)
    xs, goal, X, U = g.pack_inputs(solves)
    st_buf = b.stats_buffer(1)
    Xs, Us, sts = [X.cpu().numpy().astype(np.float64)], [U.cpu().numpy().astype(np.float64)], []
    for it in range(iters):
        b.step(xs, goal, X, U, 1, st_buf)
        torch.cuda.synchronize()
        sts.append(g.Batch.decode_stats(st_buf, M, 1)[:, 0])
        Xs.append(X.cpu().numpy().astype(np.float64))
        Us.append(U.cpu().numpy().astype(np.float64))
    b.close()
    st = np.stack(sts, axis=1)
    assert not (st["status"] & (g.ST_NONFINITE | g.ST_PCG_MAXITER)).any()
    # (The line search always steps, so a solve may end above its start.)
    down = st["merit"][:, -1] < st["merit0"][:, 0]
    print(f"merit lowered in {int(down.sum())} of {M} solves")
    assert down.mean() >= 0.95
    worst = 0.0
    for i in (0, 128, 255):
        s = solves[i]
        for it in range(iters):
            x0, u0, al = Xs[it][i], Us[it][i], float(st[i, it]["alpha"])
            dXe, dUe, _, _, _ = oracle.qp_step(s, x0, u0, mode=2)
            dXm, dUm, _, _, _ = oracle.qp_step(s, x0, u0, mode=1, pcg_tol=1e-5, pcg_max_iter=4000)
            sx, su = np.abs(x0 + al * dXe).max(), np.abs(u0 + al * dUe).max()
            e = max(np.abs(Xs[it + 1][i] - (x0 + al * dXe)).max() / sx,
                    np.abs(Us[it + 1][i] - (u0 + al * dUe)).max() / su)
            e_m = al * max(np.abs(dXm - dXe).max() / sx, np.abs(dUm - dUe).max() / su)
            worst = max(worst, e / max(1e-4, 3 * e_m))
            assert e <= max(1e-4, 3 * e_m), (i, it, e, e_m)
    print(f"worst step error / bound: {worst:.2f}")


def test_tip_reference_is_read_per_call():
    # A new reference changes the result; the old one restores it bit for bit.
    _say("task reference update")
    solves = [w.figure8_solve(7, i, n=7, N=32) for i in range(2)]
    p = g.Params(sqp_iters=2, pcg_tol=1e-7)
    b = g.Batch.from_solves(solves, p)
    xs, goal, X0, U0 = g.pack_inputs(solves)
    outs = []
    pref = torch.from_numpy(np.stack([s.pref for s in solves]).astype(np.float32)).cuda()
    for ref in (pref, pref + 0.05, pref):
        b.set_tip_reference(ref.contiguous())
        b.reset_warm_start()
        X, U = X0.clone(), U0.clone()
        b.solve(xs, goal, X, U, stats=False)
        torch.cuda.synchronize()
        outs.append(X.cpu().numpy())
    assert np.array_equal(outs[0], outs[2])
    assert np.abs(outs[0] - outs[1]).max() > 1e-3
    b.close()


def test_task_space_restrictions_are_reported():
    _say("task restrictions")
    solves = [w.figure8_solve(8, i, n=7, N=32) for i in range(2)]
    b = g.Batch.from_solves(solves)
    with pytest.raises(g.GatoError):
        b.set_mapping(7, 32, 4)
    b.set_mapping(7, 32, 2)         # kpt 2 is compiled
    b.close()
    # Long solves (N > 64) run only split, in FP64.
    long = [w.figure8_solve(8, 0, n=7, N=128)]
    with pytest.raises(g.GatoError):
        g.Batch.from_solves(long, g.Params(schur_fp64=0))
    g.Batch.from_solves(long).close()


def test_tip_positions_match_the_oracle_kinematics():
    _say("tip positions")
    solves = [w.figure8_solve(9, i, n=n, N=N) for i, (n, N) in enumerate([(7, 32), (6, 20), (3, 9)])]
    b = g.Batch.from_solves(solves)
    xs, goal, X, U = g.pack_inputs(solves)
    rng = np.random.default_rng(9)
    Xr = X.cpu().numpy()
    Xr += rng.uniform(-1.5, 1.5, Xr.shape).astype(np.float32)
    Xd = torch.from_numpy(Xr).cuda()
    P = b.tip_positions(Xd).cpu().numpy().astype(np.float64)
    b.close()
    for i, s in enumerate(solves):
        for k in range(b.N_max):
            if k < s.N:
                ref, _ = oracle.tip(s, Xr[i, k, :s.n].astype(np.float64))
                assert np.abs(P[i, k] - ref).max() <= 2e-6 * max(1.0, np.abs(ref).max()), (i, k)
            else:
                assert not P[i, k].any()


def test_uneven_task_batch_mixed_launch_equals_grouped_and_the_oracle():
    # One mixed-shape launch over DoF {3, 6, 7} and N {16, 33, 64} runs every
    # solve through the same specialisation as its grouped launch: bitwise
    # equal results; a sampled solve against the oracle at tight tolerance.
    _say("task uneven batch: mixed vs grouped")
    shapes = [(7, 16), (3, 33), (6, 64), (7, 64), (3, 16), (6, 33), (7, 33)]
    solves = [w.figure8_solve(10, i, n=n, N=N) for i, (n, N) in enumerate(shapes)]
    p = g.Params(sqp_iters=3, pcg_tol=1e-8, pcg_max_iter=3000)
    outs = []
    for mode in (g.DISPATCH_GROUPED, g.DISPATCH_MIXED):
        b = g.Batch.from_solves(solves, p)
        b.set_dispatch(mode)
        xs, goal, X, U = g.pack_inputs(solves)
        st = b.solve(xs, goal, X, U)
        outs.append((X.cpu().numpy(), U.cpu().numpy(), st))
        b.close()
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
    X, U, st = outs[1]
    for i in (0, 2, 3):
        s = solves[i]
        ex, eu, _ = _replay(s, X[i].astype(np.float64), U[i].astype(np.float64), st[i], p,
                            kkt_mode=0 if s.N <= 32 else 2)
        assert ex <= 1e-4 and eu <= 1e-4, (i, ex, eu)
    # The autotuner picks among the compiled task-space mappings.
    b = g.Batch.from_solves(solves, p)
    xs, goal, X, U = g.pack_inputs(solves)
    buckets = b.autotune(xs, goal, X, U, n_iters=1, reps=1)
    assert all(x["kpt"] in (1, 2) for x in buckets)
    b.close()


def test_figure8_closed_loop_ticks_replay_in_the_oracle():
    # MPC on the figure-8: every tick re-solves from the plant state with the
    # reference window of the tick (the horizon moves with the clock), the
    # plan shifted one knot as warm start; sampled ticks replayed in the oracle.
    _say("figure-8 closed loop ticks")
    from paper_2510_07625_amd import closed_loop
    M, N, iters, ticks = 3, 32, 2, 8
    solves = [w.figure8_solve(11, i, n=7, N=N) for i in range(M)]
    long = [w.figure8_solve(11, i, n=7, N=N + ticks) for i in range(M)]
    path = torch.from_numpy(np.stack([s.pref for s in long]).astype(np.float32)).cuda()   # [M, N + ticks, 3]
    p = g.Params(sqp_iters=iters, pcg_tol=1e-8, pcg_max_iter=3000)
    b = g.Batch.from_solves(solves, p)
    xs, goal, X0, U0 = g.pack_inputs(solves)
    b.set_trajectories(X0, U0)
    rec = (0, 3, 7)
    run = closed_loop.run(b, xs, goal, ticks, n_iters=iters, record_ticks=rec,
                          reference=lambda t: path[:, t:t + N].contiguous())
    b.close()
    assert np.isfinite(run.states.cpu().numpy()).all()
    for t in rec:
        R = run.records[t]
        np.testing.assert_array_equal(R["pref"], path[:, t:t + N].cpu().numpy())
        for i, s in enumerate(solves):
            Xp, Up = R["X_prev"][i].astype(np.float64), R["U_prev"][i].astype(np.float64)
            Xw = Xp[np.minimum(np.arange(N) + 1, N - 1)]
            Uw = Up[np.minimum(np.arange(N - 1) + 1, N - 2)]
            st = dataclasses.replace(s, xs=R["xs"][i].astype(np.float64), pref=R["pref"][i].astype(np.float64))
            ref = oracle.sqp(st, oracle.Params(sqp_iters=iters, kkt_mode=0), X=Xw, U=Uw,
                             alpha_replay=R["stats"][i]["alpha"].astype(np.float64))
            ex = np.abs(R["X"][i] - ref.X).max() / np.abs(ref.X).max()
            eu = np.abs(R["U"][i] - ref.U).max() / np.abs(ref.U).max()
            assert ex <= 1e-4 and eu <= 1e-4, (t, i, ex, eu)
