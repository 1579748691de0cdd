"""Long task-space solves (tip tracking, 6-7 DoF, N > 64) on four workgroups,
against the FP64 oracle.

Such a solve has no one-workgroup kernel. Each of four parts forms the tip
terms, the factors L_k of the dense joint blocks and the rewritten QP
(y_k = T_k^-1 x_k) of its own 32 knots and of the knots next to them, and the
parts share the PCG through device memory (the part-local split). The oracle
solves the dense-Q_k QP as Eq. (5) is written. Bars: with the GPU's accepted
steps replayed, trajectories within 1e-4 of the exact oracle (Riccati mode,
pinned against LAPACK) at PCG tolerance 1e-8, no exchange time-out; PCG counts
of the congruent systems within 2% of the oracle's dense-Q PCG at tolerance
1e-5; graph replay identical to the eager launch; the limits reported.
"""
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


def _solve(solves, p):
    b = g.Batch.from_solves(solves, p)
    assert b.task
    xs, goal, X, U = g.pack_inputs(solves)
    st = b.solve(xs, goal, X, U)
    out = X.cpu().numpy().astype(np.float64), U.cpu().numpy().astype(np.float64), st
    b.close()
    return out


def _replay(s, Xg, Ug, st, iters, kkt_mode=2, pcg_tol=1e-6):
    ref = oracle.sqp(s, oracle.Params(sqp_iters=iters, kkt_mode=kkt_mode, pcg_tol=pcg_tol, pcg_max_iter=8000),
                     alpha_replay=st["alpha"].astype(np.float64))
    n, N = s.n, s.N
    ex = np.abs(Xg[:N, :2 * n] - ref.X).max() / np.abs(ref.X).max()
    eu = np.abs(Ug[:N - 1, :n] - ref.U).max() / np.abs(ref.U).max()
    return ex, eu, ref


# N = 65 and 97: the last part owns one knot (65: the fourth part owns none).
@pytest.mark.parametrize("n,N", [(7, 128), (6, 100), (7, 65), (6, 97)])
def test_long_task_space_solves_match_the_oracle(n, N):
    _say(f"task split n={n} N={N}")
    solves = [w.figure8_solve(21, i, n=n, N=N) for i in range(2)] + [w.figure8_solve(21, 2, n=7, N=32)]
    iters = 5
    p = g.Params(sqp_iters=iters, pcg_tol=1e-8, pcg_max_iter=8000)
    Xg, Ug, st = _solve(solves, p)
    assert not (st["status"] & (g.ST_NONFINITE | g.ST_EXCHANGE | g.ST_PCG_MAXITER)).any(), st["status"]
    for i, s in enumerate(solves):
        ex, eu, ref = _replay(s, Xg[i], Ug[i], st[i], iters)
        print(f"solve {i} (n={s.n}, N={s.N}): traj err X {ex:.2e} U {eu:.2e}; pcg its {st[i]['pcg_iters'].tolist()}")
        assert ex <= 1e-4 and eu <= 1e-4, (i, ex, eu)
        assert st[i]["merit"][-1] < st[i]["merit0"][0]
        # The merit at the start of every iteration, summed over the parts (tip term included).
        for it, L in enumerate(ref.logs):
            assert abs(st[i]["merit0"][it] - L["merit0"]) <= 2e-4 * abs(L["merit0"]) + 1e-4, (i, it)


def test_long_task_space_pcg_counts_match_the_dense_system():
    # From the same iterate and a zero start, the split PCG on the rewritten
    # system needs the oracle's dense-Q PCG count at the same tolerance, up to
    # rounding: a wrong halo row, factor or preconditioner block would change it.
    _say("task split pcg counts")
    solves = [w.figure8_solve(22, i, n=7, N=128) for i in range(3)]
    p = g.Params(sqp_iters=1, pcg_tol=1e-5, pcg_max_iter=8000)
    Xg, Ug, st = _solve(solves, p)
    for i, s in enumerate(solves):
        _, _, ref = _replay(s, Xg[i], Ug[i], st[i], 1, kkt_mode=1, pcg_tol=1e-5)
        a, b_ = int(st[i]["pcg_iters"][0]), int(ref.logs[0]["pcg_iters"])
        print(f"solve {i}: gpu {a}, oracle {b_}")
        assert abs(a - b_) <= max(2, 0.02 * b_), (i, a, b_)


def test_long_task_space_graph_replay_equals_eager():
    # gato_step_graph builds the split launch as a cooperative graph node;
    # every replay (eager launches in between) equals the eager launch bit for bit.
    _say("task split graph replay")
    shapes = [(7, 128), (6, 80), (7, 32), (3, 100), (6, 16)]
    solves = [w.figure8_solve(23, i, n=n, N=N) for i, (n, N) in enumerate(shapes)]
    p = g.Params(sqp_iters=2, pcg_tol=1e-7, pcg_max_iter=8000)
    b = g.Batch.from_solves(solves, p)
    xs, goal, X0, U0 = g.pack_inputs(solves)
    X, U = torch.empty_like(X0), torch.empty_like(U0)
    st = b.stats_buffer(2)

    def run(graph):
        X.copy_(X0)
        U.copy_(U0)
        b.reset_warm_start()
        b.step(xs, goal, X, U, 2, st, graph=graph)
        torch.cuda.synchronize()
        return (X.cpu().numpy().copy(), U.cpu().numpy().copy(), b.get_multipliers().cpu().numpy(),
                g.Batch.decode_stats(st, b.M, 2))

    ref = run(False)
    assert not (ref[3]["status"] & (g.ST_EXCHANGE | g.ST_NONFINITE)).any()
    for _ in range(3):
        for a_, b_ in zip(ref, run(True)):
            np.testing.assert_array_equal(a_, b_)
        for a_, b_ in zip(ref, run(False)):
            np.testing.assert_array_equal(a_, b_)
    b.close()


def test_long_task_space_limits_are_reported():
    _say("task split limits")
    long = [w.figure8_solve(24, i, n=7, N=128) for i in range(2)]
    with pytest.raises(g.GatoError):
        g.Batch.from_solves(long, g.Params(schur_fp64=0))      # the part-local form is FP64
    solves = long + [w.figure8_solve(24, 2, n=7, N=32)]
    b = g.Batch.from_solves(solves)
    with pytest.raises(g.GatoError):
        b.set_split(1)                                           # no one-workgroup kernel
    with pytest.raises(g.GatoError):
        b.set_mapping(7, 32, 4)
    b.set_mapping(7, 128, 4)                                     # its only mapping
    xs, goal, X, U = g.pack_inputs(solves)
    buckets = b.autotune(xs, goal, X, U, n_iters=1, reps=1)
    assert {(x["N"], x["kpt"]) for x in buckets} == {(128, 4), (32, 1)} or \
        {(x["N"], x["kpt"]) for x in buckets} == {(128, 4), (32, 2)}
    slots = torch.arange(len(solves), dtype=torch.int32, device="cuda")
    with pytest.raises(g.GatoError):
        b.serve_step(slots, xs, goal)
    b.close()


def test_long_task_space_batch_beyond_one_launch_runs_in_ranges():
    # 70 long solves need 280 workgroups at once, more than the device holds:
    # the step runs as consecutive cooperative launches of whole solves, eagerly
    # and as graph nodes. Solves are independent, so every solve's result equals
    # the same solve's in a batch of four bit for bit, and graph replays equal
    # the eager launches.
    _say("task split beyond one launch")
    distinct = [w.figure8_solve(25, i, n=7, N=128) for i in range(4)]
    many = [w.figure8_solve(25, i % 4, n=7, N=128) for i in range(70)]
    p = g.Params(sqp_iters=2, pcg_tol=1e-7, pcg_max_iter=8000)

    def run(solves, graph):
        b = g.Batch.from_solves(solves, p)
        xs, goal, X, U = g.pack_inputs(solves)
        st = b.stats_buffer(p.sqp_iters)
        b.reset_warm_start()
        b.step(xs, goal, X, U, p.sqp_iters, st, graph=graph)
        torch.cuda.synchronize()
        out = X.cpu().numpy(), U.cpu().numpy(), g.Batch.decode_stats(st, len(solves), p.sqp_iters)
        b.close()
        return out

    Xs, Us, ss = run(distinct, False)
    for graph in (False, True):
        X, U, st = run(many, graph)
        assert not (st["status"] & (g.ST_EXCHANGE | g.ST_NONFINITE)).any()
        for i in range(len(many)):
            np.testing.assert_array_equal(X[i], Xs[i % 4])
            np.testing.assert_array_equal(U[i], Us[i % 4])
            np.testing.assert_array_equal(st["pcg_iters"][i], ss["pcg_iters"][i % 4])


def test_full_size_uneven_task_batch_step_by_step():
    # The uneven task-space launch of the benchmark: 128 solves of 3-7 DoF and
    # 16-128 knots tracking figure-8s (22 long ones split), PCG tolerance 1e-5,
    # 10 SQP iterations taken one per call. Each GPU step of the sampled
    # solves (every long bucket, and the slowest-PCG long solve), from the
    # GPU's own iterate, must match the exact step of that iterate within
    # max(1e-4, 3 e_m), e_m the error of the FP64 method's own PCG at the same
    # tolerance from the same (zero) start.
    _say("task uneven full size, step by step")
    M, iters = 128, 10
    solves = w.figure8_uneven_batch(0, M=M)
    p = g.Params(sqp_iters=iters, pcg_tol=1e-5, pcg_max_iter=1000, warm_lambda=0)
    b = g.Batch.from_solves(solves, p)
    xs, goal, X, U = g.pack_inputs(solves)
    st_buf = b.stats_buffer(1)
    Xs, Us, sts = [X.cpu().numpy().astype(np.float64)], [U.cpu().numpy().astype(np.float64)], []
    for _ in range(iters):
        b.step(xs, goal, X, U, 1, st_buf)
        torch.cuda.synchronize()
        sts.append(g.Batch.decode_stats(st_buf, M, 1)[:, 0])
        Xs.append(X.cpu().numpy().astype(np.float64))
        Us.append(U.cpu().numpy().astype(np.float64))
    b.close()
    st = np.stack(sts, axis=1)
    assert not (st["status"] & (g.ST_NONFINITE | g.ST_PCG_MAXITER | g.ST_EXCHANGE)).any()
    long = [i for i, s in enumerate(solves) if s.n >= 6 and s.N > 64]
    pcg = st["pcg_iters"].sum(axis=1)
    idx = sorted({long[0], long[-1], max(long, key=lambda i: pcg[i])} |
                 {next(i for i in long if (solves[i].n, solves[i].N) == key)
                  for key in {(solves[i].n, solves[i].N) for i in long}})
    worst = 0.0
    for i in idx:
        s = solves[i]
        n, N = s.n, s.N
        for it in range(iters):
            x0, u0 = Xs[it][i, :N, :2 * n], Us[it][i, :N - 1, :n]
            x1, u1 = Xs[it + 1][i, :N, :2 * n], Us[it + 1][i, :N - 1, :n]
            al = float(st[i, it]["alpha"])
            dXe, dUe, _, _, _ = oracle.qp_step(s, x0, u0, mode=2)
            dXm, dUm, _, _, _ = oracle.qp_step(s, x0, u0, mode=1, pcg_tol=1e-5, pcg_max_iter=8000)
            sx, su = np.abs(x0 + al * dXe).max(), np.abs(u0 + al * dUe).max()
            e = max(np.abs(x1 - (x0 + al * dXe)).max() / sx, np.abs(u1 - (u0 + al * dUe)).max() / su)
            e_m = al * max(np.abs(dXm - dXe).max() / sx, np.abs(dUm - dUe).max() / su)
            worst = max(worst, e / max(1e-4, 3 * e_m))
            assert e <= max(1e-4, 3 * e_m), (i, n, N, it, e, e_m)
    print(f"{len(idx)} long solves sampled; worst step error / bound: {worst:.2f}")
