"""Accuracy of the GPU path against the FP64 oracle on the benchmark's workloads.

A report, not a test (pytest does not collect it): run it on an MI355X as
``python tests/accuracy_report.py`` and it prints one JSON line with

* the headline launch (M = 256 7-DoF chains, N = 32, 10 SQP iterations, PCG
  tolerance 1e-5): the trajectory error of every solve against the exact
  oracle (dense KKT LU) and against the oracle running the same method (Schur
  + PCG at the same tolerance), the oracle replaying the GPU's accepted steps
  and PCG iteration counts; the FP64 method's own distance from the exact
  solve;
* every precision setting: the same trajectory error, and the KKT-solution
  error on identical QP data (the oracle's LQ data rounded once to FP32);
* the uneven batch in its three precision settings: per (DoF, N) bucket,
  sampled solves against the same-method and the exact oracle;
* the closed-loop batch: sampled ticks replayed in the oracle from the same
  plant state and warm start, and the oracle's own closed loop for 150 ticks;
* the task-space (figure-8) launch: sampled trajectories and, step by step,
  each GPU step against the exact step of the GPU's own iterate;
* the uneven batch with figure-8 tracking (long solves split): per (DoF, N)
  bucket, the same step-by-step errors.

The benchmark itself never runs the oracle (apart from its CPU-throughput
leg); these are the figures quoted beside its numbers.
"""
from __future__ import annotations

import dataclasses
import json
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workload as w  # noqa: E402

PRECISIONS = (dict(schur_fp64=1), dict(schur_fp64=0), dict(schur_fp64=0, fp64_block_inv=1),
              dict(schur_fp64=0, fp64_dot=1), dict(schur_fp64=0, fp64_block_inv=1, fp64_dot=1))


def _rel(X, U, ref_X, ref_U):
    return max(np.abs(X - ref_X).max() / np.abs(ref_X).max(), np.abs(U - ref_U).max() / np.abs(ref_U).max())


def _launch(g, torch, solves, params):
    b = g.Batch.from_solves(solves, params)
    xs, goal, X, U = g.pack_inputs(solves)
    st = b.stats_buffer(params.sqp_iters)
    b.reset_warm_start()
    b.step(xs, goal, X, U, params.sqp_iters, st)
    torch.cuda.synchronize()
    out = (X.cpu().numpy().astype(np.float64), U.cpu().numpy().astype(np.float64),
           g.Batch.decode_stats(st, len(solves), params.sqp_iters))
    b.close()
    return out


def trajectories(g, torch, solves, params, idx, exact_mode=0, replay_counts=True):
    """Sampled solves of one launch against the exact oracle and against the
    same-method FP64 oracle replaying the GPU's accepted steps and (with
    replay_counts) its PCG iteration counts. (The task-space kernel runs its
    PCG on a congruent rewritten system, whose stopping decisions in floating
    point are its own, so its comparison keeps the oracle's own counts.)"""
    X, U, st = _launch(g, torch, solves, params)

    def one(i):
        s = solves[i]
        al = st[i]["alpha"].astype(np.float64)
        common = dict(sqp_iters=params.sqp_iters, mu=params.mu, beta=params.beta, n_alpha=params.n_alpha)
        exact = oracle.sqp(s, oracle.Params(kkt_mode=exact_mode, **common), alpha_replay=al)
        same = oracle.sqp(s, oracle.Params(kkt_mode=1, pcg_tol=params.pcg_tol, warm_lambda=params.warm_lambda,
                                           pcg_max_iter=params.pcg_max_iter, **common), alpha_replay=al,
                          pcg_replay=[int(c) for c in st[i]["pcg_iters"]] if replay_counts else None)
        return (_rel(X[i], U[i], exact.X, exact.U), _rel(X[i], U[i], same.X, same.U),
                _rel(same.X, same.U, exact.X, exact.U))

    oracle.lib()
    with ThreadPoolExecutor(16) as ex:
        errs = list(ex.map(one, idx))
    e_exact, e_same, e_method = zip(*errs)
    return dict(max_rel_traj_err_vs_exact=float(max(e_exact)), max_rel_traj_err_vs_same_method=float(max(e_same)),
                median_rel_traj_err_vs_same_method=float(np.median(e_same)),
                same_method_vs_exact=float(max(e_method)), solves=len(idx),
                status_bits_set=int((st["status"] != 0).sum()))


def kkt_error(g, torch, params, n_solves=3, seed=12):
    solves = [w.chain_solve(seed, i) for i in range(n_solves)]
    n, N = solves[0].n, solves[0].N
    nx, nu, M = 2 * n, n, n_solves
    f32 = lambda a: np.asarray(a, np.float64).astype(np.float32)
    data = [{k: f32(v) for k, v in oracle.lq(s, s.X0, s.U0).items()} for s in solves]
    dev = lambda key, shape: torch.from_numpy(np.stack([d[key] for d in data]).reshape(shape)).cuda()
    b = g.Batch.from_solves(solves, params)
    dX, dU, _, its = (t.cpu().numpy() for t in b.debug_kkt(
        dev("A", (M, N - 1, nx, nx)), dev("B", (M, N - 1, nx, nu)), dev("e", (M, N - 1, nx)),
        dev("q", (M, N, nx)), dev("r", (M, N - 1, nu)), dev("c0", (M, nx))))
    b.close()
    worst = 0.0
    for i, s in enumerate(solves):
        d = {k: v.astype(np.float64) for k, v in data[i].items()}
        Qh = np.array([(s.Qd if k < N - 1 else s.QNd) for k in range(N)])
        rX, rU, _, _ = oracle.kkt_from_lq(d["A"], d["B"], d["e"], d["q"], d["r"], d["c0"], Qh, s.Rd)
        ref = np.concatenate([rX.ravel(), rU.ravel()])
        got = np.concatenate([dX[i].ravel(), dU[i].ravel()])
        worst = max(worst, float(np.abs(got - ref).max() / np.abs(ref).max()))
    return worst, int(its.max())


def closed_loop(g, torch, M=256, N=64, ticks=1000, iters=3, sample=8, oracle_ticks=150, seed=0):
    """The benchmark's closed-loop batch (same seeds and impulses), checked."""
    from paper_2510_07625_amd import closed_loop as cl
    solves = w.chain_batch(seed, M, N=N)
    b = g.Batch.from_solves(solves, g.Params(sqp_iters=iters, pcg_tol=1e-5))
    xs, goal, X0, U0 = g.pack_inputs(solves)
    b.set_trajectories(X0, U0)
    rng = np.random.default_rng([seed, 5])
    kicks = {t: torch.from_numpy(rng.normal(0.0, 5.0, (M, 7)).astype(np.float32)).cuda()
             for t in range(100, ticks, 100)}
    idx = np.linspace(0, M - 1, sample).astype(int)
    rec = sorted({0, 100, 101, ticks // 2, ticks - 1} & set(range(ticks)))
    run = cl.run(b, xs, goal, ticks, n_iters=iters, disturbance=kicks.get, record_ticks=rec)
    b.close()
    q = run.states.cpu().numpy()[:, :, :7].astype(np.float64)
    qg = np.stack([s.qgoal for s in solves])
    track = np.linalg.norm(q - qg[None], axis=2)
    errs, errs_same = [], []
    for t in rec:
        R = run.records[t]
        for i in idx:
            s = solves[i]
            Xw = R["X_prev"][i].astype(np.float64)[np.minimum(np.arange(N) + 1, N - 1)]
            Uw = R["U_prev"][i].astype(np.float64)[np.minimum(np.arange(N - 1) + 1, N - 2)]
            st = dataclasses.replace(s, xs=R["xs"][i].astype(np.float64))
            al = R["stats"][i]["alpha"].astype(np.float64)
            ref = oracle.sqp(st, oracle.Params(sqp_iters=iters, kkt_mode=2), X=Xw, U=Uw, alpha_replay=al)
            errs.append(_rel(R["X"][i], R["U"][i], ref.X, ref.U))
            lam_w = R["lam_prev"][i][np.minimum(np.arange(N) + 1, N - 1)]
            same = oracle.sqp(st, oracle.Params(sqp_iters=iters, kkt_mode=1, pcg_tol=1e-5), X=Xw, U=Uw, lam=lam_w,
                              alpha_replay=al, pcg_replay=[int(c) for c in R["stats"][i]["pcg_iters"]])
            errs_same.append(_rel(R["X"][i], R["U"][i], same.X, same.U))

    def oracle_loop(i):
        s = solves[i]
        x, X, U = s.xs.copy(), s.X0.copy(), s.U0.copy()
        out = [np.linalg.norm(x[:7] - s.qgoal)]
        for t in range(oracle_ticks):
            Xw, Uw = X[np.minimum(np.arange(N) + 1, N - 1)], U[np.minimum(np.arange(N - 1) + 1, N - 2)]
            r = oracle.sqp(dataclasses.replace(s, xs=x), oracle.Params(sqp_iters=iters, kkt_mode=2), X=Xw, U=Uw)
            X, U = r.X, r.U
            tau = U[0] + (kicks[t][i].cpu().numpy().astype(np.float64) if t in kicks else 0.0)
            x = oracle.plant_rk4(s, x, tau, 0.01, 10)
            out.append(np.linalg.norm(x[:7] - s.qgoal))
        return np.array(out)

    oracle.lib()
    with ThreadPoolExecutor(len(idx)) as ex:
        otrack = np.stack(list(ex.map(oracle_loop, idx)), axis=1)
    gtrack = track[:oracle_ticks + 1, idx]
    return dict(tick_replay_max_rel_err_vs_exact=float(max(errs)),
                tick_replay_max_rel_err_vs_same_method=float(max(errs_same)), ticks_replayed=rec,
                instances=[int(i) for i in idx],
                oracle_loop=dict(ticks=oracle_ticks, max_abs_tracking_diff_rad=float(np.abs(otrack - gtrack).max()),
                                 mean_tracking_gpu=float(gtrack.mean()), mean_tracking_oracle=float(otrack.mean())))


def task_space(g, torch, M=256, iters=10, idx=(0, 128, 255)):
    solves = w.figure8_batch(0, M)
    params = g.Params(sqp_iters=iters, pcg_tol=1e-5, pcg_max_iter=1000)
    traj = trajectories(g, torch, solves, params, idx, exact_mode=2, replay_counts=False)
    # Step by step from the GPU's own iterates (cold PCG starts on both sides).
    p1 = g.Params(sqp_iters=iters, pcg_tol=1e-5, pcg_max_iter=1000, warm_lambda=0)
    b = g.Batch.from_solves(solves, p1)
    xs, goal, X, U = g.pack_inputs(solves)
    st_buf = b.stats_buffer(1)
    worst, worst_m = 0.0, 0.0
    for it in range(iters):
        x0, u0 = X.cpu().numpy().astype(np.float64), U.cpu().numpy().astype(np.float64)
        b.step(xs, goal, X, U, 1, st_buf)
        torch.cuda.synchronize()
        st = g.Batch.decode_stats(st_buf, M, 1)[:, 0]
        x1, u1 = X.cpu().numpy().astype(np.float64), U.cpu().numpy().astype(np.float64)
        for i in idx:
            s, al = solves[i], float(st[i]["alpha"])
            dXe, dUe, _, _, _ = oracle.qp_step(s, x0[i], u0[i], mode=2)
            dXm, dUm, _, _, _ = oracle.qp_step(s, x0[i], u0[i], mode=1, pcg_tol=1e-5, pcg_max_iter=4000)
            sx, su = np.abs(x0[i] + al * dXe).max(), np.abs(u0[i] + al * dUe).max()
            worst = max(worst, np.abs(x1[i] - (x0[i] + al * dXe)).max() / sx,
                        np.abs(u1[i] - (u0[i] + al * dUe)).max() / su)
            worst_m = max(worst_m, al * max(np.abs(dXm - dXe).max() / sx, np.abs(dUm - dUe).max() / su))
    b.close()
    traj.update(step_max_rel_err_vs_exact=float(worst), step_max_rel_err_same_method=float(worst_m))
    return traj


def task_uneven(g, torch, M=128, iters=10, seed=0, per_bucket=2):
    """The uneven batch with figure-8 tip tracking (its long solves split,
    part-local), step by step from the GPU's own iterates with cold PCG starts
    on both sides, as for the task-space launch: per (DoF, N) bucket, the
    largest error of a GPU step of `per_bucket` sampled solves against the
    exact step of the same iterate, beside the FP64 method's own error (its
    PCG at the same tolerance)."""
    solves = w.figure8_uneven_batch(seed, M=M)
    buckets = {}
    for i, s in enumerate(solves):
        buckets.setdefault((s.n, s.N), []).append(i)
    idx = sorted(i for v in buckets.values() for i in v[:per_bucket])
    p1 = g.Params(sqp_iters=iters, pcg_tol=1e-5, pcg_max_iter=1000, warm_lambda=0)
    b = g.Batch.from_solves(solves, p1)
    xs, goal, X, U = g.pack_inputs(solves)
    st_buf = b.stats_buffer(1)
    err = {i: [0.0, 0.0] for i in idx}
    bits = 0
    oracle.lib()
    for it in range(iters):
        x0, u0 = X.cpu().numpy().astype(np.float64), U.cpu().numpy().astype(np.float64)
        b.step(xs, goal, X, U, 1, st_buf)
        torch.cuda.synchronize()
        st = g.Batch.decode_stats(st_buf, M, 1)[:, 0]
        bits += int((st["status"] & (g.ST_NONFINITE | g.ST_EXCHANGE | g.ST_PCG_MAXITER) != 0).sum())
        x1, u1 = X.cpu().numpy().astype(np.float64), U.cpu().numpy().astype(np.float64)

        def one(i):
            s, al = solves[i], float(st[i]["alpha"])
            n, N = s.n, s.N
            xa, ua, xb, ub = x0[i, :N, :2 * n], u0[i, :N - 1, :n], x1[i, :N, :2 * n], u1[i, :N - 1, :n]
            dXe, dUe, _, _, _ = oracle.qp_step(s, xa, ua, mode=2)
            dXm, dUm, _, _, _ = oracle.qp_step(s, xa, ua, mode=1, pcg_tol=1e-5, pcg_max_iter=8000)
            sx, su = np.abs(xa + al * dXe).max(), np.abs(ua + al * dUe).max()
            e = max(np.abs(xb - (xa + al * dXe)).max() / sx, np.abs(ub - (ua + al * dUe)).max() / su)
            e_m = al * max(np.abs(dXm - dXe).max() / sx, np.abs(dUm - dUe).max() / su)
            return i, e, e_m

        with ThreadPoolExecutor(16) as ex:
            for i, e, e_m in ex.map(one, idx):
                err[i][0] = max(err[i][0], e)
                err[i][1] = max(err[i][1], e_m)
    b.close()
    out = {f"{n}x{N}": dict(step_vs_exact=float(max(err[i][0] for i in v[:per_bucket])),
                            method_step_vs_exact=float(max(err[i][1] for i in v[:per_bucket])), count=len(v))
           for (n, N), v in sorted(buckets.items())}
    out["failure_bits_set"] = bits
    return out


def uneven(g, torch, M=128, seed=0, per_bucket=2):
    """The uneven batch of the benchmark (one mixed-shape launch, long solves
    split) in each of its precision settings: per (DoF, N) bucket, the largest
    error of `per_bucket` sampled solves against the same-method FP64 oracle
    and against the exact (Riccati) oracle."""
    solves = w.uneven_batch(seed, M=M)
    buckets = {}
    for i, s in enumerate(solves):
        buckets.setdefault((s.n, s.N), []).append(i)
    idx = sorted(i for v in buckets.values() for i in v[:per_bucket])
    out = {}
    for name, kw in (("fp64-schur", dict(schur_fp64=1)), ("fp32+fp64-inv", dict(schur_fp64=0, fp64_block_inv=1)),
                     ("fp32", dict(schur_fp64=0))):
        params = g.Params(sqp_iters=10, pcg_tol=1e-5, **kw)
        b = g.Batch.from_solves(solves, params)
        b.set_dispatch(g.DISPATCH_MIXED)
        xs, goal, X, U = g.pack_inputs(solves)
        st = b.stats_buffer(10)
        b.reset_warm_start()
        b.step(xs, goal, X, U, 10, st)
        torch.cuda.synchronize()
        X, U = X.cpu().numpy().astype(np.float64), U.cpu().numpy().astype(np.float64)
        st = g.Batch.decode_stats(st, M, 10)
        b.close()

        def one(i):
            s = solves[i]
            al = st[i]["alpha"].astype(np.float64)
            common = dict(sqp_iters=10, mu=params.mu, beta=params.beta, n_alpha=params.n_alpha)
            exact = oracle.sqp(s, oracle.Params(kkt_mode=2, **common), alpha_replay=al)
            same = oracle.sqp(s, oracle.Params(kkt_mode=1, pcg_tol=params.pcg_tol, **common), alpha_replay=al,
                              pcg_replay=[int(c) for c in st[i]["pcg_iters"]])
            n, N = s.n, s.N
            Xi, Ui = X[i, :N, :2 * n], U[i, :N - 1, :n]
            return _rel(Xi, Ui, same.X, same.U), _rel(Xi, Ui, exact.X, exact.U)

        oracle.lib()
        with ThreadPoolExecutor(16) as ex:
            errs = dict(zip(idx, ex.map(one, idx)))
        out[name] = {f"{n}x{N}": dict(vs_same_method=float(max(errs[i][0] for i in v[:per_bucket])),
                                      vs_exact=float(max(errs[i][1] for i in v[:per_bucket])), count=len(v))
                     for (n, N), v in sorted(buckets.items())}
        out[name]["status_bits_set"] = int((st["status"] != 0).sum())
        print("# uneven", name, out[name], file=sys.stderr, flush=True)
    return out


def main():
    import torch
    import paper_2510_07625_amd as g
    torch.cuda.set_device(0)
    out = {}
    solves = w.chain_batch(0, 256)
    params = g.Params(sqp_iters=10, pcg_tol=1e-5)
    out["headline"] = trajectories(g, torch, solves, params, range(256))
    print("# headline", out["headline"], file=sys.stderr, flush=True)
    prec = []
    for kw in PRECISIONS:
        p = g.Params(sqp_iters=10, pcg_tol=1e-5, **kw)
        t = trajectories(g, torch, solves[:32], p, (0, 31))
        kkt, its = kkt_error(g, torch, g.Params(pcg_tol=1e-5, **kw))
        prec.append(dict(precision=p.precision(), max_rel_traj_err_vs_exact=t["max_rel_traj_err_vs_exact"],
                         kkt_rel_err=kkt, kkt_pcg_iters=its))
        print("# precision", prec[-1], file=sys.stderr, flush=True)
    out["precision"] = prec
    out["uneven"] = uneven(g, torch)
    out["closed_loop"] = closed_loop(g, torch)
    print("# closed loop", out["closed_loop"], file=sys.stderr, flush=True)
    out["task_space"] = task_space(g, torch)
    print("# task space", out["task_space"], file=sys.stderr, flush=True)
    out["task_uneven"] = task_uneven(g, torch)
    print("# task uneven", out["task_uneven"], file=sys.stderr, flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
