"""Parity checks of a GPU solve against the FP64 oracle (test helper).

At the benchmark's PCG tolerance the method itself (Schur complement + stair
preconditioner + PCG stopped at tolerance eps, Sec. II-B) departs from the
exact QP solve. The bar that catches a kernel error is therefore the oracle
running the *same method* in FP64 (Schur + PCG mode, same tolerance, same cap,
same warm start), replaying the GPU's decisions that floating point takes (the
accepted step of Eq. (7) and the PCG stopping iteration of reading R6: two
implementations that round differently can stop one iteration apart, and at a
truncated PCG one iteration moves the step by about as much as the truncation
itself):

  * max relative trajectory error X, U  <= 1e-4 (the target of the method);
  * every accepted step a valid argmin of Eq. (7) on the oracle's merits (ties
    at FP32 merit resolution accepted), and the merit before each step within
    1e-4 of the oracle's;
  * every PCG count a valid stop: at the GPU's count the oracle's stopping
    value r^T P r / (eps^2 gamma~^T P gamma~) is at most STOP_BAND, and one
    iteration earlier above 1 / STOP_BAND (or the GPU reported its cap).

How far the GPU and that same-method oracle sit from the exact solve (Riccati
mode, pinned against LAPACK) is computed as well and reported, not asserted.
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle

TRAJ_TOL = 1e-4
MERIT_TIE = 1e-5
# A factor 2 in the preconditioned residual norm either side of the threshold:
# the GPU evaluates the rule on its own (FP32-data, FP64-vector) iterates.
STOP_BAND = 4.0
ST_PCG_MAXITER = 1


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def check(s, Xg, Ug, st, p_gpu, X0=None, U0=None, lam0=None, tol=TRAJ_TOL, exact=True, label=""):
    """Replays the GPU's steps in the same-method FP64 oracle and asserts the
    bars above. st: the solve's per-iteration statistics (structured array).
    Returns a dict of errors (same-method, exact, and the method's own departure
    from the exact solve)."""
    iters = len(st)
    alphas = st["alpha"].astype(np.float64)
    kw = dict(sqp_iters=iters, mu=p_gpu.mu, beta=p_gpu.beta, n_alpha=p_gpu.n_alpha, rho=p_gpu.rho,
              rho_adapt=0, warm_lambda=p_gpu.warm_lambda)
    counts = [int(c) for c in st["pcg_iters"]]
    pm = oracle.Params(kkt_mode=1, pcg_tol=p_gpu.pcg_tol, pcg_max_iter=p_gpu.pcg_max_iter, **kw)
    same = oracle.sqp(s, pm, X=X0, U=U0, lam=lam0, alpha_replay=alphas, pcg_replay=counts)
    own = oracle.sqp(s, pm, X=X0, U=U0, lam=lam0, alpha_replay=alphas)
    n, N = s.n, s.N
    Xg, Ug = Xg[:N, :2 * n], Ug[:N - 1, :n]
    out = dict(label=label, e_same=max(rel(Xg, same.X), rel(Ug, same.U)),
               e_same_own_stop=max(rel(Xg, own.X), rel(Ug, own.U)),
               pcg_gpu=counts, pcg_oracle=[int(L["pcg_iters"]) for L in own.logs],
               stop_at_count=max(L["pcg_stop"] for L in same.logs),
               stop_before_count=min(L["pcg_stop_prev"] for L, c in zip(same.logs, counts) if c > 0)
               if any(c > 0 for c in counts) else float("inf"))
    bad_stop = []
    for it, (L, c) in enumerate(zip(same.logs, counts)):
        if int(st["status"][it]) & ST_PCG_MAXITER:
            continue
        if not (L["pcg_stop"] <= STOP_BAND and (c == 0 or L["pcg_stop_prev"] > 1.0 / STOP_BAND)):
            bad_stop.append((it, c, float(L["pcg_stop"]), float(L["pcg_stop_prev"])))
    out["stop_invalid"] = bad_stop
    bad_alpha = []
    for it, L in enumerate(same.logs):
        ms = L["merits"]
        i_gpu = int(round(-np.log2(alphas[it]) / np.log2(p_gpu.beta)))
        if ms[i_gpu] - ms.min() > MERIT_TIE * abs(ms.min()) + 1e-6:
            bad_alpha.append((it, i_gpu, int(np.argmin(ms)), float(ms[i_gpu]), float(ms.min())))
        assert abs(st["merit0"][it] - L["merit0"]) <= 1e-4 * abs(L["merit0"]) + 1e-4, \
            (label, it, float(st["merit0"][it]), L["merit0"])
    out["alpha_invalid"] = bad_alpha
    if exact:
        ex = oracle.sqp(s, oracle.Params(kkt_mode=2, **kw), X=X0, U=U0, alpha_replay=alphas)
        out["e_exact"] = max(rel(Xg, ex.X), rel(Ug, ex.U))
        out["e_ref"] = max(rel(same.X, ex.X), rel(same.U, ex.U))
    assert out["e_same"] <= tol, out
    assert not bad_alpha, out
    assert not bad_stop, out
    return out


def check_many(cases, threads=16):
    """Runs check(**case) for every case on a thread pool (the oracle releases
    the GIL); returns the list of results in order."""
    with ThreadPoolExecutor(max_workers=threads) as ex:
        futs = [ex.submit(check, **c) for c in cases]
        return [f.result() for f in futs]


def sample_indices(M, pcg_totals, count=16):
    """count solves of a batch: evenly spread, plus the slowest and the fastest
    PCG solve (the slowest sets the launch time)."""
    idx = set(int(i) for i in np.linspace(0, M - 1, max(count - 2, 1)).round())
    idx.add(int(np.argmax(pcg_totals)))
    idx.add(int(np.argmin(pcg_totals)))
    return sorted(idx)


def report(results, title):
    w = max(r["e_same"] for r in results)
    line = (f"{title}: {len(results)} solves, max error vs same-method FP64 oracle {w:.2e} "
            f"(its own PCG stops: {max(r['e_same_own_stop'] for r in results):.2e}; stopping value at the "
            f"GPU's counts {max(r['stop_at_count'] for r in results):.2f} max, one before "
            f"{min(r['stop_before_count'] for r in results):.2f} min)")
    if all("e_exact" in r for r in results):
        line += (f"; vs exact oracle {max(r['e_exact'] for r in results):.2e} (the FP64 method itself "
                 f"{max(r['e_ref'] for r in results):.2e})")
    print(line, flush=True)
    return line
