"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (from the target precision of the method; FP32 bulk arithmetic):
  * QP data (A, B, e) of the LQ stage: |gpu - oracle| <= 2e-5 * max(1, |oracle|).
  * KKT solution on identical QP data (the oracle's FP64 data rounded once to
    FP32 on both sides): ||dZ_gpu - dZ_ora||_inf <= 1e-5 ||dZ_ora||_inf.
  * Trajectory after the SQP iterations, with the oracle replaying the GPU's
    accepted steps: max|X_gpu - X_ora| <= 1e-4 max|X_ora| (same for U).
"""
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


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _f32(a):
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


def _qh(s, rho=0.0):
    return np.array([(s.Qd if k < s.N - 1 else s.QNd) + rho for k in range(s.N)])


@pytest.mark.parametrize("n,N,M", [(7, 32, 3), (3, 16, 2), (6, 40, 2), (7, 64, 2), (7, 128, 1), (3, 100, 2),
                                   (7, 2, 2)])
def test_lq_stage_parity(n, N, M):
    _say(f"lq n={n} N={N} M={M}")
    solves = [w.chain_solve(11, i, n=n, N=N) for i in range(M)]
    rng = np.random.default_rng(n * 1000 + N)
    for s in solves:  # off-manifold iterate so every term is non-trivial
        s.X0 = s.X0 + rng.normal(0, 0.1, s.X0.shape)
        s.U0 = rng.normal(0, 2.0, s.U0.shape)
    b = g.Batch.from_solves(solves)
    xs, goal, X, U = g.pack_inputs(solves)
    A, B, e = (t.cpu().numpy().astype(np.float64) for t in b.debug_lq(xs, goal, X, U))
    torch.cuda.synchronize()
    for i, s in enumerate(solves):
        L = oracle.lq(s, _f32(s.X0), _f32(s.U0))
        nx, nu = 2 * n, n
        for name, got, ref in (("A", A[i, :N - 1, :nx, :nx], L["A"]), ("B", B[i, :N - 1, :nx, :nu], L["B"]),
                               ("e", e[i, :N - 1, :nx], L["e"])):
            err = np.abs(got - ref).max()
            assert err <= 2e-5 * max(1.0, np.abs(ref).max()), (name, i, err)
    b.close()


@pytest.mark.parametrize("n,N,M,fp64", [(7, 32, 4, 1), (3, 12, 3, 1), (7, 64, 2, 1), (7, 128, 1, 1),
                                        (6, 33, 2, 1), (7, 2, 2, 1)])
def test_kkt_parity_on_identical_qp_data(n, N, M, fp64):
    _say(f"kkt n={n} N={N} M={M} fp64={fp64}")
    solves = [w.chain_solve(12, i, n=n, N=N) for i in range(M)]
    nx, nu = 2 * n, n
    data = [oracle.lq(s, s.X0, s.U0) for s in solves]
    cast = [{k: _f32(v) for k, v in d.items()} for d in data]
    b = g.Batch.from_solves(solves, g.Params(pcg_tol=1e-9, schur_fp64=fp64))
    dev = lambda key, shape: torch.from_numpy(np.stack([c[key] for c in cast]).astype(np.float32).reshape(shape)).cuda()
    A = dev("A", (M, N - 1, nx, nx))
    B = dev("B", (M, N - 1, nx, nu))
    e = dev("e", (M, N - 1, nx))
    q = dev("q", (M, N, nx))
    r = dev("r", (M, N - 1, nu))
    c0 = dev("c0", (M, nx))
    dX, dU, lam, its = b.debug_kkt(A, B, e, q, r, c0)
    dX, dU, lam, its = dX.cpu().numpy(), dU.cpu().numpy(), lam.cpu().numpy(), its.cpu().numpy()
    for i, s in enumerate(solves):
        c = cast[i]
        mode = 2 if N > 64 else 0
        rX, rU, rl, _ = oracle.kkt_from_lq(c["A"], c["B"], c["e"], c["q"], c["r"], c["c0"], _qh(s), s.Rd, mode=mode)
        ref = np.concatenate([rX.ravel(), rU.ravel()])
        got = np.concatenate([dX[i].ravel(), dU[i].ravel()])
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert err <= 1e-5, (i, err, int(its[i]))
        assert 0 < its[i] <= N * nx
    b.close()


PRECISIONS = {"fp64-schur": dict(schur_fp64=1), "fp32": dict(schur_fp64=0),
              "fp32+fp64-inv": dict(schur_fp64=0, fp64_block_inv=1), "fp32+fp64-dot": dict(schur_fp64=0, fp64_dot=1),
              "fp32+fp64-inv+fp64-dot": dict(schur_fp64=0, fp64_block_inv=1, fp64_dot=1)}


def test_precision_toggles_kkt_error():
    # KKT-solution error on identical QP data for every precision setting.
    # The FP64 Schur/PCG variant meets 1e-5. With S~ formed and stored in FP32
    # the error stalls near 1e-3 (kappa(S~) ~ 1e5-1e6 here); the FP64 block
    # inverse and FP64 inner products are reported beside it.
    _say("kkt precision toggles")
    n, N, M = 7, 32, 3
    solves = [w.chain_solve(12, i, n=n, N=N) for i in range(M)]
    nx, nu = 2 * n, n
    cast = [{k: _f32(v) for k, v in oracle.lq(s, s.X0, s.U0).items()} for s in solves]
    dev = lambda key, shape: torch.from_numpy(np.stack([c[key] for c in cast]).astype(np.float32).reshape(shape)).cuda()
    args = (dev("A", (M, N - 1, nx, nx)), dev("B", (M, N - 1, nx, nu)), dev("e", (M, N - 1, nx)),
            dev("q", (M, N, nx)), dev("r", (M, N - 1, nu)), dev("c0", (M, nx)))
    refs = []
    for i, s in enumerate(solves):
        c = cast[i]
        rX, rU, _, _ = oracle.kkt_from_lq(c["A"], c["B"], c["e"], c["q"], c["r"], c["c0"], _qh(s), s.Rd)
        refs.append(np.concatenate([rX.ravel(), rU.ravel()]))
    errs, iters = {}, {}
    for name, kw in PRECISIONS.items():
        b = g.Batch.from_solves(solves, g.Params(pcg_tol=1e-7, **kw))
        dX, dU, _, its = (t.cpu().numpy() for t in b.debug_kkt(*args))
        b.close()
        worst = 0.0
        for i in range(M):
            got = np.concatenate([dX[i].ravel(), dU[i].ravel()])
            worst = max(worst, np.abs(got - refs[i]).max() / np.abs(refs[i]).max())
        errs[name], iters[name] = worst, int(its.max())
    print("KKT-solution error (PCG tol 1e-7): " + ", ".join(f"{k} {v:.2e} ({iters[k]} its)" for k, v in errs.items()))
    assert errs["fp64-schur"] <= 1e-5
    assert errs["fp32"] > 1e-5
    for k, v in errs.items():
        assert np.isfinite(v) and v < 1e-1, (k, v)


def _run_gpu(solves, params, X=None, U=None):
    b = g.Batch.from_solves(solves, params)
    xs, goal, Xd, Ud = g.pack_inputs(solves)
    if X is not None:
        Xd.copy_(torch.from_numpy(X.astype(np.float32)))
        Ud.copy_(torch.from_numpy(U.astype(np.float32)))
    st = b.solve(xs, goal, Xd, Ud)
    out = Xd.cpu().numpy().astype(np.float64), Ud.cpu().numpy().astype(np.float64), st
    b.close()
    return out


def _replay_check(s, Xg, Ug, st, p_gpu, tol=1e-4, check_merit=True):
    """Oracle replays the GPU's accepted steps; returns the trajectory errors."""
    alphas = st["alpha"].astype(np.float64)
    po = oracle.Params(sqp_iters=p_gpu.sqp_iters, kkt_mode=0 if s.N <= 64 else 2, mu=p_gpu.mu, beta=p_gpu.beta,
                       n_alpha=p_gpu.n_alpha)
    ref = oracle.sqp(s, po, alpha_replay=alphas)
    n, N = s.n, s.N
    ex = np.abs(Xg[:N, :2 * n] - ref.X).max() / np.abs(ref.X).max()
    eu = np.abs(Ug[:N - 1, :n] - ref.U).max() / np.abs(ref.U).max()
    assert ex <= tol and eu <= tol, (ex, eu, tol)
    for it, L in enumerate(ref.logs):
        ms = L["merits"]
        i_gpu = int(round(-np.log2(alphas[it]) / np.log2(p_gpu.beta)))
        if check_merit and i_gpu != int(np.argmin(ms)):
            # Either candidate is a correct argmin when the merits tie at FP32 resolution.
            assert ms[i_gpu] - ms.min() <= 1e-5 * abs(ms.min()) + 1e-6, (it, ms, i_gpu)
        if check_merit:
            assert abs(st["merit0"][it] - L["merit0"]) <= 1e-4 * abs(L["merit0"]) + 1e-4, (it, st["merit0"][it],
                                                                                           L["merit0"])
    return ex, eu


# (7, 128): the longest horizon, four knots per lane group with the Schur rows
# read back from the workspace; (7, 2): a single control, no off-diagonal blocks;
# (7, 33): two knots per lane group with a single knot in the second pass.
@pytest.mark.parametrize("n,N,M", [(7, 32, 3), (3, 20, 2), (6, 48, 2), (7, 64, 1), (7, 128, 1), (7, 2, 2),
                                   (7, 33, 2)])
def test_sqp_trajectory_parity_tight_tolerance(n, N, M):
    # PCG tolerance 1e-7: the exact (dense LU) oracle is the reference, 1e-4.
    _say(f"sqp tight n={n} N={N} M={M}")
    solves = [w.chain_solve(0, i, n=n, N=N) for i in range(M)]
    p = g.Params(sqp_iters=10, pcg_tol=1e-7)
    Xg, Ug, st = _run_gpu(solves, p)
    assert st.shape == (M, 10)
    for i, s in enumerate(solves):
        _replay_check(s, Xg[i], Ug[i], st[i], p)
        assert not (st[i]["status"] & (g.ST_NONFINITE | g.ST_PCG_MAXITER)).any()
        assert st[i]["merit"][-1] < st[i]["merit0"][0]


# The line search of Eq. (7) at its limits: one candidate (the full step only)
# and the largest candidate set, with a step ratio other than the default; and
# a lighter weight mu of the constraint violation in the merit of Eq. (3).
@pytest.mark.parametrize("n_alpha,beta,mu", [(1, 2.0, 10.0), (16, 1.5, 10.0), (8, 2.0, 1.0)])
def test_line_search_candidate_count_limits(n_alpha, beta, mu):
    _say(f"line search n_alpha={n_alpha} beta={beta} mu={mu}")
    solves = [w.chain_solve(3, i, n=6, N=24) for i in range(2)]
    p = g.Params(sqp_iters=6, pcg_tol=1e-7, n_alpha=n_alpha, beta=beta, mu=mu)
    Xg, Ug, st = _run_gpu(solves, p)
    for i, s in enumerate(solves):
        _replay_check(s, Xg[i], Ug[i], st[i], p)
        assert not (st[i]["status"] & (g.ST_NONFINITE | g.ST_PCG_MAXITER)).any()
    candidates = beta ** -np.arange(n_alpha, dtype=np.float64)
    for a in st["alpha"].ravel():
        assert np.isclose(candidates, float(a), rtol=1e-6).any(), (a, candidates)
    if n_alpha == 1:
        assert (st["alpha"] == 1.0).all()


@pytest.mark.parametrize("n,N,M", [(7, 32, 4), (6, 48, 2)])
def test_sqp_trajectory_at_config_tolerance(n, N, M):
    # PCG tolerance 1e-5 (the benchmark setting). The reference is the oracle
    # running the same method in FP64 (Schur complement + stair preconditioner
    # + PCG at 1e-5, same warm start) over the GPU's accepted steps: trajectory
    # within 1e-4 and every accepted step a valid argmin of its merits. The
    # distance of both to the exact solve is printed.
    _say(f"sqp config-tol n={n} N={N} M={M}")
    solves = [w.chain_solve(0, i, n=n, N=N) for i in range(M)]
    p = g.Params(sqp_iters=10, pcg_tol=1e-5)
    Xg, Ug, st = _run_gpu(solves, p)
    res = _parity.check_many([dict(s=s, Xg=Xg[i], Ug=Ug[i], st=st[i], p_gpu=p, label=f"solve {i}")
                              for i, s in enumerate(solves)])
    _parity.report(res, f"n={n} N={N} at PCG tol 1e-5")


def test_full_size_batch_sampled_solves():
    # The benchmark's launch: M = 256 seeded 7-DoF chains, N = 32, 10 SQP
    # iterations, PCG tol 1e-5, one workgroup per solve (bench.py's step with
    # the iterate restored and the warm start cleared). Eighteen solves (evenly
    # spread, plus the slowest and the fastest PCG solve) are replayed in the
    # same-method FP64 oracle. The per-iteration statistics of every solve must
    # be clean.
    _say("full size M=256")
    M = 256
    solves = w.chain_batch(0, M)
    p = g.Params(sqp_iters=10, pcg_tol=1e-5)
    b = g.Batch.from_solves(solves, p)
    xs, goal, X, U = g.pack_inputs(solves)
    st_buf = b.stats_buffer(10)
    b.reset_warm_start()
    b.step(xs, goal, X, U, 10, st_buf)
    torch.cuda.synchronize()
    st = g.Batch.decode_stats(st_buf, M, 10)
    Xg, Ug = X.cpu().numpy().astype(np.float64), U.cpu().numpy().astype(np.float64)
    b.close()
    assert not (st["status"] & (g.ST_NONFINITE | g.ST_PCG_MAXITER)).any()
    tot = st["pcg_iters"].sum(axis=1)
    idx = _parity.sample_indices(M, tot, count=18)
    assert int(np.argmax(tot)) in idx and len(idx) >= 16
    res = _parity.check_many([dict(s=solves[i], Xg=Xg[i], Ug=Ug[i], st=st[i], p_gpu=p, label=f"solve {i}")
                              for i in idx])
    _parity.report(res, f"M=256 batch (slowest PCG solve {int(np.argmax(tot))}: {int(tot.max())} iterations)")


def test_uneven_batch_matches_single_solves():
    _say("uneven batch")
    solves = w.uneven_batch(5, M=6, horizons=(16, 32, 64))
    p = g.Params(sqp_iters=3)
    Xb, Ub, stb = _run_gpu(solves, p)
    for i, s in enumerate(solves):
        Xs, Us, sts = _run_gpu([s], p)
        n, N = s.n, s.N
        np.testing.assert_array_equal(Xb[i, :N, :2 * n], Xs[0, :N, :2 * n])
        np.testing.assert_array_equal(Ub[i, :N - 1, :n], Us[0, :N - 1, :n])
        np.testing.assert_array_equal(stb[i], sts[0])
        # Padding beyond the solve's own shape is left untouched (zeros from pack_inputs).
        assert not Xb[i, N:].any() and not Xb[i, :, 2 * n:].any()


def test_plain_launches_equal_batched_launch():
    _say("plain vs batched")
    solves = [w.chain_solve(2, i) for i in range(4)]
    p = g.Params(sqp_iters=2)
    b = g.Batch.from_solves(solves, p)
    xs, goal, X1, U1 = g.pack_inputs(solves)
    X2, U2 = X1.clone(), U1.clone()
    b.step(xs, goal, X1, U1, 2)
    b.reset_warm_start()
    b.step(xs, goal, X2, U2, 2, plain=True)
    torch.cuda.synchronize()
    assert torch.equal(X1, X2) and torch.equal(U1, U2)
    b.close()


def test_batch_of_more_solves_than_cus_is_batch_invariant():
    # 600 solves: more workgroups than the chip holds at once (LDS allows one
    # per CU), so later solves start as earlier ones finish. Every solve must
    # come out bit for bit as in a batch of its own, and sampled solves match
    # the oracle.
    _say("M=600 batch invariance")
    M = 600
    solves = w.chain_batch(21, M, N=16)
    p = g.Params(sqp_iters=3, pcg_tol=1e-7)
    b = g.Batch.from_solves(solves, p)
    xs, goal, X, U = g.pack_inputs(solves)
    st = b.solve(xs, goal, X, U)
    b.close()
    Xb, Ub = X.cpu().numpy(), U.cpu().numpy()
    for i in (0, 257, 599):
        b1 = g.Batch.from_solves([solves[i]], p)
        xs1, goal1, X1, U1 = g.pack_inputs([solves[i]])
        b1.solve(xs1, goal1, X1, U1)
        b1.close()
        assert np.array_equal(X1.cpu().numpy()[0], Xb[i]) and np.array_equal(U1.cpu().numpy()[0], Ub[i]), i
        _replay_check(solves[i], Xb[i].astype(np.float64), Ub[i].astype(np.float64), st[i], p)


def test_double_integrator_one_step_is_the_lq_optimum():
    _say("double integrator")
    s = w.double_integrator_solve(3, 0, n=3, N=12, spring_k=1.0)
    X0 = np.zeros((s.N, 6))
    X0[0] = s.xs
    for k in range(s.N - 1):
        X0[k + 1] = oracle.step(s, X0[k], s.U0[k])
    X0 = _f32(X0)
    p = g.Params(sqp_iters=1, pcg_tol=1e-9)
    Xg, Ug, st = _run_gpu([s], p, X=X0[None], U=_f32(s.U0)[None])
    ref = oracle.sqp(s, oracle.Params(sqp_iters=1, kkt_mode=0), X=X0, U=_f32(s.U0))
    assert st[0]["alpha"][0] == 1.0
    assert np.abs(Xg[0] - ref.X).max() <= 1e-5 * np.abs(ref.X).max()
    assert np.abs(Ug[0] - ref.U).max() <= 1e-5 * np.abs(ref.U).max()


def test_status_bits_are_per_solve():
    _say("status bits")
    solves = [w.chain_solve(4, i) for i in range(3)]
    solves[1].xs = solves[1].xs.copy()
    solves[1].xs[3] = np.nan
    p = g.Params(sqp_iters=2)
    Xg, Ug, st = _run_gpu(solves, p)
    assert (st[1]["status"] & g.ST_NONFINITE).all()
    assert not (st[0]["status"] & g.ST_NONFINITE).any() and not (st[2]["status"] & g.ST_NONFINITE).any()
    ok = [solves[0], solves[2]]
    Xo, Uo, sto = _run_gpu(ok, p)
    np.testing.assert_array_equal(Xg[[0, 2]], Xo)
    _, _, st2 = _run_gpu([w.chain_solve(4, 0)], g.Params(sqp_iters=1, pcg_max_iter=1))
    assert st2[0]["status"][0] & g.ST_PCG_MAXITER
    assert st2[0]["pcg_iters"][0] == 1
