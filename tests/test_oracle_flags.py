"""Pins of the oracle's line-search status flag (NO_DESCENT, reading R11 of
Eq. (7)), of its KKT residual (the residual of Eq. (2) that every SQP
iteration records) and of its block-tridiagonal PCG products (CPU only).

Each case fixes the expected value by construction, not by re-running the
oracle's own formula:
  * a problem whose QP right-hand side is exactly zero (every candidate merit
    equals the current one, so no candidate lowers it: the flag is set);
  * a problem at the global minimum of the cost with an infeasible start and
    mu = 0 (every step raises the merit: the flag is set);
  * a linear chain started on a feasible rollout (the merit is a convex
    quadratic in alpha minimised at alpha = 1: the flag is clear);
  * a linear chain whose full step overshoots while shorter steps descend (the
    flag follows the best candidate, not alpha = 1);
  * KKT residuals of the LAPACK solution, of the zero vector and of single
    perturbed entries, whose values follow from the assembled G, g, C, c.
"""
import numpy as np
import pytest

import oracle
import workload as w

ST_NO_DESCENT = oracle.ST_NO_DESCENT


def _at_goal(s, X=None):
    """Every knot at [q_goal; 0], zero controls."""
    xg = np.concatenate([s.qgoal, np.zeros(s.n)])
    return np.tile(xg, (s.N, 1)), np.zeros((s.N - 1, s.n))


def _J(s, X, U):
    # Eq. (1)'s cost written out: stage terms, control terms, terminal term.
    xg = np.concatenate([s.qgoal, np.zeros(s.n)])
    d = X - xg
    return (0.5 * (s.Qd * d[:-1] ** 2).sum() + 0.5 * (s.Rd * U ** 2).sum() + 0.5 * (s.QNd * d[-1] ** 2).sum())


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_no_descent_is_set_when_the_step_is_zero(oracle_lib, mode):
    # q'' = u (no springs) with the iterate at the goal, at rest, zero controls
    # and x_s = x_0: the defects, gradients and c_0 are exactly zero, so the QP
    # step is exactly zero and every candidate's merit equals the current merit
    # (0). No candidate is strictly lower: NO_DESCENT.
    s = w.double_integrator_solve(0, 3, n=3, N=6, spring_k=0.0)
    X, U = _at_goal(s)
    s.xs = X[0].copy()
    r = oracle.sqp(s, oracle.Params(sqp_iters=1, kkt_mode=mode, pcg_tol=1e-8), X=X, U=U)
    L = r.logs[0]
    assert L["merit0"] == 0.0
    assert np.all(L["merits"] == 0.0)
    assert L["status"] & ST_NO_DESCENT
    assert L["argmin"] == 0 and L["alpha"] == 1.0     # ties go to the larger step
    np.testing.assert_array_equal(r.X, X)


def test_no_descent_is_set_when_every_step_raises_the_merit(oracle_lib):
    # mu = 0 (merit = cost). The iterate sits at the global minimum of the cost
    # (J = 0) but x_0 != x_s, so the QP step must move x_0 (its first
    # constraint row fixes dx_0 = x_s - x_0) and every candidate has J > 0.
    s = w.double_integrator_solve(0, 4, n=2, N=5, spring_k=1.0)
    X, U = _at_goal(s)
    s.xs = X[0] + np.array([0.3, -0.2, 0.1, 0.05])
    r = oracle.sqp(s, oracle.Params(sqp_iters=1, kkt_mode=0, mu=0.0), X=X, U=U)
    L = r.logs[0]
    assert L["merit0"] == 0.0
    assert np.all(L["merits"] > 0.0)
    assert L["status"] & ST_NO_DESCENT
    # The step is still taken (Eq. (7) is a plain argmin over the candidates).
    assert np.abs(r.X - X).max() > 0.0


def test_no_descent_is_clear_on_a_feasible_linear_start(oracle_lib):
    # Linear dynamics from a feasible rollout: every candidate is feasible, the
    # merit is the convex quadratic J(Z + alpha dZ) with its minimum at alpha = 1
    # and strictly decreasing towards it.
    s = w.double_integrator_solve(0, 5, n=3, N=8, spring_k=1.0)
    X = np.zeros((s.N, 6))
    X[0] = s.xs
    for k in range(s.N - 1):
        X[k + 1] = oracle.step(s, X[k], s.U0[k])
    r = oracle.sqp(s, oracle.Params(sqp_iters=1, kkt_mode=0), X=X, U=s.U0)
    L = r.logs[0]
    assert not (L["status"] & ST_NO_DESCENT)
    m = L["merits"]
    assert np.all(np.diff(m) > 0) and m[0] < L["merit0"]


def test_no_descent_follows_the_best_candidate_not_the_full_step(oracle_lib):
    # mu = 0 on a linear chain started off the goal with an infeasible x_0: the
    # full step overshoots (merit above the current one) while a shorter step
    # descends, so the flag stays clear. The candidate merits are recomputed
    # here from Eq. (1)'s cost at X + alpha dX, U + alpha dU.
    s = w.double_integrator_solve(1, 3, n=2, N=5, spring_k=0.0)
    rng = np.random.default_rng(3)
    X, U = _at_goal(s)
    X = X + rng.normal(0, 0.3, X.shape)
    U = U + rng.normal(0, 0.3, U.shape)
    r = oracle.sqp(s, oracle.Params(sqp_iters=1, kkt_mode=0, mu=0.0), X=X, U=U)
    L = r.logs[0]
    dX, dU, _, _, _ = oracle.qp_step(s, X, U, mode=0)
    ms = np.array([_J(s, X + 2.0 ** -i * dX, U + 2.0 ** -i * dU) for i in range(8)])
    np.testing.assert_allclose(L["merits"], ms, rtol=1e-12)
    assert abs(L["merit0"] - _J(s, X, U)) <= 1e-12 * _J(s, X, U)
    assert ms[0] > 1.5 * L["merit0"] and ms.min() < 0.9 * L["merit0"]
    assert not (L["status"] & ST_NO_DESCENT)
    assert L["argmin"] == int(np.argmin(ms)) > 0


def _kkt_parts(n=3, N=5, seed=2):
    s = w.chain_solve(seed, 0, n=n, N=N)
    rng = np.random.default_rng(seed)
    X = s.X0 + rng.normal(0, 0.2, s.X0.shape)
    U = rng.normal(0, 1.0, s.U0.shape)
    G, g, C, c = oracle.kkt_parts(s, X, U)
    nz, nc = G.shape[0], C.shape[0]
    K = np.block([[G, C.T], [C, np.zeros((nc, nc))]])
    sol = np.linalg.solve(K, np.concatenate([-g, c]))
    return s, X, U, G, g, C, c, sol[:nz], -sol[nz:]


def test_kkt_residual_of_known_vectors(oracle_lib):
    # Residual r = [G dZ + g - C^T lambda; C dZ - c], inf-norm.
    s, X, U, G, g, C, c, dZ, lam = _kkt_parts()
    base = oracle.kkt_residual(s, X, U, dZ, lam)
    assert base <= 1e-11 * max(np.abs(g).max(), np.abs(c).max())
    # The zero vector leaves the right-hand side: max(|g|, |c|).
    r0 = oracle.kkt_residual(s, X, U, np.zeros_like(dZ), np.zeros_like(lam))
    assert r0 == pytest.approx(max(np.abs(g).max(), np.abs(c).max()), rel=1e-14)
    # One multiplier moved by d changes only the stationarity rows, by -d C[j, :].
    d = 1e-2
    for j in (0, 7, lam.size - 1):
        lp = lam.copy()
        lp[j] += d
        want = d * np.abs(C[j]).max()
        assert oracle.kkt_residual(s, X, U, dZ, lp) == pytest.approx(want, rel=1e-8, abs=1e-11)
    # One entry of dZ moved by d changes the stationarity rows by d G[:, i] and
    # the feasibility rows by d C[:, i]: the last state entry (Q_N on the
    # diagonal of G dominates) and the first control entry (the B_0 column of C
    # dominates R).
    nx, nu = 2 * s.n, s.n
    for i in (dZ.size - 1, nx):
        zp = dZ.copy()
        zp[i] += d
        want = d * max(np.abs(G[:, i]).max(), np.abs(C[:, i]).max())
        assert oracle.kkt_residual(s, X, U, zp, lam) == pytest.approx(want, rel=1e-8, abs=1e-11)
    assert np.abs(G[:, dZ.size - 1]).max() > np.abs(C[:, dZ.size - 1]).max()
    assert np.abs(C[:, nx]).max() > np.abs(G[:, nx]).max()


def test_logged_kkt_residual_is_that_of_the_step(oracle_lib):
    # The residual an SQP iteration logs is the residual of its own step.
    s, X, U, G, g, C, c, dZ, lam = _kkt_parts(n=3, N=6, seed=4)
    r = oracle.sqp(s, oracle.Params(sqp_iters=1, kkt_mode=1, pcg_tol=1e-3), X=X, U=U)
    dX, dU, lam1, _, res = oracle.qp_step(s, X, U, mode=1, pcg_tol=1e-3)
    dz = np.concatenate([np.concatenate([dX[k], dU[k]]) for k in range(s.N - 1)] + [dX[-1]])
    want = oracle.kkt_residual(s, X, U, dz, lam1)
    assert want > 1e-8              # an inexact PCG step leaves a visible residual
    assert r.logs[0]["kkt_res"] == pytest.approx(want, rel=1e-12)
    assert res == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("n,N", [(7, 32), (3, 20)])
def test_pcg_on_the_block_tridiagonal_system_equals_the_dense_products(oracle_lib, n, N):
    # The SQP's PCG multiplies S~ and P block row by block row; the same PCG on
    # the dense matrices (every entry of every row) must give the same bits.
    s = w.chain_solve(6, 1, n=n, N=N)
    S, gam, P = oracle.schur(s, s.X0, s.U0)
    dim = N * 2 * n
    nb = 2 * n
    band = np.zeros((dim, dim), bool)
    for b in range(N):
        band[b * nb:(b + 1) * nb, max(b - 1, 0) * nb:min(b + 2, N) * nb] = True
    assert not S[~band].any() and not P[~band].any()
    lam_d, it_d, _ = oracle.pcg_dense(S, P, gam, tol=1e-6)
    _, _, lam_t, it_t, _ = oracle.qp_step(s, s.X0, s.U0, mode=1, pcg_tol=1e-6)
    assert it_d == it_t
    np.testing.assert_array_equal(lam_d, lam_t.ravel())
