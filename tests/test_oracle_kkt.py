"""Pins of the oracle's QP solve, Schur complement, preconditioner, PCG, Riccati
mode and line search (CPU only).

Independent checks: numpy/LAPACK solves of the assembled KKT system, dense
matrix products of Eq. (4), a hand-worked one-knot example, eigenvalues, and a
numpy-assembled QP for the linear double-integrator chain.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workload as w

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _solve(n=3, N=5, seed=1, i=0):
    s = w.chain_solve(seed, i, n=n, N=N)
    rng = np.random.default_rng(seed + 100 * i)
    # A point off the dynamics manifold so every term of Eq. (1) is active.
    X = s.X0 + rng.normal(0, 0.2, s.X0.shape)
    U = rng.normal(0, 1.0, s.U0.shape)
    return s, X, U


def _dense_kkt(s, X, U, rho=0.0):
    G, g, C, c = oracle.kkt_parts(s, X, U, rho)
    nz, nc = G.shape[0], C.shape[0]
    K = np.block([[G, C.T], [C, np.zeros((nc, nc))]])
    sol = np.linalg.solve(K, np.concatenate([-g, c]))
    return sol[:nz], -sol[nz:], (G, g, C, c)


@pytest.mark.parametrize("n,N", [(3, 5), (7, 4), (2, 2)])
def test_dense_kkt_matches_lapack(oracle_lib, n, N):
    s, X, U = _solve(n, N)
    dZ_ref, lam_ref, _ = _dense_kkt(s, X, U)
    dX, dU, lam, _, res = oracle.qp_step(s, X, U, mode=0)
    dX_ref, dU_ref = oracle.split_dz(s, dZ_ref)
    np.testing.assert_allclose(dX, dX_ref, atol=1e-10 * np.abs(dX_ref).max())
    np.testing.assert_allclose(dU, dU_ref, atol=1e-10 * np.abs(dU_ref).max())
    np.testing.assert_allclose(lam.ravel(), lam_ref, atol=1e-10 * np.abs(lam_ref).max())
    assert res < 1e-10


def test_kkt_structure(oracle_lib):
    # G block diagonal [Q_0 R_0 Q_1 ... Q_N]; C has I on the state diagonal and
    # -A_k, -B_k below it (Eq. (2)).
    s, X, U = _solve(3, 4)
    G, g, C, c = oracle.kkt_parts(s, X, U, rho=0.5)
    lq = oracle.lq(s, X, U, rho=0.5)
    nx, nu = 6, 3
    assert np.count_nonzero(G - np.diag(np.diag(G))) == 0
    np.testing.assert_allclose(np.diag(G)[:nx], s.Qd + 0.5)
    np.testing.assert_allclose(np.diag(G)[nx:nx + nu], s.Rd)
    np.testing.assert_allclose(np.diag(G)[-nx:], s.QNd + 0.5)
    np.testing.assert_allclose(C[nx:2 * nx, :nx], -lq["A"][0])
    np.testing.assert_allclose(C[nx:2 * nx, nx:nx + nu], -lq["B"][0])
    np.testing.assert_allclose(C[nx:2 * nx, nx + nu:2 * nx + nu], np.eye(nx))
    np.testing.assert_allclose(c[:nx], s.xs - X[0])
    np.testing.assert_allclose(c[nx:2 * nx], oracle.step(s, X[0], U[0]) - X[1])
    xg = np.concatenate([s.qgoal, np.zeros(3)])
    np.testing.assert_allclose(g[:nx], s.Qd * (X[0] - xg))


def test_one_knot_sign_example(oracle_lib):
    ex = json.load(open(os.path.join(GOLDEN, "one_knot_sign_example.json")))
    s = w.double_integrator_solve(0, 0, n=1, N=1, spring_k=0.0)
    s.QNd = np.array(ex["Q_diag"])
    s.qgoal = np.array([ex["goal_q"]])
    s.xs = np.array(ex["xs"])
    X = np.array([ex["x0"]])
    U = np.zeros((0, 1))
    lq = oracle.lq(s, X, U)
    np.testing.assert_allclose(lq["q"][0], ex["q_grad"])
    np.testing.assert_allclose(lq["c0"], ex["c"])
    for mode in (0, 1, 2):
        dX, _, lam, _, _ = oracle.qp_step(s, X, U, mode=mode, pcg_tol=1e-14)
        np.testing.assert_allclose(dX[0], ex["dx"], atol=1e-14)
        np.testing.assert_allclose(lam[0], ex["lambda"], atol=1e-14)
    # Eq. (4) read literally: S = -C G^-1 C^T, gamma = c - C G^-1 g.
    Q = np.diag(ex["Q_diag"])
    S_lit = -np.linalg.inv(Q)
    gam_lit = np.array(ex["c"]) - np.linalg.inv(Q) @ np.array(ex["q_grad"])
    lam_lit = np.linalg.solve(S_lit, gam_lit)
    dx_lit = -np.linalg.inv(Q) @ (np.array(ex["q_grad"]) - lam_lit)
    np.testing.assert_allclose(dx_lit, ex["paper_literal_dx"], atol=1e-14)


@pytest.mark.parametrize("n,N", [(3, 4), (2, 3)])
def test_schur_blocks_equal_dense_products(oracle_lib, n, N):
    s, X, U = _solve(n, N, seed=3)
    S, gam, P = oracle.schur(s, X, U, rho=0.2)
    G, g, C, c = oracle.kkt_parts(s, X, U, rho=0.2)
    Gi = np.linalg.inv(G)
    np.testing.assert_allclose(S, C @ Gi @ C.T, atol=1e-12 * np.abs(S).max())
    np.testing.assert_allclose(gam, c + C @ Gi @ g, atol=1e-12 * np.abs(gam).max())
    # Block tridiagonal and symmetric.
    nx = 2 * n
    for bi in range(N):
        for bj in range(N):
            if abs(bi - bj) > 1:
                assert not S[bi * nx:(bi + 1) * nx, bj * nx:(bj + 1) * nx].any()
                assert not P[bi * nx:(bi + 1) * nx, bj * nx:(bj + 1) * nx].any()
    np.testing.assert_allclose(S, S.T, atol=1e-13 * np.abs(S).max())
    # P = D^-1 - D^-1 O D^-1 with D, O the block diagonal / off-diagonal of S~.
    D = np.zeros_like(S)
    for k in range(N):
        D[k * nx:(k + 1) * nx, k * nx:(k + 1) * nx] = S[k * nx:(k + 1) * nx, k * nx:(k + 1) * nx]
    Di = np.linalg.inv(D)
    np.testing.assert_allclose(P, Di - Di @ (S - D) @ Di, atol=1e-10 * np.abs(P).max())
    assert np.linalg.eigvalsh(S).min() > 0
    assert np.linalg.eigvalsh(0.5 * (P + P.T)).min() > 0
    # Eq. (4)'s multipliers solve the KKT system.
    dZ_ref, lam_ref, _ = _dense_kkt(s, X, U, rho=0.2)
    np.testing.assert_allclose(np.linalg.solve(S, gam), lam_ref, atol=1e-9 * np.abs(lam_ref).max())


def test_stair_preconditioner_entrywise_form(oracle_lib):
    # Eq. (6): blocks Q_0, theta_k^-1 on the diagonal and
    # -theta_0^-1 phi_0 Q_0 / -theta_1^-1 phi_1 theta_0^-1 below it (sign per R3).
    s, X, U = _solve(2, 3, seed=8)
    S, gam, P = oracle.schur(s, X, U)
    nx = 4
    blk = lambda M, i, j: M[i * nx:(i + 1) * nx, j * nx:(j + 1) * nx]
    Q0 = np.diag(s.Qd)
    th0, th1 = blk(S, 1, 1), blk(S, 2, 2)
    ph0, ph1 = blk(S, 1, 0), blk(S, 2, 1)
    np.testing.assert_allclose(blk(P, 0, 0), Q0, atol=1e-12)
    np.testing.assert_allclose(blk(P, 1, 1), np.linalg.inv(th0), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(blk(P, 1, 0), -np.linalg.inv(th0) @ ph0 @ Q0, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(blk(P, 2, 1), -np.linalg.inv(th1) @ ph1 @ np.linalg.inv(th0), rtol=1e-9,
                               atol=1e-12)


@pytest.mark.parametrize("n,N", [(2, 2), (3, 3), (3, 4)])
def test_pcg_reaches_dense_solution(oracle_lib, n, N):
    s, X, U = _solve(n, N, seed=4)
    S, gam, P = oracle.schur(s, X, U)
    lam, it, hit = oracle.pcg_dense(S, P, gam, tol=1e-14)
    ref = np.linalg.solve(S, gam)
    np.testing.assert_allclose(lam, ref, atol=1e-11 * np.abs(ref).max())
    assert not hit and it <= N * 2 * n


def test_pcg_stopping_rule_and_cap(oracle_lib):
    s, X, U = _solve(3, 6, seed=5)
    S, gam, P = oracle.schur(s, X, U)
    lam, it, hit = oracle.pcg_dense(S, P, gam, tol=1e-4)
    r = gam - S @ lam
    assert r @ P @ r <= (1e-4) ** 2 * (gam @ P @ gam) * (1 + 1e-9)
    _, it1, hit1 = oracle.pcg_dense(S, P, gam, tol=1e-14, max_iter=2)
    assert it1 == 2 and hit1


@pytest.mark.parametrize("n,N", [(3, 6), (7, 5)])
def test_riccati_matches_dense_kkt(oracle_lib, n, N):
    s, X, U = _solve(n, N, seed=6)
    dZ_ref, lam_ref, _ = _dense_kkt(s, X, U)
    dX_ref, dU_ref = oracle.split_dz(s, dZ_ref)
    dX, dU, lam, _, res = oracle.qp_step(s, X, U, mode=2)
    np.testing.assert_allclose(dX, dX_ref, atol=1e-9 * np.abs(dX_ref).max())
    np.testing.assert_allclose(dU, dU_ref, atol=1e-9 * np.abs(dU_ref).max())
    np.testing.assert_allclose(lam.ravel(), lam_ref, atol=1e-9 * np.abs(lam_ref).max())
    assert res < 1e-9


def _rollout(s, U):
    X = np.zeros((s.N, 2 * s.n))
    X[0] = s.xs
    for k in range(s.N - 1):
        X[k + 1] = oracle.step(s, X[k], U[k])
    return X


def test_double_integrator_one_iteration_is_the_lqr_optimum(oracle_lib):
    # Linear dynamics from a feasible rollout: c = 0 for every step length, so the
    # merit is a convex quadratic in alpha minimised at alpha = 1, and one SQP
    # iteration lands on the optimum of the (exactly quadratic) problem. The
    # optimum is computed here independently from a numpy-assembled QP.
    s = w.double_integrator_solve(0, 1, n=3, N=8, spring_k=1.0)
    U0 = s.U0
    X0 = _rollout(s, U0)
    res = oracle.sqp(s, oracle.Params(sqp_iters=1, kkt_mode=0), X=X0, U=U0)
    assert res.logs[0]["alpha"] == 1.0
    n, N, h, k = 3, s.N, s.dt, s.spring_k
    T = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    A = np.block([[np.eye(n), h * np.eye(n)], [-h * k * T, np.eye(n)]])
    B = np.vstack([np.zeros((n, n)), h * np.eye(n)])
    nx = 2 * n
    # Unknowns [x_0..x_{N-1}, u_0..u_{N-2}] in absolute coordinates.
    nvar = N * nx + (N - 1) * n
    H = np.zeros((nvar, nvar))
    f = np.zeros(nvar)
    xg = np.concatenate([s.qgoal, np.zeros(n)])
    for kk in range(N):
        W = s.Qd if kk < N - 1 else s.QNd
        H[kk * nx:(kk + 1) * nx, kk * nx:(kk + 1) * nx] = np.diag(W)
        f[kk * nx:(kk + 1) * nx] = -W * xg
    for kk in range(N - 1):
        o = N * nx + kk * n
        H[o:o + n, o:o + n] = np.diag(s.Rd)
    E = np.zeros((N * nx, nvar))
    e = np.zeros(N * nx)
    E[:nx, :nx] = np.eye(nx)
    e[:nx] = s.xs
    for kk in range(N - 1):
        r = (kk + 1) * nx
        E[r:r + nx, (kk + 1) * nx:(kk + 2) * nx] = np.eye(nx)
        E[r:r + nx, kk * nx:(kk + 1) * nx] = -A
        E[r:r + nx, N * nx + kk * n:N * nx + (kk + 1) * n] = -B
    K = np.block([[H, E.T], [E, np.zeros((N * nx, N * nx))]])
    sol = np.linalg.solve(K, np.concatenate([-f, e]))
    X_opt = sol[:N * nx].reshape(N, nx)
    U_opt = sol[N * nx:nvar].reshape(N - 1, n)
    np.testing.assert_allclose(res.X, X_opt, atol=1e-10)
    np.testing.assert_allclose(res.U, U_opt, atol=1e-10)
    for mode in (1, 2):
        r2 = oracle.sqp(s, oracle.Params(sqp_iters=1, kkt_mode=mode, pcg_tol=1e-13), X=X0, U=U0)
        np.testing.assert_allclose(r2.X, X_opt, atol=1e-9)
        np.testing.assert_allclose(r2.U, U_opt, atol=1e-8)


def test_line_search_merits_and_argmin(oracle_lib):
    s, X, U = _solve(3, 6, seed=7)
    p = oracle.Params(sqp_iters=1, kkt_mode=0)
    res = oracle.sqp(s, p, X=X, U=U)
    L = res.logs[0]
    dX, dU, _, _, _ = oracle.qp_step(s, X, U, mode=0)
    m0 = oracle.merit(s, X, U, p.mu)[0]
    assert abs(L["merit0"] - m0) < 1e-12 * abs(m0)
    ms = [oracle.merit(s, X + 2.0 ** -i * dX, U + 2.0 ** -i * dU, p.mu)[0] for i in range(p.n_alpha)]
    np.testing.assert_allclose(L["merits"], ms, rtol=1e-12)
    assert L["argmin"] == int(np.argmin(ms))
    assert L["alpha"] == 2.0 ** -int(np.argmin(ms))
    np.testing.assert_allclose(res.X, X + L["alpha"] * dX, atol=1e-13)
    # Merit of Eq. (3): J + mu ||c||_1 with the nonlinear defects.
    xg = np.concatenate([s.qgoal, np.zeros(3)])
    J = sum(0.5 * (s.Qd * (X[k] - xg) ** 2).sum() + 0.5 * (s.Rd * U[k] ** 2).sum() for k in range(s.N - 1))
    J += 0.5 * (s.QNd * (X[-1] - xg) ** 2).sum()
    c1 = np.abs(s.xs - X[0]).sum() + sum(np.abs(oracle.step(s, X[k], U[k]) - X[k + 1]).sum() for k in range(s.N - 1))
    assert abs(m0 - (J + p.mu * c1)) < 1e-12 * abs(m0)


def test_sqp_converges_to_a_kkt_point(oracle_lib):
    # After enough iterations the nonlinear constraints hold and the QP step
    # vanishes (stationarity of the Lagrangian).
    s = w.chain_solve(0, 2, n=3, N=8)
    res = oracle.sqp(s, oracle.Params(sqp_iters=25, kkt_mode=2))
    assert res.logs[-1]["c1"] < 1e-9
    dX, dU, _, _, _ = oracle.qp_step(s, res.X, res.U, mode=0)
    assert max(np.abs(dX).max(), np.abs(dU).max()) < 1e-7
    merits = [L["merit"] for L in res.logs]
    assert merits[-1] <= merits[0]


def test_schur_pcg_mode_tracks_dense_mode(oracle_lib):
    s = w.chain_solve(0, 0, n=7, N=16)
    a = oracle.sqp(s, oracle.Params(sqp_iters=4, kkt_mode=0))
    b = oracle.sqp(s, oracle.Params(sqp_iters=4, kkt_mode=1, pcg_tol=1e-10))
    scale = np.abs(a.X).max()
    assert np.abs(a.X - b.X).max() < 1e-6 * scale
    assert all(L["pcg_iters"] > 0 for L in b.logs[:2])


@pytest.mark.parametrize("n,N", [(3, 128), (7, 64)])
def test_riccati_is_stable_on_long_horizons(oracle_lib, n, N):
    # Open-loop-unstable chains over long horizons: the Riccati mode must still
    # agree with a LAPACK solve of the assembled KKT system.
    s = w.chain_solve(12, 0, n=n, N=N)
    dZ_ref, lam_ref, _ = _dense_kkt(s, s.X0, s.U0)
    dX_ref, dU_ref = oracle.split_dz(s, dZ_ref)
    dX, dU, lam, _, res = oracle.qp_step(s, s.X0, s.U0, mode=2)
    np.testing.assert_allclose(dX, dX_ref, atol=1e-8 * np.abs(dX_ref).max())
    np.testing.assert_allclose(dU, dU_ref, atol=1e-8 * np.abs(dU_ref).max())
    np.testing.assert_allclose(lam.ravel(), lam_ref, atol=1e-8 * np.abs(lam_ref).max())
    assert res < 1e-9


def test_rho_damps_only_the_hessian_and_adapts_with_the_line_search(oracle_lib):
    # rho is added to the diagonal of every Q_k in the QP Hessian only (the
    # gradient and the merit keep the undamped Q). The step of one iteration is
    # checked against a numpy-assembled damped KKT system. With rho_adapt, rho
    # is divided by 3 after an iteration whose best candidate lowers the merit
    # and doubled otherwise; descent_replay overrides that decision.
    s = w.double_integrator_solve(0, 2, n=3, N=6, spring_k=1.0)
    X0 = _rollout(s, s.U0)
    rho = 0.7
    G, g, C, c = oracle.kkt_parts(s, X0, s.U0, rho=0.0)
    nx, N = 6, s.N
    Gd = G.copy()
    idx = np.diag_indices_from(Gd)
    # State blocks of the unknown ordering [x_0, u_0, x_1, u_1, ..., x_{N-1}].
    is_state = np.zeros(G.shape[0], bool)
    off = 0
    for k in range(N):
        is_state[off:off + nx] = True
        off += nx + (3 if k < N - 1 else 0)
    Gd[idx] += np.where(is_state, rho, 0.0)
    m = C.shape[0]
    K = np.block([[Gd, C.T], [C, np.zeros((m, m))]])
    dZ = np.linalg.solve(K, np.concatenate([-g, c]))[:G.shape[0]]
    dX, dU = oracle.split_dz(s, dZ)
    res = oracle.sqp(s, oracle.Params(sqp_iters=1, kkt_mode=0, rho=rho), X=X0, U=s.U0,
                     alpha_replay=np.array([1.0]))
    np.testing.assert_allclose(res.X, X0 + dX, atol=1e-11)
    np.testing.assert_allclose(res.U, s.U0 + dU, atol=1e-11)
    # Adaptation bookkeeping over a nonlinear chain.
    sc = w.chain_solve(5, 0, n=3, N=12)
    r = oracle.sqp(sc, oracle.Params(sqp_iters=8, kkt_mode=0, rho=1.0, rho_adapt=1))
    seq = [L["rho"] for L in r.logs]
    assert seq[0] == 1.0
    for i in range(1, 8):
        nd = r.logs[i - 1]["status"] & 4
        assert seq[i] == pytest.approx(seq[i - 1] * 2.0 if nd else seq[i - 1] / 3.0, rel=1e-15)
    forced = [1, 0, 0, 1, 1, 1, 0, 1]
    r2 = oracle.sqp(sc, oracle.Params(sqp_iters=8, kkt_mode=0, rho=1.0, rho_adapt=1), descent_replay=forced)
    want = [1.0]
    for d in forced[:-1]:
        want.append(want[-1] / 3.0 if d else want[-1] * 2.0)
    np.testing.assert_allclose([L["rho"] for L in r2.logs], want, rtol=1e-15)
