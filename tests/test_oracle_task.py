"""Pins of the oracle's task-space (tip tracking) cost (CPU only).

Independent checks: the numpy kinematics of tests/_fk.py, central finite
differences of the tip position and of the cost, the Hessian of the cost at a
zero tracking residual (where the Gauss-Newton term is exact), numpy/LAPACK
solves and dense products of the assembled KKT system with its dense state
Hessian blocks, and convergence to a stationary point of the nonlinear
problem.
"""
import numpy as np
import pytest

import oracle
import workload as w

from . import _fk


def _fig8(n=7, N=6, seed=2, i=0, off=0.2):
    s = w.figure8_solve(seed, i, n=n, N=N)
    rng = np.random.default_rng(seed + 31 * i)
    X = s.X0 + rng.normal(0, off, s.X0.shape)
    U = rng.normal(0, 1.0, s.U0.shape)
    return s, X, U


@pytest.mark.parametrize("n", [3, 6, 7])
def test_tip_matches_independent_kinematics(oracle_lib, n):
    s = w.figure8_solve(1, 3, n=n, N=4)
    rng = np.random.default_rng(n)
    for _ in range(5):
        q = rng.uniform(-2, 2, n)
        p, J = oracle.tip(s, q)
        np.testing.assert_allclose(p, _fk.tip(s.links, q), atol=1e-14)
        np.testing.assert_allclose(J, _fk.tip_jacobian(s.links, q), atol=1e-14)


def test_tip_jacobian_matches_finite_differences(oracle_lib):
    s = w.figure8_solve(0, 1, n=7, N=4)
    q = np.random.default_rng(0).uniform(-1.5, 1.5, 7)
    _, J = oracle.tip(s, q)
    h = 1e-6
    Jfd = np.stack([(oracle.tip(s, q + h * e)[0] - oracle.tip(s, q - h * e)[0]) / (2 * h) for e in np.eye(7)], 1)
    np.testing.assert_allclose(J, Jfd, atol=1e-8)


def test_figure8_reference_is_reachable_and_closed(oracle_lib):
    # The centre lies within reach; one period of the figure returns to its start.
    s = w.figure8_solve(0, 0, n=7, N=201, dt=0.01)
    L = s.links[:, 0].sum()
    assert np.linalg.norm(s.pref, axis=1).max() < 0.75 * L
    np.testing.assert_allclose(s.pref[200], s.pref[0], atol=1e-12)
    # Gerono lemniscate: the vertical offset is the horizontal one times cos(th).
    assert np.ptp(s.pref[:, 2]) > 0 and np.ptp(s.pref[:, :2]) > 0


def test_gradient_is_the_cost_gradient(oracle_lib):
    # q_k of the QP (Eq. (1)) is dJ/dx_k, the tip term included.
    s, X, U = _fig8()
    q = oracle.lq(s, X, U)["q"]
    h = 1e-6
    for k in (0, 2, s.N - 1):
        for i in range(2 * s.n):
            Xp, Xm = X.copy(), X.copy()
            Xp[k, i] += h
            Xm[k, i] -= h
            d = (oracle.merit(s, Xp, U)[1] - oracle.merit(s, Xm, U)[1]) / (2 * h)
            assert abs(d - q[k, i]) <= 1e-6 * max(1.0, abs(q[k, i])), (k, i, d, q[k, i])


def test_hessian_blocks_are_diag_plus_gauss_newton(oracle_lib):
    s, X, U = _fig8()
    Qf = oracle.lq_hessian(s, X, U, rho=0.3)
    n = s.n
    for k in range(s.N):
        Wd = s.Wee if k < s.N - 1 else s.WeeN
        Qd = s.Qd if k < s.N - 1 else s.QNd
        J = _fk.tip_jacobian(s.links, X[k, :n])
        ref = np.diag(Qd + 0.3)
        ref[:n, :n] += J.T @ np.diag(Wd) @ J
        np.testing.assert_allclose(Qf[k], ref, atol=1e-12 * np.abs(ref).max())
    # The dense G of Eq. (2) carries these blocks.
    G, _, _, _ = oracle.kkt_parts(s, X, U, rho=0.3)
    nx, nu = 2 * n, n
    for k in range(s.N):
        o = k * (nx + nu)
        np.testing.assert_allclose(G[o:o + nx, o:o + nx], Qf[k], atol=0)


def test_gauss_newton_is_the_exact_hessian_at_zero_residual(oracle_lib):
    # With the reference placed at the current tip positions the residual term
    # of the Hessian vanishes, so Q_k must equal the finite-difference Hessian.
    s, X, U = _fig8(N=4)
    s.pref = np.stack([_fk.tip(s.links, X[k, :s.n]) for k in range(s.N)])
    Qf = oracle.lq_hessian(s, X, U)
    h = 1e-4
    nx = 2 * s.n
    for k in (1, s.N - 1):
        H = np.zeros((nx, nx))
        for i in range(nx):
            Xp, Xm = X.copy(), X.copy()
            Xp[k, i] += h
            Xm[k, i] -= h
            H[:, i] = (oracle.lq(s, Xp, U)["q"][k] - oracle.lq(s, Xm, U)["q"][k]) / (2 * h)
        # (The gradient's own derivative includes the residual term, zero here.)
        np.testing.assert_allclose(H, Qf[k], atol=1e-6 * np.abs(Qf[k]).max())


@pytest.mark.parametrize("n,N", [(3, 4), (7, 3)])
def test_schur_with_dense_hessian_equals_dense_products(oracle_lib, n, N):
    s, X, U = _fig8(n=n, N=N, seed=5)
    S, gam, P = oracle.schur(s, X, U, rho=0.1)
    G, g, C, c = oracle.kkt_parts(s, X, U, rho=0.1)
    Gi = np.linalg.inv(G)
    np.testing.assert_allclose(S, C @ Gi @ C.T, atol=1e-12 * np.abs(S).max())
    np.testing.assert_allclose(gam, c + C @ Gi @ g, atol=1e-12 * np.abs(gam).max())
    nx = 2 * n
    D = np.zeros_like(S)
    for k in range(N):
        D[k * nx:(k + 1) * nx, k * nx:(k + 1) * nx] = S[k * nx:(k + 1) * nx, k * nx:(k + 1) * nx]
    Di = np.linalg.inv(D)
    np.testing.assert_allclose(P, Di - Di @ (S - D) @ Di, atol=1e-10 * np.abs(P).max())
    # The (0, 0) block is the dense Q_0^-1, not a diagonal. (For three joints
    # the tip Jacobian's columns happen to be orthogonal.)
    Q0i = S[:nx, :nx]
    assert n < 6 or np.abs(Q0i[:n, :n] - np.diag(np.diag(Q0i[:n, :n]))).max() > 1e-3 * np.abs(Q0i).max()


def test_all_kkt_modes_agree_with_lapack(oracle_lib):
    s, X, U = _fig8(n=7, N=8, seed=6)
    G, g, C, c = oracle.kkt_parts(s, X, U)
    nz, nc = G.shape[0], C.shape[0]
    K = np.block([[G, C.T], [C, np.zeros((nc, nc))]])
    sol = np.linalg.solve(K, np.concatenate([-g, c]))
    dX_ref, dU_ref = oracle.split_dz(s, sol[:nz])
    lam_ref = -sol[nz:].reshape(s.N, -1)
    scale = max(np.abs(dX_ref).max(), np.abs(dU_ref).max())
    # (The tip term makes S~ far worse conditioned than the joint-space one:
    # FP64 PCG needs more than N nx iterations and levels off near 1e-9.)
    for mode, tol in ((0, 1e-10), (1, 1e-7), (2, 1e-9)):
        dX, dU, lam, _, res = oracle.qp_step(s, X, U, mode=mode, pcg_tol=1e-12, pcg_max_iter=2000)
        assert np.abs(dX - dX_ref).max() <= tol * scale, mode
        assert np.abs(dU - dU_ref).max() <= tol * scale, mode
        assert np.abs(lam - lam_ref).max() <= tol * np.abs(lam_ref).max(), mode
        assert res < 1e-6


def test_task_space_sqp_converges_to_a_stationary_point(oracle_lib):
    s = w.figure8_solve(0, 2, n=3, N=16, dt=0.05)
    res = oracle.sqp(s, oracle.Params(sqp_iters=60, kkt_mode=2))
    assert res.logs[-1]["c1"] < 1e-9
    dX, dU, _, _, _ = oracle.qp_step(s, res.X, res.U, mode=0)
    assert max(np.abs(dX).max(), np.abs(dU).max()) < 1e-7
    # The tip ends much closer to the figure than the joint-space optimum of
    # the same problem (tip weights removed) takes it.
    plain = w.figure8_solve(0, 2, n=3, N=16, dt=0.05)
    plain.Wee = plain.WeeN = plain.pref = None
    rp = oracle.sqp(plain, oracle.Params(sqp_iters=60, kkt_mode=2))
    err = lambda X: np.linalg.norm([_fk.tip(s.links, x[:3]) - p for x, p in zip(X, s.pref)], axis=1)
    assert err(res.X).mean() < 0.7 * err(rp.X).mean()
    assert err(res.X)[-1] < 0.6 * err(rp.X)[-1]


def test_zero_tip_weights_reduce_to_the_joint_space_problem(oracle_lib):
    s, X, U = _fig8(n=7, N=6, seed=4)
    s0 = w.figure8_solve(4, 0, n=7, N=6)
    s0.Wee = np.zeros(3)
    s0.WeeN = np.zeros(3)
    plain = w.figure8_solve(4, 0, n=7, N=6)
    plain.Wee = plain.WeeN = plain.pref = None
    a = oracle.qp_step(s0, X, U, mode=0)
    b = oracle.qp_step(plain, X, U, mode=0)
    np.testing.assert_allclose(a[0], b[0], atol=1e-13 * np.abs(b[0]).max())
    np.testing.assert_allclose(a[2], b[2], atol=1e-13 * np.abs(b[2]).max())
