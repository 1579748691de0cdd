"""Pins of the oracle's rigid-body dynamics and discretisation (CPU only).

The oracle's inverse dynamics is a Newton-Euler recursion in base coordinates.
It is checked here against things it does not share code with: textbook closed
forms of a two-link chain, the Lagrangian form of the dynamics built from
geometric Jacobians (tests/_fk.py), and finite differences.
"""
import numpy as np
import pytest

import oracle
import workload as w
from tests import _fk


def _chain(n, seed=0, i=0):
    return w.chain_solve(seed, i, n=n, N=4)


def test_two_link_closed_forms(oracle_lib):
    # Joint 0 about the vertical z axis, joint 1 about y: link 1 is an inverted
    # pendulum on a turntable. With the COM of link 1 at l1/2:
    #   M11 = Iyy1 + m1 (l1/2)^2,  M01 = 0,
    #   M00 = Izz0 + Ixx1 sin^2 q1 + Izz1 cos^2 q1 + m1 (l1/2 sin q1)^2,
    #   gravity torque on joint 1 = -m1 g (l1/2) sin q1, none on joint 0.
    s = _chain(2)
    l1, m1, Ixx1, Iyy1, Izz1 = s.links[1]
    Izz0 = s.links[0][4]
    g = 9.81
    for q in ([0.3, 0.0], [-1.1, 0.7], [2.0, -2.5]):
        q = np.array(q)
        M = oracle.mass_matrix(s, q)
        s1, c1 = np.sin(q[1]), np.cos(q[1])
        M00 = Izz0 + Ixx1 * s1 ** 2 + Izz1 * c1 ** 2 + m1 * (0.5 * l1 * s1) ** 2
        M11 = Iyy1 + m1 * (0.5 * l1) ** 2
        np.testing.assert_allclose(M, [[M00, 0.0], [0.0, M11]], atol=1e-13)
        tau = oracle.inverse_dynamics(s, q, np.zeros(2), np.zeros(2))
        np.testing.assert_allclose(tau, [0.0, -m1 * g * 0.5 * l1 * s1], atol=1e-12)


@pytest.mark.parametrize("n", [1, 3, 7])
def test_mass_matrix_matches_jacobian_form(oracle_lib, n):
    s = _chain(n, seed=4)
    rng = np.random.default_rng(n)
    for _ in range(5):
        q = rng.uniform(-np.pi, np.pi, n)
        M = oracle.mass_matrix(s, q)
        np.testing.assert_allclose(M, _fk.mass_matrix(s.links, q), rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(M, M.T, atol=1e-13)
        assert np.linalg.eigvalsh(M).min() > 0


@pytest.mark.parametrize("n", [2, 3, 7])
def test_inverse_dynamics_matches_lagrangian(oracle_lib, n):
    s = _chain(n, seed=5)
    rng = np.random.default_rng(10 + n)
    for _ in range(3):
        q, qd, qdd = rng.uniform(-1.5, 1.5, n), rng.normal(0, 1.0, n), rng.normal(0, 2.0, n)
        tau = oracle.inverse_dynamics(s, q, qd, qdd)
        ref = _fk.lagrangian_id(s.links, q, qd, qdd)
        np.testing.assert_allclose(tau, ref, rtol=1e-7, atol=1e-7 * np.abs(ref).max())


def test_forward_inverse_consistency(oracle_lib):
    s = _chain(7, seed=6)
    rng = np.random.default_rng(3)
    for _ in range(5):
        q, qd, tau = rng.uniform(-1, 1, 7), rng.normal(0, 1, 7), rng.normal(0, 5, 7)
        qdd = oracle.forward_dynamics(s, q, qd, tau)
        np.testing.assert_allclose(oracle.inverse_dynamics(s, q, qd, qdd), tau, atol=1e-11)


def test_power_balance(oracle_lib):
    # Along qdd = FD(q, qd, tau): d/dt (1/2 qd^T M qd + V) = qd^T tau.
    s = _chain(7, seed=7)
    rng = np.random.default_rng(8)
    q, qd, tau = rng.uniform(-1, 1, 7), rng.normal(0, 1, 7), rng.normal(0, 3, 7)
    qdd = oracle.forward_dynamics(s, q, qd, tau)
    h = 1e-5
    def energy(t):
        qt, qdt = q + t * qd + 0.5 * t * t * qdd, qd + t * qdd
        return 0.5 * qdt @ _fk.mass_matrix(s.links, qt) @ qdt + _fk.potential(s.links, qt)
    dEdt = (energy(h) - energy(-h)) / (2 * h)
    assert abs(dEdt - qd @ tau) < 1e-6 * max(1.0, abs(qd @ tau))


@pytest.mark.parametrize("n", [3, 7])
def test_fd_derivatives_match_finite_differences(oracle_lib, n):
    s = _chain(n, seed=9)
    rng = np.random.default_rng(20 + n)
    q, qd, tau = rng.uniform(-1, 1, n), rng.normal(0, 0.5, n), rng.normal(0, 3, n)
    qdd, dq, dqd, Minv = oracle.fd_derivatives(s, q, qd, tau)
    h = 1e-6
    Jq, Jqd, Jt = np.zeros((n, n)), np.zeros((n, n)), np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = h
        Jq[:, j] = (oracle.forward_dynamics(s, q + e, qd, tau) - oracle.forward_dynamics(s, q - e, qd, tau)) / (2 * h)
        Jqd[:, j] = (oracle.forward_dynamics(s, q, qd + e, tau) - oracle.forward_dynamics(s, q, qd - e, tau)) / (2 * h)
        Jt[:, j] = (oracle.forward_dynamics(s, q, qd, tau + e) - oracle.forward_dynamics(s, q, qd, tau - e)) / (2 * h)
    for a, b in ((dq, Jq), (dqd, Jqd), (Minv, Jt)):
        np.testing.assert_allclose(a, b, rtol=1e-6, atol=1e-6 * np.abs(b).max())
    np.testing.assert_allclose(Minv, np.linalg.inv(oracle.mass_matrix(s, q)), rtol=1e-10, atol=1e-12)


def test_euler_step_and_jacobians(oracle_lib):
    s = _chain(7, seed=11)
    rng = np.random.default_rng(5)
    x, u = np.concatenate([rng.uniform(-1, 1, 7), rng.normal(0, 0.3, 7)]), rng.normal(0, 2, 7)
    xn, A, B = oracle.step_jacobians(s, x, u)
    qdd = oracle.forward_dynamics(s, x[:7], x[7:], u)
    np.testing.assert_allclose(xn, np.concatenate([x[:7] + s.dt * x[7:], x[7:] + s.dt * qdd]), atol=1e-14)
    h = 1e-6
    for j in range(14):
        e = np.zeros(14)
        e[j] = h
        col = (oracle.step(s, x + e, u) - oracle.step(s, x - e, u)) / (2 * h)
        np.testing.assert_allclose(A[:, j], col, rtol=1e-6, atol=1e-9)
    for j in range(7):
        e = np.zeros(7)
        e[j] = h
        col = (oracle.step(s, x, u + e) - oracle.step(s, x, u - e)) / (2 * h)
        np.testing.assert_allclose(B[:, j], col, rtol=1e-6, atol=1e-10)
    # Explicit Euler structure: top rows [I, hI] and [0].
    np.testing.assert_array_equal(A[:7, :7], np.eye(7))
    np.testing.assert_array_equal(A[:7, 7:], s.dt * np.eye(7))
    np.testing.assert_array_equal(B[:7], np.zeros((7, 7)))


def test_double_integrator_chain_is_linear(oracle_lib):
    s = w.double_integrator_solve(0, 0, n=4, N=5, spring_k=1.0)
    T = 2 * np.eye(4) - np.eye(4, k=1) - np.eye(4, k=-1)
    rng = np.random.default_rng(2)
    x, u = rng.normal(size=8), rng.normal(size=4)
    xn, A, B = oracle.step_jacobians(s, x, u)
    h = s.dt
    A_ref = np.block([[np.eye(4), h * np.eye(4)], [-h * s.spring_k * T, np.eye(4)]])
    B_ref = np.vstack([np.zeros((4, 4)), h * np.eye(4)])
    np.testing.assert_allclose(A, A_ref, atol=1e-15)
    np.testing.assert_allclose(B, B_ref, atol=1e-15)
    np.testing.assert_allclose(xn, A_ref @ x + B_ref @ u, atol=1e-14)
