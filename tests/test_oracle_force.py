"""Pins of the oracle's external end-effector force (the disturbance model of
the hypothesize-and-test case study, Sec. IV-D).

A force f on the tip of the last link changes the joint torques by -J(q)^T f,
with J the tip's positional Jacobian from the independent forward kinematics
of tests/_fk.py (itself checked against central differences of the tip
position); forward-dynamics derivatives with the force match central
differences; and the power balance gains the force's power f . v_tip.
"""
import dataclasses

import numpy as np

import oracle
import workload as w

from . import _fk


def _with_force(s, f):
    return dataclasses.replace(s, fext=tuple(float(v) for v in f))


def test_tip_jacobian_matches_finite_differences():
    s = w.chain_solve(8, 0, n=7)
    q = np.random.default_rng(1).uniform(-1, 1, 7)
    J = _fk.tip_jacobian(s.links, q)
    h = 1e-6
    Jfd = np.stack([(_fk.tip(s.links, q + h * e) - _fk.tip(s.links, q - h * e)) / (2 * h) for e in np.eye(7)], 1)
    np.testing.assert_allclose(J, Jfd, atol=1e-8)


def test_force_enters_as_minus_j_transpose_f():
    rng = np.random.default_rng(2)
    for n in (3, 6, 7):
        s = w.chain_solve(9, n, n=n)
        q, qd, qdd = rng.uniform(-1, 1, n), rng.normal(0, 1, n), rng.normal(0, 1, n)
        f = rng.normal(0, 10, 3)
        t0 = oracle.inverse_dynamics(s, q, qd, qdd)
        t1 = oracle.inverse_dynamics(_with_force(s, f), q, qd, qdd)
        np.testing.assert_allclose(t1 - t0, -_fk.tip_jacobian(s.links, q).T @ f, atol=1e-10)
        # The inertia matrix does not depend on the force.
        np.testing.assert_allclose(oracle.mass_matrix(_with_force(s, f), q), oracle.mass_matrix(s, q), atol=1e-12)


def test_forward_dynamics_derivatives_with_force():
    rng = np.random.default_rng(3)
    s = _with_force(w.chain_solve(10, 0, n=7), rng.normal(0, 20, 3))
    q, qd, tau = rng.uniform(-1, 1, 7), rng.normal(0, 1, 7), rng.normal(0, 3, 7)
    _, dq, dqd, _ = oracle.fd_derivatives(s, q, qd, tau)
    h = 1e-6
    for j in range(7):
        e = np.eye(7)[j]
        num_q = (oracle.forward_dynamics(s, q + h * e, qd, tau) - oracle.forward_dynamics(s, q - h * e, qd, tau)) / (2 * h)
        num_qd = (oracle.forward_dynamics(s, q, qd + h * e, tau) - oracle.forward_dynamics(s, q, qd - h * e, tau)) / (2 * h)
        np.testing.assert_allclose(dq[:, j], num_q, rtol=1e-6, atol=1e-6 * np.abs(num_q).max())
        np.testing.assert_allclose(dqd[:, j], num_qd, rtol=1e-6, atol=1e-6 * np.abs(num_qd).max())


def test_power_balance_with_force():
    # d/dt (kinetic + potential) = qd . tau + f . v_tip along the motion.
    rng = np.random.default_rng(4)
    s0 = w.chain_solve(11, 0, n=6)
    f = rng.normal(0, 15, 3)
    s = _with_force(s0, f)
    q, qd, tau = rng.uniform(-1, 1, 6), rng.normal(0, 1, 6), rng.normal(0, 2, 6)

    def energy(qq, qqd):
        return 0.5 * qqd @ _fk.mass_matrix(s0.links, qq) @ qqd + _fk.potential(s0.links, qq)

    qdd = oracle.forward_dynamics(s, q, qd, tau)
    h = 1e-6
    dE = (energy(q + h * qd, qd + h * qdd) - energy(q - h * qd, qd - h * qdd)) / (2 * h)
    v_tip = _fk.tip_jacobian(s0.links, q) @ qd
    assert abs(dE - (qd @ tau + f @ v_tip)) <= 1e-6 * max(1.0, abs(dE))


def test_hypothesis_selection_picks_the_force_that_explains_the_step(oracle_lib):
    # The measured state is the plant's own step under force 3 of the list:
    # that hypothesis is at distance 0 and wins; a duplicate of it later in the
    # list ties and loses to the earlier index; distances are those of the
    # individual predictions.
    import dataclasses
    s = w.chain_solve(8, 0, n=7, N=4)
    rng = np.random.default_rng(8)
    x = np.concatenate([rng.uniform(-1, 1, 7), rng.normal(0, 0.3, 7)])
    tau = rng.normal(0, 2, 7)
    forces = rng.normal(0, 15, (6, 3))
    forces[5] = forces[3]
    meas = oracle.plant_rk4(dataclasses.replace(s, fext=tuple(forces[3])), x, tau, 0.01, 10)
    j, d = oracle.hypothesis_select(s, x, tau, forces, meas)
    assert j == 3 and d[3] == 0.0 and d[5] == 0.0
    assert np.all(np.delete(d, [3, 5]) > 1e-6)
    other = oracle.plant_rk4(dataclasses.replace(s, fext=tuple(forces[1])), x, tau, 0.01, 10)
    assert d[1] == np.linalg.norm(other - meas)
