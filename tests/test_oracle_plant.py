"""Pins of the oracle's closed-loop plant (RK4 on the continuous dynamics, Sec. IV-E).

* Linear spring chain: x' = A x + b is solved exactly by the matrix exponential
  of the augmented system, which RK4 must match to rounding.
* Nonlinear chain: the error against a fine-step solution falls by 2^4 when the
  step halves (fourth order).
* Nonlinear chain, zero torque: kinetic plus potential energy, both computed
  from the independent forward kinematics of tests/_fk.py, is conserved.
"""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle
import workload as w

from . import _fk


def test_rk4_matches_the_matrix_exponential_on_the_linear_chain():
    for n, ks in ((3, 1.0), (4, 0.0), (2, 3.0)):
        s = w.double_integrator_solve(7, n, n=n, N=4, spring_k=ks)
        T = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
        A = np.block([[np.zeros((n, n)), np.eye(n)], [-ks * T, np.zeros((n, n))]])
        rng = np.random.default_rng(n)
        x0, u = rng.normal(size=2 * n), rng.normal(size=n)
        h = 0.01
        aug = np.zeros((2 * n + 1, 2 * n + 1))
        aug[:2 * n, :2 * n] = A
        aug[n:2 * n, 2 * n] = u
        exact = (expm(aug * h) @ np.concatenate([x0, [1.0]]))[:2 * n]
        got = oracle.plant_rk4(s, x0, u, h=h, substeps=10)
        np.testing.assert_allclose(got, exact, rtol=1e-12, atol=1e-13)


def test_rk4_is_fourth_order_on_the_chain():
    s = w.chain_solve(3, 0, n=7)
    x0 = np.concatenate([s.xs[:7], [0.5, -0.3, 0.2, 0.1, -0.4, 0.3, 0.2]])
    tau = np.linspace(-2.0, 2.0, 7)
    ref = oracle.plant_rk4(s, x0, tau, h=0.05, substeps=800)
    errs = [np.abs(oracle.plant_rk4(s, x0, tau, h=0.05, substeps=k) - ref).max() for k in (10, 20)]
    assert 12.0 < errs[0] / errs[1] < 20.0, errs


def test_rk4_conserves_energy_without_torque():
    s = w.chain_solve(4, 1, n=6)

    def energy(x):
        q, qd = x[:6], x[6:]
        return 0.5 * qd @ _fk.mass_matrix(s.links, q) @ qd + _fk.potential(s.links, q)

    x = np.concatenate([s.xs[:6], np.full(6, 0.3)])
    e0 = energy(x)
    for _ in range(50):                       # 0.5 s of free motion at 1 kHz
        x = oracle.plant_rk4(s, x, np.zeros(6), h=0.01, substeps=10)
    assert abs(energy(x) - e0) <= 1e-8 * max(1.0, abs(e0))


def test_rk4_rejects_zero_substeps():
    s = w.chain_solve(0, 0, n=3)
    with pytest.raises(FloatingPointError):
        oracle.plant_rk4(s, s.xs, np.zeros(3), substeps=0)
