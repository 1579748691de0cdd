"""Pins of the oracle's PCG-count replay (CPU only).

The PCG stopping iteration of Sec. II-B is an integer that floating point
decides (the rule of reading R6 compares r^T P r with tol^2 gamma~^T P gamma~),
so two correct implementations that round differently may stop one iteration
apart. For parity the oracle can therefore replay another implementation's
count, and reports where its own rule stands at that count. These tests fix
the replay's behaviour by construction:
  * replaying the oracle's own counts changes nothing, bit for bit, and the
    rule first holds at the last replayed iteration;
  * with zero PCG iterations from zero multipliers the step is
    dZ = -G^-1 g (Eq. (4) with lambda = 0), which moves every knot onto
    [q_goal; 0] and every control to zero at alpha = 1;
  * replaying as many iterations as the system's dimension (conjugate
    gradients terminate in at most that many steps in exact arithmetic) gives
    the exact KKT solution of the dense LU solve;
  * fewer iterations than the rule needs leave the rule unmet.
"""
import numpy as np

import oracle
import workload as w


def _run(s, mode, iters=3, tol=1e-5, **kw):
    return oracle.sqp(s, oracle.Params(sqp_iters=iters, kkt_mode=mode, pcg_tol=tol), **kw)


def test_replaying_own_counts_is_bit_identical():
    s = w.chain_solve(0, 3, n=7, N=32)
    own = _run(s, 1)
    counts = [L["pcg_iters"] for L in own.logs]
    assert min(counts) > 0
    rep = _run(s, 1, pcg_replay=counts, alpha_replay=[L["alpha"] for L in own.logs])
    assert np.array_equal(own.X, rep.X) and np.array_equal(own.U, rep.U) and np.array_equal(own.lam, rep.lam)
    for L in rep.logs:
        assert L["pcg_stop"] <= 1.0 < L["pcg_stop_prev"], L


def test_zero_iterations_from_zero_multipliers_step_onto_the_goal():
    s = w.chain_solve(1, 0, n=6, N=16)
    r = _run(s, 1, iters=1, pcg_replay=[0], alpha_replay=[1.0])
    xg = np.concatenate([s.qgoal, np.zeros(s.n)])
    np.testing.assert_allclose(r.X, np.tile(xg, (s.N, 1)), rtol=0, atol=1e-12)
    np.testing.assert_allclose(r.U, 0.0, rtol=0, atol=1e-12)
    assert np.all(r.lam == 0.0)
    assert np.isinf(r.logs[0]["pcg_stop_prev"]) and r.logs[0]["pcg_stop"] > 1.0


def test_full_dimension_replay_reaches_the_dense_solution():
    s = w.chain_solve(2, 1, n=3, N=8)
    dim = s.N * 2 * s.n
    dense = _run(s, 0, iters=2)
    alphas = [L["alpha"] for L in dense.logs]
    rep = _run(s, 1, iters=2, pcg_replay=[dim, dim], alpha_replay=alphas)
    scale = np.abs(dense.X).max()
    assert np.abs(rep.X - dense.X).max() <= 1e-9 * scale
    assert np.abs(rep.U - dense.U).max() <= 1e-9 * max(np.abs(dense.U).max(), 1.0)
    for L in rep.logs:
        assert L["pcg_stop"] <= 1e-6


def test_short_replay_leaves_the_rule_unmet():
    s = w.chain_solve(0, 5, n=7, N=32)
    own = _run(s, 1, iters=2)
    counts = [L["pcg_iters"] for L in own.logs]
    short = [max(c // 2, 1) for c in counts]
    rep = _run(s, 1, iters=2, pcg_replay=short, alpha_replay=[L["alpha"] for L in own.logs])
    for L, c in zip(rep.logs, short):
        assert L["pcg_iters"] == c
        assert L["pcg_stop"] > 1.0
