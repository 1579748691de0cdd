"""Batched rho sweep with line-search-driven rho adaptation (Sec. IV-C) on the GPU.

M copies of one problem start from log-spaced rho in [1e-8, 1e1] and adapt rho
after every SQP iteration. Each solve is replayed in the FP64 oracle with the
GPU's accepted steps and descent decisions: trajectories to the 1e-4 bar, and
the same rho sequence.
"""
import sys

import numpy as np
import pytest

import oracle
import workload as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2510_07625_amd as g  # noqa: E402


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("zero_init", [False, True])
def test_rho_sweep_with_adaptation_matches_the_oracle(zero_init):
    _say(f"rho sweep zero_init={zero_init}")
    M, iters = 8, 6
    base = w.chain_solve(41, 0, n=7, N=32, zero_init=zero_init)
    solves = [base] * M
    rho0 = np.logspace(-8, 1, M)
    b = g.Batch.from_solves(solves, g.Params(sqp_iters=iters, pcg_tol=1e-7, rho_adapt=1))
    b.set_rho(rho0)
    xs, goal, X, U = g.pack_inputs(solves)
    st = b.solve(xs, goal, X, U)
    rho_end = b.get_rho()
    Xg, Ug = X.cpu().numpy().astype(np.float64), U.cpu().numpy().astype(np.float64)
    b.close()
    for i in range(M):
        s = st[i]
        descent = [0 if (v & (g.ST_NO_DESCENT | g.ST_NONFINITE)) else 1 for v in s["status"]]
        ref = oracle.sqp(base, oracle.Params(sqp_iters=iters, kkt_mode=0, rho=rho0[i], rho_adapt=1),
                         alpha_replay=s["alpha"].astype(np.float64), descent_replay=descent)
        np.testing.assert_allclose(s["rho"], [L["rho"] for L in ref.logs], rtol=1e-6)
        last = ref.logs[-1]["rho"]
        want_end = last / 3.0 if descent[-1] else min(2.0 * last, 1e8)
        assert rho_end[i] == pytest.approx(want_end, rel=1e-12)
        ex = np.abs(Xg[i] - ref.X).max() / np.abs(ref.X).max()
        eu = np.abs(Ug[i] - ref.U).max() / np.abs(ref.U).max()
        assert ex <= 1e-4 and eu <= 1e-4, (i, rho0[i], ex, eu)
