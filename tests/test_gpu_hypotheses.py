"""Batched hypothesize-and-test over tip forces (Sec. IV-D) on the GPU.

The estimate is judged where the data can see it: the joint torque the
estimated force produces, J(q)^T f_est, approaches the true force's
J(q)^T f_true (force components that the joints cannot feel at a posture are
not observable from one step). The hypothesis batch also tracks the goal
better than a single solve that assumes no force.
"""
import sys

import numpy as np
import pytest

import workload as w

from . import _fk

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2510_07625_amd as g  # noqa: E402
from paper_2510_07625_amd import hypotheses  # noqa: E402


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _run(H, P=2, ticks=80, seed=90):
    base = [w.chain_solve(seed, p, n=7, N=32) for p in range(P)]
    solves = [s for s in base for _ in range(H)]
    b = g.Batch.from_solves(solves, g.Params(sqp_iters=2))
    xs, goal, X, U = g.pack_inputs(solves)
    b.set_trajectories(X, U)
    f_true = np.tile([[8.0, -12.0, -25.0]], (P, 1))
    r = hypotheses.run(b, P, H, xs[::H].contiguous(), goal[::H].contiguous(), ticks, lambda t: f_true, sigma=12.0)
    b.close()
    qg = np.stack([s.qgoal for s in base])
    q = r.states[:, :, :7].astype(np.float64)
    track = np.linalg.norm(q - qg[None], axis=2)                       # [ticks + 1, P]
    terr = np.zeros(track.shape)
    for t in range(q.shape[0]):
        for p in range(P):
            J = _fk.tip_jacobian(base[p].links, q[t, p])
            terr[t, p] = np.linalg.norm(J.T @ (r.estimates[t, p] - f_true[p])) / np.linalg.norm(J.T @ f_true[p])
    return r, terr, track


def test_hypotheses_explain_the_disturbance_and_track_better():
    _say("hypotheses")
    r, terr, track = _run(16)
    _, _, track1 = _run(1)
    print(f"relative torque error of the estimate: start {terr[0]}, last 10 ticks {terr[-10:].mean(axis=0)}")
    print(f"tracking, last 20 ticks: 16 hypotheses {track[-20:].mean():.4f} rad, one solve {track1[-20:].mean():.4f} rad")
    assert np.isfinite(r.states).all()
    assert (terr[-10:].mean(axis=0) < 0.5 * terr[0]).all()
    assert track[-20:].mean() < track1[-20:].mean()
