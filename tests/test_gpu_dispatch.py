"""Uneven batches: mixed-shape launch, per-bucket mapping, autotuner, HIP graph.

Every mapping of a solve (knots per lane group, mixed or per-shape launch,
eager or graph) runs the same arithmetic on the same data; results must agree
to the trajectory tolerance (1e-4 relative, oracle-replayed) and, where the
reduction order is the same, bit for bit.
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


def _run(b, solves, iters, graph=False, reps=1):
    xs, goal, X0, U0 = g.pack_inputs(solves)
    st = b.stats_buffer(iters)
    for _ in range(reps):
        X, U = X0.clone(), U0.clone()
        b.reset_warm_start()
        b.step(xs, goal, X, U, iters, st, graph=graph)
        torch.cuda.synchronize()
    return X.cpu().numpy().astype(np.float64), U.cpu().numpy().astype(np.float64), g.Batch.decode_stats(st, b.M, iters)


def _oracle_check(s, Xg, Ug, st, iters, tol=1e-4):
    po = oracle.Params(sqp_iters=iters, kkt_mode=0 if s.N <= 32 else 2)
    ref = oracle.sqp(s, po, alpha_replay=st["alpha"].astype(np.float64))
    n, N = s.n, s.N
    ex = np.abs(Xg[:N, :2 * n] - ref.X).max() / np.abs(ref.X).max()
    eu = np.abs(Ug[:N - 1, :n] - ref.U).max() / np.abs(ref.U).max()
    assert ex <= tol and eu <= tol, (s.n, s.N, ex, eu)


def test_mixed_launch_equals_grouped_launches():
    _say("mixed vs grouped")
    solves = w.uneven_batch(11, M=12, horizons=(16, 32, 64, 128))
    p = g.Params(sqp_iters=2, pcg_tol=1e-7)
    b = g.Batch.from_solves(solves, p)
    assert len({(s.n, s.N) for s in solves}) > 1
    b.set_dispatch(g.DISPATCH_GROUPED)
    Xa, Ua, sa = _run(b, solves, 2)
    b.set_dispatch(g.DISPATCH_MIXED)
    Xb, Ub, sb = _run(b, solves, 2)
    b.close()
    np.testing.assert_array_equal(Xa, Xb)
    np.testing.assert_array_equal(Ua, Ub)
    np.testing.assert_array_equal(sa["pcg_iters"], sb["pcg_iters"])
    for i in (0, 5, 11):
        _oracle_check(solves[i], Xb[i], Ub[i], sb[i], 2)


@pytest.mark.parametrize("n,N,kpts", [(7, 32, (1, 2, 4)), (6, 64, (2, 4)), (3, 48, (1, 2))])
def test_every_mapping_matches_the_oracle(n, N, kpts):
    _say(f"mappings n={n} N={N}")
    solves = [w.chain_solve(21, i, n=n, N=N) for i in range(2)]
    p = g.Params(sqp_iters=3, pcg_tol=1e-7)
    b = g.Batch.from_solves(solves, p)
    for kpt in kpts:
        b.set_mapping(n, N, kpt)
        assert b.buckets()[0]["kpt"] == kpt
        Xg, Ug, st = _run(b, solves, 3)
        for i, s in enumerate(solves):
            _oracle_check(s, Xg[i], Ug[i], st[i], 3)
    with pytest.raises(g.GatoError):
        b.set_mapping(n, N, 8)
    b.close()


def test_autotune_picks_an_allowed_mapping_and_keeps_results():
    _say("autotune")
    solves = w.uneven_batch(12, M=16, horizons=(16, 32, 64, 128))
    p = g.Params(sqp_iters=2, pcg_tol=1e-7)
    b = g.Batch.from_solves(solves, p)
    xs, goal, X0, U0 = g.pack_inputs(solves)
    X0c, U0c = X0.clone(), U0.clone()
    bk = b.autotune(xs, goal, X0, U0, n_iters=1, reps=2)
    assert torch.equal(X0, X0c) and torch.equal(U0, U0c)          # inputs untouched
    assert sum(x["count"] for x in bk) == len(solves)
    for x in bk:
        G = 16 if x["n_dof"] > 4 else 8
        assert x["kpt"] in (1, 2, 4) and x["kpt"] * (512 // G) >= x["N"] and x["tuned_ms"] > 0
    print("autotuned:", bk)
    Xg, Ug, st = _run(b, solves, 2)
    b.close()
    for i, s in enumerate(solves):
        _oracle_check(s, Xg[i], Ug[i], st[i], 2)


def test_graph_replays_equal_the_eager_step():
    _say("graph")
    solves = w.uneven_batch(13, M=8, horizons=(16, 32, 64))
    p = g.Params(sqp_iters=2)
    b = g.Batch.from_solves(solves, p)
    Xe, Ue, se = _run(b, solves, 2)
    xs, goal, X0, U0 = g.pack_inputs(solves)
    X, U = X0.clone(), U0.clone()
    st = b.stats_buffer(2)
    for rep in range(4):                     # replays, with eager work and syncs between them
        X.copy_(X0)
        U.copy_(U0)
        b.reset_warm_start()
        b.step(xs, goal, X, U, 2, st, graph=True)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(X.cpu().numpy(), Xe.astype(np.float32))
        np.testing.assert_array_equal(U.cpu().numpy(), Ue.astype(np.float32))
        np.testing.assert_array_equal(g.Batch.decode_stats(st, b.M, 2)["alpha"], se["alpha"])
        _ = (X0 * 2).sum().item()            # unrelated eager work between replays
    b.close()
