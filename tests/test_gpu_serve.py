"""Serving path on the GPU: warm-start shift, batch invariance and a served run."""
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
from paper_2510_07625_amd.serve import GpuExecutor, NativeScheduler, Request, Scheduler  # noqa: E402


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _pool(P, seed=0, **kw):
    solves = w.chain_batch(seed, P)
    b = g.Batch.from_solves(solves, g.Params(**kw))
    xs, goal, X, U = g.pack_inputs(solves)
    return solves, b, xs, goal, X, U


def test_shifted_serve_step_equals_step_on_shifted_trajectory():
    _say("serve shift")
    solves, b, xs, goal, X, U = _pool(4, seed=1, sqp_iters=2, warm_lambda=0)
    b.step(xs, goal, X, U, 2)                   # some non-trivial trajectories
    b.set_trajectories(X, U)
    slots = torch.tensor([2, 0], dtype=torch.int32, device="cuda")
    Xo = torch.zeros((2,) + tuple(X.shape[1:]), device="cuda")
    Uo = torch.zeros((2,) + tuple(U.shape[1:]), device="cuda")
    b.serve_step(slots, xs[[2, 0]].contiguous(), goal[[2, 0]].contiguous(), n_iters=1, shift=1, Xout=Xo, Uout=Uo)
    Xs = torch.cat([X[:, 1:], X[:, -1:]], dim=1).contiguous()
    Us = torch.cat([U[:, 1:], U[:, -1:]], dim=1).contiguous()
    b.step(xs, goal, Xs, Us, 1)
    torch.cuda.synchronize()
    assert torch.equal(Xo[0], Xs[2]) and torch.equal(Xo[1], Xs[0])
    assert torch.equal(Uo[0], Us[2]) and torch.equal(Uo[1], Us[0])
    Xr, Ur = b.get_trajectories()
    assert torch.equal(Xr[2], Xs[2]) and torch.equal(Xr[1], X[1])   # untouched slots keep their state
    b.close()


def test_result_is_the_same_alone_and_in_the_mix():
    _say("serve batch invariance")
    solves, b, xs, goal, X, U = _pool(8, seed=2)
    b.set_trajectories(X, U)
    outs = []
    for slots in ([5], [1, 5, 7, 3]):
        b.set_trajectories(X, U)
        b.reset_warm_start()
        sl = torch.tensor(slots, dtype=torch.int32, device="cuda")
        Xo = torch.zeros((len(slots),) + tuple(X.shape[1:]), device="cuda")
        b.serve_step(sl, xs[slots].contiguous(), goal[slots].contiguous(), n_iters=2, shift=1, Xout=Xo)
        torch.cuda.synchronize()
        outs.append(Xo[slots.index(5)].clone())
    assert torch.equal(outs[0], outs[1])
    b.close()


def test_served_resolve_matches_the_oracle():
    _say("serve parity")
    solves, b, xs, goal, X, U = _pool(3, seed=3, pcg_tol=1e-7)
    b.set_trajectories(X, U)
    sl = torch.tensor([0, 1, 2], dtype=torch.int32, device="cuda")
    st = torch.zeros(3 * 3 * g.STATS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    Xo = torch.zeros_like(X)
    Uo = torch.zeros_like(U)
    b.serve_step(sl, xs, goal, n_iters=3, shift=0, Xout=Xo, Uout=Uo, d_stats=st)
    stats = g.Batch.decode_stats(st, 3, 3)
    Xg, Ug = Xo.cpu().numpy(), Uo.cpu().numpy()
    for i, s in enumerate(solves):
        ref = oracle.sqp(s, oracle.Params(sqp_iters=3, kkt_mode=0), alpha_replay=stats[i]["alpha"].astype(float))
        assert np.abs(Xg[i] - ref.X).max() <= 1e-4 * np.abs(ref.X).max()
        assert np.abs(Ug[i] - ref.U).max() <= 1e-4 * np.abs(ref.U).max()
    b.close()


def test_short_served_run():
    _say("served run")
    P = 32
    solves, b, xs, goal, X, U = _pool(P, seed=4)
    b.set_trajectories(X, U)
    ex = GpuExecutor(b, slots=3, n_iters=1)
    g_ = np.random.default_rng(0)
    reqs = []
    t = 0.0
    for i in range(300):
        t += g_.exponential(1 / 5000)
        inst = int(g_.integers(P))
        reqs.append(Request(i, inst, t, solves[inst].qgoal + g_.normal(0, 0.05, 7)))
    sch = Scheduler(ex, np.stack([s.xs for s in solves]), deadline_s=1e-3)
    rep = sch.run(reqs)
    ex.close()
    s = rep.summary()
    print("served:", s)
    assert s["completed"] == 300 and s["rejected"] == 0
    assert all((c.status & g.ST_NONFINITE) == 0 for c in rep.completions)
    b.close()


def test_serve_context_equals_the_serve_step():
    _say("serve context")
    solves, b1, xs, goal, X, U = _pool(6, seed=6)
    b2 = g.Batch.from_solves(solves, g.Params())
    b1.set_trajectories(X, U)
    b2.set_trajectories(X, U)
    sl = [4, 1, 3]
    ctx = g.ServeContext(b1, capacity=4, n_iters=2)
    ctx.slots[:3] = sl
    ctx.xs[:3] = xs[sl].cpu().numpy()
    ctx.goal[:3] = goal[sl].cpu().numpy()
    ctx.submit(3, shift=1)
    while not ctx.done():
        pass
    Xo = torch.zeros((3,) + tuple(X.shape[1:]), device="cuda")
    Uo = torch.zeros((3,) + tuple(U.shape[1:]), device="cuda")
    st = torch.zeros(3 * 2 * g.STATS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    b2.serve_step(torch.tensor(sl, dtype=torch.int32, device="cuda"), xs[sl].contiguous(), goal[sl].contiguous(),
                  n_iters=2, shift=1, Xout=Xo, Uout=Uo, d_stats=st)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ctx.x1[:3], Xo[:, 1].cpu().numpy())
    np.testing.assert_array_equal(ctx.u0[:3], Uo[:, 0].cpu().numpy())
    np.testing.assert_array_equal(ctx.stats[:3]["alpha"], g.Batch.decode_stats(st, 3, 2)["alpha"])
    Xf, Uf = ctx.trajectories()
    np.testing.assert_array_equal(Xf, Xo.cpu().numpy())
    np.testing.assert_array_equal(Uf, Uo.cpu().numpy())
    ctx.slots[0] = 99                                     # outside 0..M-1: rejected on the host
    with pytest.raises(g.GatoError):
        ctx.submit(1)
    ctx.close()
    b1.close()
    b2.close()


def _stream(P, solves, n, rate, seed):
    g_ = np.random.default_rng(seed)
    reqs, t = [], 0.0
    for i in range(n):
        t += g_.exponential(1 / rate)
        inst = int(g_.integers(P))
        reqs.append(Request(i, inst, t, solves[inst].qgoal + g_.normal(0, 0.05, 7)))
    return reqs


def test_native_loop_ends_in_the_same_states_as_the_python_loop():
    # A request's result depends only on its instance's own history (its FIFO
    # order, start states and warm starts), never on which launch it joined,
    # so both loops must leave every instance in the bit-identical state.
    _say("native serve loop vs python loop")
    P = 24
    solves, b1, xs, goal, X, U = _pool(P, seed=7)
    b2 = g.Batch.from_solves(solves, g.Params())
    b1.set_trajectories(X, U)
    b2.set_trajectories(X, U)
    reqs = _stream(P, solves, 400, 20000.0, seed=1)
    x0 = np.stack([s.xs for s in solves])
    ex = GpuExecutor(b1, slots=3, n_iters=2)
    py = Scheduler(ex, x0, deadline_s=1e-3)
    rp = py.run(reqs)
    ex.close()
    nat = NativeScheduler(b2, x0, slots=3, n_iters=2)
    rn = nat.run(reqs)
    sp, sn = rp.summary(), rn.summary()
    print("python:", sp)
    print("native:", sn)
    assert sn["completed"] == sp["completed"] == 400 and sn["rejected"] == 0
    np.testing.assert_array_equal(nat.state, py.state.astype(np.float32))
    # The control of each instance's last request agrees too.
    last_p = {c.instance: c for c in sorted(rp.completions, key=lambda c: c.rid)}
    last_n = {c.instance: c for c in sorted(rn.completions, key=lambda c: c.rid)}
    for i in last_p:
        np.testing.assert_array_equal(last_n[i].u0, last_p[i].u0)
        assert last_n[i].status == last_p[i].status
    assert all(c.launched >= c.arrival and c.done > c.launched for c in rn.completions)
    assert 1 <= rn.launches <= 400 and 1 <= rn.max_inflight <= 3
    b1.close()
    b2.close()


def test_native_loop_rejects_beyond_the_queue_limit():
    _say("native serve loop queue limit")
    P = 8
    solves, b, xs, goal, X, U = _pool(P, seed=8)
    b.set_trajectories(X, U)
    reqs = [Request(i, i % P, 0.0, solves[i % P].qgoal) for i in range(64)]   # one burst
    nat = NativeScheduler(b, np.stack([s.xs for s in solves]), slots=2, n_iters=1, queue_limit=10)
    rep = nat.run(reqs)
    assert len(rep.rejected) == 54 and len(rep.completions) == 10
    assert sorted(c.rid for c in rep.completions) == list(range(10))
    b.close()


def test_shift_then_serve_equals_serve_with_shift_and_multipliers_round_trip():
    _say("shift warm start")
    solves, b1, xs, goal, X, U = _pool(5, seed=12, sqp_iters=2)
    b2 = g.Batch.from_solves(solves, g.Params(sqp_iters=2))
    for b in (b1, b2):
        b.step(xs, goal, X.clone(), U.clone(), 1)       # non-trivial multipliers in both
        b.set_trajectories(X, U)
    lam = b1.get_multipliers()
    b2.set_multipliers(lam)
    torch.cuda.synchronize()
    assert torch.equal(b2.get_multipliers(), lam) and lam.abs().max() > 0
    sl = torch.tensor([3, 0, 4], dtype=torch.int32, device="cuda")
    outs = []
    for b, shift in ((b1, 1), (b2, 0)):
        if shift == 0:
            b.shift_warm_start(sl)
        Xo = torch.zeros((3,) + tuple(X.shape[1:]), device="cuda")
        Uo = torch.zeros((3,) + tuple(U.shape[1:]), device="cuda")
        b.serve_step(sl, xs[[3, 0, 4]].contiguous(), goal[[3, 0, 4]].contiguous(), n_iters=2, shift=shift,
                     Xout=Xo, Uout=Uo)
        torch.cuda.synchronize()
        outs.append((Xo, Uo, b.get_multipliers()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    assert torch.equal(outs[0][2], outs[1][2])
    b1.close()
    b2.close()
