"""External tip force (the disturbance hypotheses of Sec. IV-D) on the GPU:
LQ data, SQP trajectories and the plant against the FP64 oracle with the same
force."""
import dataclasses
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


def _f32(a):
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


def _forced(seed, M, n=7, N=32, scale=20.0):
    rng = np.random.default_rng(seed)
    return [dataclasses.replace(w.chain_solve(seed, i, n=n, N=N),
                                fext=tuple(float(v) for v in _f32(rng.normal(0, scale, 3)))) for i in range(M)]


@pytest.mark.parametrize("n,N,M", [(7, 32, 3), (3, 16, 2), (6, 48, 2), (7, 128, 1)])
def test_lq_stage_parity_with_force(n, N, M):
    _say(f"lq force n={n} N={N}")
    solves = _forced(60 + n, M, n=n, N=N)
    rng = np.random.default_rng(n)
    for s in solves:
        s.X0 = s.X0 + rng.normal(0, 0.1, s.X0.shape)
        s.U0 = rng.normal(0, 2.0, s.U0.shape)
    b = g.Batch.from_solves(solves)
    xs, goal, X, U = g.pack_inputs(solves)
    A, B, e = (t.cpu().numpy().astype(np.float64) for t in b.debug_lq(xs, goal, X, U))
    b.close()
    for i, s in enumerate(solves):
        L = oracle.lq(s, _f32(s.X0), _f32(s.U0))
        nx, nu = 2 * n, n
        for name, got, ref in (("A", A[i, :N - 1, :nx, :nx], L["A"]), ("B", B[i, :N - 1, :nx, :nu], L["B"]),
                               ("e", e[i, :N - 1, :nx], L["e"])):
            err = np.abs(got - ref).max()
            assert err <= 2e-5 * max(1.0, np.abs(ref).max()), (name, i, err)


def test_sqp_trajectory_parity_with_force():
    _say("sqp force")
    solves = _forced(70, 3)
    b = g.Batch.from_solves(solves, g.Params(sqp_iters=4, pcg_tol=1e-7))
    xs, goal, X, U = g.pack_inputs(solves)
    st = b.solve(xs, goal, X, U)
    Xg, Ug = X.cpu().numpy().astype(np.float64), U.cpu().numpy().astype(np.float64)
    b.close()
    for i, s in enumerate(solves):
        ref = oracle.sqp(s, oracle.Params(sqp_iters=4, kkt_mode=0), alpha_replay=st[i]["alpha"].astype(np.float64))
        ex = np.abs(Xg[i] - ref.X).max() / np.abs(ref.X).max()
        eu = np.abs(Ug[i] - ref.U).max() / np.abs(ref.U).max()
        assert ex <= 1e-4 and eu <= 1e-4, (i, ex, eu)


def test_plant_true_force_overrides_the_slot_force():
    _say("plant force")
    solves = _forced(80, 4)
    b = g.Batch.from_solves(solves)
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, (4, 14)).astype(np.float32)
    tau = rng.normal(0, 3, (4, 7)).astype(np.float32)
    true_f = rng.normal(0, 30, (4, 3)).astype(np.float32)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(tau).cuda()
    own = b.plant_step(xd, td).cpu().numpy()
    over = b.plant_step(xd, td, fext=torch.from_numpy(true_f).cuda()).cpu().numpy()
    b.close()
    for i, s in enumerate(solves):
        r_own = oracle.plant_rk4(s, x[i].astype(np.float64), tau[i].astype(np.float64), 0.01, 10)
        r_true = oracle.plant_rk4(dataclasses.replace(s, fext=tuple(true_f[i].astype(np.float64))),
                                  x[i].astype(np.float64), tau[i].astype(np.float64), 0.01, 10)
        np.testing.assert_allclose(own[i], r_own, rtol=2e-6, atol=2e-6)
        np.testing.assert_allclose(over[i], r_true, rtol=2e-6, atol=2e-6)
