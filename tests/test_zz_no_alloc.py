"""The allocation-free entry point gato_solve_static against gato_solve.

gato_solve_static runs the same kernels as gato_solve with the statistics
staged in the library's static device array instead of a buffer the batch
allocates, so trajectories and statistics must agree bit for bit. Two calls in
a row share the array: the second, smaller one must not see the first one's
contents. A statistics request beyond the array's size is refused before
anything is launched.
"""
import sys

import numpy as np
import pytest

import workload as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2510_07625_amd as g  # noqa: E402


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _both(solves, params):
    """Runs gato_solve and gato_solve_static from the same inputs and warm start."""
    b = g.Batch.from_solves(solves, params)
    xs, goal, X0, U0 = g.pack_inputs(solves)
    Xa, Ua = X0.clone(), U0.clone()
    b.reset_warm_start()
    sa = b.solve(xs, goal, Xa, Ua)
    Xb, Ub = X0.clone(), U0.clone()
    b.reset_warm_start()
    sb = b.solve_static(xs, goal, Xb, Ub)
    # Without statistics the static form must leave the same trajectories.
    Xc, Uc = X0.clone(), U0.clone()
    b.reset_warm_start()
    b.solve_static(xs, goal, Xc, Uc, stats=False)
    torch.cuda.synchronize()
    b.close()
    return (Xa.cpu().numpy(), Ua.cpu().numpy(), sa), (Xb.cpu().numpy(), Ub.cpu().numpy(), sb), \
        (Xc.cpu().numpy(), Uc.cpu().numpy())


def _same(a, b, c):
    Xa, Ua, sa = a
    Xb, Ub, sb = b
    Xc, Uc = c
    assert np.array_equal(Xa, Xb) and np.array_equal(Ua, Ub)
    assert np.array_equal(Xa, Xc) and np.array_equal(Ua, Uc)
    assert sa.shape == sb.shape
    assert sa.tobytes() == sb.tobytes()


def test_static_solve_equals_solve_twice_second_smaller():
    _say("static solve: 48 7-DoF N = 32 solves, 4 SQP iterations")
    first = w.chain_batch(0, 48)
    a, b, c = _both(first, g.Params(sqp_iters=4))
    _same(a, b, c)
    assert (a[2]["pcg_iters"] > 0).all()
    _say("static solve: 10 uneven solves (a split N = 128 solve among them), 2 SQP iterations")
    second = w.uneven_batch(5, M=10, horizons=(16, 32, 128))
    assert any(s.N == 128 and s.n >= 6 for s in second)
    a, b, c = _both(second, g.Params(sqp_iters=2))
    _same(a, b, c)
    assert b[2].shape == (10, 2)
    assert not (b[2]["status"] & (g.ST_EXCHANGE | g.ST_NONFINITE)).any()


def test_static_solve_refuses_statistics_beyond_its_staging():
    _say("static solve: statistics beyond the staging are refused")
    solves = [w.chain_solve(0, i, n=3, N=2) for i in range(6554)]
    b = g.Batch.from_solves(solves, g.Params(sqp_iters=10))
    xs, goal, X, U = g.pack_inputs(solves)
    with pytest.raises(g.GatoError) as ei:
        b.solve_static(xs, goal, X, U)
    assert ei.value.code == -1 and "static" in str(ei.value)
    b.close()
