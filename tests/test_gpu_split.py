"""Long solves split across four workgroups (gato_set_split) against the oracle
and against the one-workgroup form.

Each part of a split solve holds the PCG rows of 32 knots and exchanges halo
rows and inner products with the other parts at every PCG iteration; the PCG
is the same method (Sec. III-B), with its inner products summed per part
first. Bars: the oracle replay of the accepted steps within 1e-4 (PCG
tolerance 1e-7, as the other trajectory tests), no exchange time-out, and the
multipliers within 1e-5 of the one-workgroup form (both stop at the PCG
tolerance) while not bit-identical to it (the split path ran).
"""
import sys

import numpy as np
import pytest

import oracle
import workload as w

from . import _parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2510_07625_amd as g  # noqa: E402


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _run(solves, p, parts, dispatch=None):
    b = g.Batch.from_solves(solves, p)
    b.set_split(parts)
    if dispatch is not None:
        b.set_dispatch(dispatch)
    xs, goal, X, U = g.pack_inputs(solves)
    st = b.stats_buffer(p.sqp_iters)
    b.reset_warm_start()
    b.step(xs, goal, X, U, p.sqp_iters, st)
    torch.cuda.synchronize()
    lam_d = b.get_multipliers()
    torch.cuda.synchronize()
    lam = lam_d.cpu().numpy()
    out = (X.cpu().numpy().astype(np.float64), U.cpu().numpy().astype(np.float64),
           g.Batch.decode_stats(st, b.M, p.sqp_iters), lam)
    b.close()
    return out


def _replay(s, Xg, Ug, st, iters):
    ref = oracle.sqp(s, oracle.Params(sqp_iters=iters, kkt_mode=2), alpha_replay=st["alpha"].astype(np.float64))
    n, N = s.n, s.N
    ex = np.abs(Xg[:N, :2 * n] - ref.X).max() / np.abs(ref.X).max()
    eu = np.abs(Ug[:N - 1, :n] - ref.U).max() / np.abs(ref.U).max()
    return ex, eu


# N = 128: four full parts; 100: the last part holds 4 knots; 80: the last part
# holds none (it still takes part in every exchange); 65: the third part holds a
# single knot (a left neighbour only) and the last none; 97: the last part holds
# a single knot.
@pytest.mark.parametrize("n,N", [(7, 128), (6, 100), (7, 80), (7, 65), (6, 97)])
def test_split_solve_matches_the_oracle_and_the_one_workgroup_form(n, N):
    _say(f"split n={n} N={N}")
    solves = [w.chain_solve(31, i, n=n, N=N) for i in range(2)]
    p = g.Params(sqp_iters=5, pcg_tol=1e-7)
    Xs, Us, ss, ls = _run(solves, p, 4)
    X1, U1, s1, l1 = _run(solves, p, 1)
    assert not (ss["status"] & (g.ST_EXCHANGE | g.ST_NONFINITE | g.ST_PCG_MAXITER)).any(), ss["status"]
    for i, s in enumerate(solves):
        ex, eu = _replay(s, Xs[i], Us[i], ss[i], p.sqp_iters)
        print(f"solve {i}: split vs oracle X {ex:.2e} U {eu:.2e}; PCG its split {ss[i]['pcg_iters'].tolist()} "
              f"one-workgroup {s1[i]['pcg_iters'].tolist()}")
        assert ex <= 1e-4 and eu <= 1e-4, (i, ex, eu)
    # The same method: equal step sizes, multipliers close but summed in another
    # order. The four parts hold the preconditioner's D^-1 rows in FP64 like
    # the FP64 oracle, the one-workgroup form at four knots per lane group in
    # FP32 (which slows PCG by a few percent), so the split's PCG totals are
    # held to the same-method oracle's (within 5%: near the stopping value the
    # residual decreases slowly and rounding moves single counts) and the
    # one-workgroup totals are printed.
    np.testing.assert_array_equal(ss["alpha"], s1["alpha"])
    ts, t1 = ss["pcg_iters"].sum(axis=1), s1["pcg_iters"].sum(axis=1)
    to = np.array([sum(L["pcg_iters"] for L in oracle.sqp(
        s, oracle.Params(sqp_iters=p.sqp_iters, kkt_mode=1, pcg_tol=p.pcg_tol),
        alpha_replay=ss[i]["alpha"].astype(np.float64)).logs) for i, s in enumerate(solves)])
    print(f"PCG totals: split {ts.tolist()}, FP64 oracle {to.tolist()}, one workgroup {t1.tolist()}")
    assert np.all(np.abs(ts - to) <= 0.05 * to), (ts, to, t1)
    # Both stop at the PCG tolerance 1e-7 (R6), so their multipliers may differ
    # at that tolerance's order.
    scale = np.abs(l1).max()
    assert np.abs(ls - l1).max() <= 1e-5 * scale
    assert not np.array_equal(ls, l1), "the split path did not run"


def test_split_line_search_with_the_largest_candidate_set():
    # Sixteen step candidates: every part's partial merits and flags
    # (n_alpha + 3 values) fill the sums region of its exchange slot.
    _say("split n_alpha=16")
    solves = [w.chain_solve(31, i, n=6, N=100) for i in range(2)]
    p = g.Params(sqp_iters=4, pcg_tol=1e-7, n_alpha=16, beta=1.5)
    Xs, Us, ss, _ = _run(solves, p, 4)
    assert not (ss["status"] & (g.ST_EXCHANGE | g.ST_NONFINITE | g.ST_PCG_MAXITER)).any(), ss["status"]
    for i, s in enumerate(solves):
        ref = oracle.sqp(s, oracle.Params(sqp_iters=p.sqp_iters, kkt_mode=2, n_alpha=16, beta=1.5),
                         alpha_replay=ss[i]["alpha"].astype(np.float64))
        ex = np.abs(Xs[i][:s.N, :2 * s.n] - ref.X).max() / np.abs(ref.X).max()
        eu = np.abs(Us[i][:s.N - 1, :s.n] - ref.U).max() / np.abs(ref.U).max()
        print(f"solve {i}: alphas {ss[i]['alpha'].tolist()}, X {ex:.2e} U {eu:.2e}")
        assert ex <= 1e-4 and eu <= 1e-4, (i, ex, eu)
        for it, L in enumerate(ref.logs):
            ms = L["merits"]
            j = int(round(-np.log(float(ss[i]["alpha"][it])) / np.log(1.5)))
            assert ms[j] - ms.min() <= 1e-5 * abs(ms.min()) + 1e-6, (i, it, j, int(np.argmin(ms)))


@pytest.mark.parametrize("fp64", [1, 0])
def test_split_uneven_batch_mixed_equals_grouped(fp64):
    # Split and one-workgroup solves in one mixed-shape launch, and per shape group.
    _say(f"split uneven fp64={fp64}")
    solves = w.uneven_batch(33, M=10, horizons=(16, 64, 128))
    assert any(s.N > 64 and s.n >= 6 for s in solves)
    p = g.Params(sqp_iters=3, pcg_tol=1e-7 if fp64 else 1e-5, schur_fp64=fp64)
    Xm, Um, sm, lm = _run(solves, p, 4, g.DISPATCH_MIXED)
    Xg, Ug, sg, lg = _run(solves, p, 4, g.DISPATCH_GROUPED)
    np.testing.assert_array_equal(Xm, Xg)
    np.testing.assert_array_equal(Um, Ug)
    np.testing.assert_array_equal(lm, lg)
    assert not (sm["status"] & (g.ST_EXCHANGE | g.ST_NONFINITE)).any()
    if fp64:
        for i, s in enumerate(solves):
            if s.N > 64 and s.n >= 6:
                ex, eu = _replay(s, Xm[i], Um[i], sm[i], p.sqp_iters)
                assert ex <= 1e-4 and eu <= 1e-4, (i, ex, eu)


def test_split_fp32_variant_matches_the_one_workgroup_form():
    # The all-FP32 variant (standard PCG arrangement, four exchanges per
    # iteration). With its Schur rows rounded to FP32 that variant departs from
    # the exact solution by about 1e-3 whatever the summation order, so the bar
    # is its own: the split as close to the exact oracle as the one-workgroup
    # FP32 form (within a factor 3), each replayed with its own steps.
    _say("split fp32")
    solves = [w.chain_solve(39, i, n=7, N=128) for i in range(2)]
    p = g.Params(sqp_iters=3, pcg_tol=1e-5, schur_fp64=0)
    Xs, Us, ss, ls = _run(solves, p, 4)
    X1, U1, s1, l1 = _run(solves, p, 1)
    assert not (ss["status"] & (g.ST_EXCHANGE | g.ST_NONFINITE)).any(), ss["status"]
    assert not np.array_equal(ls, l1), "the split path did not run"
    for i, s in enumerate(solves):
        ex, eu = _replay(s, Xs[i], Us[i], ss[i], p.sqp_iters)
        ox, ou = _replay(s, X1[i], U1[i], s1[i], p.sqp_iters)
        d = max(_parity.rel(Xs[i, :s.N, :14], X1[i, :s.N, :14]), _parity.rel(Us[i, :s.N - 1, :7], U1[i, :s.N - 1, :7]))
        print(f"solve {i}: vs the exact oracle, split X {ex:.2e} U {eu:.2e}, one workgroup X {ox:.2e} "
              f"U {ou:.2e}; split vs one workgroup {d:.2e}; PCG its {ss[i]['pcg_iters'].tolist()} / "
              f"{s1[i]['pcg_iters'].tolist()}")
        assert max(ex, eu) <= 3 * max(ox, ou, 1e-4), (i, ex, eu, ox, ou)


def test_graph_replay_keeps_the_split():
    # A mixed-shape batch through gato_step_graph: the step is a graph of a
    # clearing kernel and the split kernel as a cooperative node. Every replay
    # (with eager launches of the same batch in between) equals the eager split
    # launch bit for bit, and differs from the one-workgroup form (so the
    # replayed kernel ran split).
    _say("split graph replay")
    solves = w.uneven_batch(33, M=10, horizons=(16, 64, 128))
    assert any(s.N > 64 and s.n >= 6 for s in solves)
    p = g.Params(sqp_iters=2, pcg_tol=1e-7)
    b = g.Batch.from_solves(solves, p)
    b.set_dispatch(g.DISPATCH_MIXED)
    xs, goal, X0, U0 = g.pack_inputs(solves)
    X, U = torch.empty_like(X0), torch.empty_like(U0)
    st = b.stats_buffer(2)

    def run(graph):
        X.copy_(X0)
        U.copy_(U0)
        b.reset_warm_start()
        b.step(xs, goal, X, U, 2, st, graph=graph)
        torch.cuda.synchronize()
        return (X.cpu().numpy().copy(), U.cpu().numpy().copy(), b.get_multipliers().cpu().numpy(),
                g.Batch.decode_stats(st, b.M, 2))

    ref = run(False)
    assert not (ref[3]["status"] & (g.ST_EXCHANGE | g.ST_NONFINITE)).any()
    for r in range(3):
        got = run(True)
        for a_, b_ in zip(ref, got):
            np.testing.assert_array_equal(a_, b_)
        again = run(False)
        for a_, b_ in zip(ref, again):
            np.testing.assert_array_equal(a_, b_)
    b.set_split(1)
    one = run(False)
    b.close()
    assert not np.array_equal(one[2], ref[2]), "the graph did not run the split kernel"


def test_split_falls_back_when_the_launch_does_not_fit():
    # 300 long solves need 1200 workgroups at once (600 with two parts): the
    # launch runs them one workgroup each, with the one-workgroup form's results.
    _say("split fallback")
    solves = [w.chain_solve(35, i % 4, n=7, N=128) for i in range(300)]
    p = g.Params(sqp_iters=1, pcg_tol=1e-5)
    Xs, Us, ss, ls = _run(solves, p, 4)
    X1, U1, s1, l1 = _run(solves, p, 1)
    np.testing.assert_array_equal(Xs, X1)
    np.testing.assert_array_equal(ls, l1)
    np.testing.assert_array_equal(ss["status"], s1["status"])


def test_split_wait_bound_reports_the_exchange_and_returns():
    # Failure handling, forced from the host: one poll per wait, so that parts
    # give up waiting for each other. Every kernel still finishes; the split
    # solves report GATO_ST_EXCHANGE, the one-workgroup solve of the same
    # launch is untouched, and the next call with the default bound is clean
    # (stale exchange words carry another launch's tag).
    _say("split wait bound")
    solves = [w.chain_solve(37, 0, n=7, N=128), w.chain_solve(37, 1, n=7, N=32)]
    p = g.Params(sqp_iters=3, pcg_tol=1e-7)
    b = g.Batch.from_solves(solves, p)
    xs, goal, X0, U0 = g.pack_inputs(solves)
    st = b.stats_buffer(3)
    b.set_split(4, 1)
    X, U = X0.clone(), U0.clone()
    b.reset_warm_start()
    b.step(xs, goal, X, U, 3, st)
    torch.cuda.synchronize()
    s_bad = g.Batch.decode_stats(st, b.M, 3)
    Xb = X.cpu().numpy()
    b.set_split(4)
    X, U = X0.clone(), U0.clone()
    b.reset_warm_start()
    b.step(xs, goal, X, U, 3, st)
    torch.cuda.synchronize()
    s_ok = g.Batch.decode_stats(st, b.M, 3)
    Xok = X.cpu().numpy()
    b.close()
    assert (s_bad["status"][0] & g.ST_EXCHANGE).any(), s_bad["status"]
    assert not (s_bad["status"][1] & g.ST_EXCHANGE).any()
    np.testing.assert_array_equal(Xb[1], Xok[1])
    assert not (s_ok["status"] & g.ST_EXCHANGE).any(), s_ok["status"]
    ex, eu = _replay(solves[0], Xok[0].astype(np.float64), U.cpu().numpy()[0].astype(np.float64), s_ok[0], 3)
    assert ex <= 1e-4 and eu <= 1e-4, (ex, eu)


# N = 70: the second part holds 6 knots in one lane-group block (p = 2).
@pytest.mark.parametrize("N", [128, 70])
def test_two_parts_per_solve_when_four_do_not_fit(N):
    # 80 long solves: four workgroups each (320) do not fit 256 CUs, two (160)
    # do. Sampled solves against the oracle; the multipliers differ from the
    # one-workgroup form at rounding level (the two-part path ran).
    _say(f"split two parts N={N}")
    solves = [w.chain_solve(41, i, n=7, N=N) for i in range(80)]
    p = g.Params(sqp_iters=2, pcg_tol=1e-7)
    Xs, Us, ss, ls = _run(solves, p, 4)
    X1, U1, s1, l1 = _run(solves, p, 1)
    assert not (ss["status"] & (g.ST_EXCHANGE | g.ST_NONFINITE)).any()
    assert not np.array_equal(ls, l1), "the split path did not run"
    assert np.abs(ls - l1).max() <= 1e-5 * np.abs(l1).max()   # PCG tolerance 1e-7 on both
    for i in (0, 41, 79):
        ex, eu = _replay(solves[i], Xs[i], Us[i], ss[i], p.sqp_iters)
        assert ex <= 1e-4 and eu <= 1e-4, (i, ex, eu)


def test_full_size_uneven_batch_sampled_solves():
    # The uneven-batch benchmark's launch: 128 seeded solves (seed 0; DoF from
    # {3, 6, 7}, N from {16, 32, 64, 128}), one mixed-shape launch with the long
    # solves split, 10 SQP iterations, PCG tolerance 1e-5. At least two solves
    # of every (DoF, N) bucket, the slowest and the fastest PCG solve are
    # replayed in the same-method FP64 oracle (bar 1e-4, valid steps); the
    # per-bucket errors (and the distance to the exact solve) are printed.
    _say("full size uneven M=128")
    solves = w.uneven_batch(0, M=128)
    p = g.Params(sqp_iters=10, pcg_tol=1e-5)
    Xg, Ug, st, _ = _run(solves, p, 4, g.DISPATCH_MIXED)
    assert not (st["status"] & (g.ST_EXCHANGE | g.ST_NONFINITE | g.ST_PCG_MAXITER)).any()
    tot = st["pcg_iters"].sum(axis=1)
    buckets = {}
    for i, s in enumerate(solves):
        buckets.setdefault((s.n, s.N), []).append(i)
    idx = {int(np.argmax(tot)), int(np.argmin(tot))}
    for key, members in buckets.items():
        idx.update(members[:2])
    idx = sorted(idx)
    assert len(idx) >= 16
    res = _parity.check_many([dict(s=solves[i], Xg=Xg[i], Ug=Ug[i], st=st[i], p_gpu=p,
                                   label=f"solve {i} (n={solves[i].n}, N={solves[i].N})") for i in idx])
    for key in sorted(buckets):
        rs = [r for i, r in zip(idx, res) if (solves[i].n, solves[i].N) == key]
        print(f"bucket n={key[0]} N={key[1]}: {len(rs)} sampled, vs same-method {max(r['e_same'] for r in rs):.2e}, "
              f"vs exact {max(r['e_exact'] for r in rs):.2e}")
    _parity.report(res, f"uneven M=128 (slowest PCG solve {int(np.argmax(tot))}, N={solves[int(np.argmax(tot))].N})")
