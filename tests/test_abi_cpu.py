"""Host-side checks of the C-ABI library (no GPU needed): exports, workspace
sizing, defaults and argument validation (which returns before any HIP call)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2510_07625_amd as g

pytestmark = pytest.mark.skipif(not os.path.exists(g.LIB_PATH), reason="libgato.so not built")


def _declared():
    import glob
    headers = sorted(glob.glob(os.path.join(os.path.dirname(g.HEADER), "*.h")))
    assert sorted(headers) == sorted(g.HEADERS)
    text = "".join(open(h).read() for h in headers)
    return sorted(set(re.findall(r"\b(gato_[a-z_0-9]+)\s*\(", text)))


def test_header_symbols_are_exported():
    names = _declared()
    assert len(names) >= 12
    L = g.lib()
    for name in names:
        assert hasattr(L, name), name
    assert set(g.EXPORTS) == set(names)


def test_default_params():
    p = g._Params()
    g.lib().gato_default_params(C.byref(p))
    assert (p.sqp_iters, p.pcg_tol, p.pcg_max_iter, p.mu, p.beta, p.n_alpha, p.rho, p.schur_fp64,
            p.warm_lambda, p.fp64_block_inv, p.fp64_dot, p.rho_adapt) == (10, 1e-5, 0, 10.0, 2.0, 8, 0.0, 1, 1, 0, 0, 0)
    d = g.Params()
    c = d.c()
    for f, _ in g._Params._fields_:
        assert getattr(c, f) == getattr(p, f), f"Params default of {f} differs from gato_default_params"
    assert g.Params().precision() == "fp64-schur"
    assert g.Params(schur_fp64=0, fp64_dot=1).precision() == "fp32+fp64-dot"


def test_workspace_bytes():
    a = g.workspace_bytes(7, 32)
    b = g.workspace_bytes(7, 64)
    assert 0 < a < b
    # A, B (fp32), inverse diagonal blocks and multipliers (fp64) at least.
    assert a >= 31 * (196 + 98) * 4 + 32 * 196 * 8 + 32 * 14 * 8
    assert g.workspace_bytes(5, 32) == 0      # no kernel compiled for 5 DoF
    assert g.workspace_bytes(7, 1) == 0
    assert g.workspace_bytes(7, 129) == 0


def _create(robots, probs, params=None):
    M = len(robots)
    rob = (g._Robot * M)(*robots)
    prob = (g._Problem * M)(*probs)
    h = C.c_void_p()
    p = (params or g.Params()).c()
    rc = g.lib().gato_batch_create(M, rob, prob, C.byref(p), None, C.byref(h))
    return rc, g.lib().gato_last_error().decode()


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def test_invalid_arguments_are_rejected_on_the_host():
    link = np.tile([0.3, 2.0, 0.05, 0.05, 0.05], (7, 1)).ravel()
    Q, R, QN = np.ones(14), np.full(7, 1e-3), np.full(14, 100.0)
    keep = [link, Q, R, QN]
    good_r = g._Robot(0, 7, _dp(link), 9.81, 0.0)
    good_p = g._Problem(32, 0.01, _dp(Q), _dp(R), _dp(QN))
    rc, _ = _create([good_r], [g._Problem(1, 0.01, _dp(Q), _dp(R), _dp(QN))])
    assert rc == g.GATO_EINVAL
    rc, msg = _create([good_r], [g._Problem(32, -0.01, _dp(Q), _dp(R), _dp(QN))])
    assert rc == g.GATO_EINVAL and "dt" in msg
    badQ = -Q
    rc, msg = _create([good_r], [g._Problem(32, 0.01, _dp(badQ), _dp(R), _dp(QN))])
    assert rc == g.GATO_EINVAL and "Q" in msg
    rc, msg = _create([good_r], [good_p], g.Params(n_alpha=0))
    assert rc == g.GATO_EINVAL and "n_alpha" in msg
    rc, msg = _create([good_r], [good_p], g.Params(beta=1.0))
    assert rc == g.GATO_EINVAL and "beta" in msg
    rc, msg = _create([g._Robot(0, 5, _dp(link), 9.81, 0.0)], [good_p])
    assert rc == g.GATO_EUNSUPPORTED
    badlink = link.copy()
    badlink[1] = 0.0
    rc, msg = _create([g._Robot(0, 7, _dp(badlink), 9.81, 0.0)], [good_p])
    assert rc == g.GATO_EINVAL and "mass" in msg
    h = C.c_void_p()
    assert g.lib().gato_batch_create(0, None, None, None, None, C.byref(h)) == g.GATO_EINVAL
    assert g.lib().gato_solve(None, None, None, None, None, None) == g.GATO_EINVAL
    rc, msg = _create([good_r], [good_p], g.Params(schur_fp64=0, fp64_dot=2))
    assert rc == g.GATO_EINVAL and "fp64_dot" in msg
    rc, msg = _create([good_r], [good_p], g.Params(schur_fp64=0, fp64_block_inv=-1))
    assert rc == g.GATO_EINVAL and "fp64_block_inv" in msg
    L = g.lib()
    n = C.c_int()
    assert L.gato_set_dispatch(None, 0) == g.GATO_EINVAL
    assert L.gato_set_split(None, 4, 0) == g.GATO_EINVAL
    assert L.gato_buckets(None, None, 0, C.byref(n)) == g.GATO_EINVAL
    assert L.gato_set_mapping(None, 7, 32, 1) == g.GATO_EINVAL
    assert L.gato_autotune(None, None, None, None, None, 1, 1) == g.GATO_EINVAL
    assert L.gato_step_graph(None, None, None, None, None, 1, None) == g.GATO_EINVAL
    assert L.gato_plant_step(None, 1, None, None, None, None, 0.01, 10, None, None, None) == g.GATO_EINVAL
    assert L.gato_set_external_force(None, None) == g.GATO_EINVAL
    assert L.gato_set_rho(None, None) == g.GATO_EINVAL and L.gato_get_rho(None, None) == g.GATO_EINVAL
    rc, msg = _create([good_r], [good_p], g.Params(rho_adapt=3))
    assert rc == g.GATO_EINVAL and "rho_adapt" in msg
    assert L.gato_set_tip_reference(None, None) == g.GATO_EINVAL
    assert L.gato_get_multipliers(None, None) == g.GATO_EINVAL
    assert L.gato_set_multipliers(None, None) == g.GATO_EINVAL
    assert L.gato_shift_warm_start(None, None, 1, None) == g.GATO_EINVAL
    assert L.gato_tip_positions(None, None, None, None) == g.GATO_EINVAL
    n = C.c_int()
    assert L.gato_serve_run(None, 1, 1, 0, None, None, None, None, 0, 0, None, None, None, None, C.byref(n)) \
        == g.GATO_EINVAL
    assert g.STATS_DTYPE.itemsize == C.sizeof(g.SolveStats) == 24
    del keep
