"""Python binding of libgato (include/gato.h): argument marshalling only.

Every step of the SQP iteration runs in the HIP kernels of libgato.so; this
module checks tensor shapes and dtypes, builds the C structs and passes device
pointers. PyTorch is used for device memory and streams only. There is no CPU
fallback: if the library is missing, loading it raises.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref
from dataclasses import dataclass, field
from typing import Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgato.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "gato.h")
HEADERS = (HEADER, os.path.join(os.path.dirname(HERE), "include", "gato_probe.h"))

GATO_OK, GATO_EINVAL, GATO_ENOMEM, GATO_EDEVICE, GATO_EUNSUPPORTED = 0, -1, -2, -3, -4
ST_PCG_MAXITER, ST_NONFINITE, ST_NO_DESCENT, ST_ADMIT_REJECT, ST_EXCHANGE = 1, 2, 4, 8, 16
MODEL_SERIAL_CHAIN, MODEL_DOUBLE_INTEGRATOR = 0, 1
MAX_DOF, MAX_KNOTS, MAX_ALPHA = 7, 128, 16
DISPATCH_AUTO, DISPATCH_GROUPED, DISPATCH_MIXED = 0, 1, 2


class GatoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gato error {code}: {msg}")
        self.code = code


class _Robot(C.Structure):
    _fields_ = [("model", C.c_int), ("n_dof", C.c_int), ("link", C.POINTER(C.c_double)),
                ("gravity", C.c_double), ("spring_k", C.c_double)]


class _Problem(C.Structure):
    _fields_ = [("N", C.c_int), ("dt", C.c_double), ("Q_diag", C.POINTER(C.c_double)),
                ("R_diag", C.POINTER(C.c_double)), ("QN_diag", C.POINTER(C.c_double)),
                ("Wee_diag", C.POINTER(C.c_double)), ("WeeN_diag", C.POINTER(C.c_double))]


class _Params(C.Structure):
    _fields_ = [("sqp_iters", C.c_int), ("pcg_tol", C.c_double), ("pcg_max_iter", C.c_int),
                ("mu", C.c_double), ("beta", C.c_double), ("n_alpha", C.c_int), ("rho", C.c_double),
                ("schur_fp64", C.c_int), ("warm_lambda", C.c_int), ("fp64_block_inv", C.c_int),
                ("fp64_dot", C.c_int), ("rho_adapt", C.c_int)]


class SolveStats(C.Structure):
    _fields_ = [("merit0", C.c_float), ("merit", C.c_float), ("alpha", C.c_float), ("pcg_iters", C.c_int),
                ("status", C.c_uint), ("rho", C.c_float)]


class Bucket(C.Structure):
    _fields_ = [("n_dof", C.c_int), ("N", C.c_int), ("count", C.c_int), ("kpt", C.c_int),
                ("tuned_ms", C.c_float)]


STATS_DTYPE = np.dtype([("merit0", np.float32), ("merit", np.float32), ("alpha", np.float32),
                        ("pcg_iters", np.int32), ("status", np.uint32), ("rho", np.float32)])

# Entry points declared in include/gato.h.
EXPORTS = ("gato_default_params", "gato_workspace_bytes", "gato_batch_create", "gato_batch_destroy",
           "gato_batch_shape", "gato_solve", "gato_step", "gato_step_plain", "gato_debug_lq",
           "gato_debug_kkt", "gato_reset_warm_start", "gato_rbd_flops", "gato_profile_phases",
           "gato_set_trajectories", "gato_get_trajectories", "gato_serve_step", "gato_plant_step",
           "gato_set_external_force", "gato_set_dispatch", "gato_set_split",
           "gato_buckets", "gato_set_mapping", "gato_autotune", "gato_step_graph", "gato_set_rho", "gato_get_rho",
           "gato_serve_ctx_create", "gato_serve_ctx_destroy", "gato_serve_ctx_buffers", "gato_serve_ctx_submit",
           "gato_serve_ctx_query", "gato_serve_ctx_trajectories", "gato_serve_run", "gato_set_tip_reference",
           "gato_tip_positions", "gato_get_multipliers", "gato_set_multipliers", "gato_shift_warm_start",
           "gato_last_error", "gato_probe_lds", "gato_select_hypotheses", "gato_solve_static")

_lib = None


def lib() -> C.CDLL:
    """Loads libgato.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2510_07625_amd/build.py "
                               "(or __graft_entry__.build()); there is no fallback path")
        L = C.CDLL(LIB_PATH)
        vp, ip = C.c_void_p, C.c_int
        L.gato_default_params.argtypes = [C.POINTER(_Params)]
        L.gato_default_params.restype = None
        L.gato_workspace_bytes.argtypes = [ip, ip, C.POINTER(_Params)]
        L.gato_workspace_bytes.restype = C.c_size_t
        L.gato_batch_create.argtypes = [ip, C.POINTER(_Robot), C.POINTER(_Problem), C.POINTER(_Params), vp,
                                        C.POINTER(vp)]
        L.gato_batch_destroy.argtypes = [vp]
        L.gato_batch_destroy.restype = None
        L.gato_batch_shape.argtypes = [vp, C.POINTER(ip), C.POINTER(ip), C.POINTER(ip)]
        L.gato_solve.argtypes = [vp, vp, vp, vp, vp, C.POINTER(SolveStats)]
        L.gato_step.argtypes = [vp, vp, vp, vp, vp, ip, vp]
        L.gato_solve_static.argtypes = [vp, vp, vp, vp, vp, C.POINTER(SolveStats)]
        L.gato_step_plain.argtypes = [vp, vp, vp, vp, vp, ip, vp]
        L.gato_debug_lq.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.gato_debug_kkt.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.gato_reset_warm_start.argtypes = [vp]
        L.gato_rbd_flops.argtypes = [ip, C.POINTER(C.c_double)]
        L.gato_profile_phases.argtypes = [vp, vp, vp, vp, vp, ip, vp]
        L.gato_set_trajectories.argtypes = [vp, vp, vp]
        L.gato_get_trajectories.argtypes = [vp, vp, vp]
        L.gato_serve_step.argtypes = [vp, ip, vp, vp, vp, ip, ip, vp, vp, vp, vp]
        L.gato_plant_step.argtypes = [vp, ip, vp, vp, vp, vp, C.c_double, ip, vp, vp, vp]
        L.gato_set_external_force.argtypes = [vp, C.POINTER(C.c_double)]
        L.gato_set_dispatch.argtypes = [vp, ip]
        L.gato_set_split.argtypes = [vp, ip, ip]
        L.gato_set_rho.argtypes = [vp, C.POINTER(C.c_double)]
        L.gato_serve_ctx_create.argtypes = [vp, ip, ip, C.POINTER(vp)]
        L.gato_serve_ctx_destroy.argtypes = [vp]
        L.gato_serve_ctx_destroy.restype = None
        L.gato_serve_ctx_buffers.argtypes = [vp] + [C.POINTER(vp)] * 6
        L.gato_serve_ctx_submit.argtypes = [vp, ip, ip]
        L.gato_serve_ctx_query.argtypes = [vp]
        L.gato_serve_ctx_trajectories.argtypes = [vp, vp, vp]
        L.gato_get_rho.argtypes = [vp, C.POINTER(C.c_double)]
        L.gato_set_tip_reference.argtypes = [vp, vp]
        L.gato_tip_positions.argtypes = [vp, vp, vp, vp]
        L.gato_get_multipliers.argtypes = [vp, vp]
        L.gato_set_multipliers.argtypes = [vp, vp]
        L.gato_shift_warm_start.argtypes = [vp, vp, ip, vp]
        L.gato_serve_run.argtypes = [vp, ip, ip, ip, vp, vp, vp, vp, ip, C.c_size_t, vp, vp, vp, vp, C.POINTER(ip)]
        L.gato_buckets.argtypes = [vp, C.POINTER(Bucket), ip, C.POINTER(ip)]
        L.gato_set_mapping.argtypes = [vp, ip, ip, ip]
        L.gato_autotune.argtypes = [vp, vp, vp, vp, vp, ip, ip]
        L.gato_step_graph.argtypes = [vp, vp, vp, vp, vp, ip, vp]
        L.gato_select_hypotheses.argtypes = [vp, ip, ip, vp, vp, vp, vp, vp, vp, vp]
        L.gato_probe_lds.argtypes = [ip, ip, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.gato_last_error.argtypes = []
        L.gato_last_error.restype = C.c_char_p
        _lib = L
    return _lib


# Live handles, released before the interpreter shuts down: serving contexts
# first (their streams may still run work on a batch's memory), then batches.
# At interpreter exit the HIP runtime itself may already be going away, so
# finalizers that run after this point release nothing.
_live_ctx: "weakref.WeakSet" = weakref.WeakSet()
_live_batches: "weakref.WeakSet" = weakref.WeakSet()


@atexit.register
def _release_all():
    for c in list(_live_ctx):
        c.close()
    for b in list(_live_batches):
        b.close()


def _check(rc: int) -> int:
    if rc < 0:
        raise GatoError(rc, lib().gato_last_error().decode())
    return rc


@dataclass
class Params:
    """Mirror of gato_params (defaults of gato_default_params)."""

    sqp_iters: int = 10
    pcg_tol: float = 1e-5
    pcg_max_iter: int = 0
    mu: float = 10.0
    beta: float = 2.0
    n_alpha: int = 8
    rho: float = 0.0
    schur_fp64: int = 1
    warm_lambda: int = 1
    fp64_block_inv: int = 0
    fp64_dot: int = 0
    rho_adapt: int = 0

    def c(self) -> _Params:
        return _Params(self.sqp_iters, self.pcg_tol, self.pcg_max_iter, self.mu, self.beta, self.n_alpha,
                       self.rho, self.schur_fp64, self.warm_lambda, self.fp64_block_inv, self.fp64_dot,
                       self.rho_adapt)

    def precision(self) -> str:
        """Short name of the precision configuration."""
        if self.schur_fp64:
            return "fp64-schur"
        parts = ["fp32"] + (["fp64-inv"] if self.fp64_block_inv else []) + (["fp64-dot"] if self.fp64_dot else [])
        return "+".join(parts)


@dataclass
class Robot:
    n_dof: int
    link: np.ndarray = None          # [n, 5] length, mass, Ixx, Iyy, Izz
    model: int = MODEL_SERIAL_CHAIN
    gravity: float = 9.81
    spring_k: float = 0.0


@dataclass
class Problem:
    N: int
    dt: float
    Q_diag: np.ndarray
    R_diag: np.ndarray
    QN_diag: np.ndarray
    Wee_diag: np.ndarray | None = None    # [3] tip tracking weights (stages), or None
    WeeN_diag: np.ndarray | None = None   # [3] at the last knot


def rbd_flops(n_dof: int):
    """(forward dynamics, one Jacobian column, one Cholesky solve) operation counts."""
    out = (C.c_double * 3)()
    _check(lib().gato_rbd_flops(int(n_dof), out))
    return tuple(out)


def sqp_iteration_flops(n: int, N: int, n_alpha: int, pcg_iters) -> float:
    """Algorithmic FLOPs of SQP iterations of one solve: what the method of
    Algorithm 1 computes, counted once, independent of how a kernel arranges it.

    pcg_iters may be an array (one entry per SQP iteration); the result is the
    sum over those iterations. Per SQP iteration:
      * dynamics and derivatives at N-1 knots: forward dynamics, 2n columns of
        the dynamics Jacobian and n columns of M^-1 (counted on the kernels'
        own rigid-body templates, rbd_flops);
      * Schur complement and preconditioner blocks (Eqs. (5)-(6)):
        N (7 nx^3 + 2 nx^2 nu);
      * per PCG iteration (Sec. II-B): one product with the block-tridiagonal
        S~ and one with the block-tridiagonal P, 2 (3N - 2) nx^2 FLOPs each,
        plus the vector updates and inner products, 10 N nx;
      * step recovery (Eq. (4)): (N - 1)(2 nx^2 + 2 nx nu) + N nx;
      * line search (Eqs. (3), (7)): n_alpha (N - 1) forward dynamics.
    """
    import numpy as _np
    f_fd, f_col, f_sol = rbd_flops(n)
    nx, nu = 2 * n, n
    lq = (N - 1) * (f_fd + 2 * n * f_col + n * f_sol)
    schur = N * (7 * nx ** 3 + 2 * nx * nx * nu)
    step = (N - 1) * (2 * nx * nx + 2 * nx * nu) + N * nx
    ls = n_alpha * (N - 1) * f_fd
    pcg_iter = 4 * (3 * N - 2) * nx * nx + 10 * N * nx
    fixed = lq + schur + step + ls
    its = _np.atleast_1d(_np.asarray(pcg_iters, dtype=_np.float64))
    return float(its.size * fixed + pcg_iter * its.sum())


def probe_lds(pattern: int, iters: int = 4096):
    """gato_probe_lds (include/gato_probe.h): delivered LDS bytes per clock per
    CU and per second over the device, for pattern 0 (distinct addresses) or 1
    (16-lane broadcast)."""
    per_clk, per_s = C.c_double(), C.c_double()
    rc = lib().gato_probe_lds(int(pattern), int(iters), C.byref(per_clk), C.byref(per_s))
    if rc != 0:
        raise GatoError(rc, "gato_probe_lds failed")
    return per_clk.value, per_s.value


def workspace_bytes(n_dof: int, N: int, params: Params | None = None) -> int:
    p = (params or Params()).c()
    return int(lib().gato_workspace_bytes(n_dof, N, C.byref(p)))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _dptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


class Batch:
    """A batch of M trajectory-optimisation solves living on one GPU."""

    def __init__(self, robots: Sequence[Robot], problems: Sequence[Problem], params: Params | None = None,
                 stream=None):
        import torch  # device memory and streams only

        if len(robots) != len(problems) or not robots:
            raise ValueError("robots and problems must be non-empty and of equal length")
        self.params = params or Params()
        self.M = len(robots)
        keep = []
        rob = (_Robot * self.M)()
        prob = (_Problem * self.M)()
        for i, (r, p) in enumerate(zip(robots, problems)):
            link = _f64(r.link if r.link is not None else np.zeros((r.n_dof, 5))).reshape(-1)
            Q, R, QN = _f64(p.Q_diag), _f64(p.R_diag), _f64(p.QN_diag)
            keep += [link, Q, R, QN]
            We = WeN = None
            if getattr(p, "Wee_diag", None) is not None:
                We, WeN = _f64(p.Wee_diag).reshape(3), _f64(p.WeeN_diag).reshape(3)
                keep += [We, WeN]
            rob[i] = _Robot(int(r.model), int(r.n_dof), link.ctypes.data_as(C.POINTER(C.c_double)),
                            float(r.gravity), float(r.spring_k))
            prob[i] = _Problem(int(p.N), float(p.dt), Q.ctypes.data_as(C.POINTER(C.c_double)),
                               R.ctypes.data_as(C.POINTER(C.c_double)), QN.ctypes.data_as(C.POINTER(C.c_double)))
            if We is not None:
                prob[i].Wee_diag = We.ctypes.data_as(C.POINTER(C.c_double))
                prob[i].WeeN_diag = WeN.ctypes.data_as(C.POINTER(C.c_double))
        self.task = any(getattr(p, "Wee_diag", None) is not None for p in problems)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        handle = C.c_void_p()
        prm = self.params.c()
        _check(lib().gato_batch_create(self.M, rob, prob, C.byref(prm), C.c_void_p(self.stream.cuda_stream),
                                       C.byref(handle)))
        self._h = handle
        _live_batches.add(self)
        M, n, N = C.c_int(), C.c_int(), C.c_int()
        _check(lib().gato_batch_shape(self._h, C.byref(M), C.byref(n), C.byref(N)))
        self.n_max, self.N_max = n.value, N.value
        self.nx_max, self.nu_max = 2 * self.n_max, self.n_max

    @classmethod
    def from_solves(cls, solves, params: Params | None = None, stream=None) -> "Batch":
        """Builds a batch from objects with the fields of workload.Solve."""
        robots = [Robot(s.n, s.links, s.model, s.gravity, s.spring_k) for s in solves]
        problems = [Problem(s.N, s.dt, s.Qd, s.Rd, s.QNd, getattr(s, "Wee", None), getattr(s, "WeeN", None))
                    for s in solves]
        b = cls(robots, problems, params, stream)
        fe = np.array([getattr(s, "fext", (0.0, 0.0, 0.0)) for s in solves], np.float64)
        if np.any(fe != 0.0):
            b.set_external_force(fe)
        if b.task:
            import torch
            pref = np.zeros((b.M, b.N_max, 3), np.float32)
            for i, s in enumerate(solves):
                if getattr(s, "pref", None) is not None:
                    pref[i, :s.N] = s.pref
            b.set_tip_reference(torch.from_numpy(pref).cuda())
        return b

    def tip_positions(self, X, stream=None):
        """gato_tip_positions: tip positions [M, N_max, 3] of trajectories X [M, N_max, nx_max]."""
        import torch
        self._chk(X, (self.M, self.N_max, self.nx_max))
        P = torch.empty((self.M, self.N_max, 3), dtype=torch.float32, device="cuda")
        st = stream.cuda_stream if stream is not None else None
        _check(lib().gato_tip_positions(self._h, _dptr(X), _dptr(P), C.c_void_p(st) if st else None))
        return P

    def set_tip_reference(self, pref):
        """gato_set_tip_reference: reference tip positions, float32 cuda tensor [M, N_max, 3]."""
        self._chk(pref, (self.M, self.N_max, 3))
        _check(lib().gato_set_tip_reference(self._h, _dptr(pref)))
        self._pref = pref          # keep it alive until the stream has copied it

    def close(self):
        """gato_batch_destroy (synchronises the device first). Idempotent."""
        if getattr(self, "_h", None):
            lib().gato_batch_destroy(self._h)
            self._h = None
        _live_batches.discard(self)

    def __del__(self, _finalizing=sys.is_finalizing):
        # (The default argument keeps the function reachable: at interpreter
        # shutdown the module's globals, sys included, may already be gone.)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    # ---- shape checks ------------------------------------------------------
    def _chk(self, t, shape, dtype=None):
        import torch
        dtype = dtype or torch.float32
        if t is None:
            raise ValueError("tensor is None")
        if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected contiguous {dtype} cuda tensor of shape {tuple(shape)}, got "
                             f"{t.dtype} {tuple(t.shape)} on {t.device}")
        return t

    def _io(self, xs, goal, X, U):
        M, N, nx, nu = self.M, self.N_max, self.nx_max, self.nu_max
        self._chk(xs, (M, nx))
        self._chk(goal, (M, nu))
        self._chk(X, (M, N, nx))
        self._chk(U, (M, N - 1, nu))

    # ---- entry points ------------------------------------------------------
    def solve(self, xs, goal, X, U, stats: bool = True):
        """gato_solve: sqp_iters iterations in place on X, U; returns per-iteration stats."""
        self._io(xs, goal, X, U)
        if stats:
            h = (SolveStats * (self.M * max(self.params.sqp_iters, 1)))()
            _check(lib().gato_solve(self._h, _dptr(xs), _dptr(goal), _dptr(X), _dptr(U), h))
            arr = np.frombuffer(h, dtype=STATS_DTYPE).copy()
            return arr.reshape(self.M, max(self.params.sqp_iters, 1))
        _check(lib().gato_solve(self._h, _dptr(xs), _dptr(goal), _dptr(X), _dptr(U), None))
        return None

    def solve_static(self, xs, goal, X, U, stats: bool = True):
        """gato_solve_static: gato_solve with the library's static statistics staging (allocates nothing)."""
        self._io(xs, goal, X, U)
        if stats:
            h = (SolveStats * (self.M * max(self.params.sqp_iters, 1)))()
            _check(lib().gato_solve_static(self._h, _dptr(xs), _dptr(goal), _dptr(X), _dptr(U), h))
            arr = np.frombuffer(h, dtype=STATS_DTYPE).copy()
            return arr.reshape(self.M, max(self.params.sqp_iters, 1))
        _check(lib().gato_solve_static(self._h, _dptr(xs), _dptr(goal), _dptr(X), _dptr(U), None))
        return None

    def step(self, xs, goal, X, U, n_iters: int, d_stats=None, plain: bool = False, graph: bool = False):
        """gato_step / gato_step_plain / gato_step_graph: asynchronous, device-side stats (uint8 tensor or None)."""
        self._io(xs, goal, X, U)
        if plain and graph:
            raise ValueError("plain and graph are exclusive")
        fn = lib().gato_step_plain if plain else (lib().gato_step_graph if graph else lib().gato_step)
        _check(fn(self._h, _dptr(xs), _dptr(goal), _dptr(X), _dptr(U), int(n_iters), _dptr(d_stats)))

    def set_rho(self, rho):
        """gato_set_rho: per-solve damping (M values)."""
        r = np.ascontiguousarray(np.broadcast_to(np.asarray(rho, np.float64), (self.M,)))
        _check(lib().gato_set_rho(self._h, r.ctypes.data_as(C.POINTER(C.c_double))))

    def get_rho(self) -> np.ndarray:
        r = np.zeros(self.M, np.float64)
        _check(lib().gato_get_rho(self._h, r.ctypes.data_as(C.POINTER(C.c_double))))
        return r

    def set_split(self, parts: int, max_polls: int = 0):
        """gato_set_split: 4 (long solves on four workgroups where the launch fits) or 1;
        max_polls bounds every wait of a part for another (0: the default)."""
        _check(lib().gato_set_split(self._h, int(parts), int(max_polls)))

    def set_dispatch(self, mode: int):
        """gato_set_dispatch: DISPATCH_AUTO, DISPATCH_GROUPED or DISPATCH_MIXED."""
        _check(lib().gato_set_dispatch(self._h, int(mode)))

    def buckets(self) -> list:
        """gato_buckets: [(n_dof, N, count, kpt, tuned_ms)] per (n_dof, N) bucket."""
        n = C.c_int()
        _check(lib().gato_buckets(self._h, None, 0, C.byref(n)))
        arr = (Bucket * max(n.value, 1))()
        _check(lib().gato_buckets(self._h, arr, n.value, C.byref(n)))
        return [dict(n_dof=b.n_dof, N=b.N, count=b.count, kpt=b.kpt, tuned_ms=b.tuned_ms) for b in arr[:n.value]]

    def set_mapping(self, n_dof: int, N: int, kpt: int):
        _check(lib().gato_set_mapping(self._h, int(n_dof), int(N), int(kpt)))

    def autotune(self, xs, goal, X, U, n_iters: int = 2, reps: int = 3) -> list:
        """gato_autotune: picks the fastest knots-per-group mapping per bucket; returns buckets()."""
        self._io(xs, goal, X, U)
        _check(lib().gato_autotune(self._h, _dptr(xs), _dptr(goal), _dptr(X), _dptr(U), int(n_iters), int(reps)))
        return self.buckets()

    PHASES = ("dynamics", "schur", "precond", "pcg", "step", "line_search")

    def profile_phases(self, xs, goal, X, U, n_iters: int):
        """Runs n_iters iterations recording per-phase device timestamps.

        Returns (wall-clock ticks per phase [M, n_iters, 6], shader cycles per
        iteration [M, n_iters]). The wall clock runs at a constant rate
        (see torch/HIP device properties for its frequency).
        """
        import torch
        self._io(xs, goal, X, U)
        clk = torch.zeros((self.M, n_iters, 8), dtype=torch.int64, device="cuda")
        _check(lib().gato_profile_phases(self._h, _dptr(xs), _dptr(goal), _dptr(X), _dptr(U), int(n_iters),
                                         _dptr(clk)))
        c = clk.cpu().numpy()
        return np.diff(c[:, :, :7], axis=2), c[:, :, 7]

    def stats_buffer(self, n_iters: int):
        import torch
        return torch.zeros(self.M * n_iters * STATS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")

    @staticmethod
    def decode_stats(buf, M: int, n_iters: int) -> np.ndarray:
        return np.frombuffer(buf.cpu().numpy().tobytes(), dtype=STATS_DTYPE).reshape(M, n_iters)

    def debug_lq(self, xs, goal, X, U):
        import torch
        self._io(xs, goal, X, U)
        M, N, nx, nu = self.M, self.N_max, self.nx_max, self.nu_max
        A = torch.zeros((M, N - 1, nx, nx), dtype=torch.float32, device="cuda")
        B = torch.zeros((M, N - 1, nx, nu), dtype=torch.float32, device="cuda")
        e = torch.zeros((M, N - 1, nx), dtype=torch.float32, device="cuda")
        _check(lib().gato_debug_lq(self._h, _dptr(xs), _dptr(goal), _dptr(X), _dptr(U), _dptr(A), _dptr(B),
                                   _dptr(e)))
        return A, B, e

    def debug_kkt(self, A, B, e, q, r, c0):
        import torch
        M, N, nx, nu = self.M, self.N_max, self.nx_max, self.nu_max
        self._chk(A, (M, N - 1, nx, nx))
        self._chk(B, (M, N - 1, nx, nu))
        self._chk(e, (M, N - 1, nx))
        self._chk(q, (M, N, nx))
        self._chk(r, (M, N - 1, nu))
        self._chk(c0, (M, nx))
        dX = torch.zeros((M, N, nx), dtype=torch.float32, device="cuda")
        dU = torch.zeros((M, N - 1, nu), dtype=torch.float32, device="cuda")
        lam = torch.zeros((M, N, nx), dtype=torch.float64, device="cuda")
        its = torch.zeros((M,), dtype=torch.int32, device="cuda")
        _check(lib().gato_debug_kkt(self._h, _dptr(A), _dptr(B), _dptr(e), _dptr(q), _dptr(r), _dptr(c0),
                                    _dptr(dX), _dptr(dU), _dptr(lam), _dptr(its)))
        return dX, dU, lam, its

    # ---- serving --------------------------------------------------------------
    def set_trajectories(self, X, U):
        self._chk(X, (self.M, self.N_max, self.nx_max))
        self._chk(U, (self.M, self.N_max - 1, self.nu_max))
        _check(lib().gato_set_trajectories(self._h, _dptr(X), _dptr(U)))

    def get_trajectories(self):
        import torch
        X = torch.empty((self.M, self.N_max, self.nx_max), dtype=torch.float32, device="cuda")
        U = torch.empty((self.M, self.N_max - 1, self.nu_max), dtype=torch.float32, device="cuda")
        _check(lib().gato_get_trajectories(self._h, _dptr(X), _dptr(U)))
        return X, U

    def serve_step(self, slots, xs, goal, n_iters: int = 1, shift: int = 1, Xout=None, Uout=None, d_stats=None,
                   stream=None):
        """gato_serve_step: slots (int32 cuda tensor [R]), xs [R, nx_max], goal [R, nu_max]."""
        import torch
        R = int(slots.shape[0])
        self._chk(slots, (R,), torch.int32)
        self._chk(xs, (R, self.nx_max))
        self._chk(goal, (R, self.nu_max))
        if Xout is not None:
            self._chk(Xout, (R, self.N_max, self.nx_max))
        if Uout is not None:
            self._chk(Uout, (R, self.N_max - 1, self.nu_max))
        st = stream.cuda_stream if stream is not None else None
        _check(lib().gato_serve_step(self._h, R, _dptr(slots), _dptr(xs), _dptr(goal), int(n_iters), int(shift),
                                     _dptr(Xout), _dptr(Uout), _dptr(d_stats), C.c_void_p(st) if st else None))

    def plant_step(self, x, tau, h: float = 0.01, substeps: int = 10, slots=None, xn=None, status=None,
                   stream=None, fext=None):
        """gato_plant_step: RK4 plant over h for R instances (x [R, nx_max], tau [R, nu_max],
        optional true tip force fext [R, 3]); returns xn."""
        import torch
        R = int(x.shape[0])
        self._chk(x, (R, self.nx_max))
        self._chk(tau, (R, self.nu_max))
        if fext is not None:
            self._chk(fext, (R, 3))
        if slots is not None:
            self._chk(slots, (R,), torch.int32)
        if xn is None:
            xn = torch.empty_like(x)
        self._chk(xn, (R, self.nx_max))
        if status is not None:
            self._chk(status, (R,), torch.int32)
        st = stream.cuda_stream if stream is not None else None
        _check(lib().gato_plant_step(self._h, R, _dptr(slots), _dptr(x), _dptr(tau), _dptr(fext), float(h),
                                     int(substeps), _dptr(xn), _dptr(status), C.c_void_p(st) if st else None))
        return xn

    def set_external_force(self, f):
        """gato_set_external_force: per-solve tip force [M, 3] (base frame, N)."""
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(f, np.float64), (self.M, 3)))
        _check(lib().gato_set_external_force(self._h, a.ctypes.data_as(C.POINTER(C.c_double))))

    def select_hypotheses(self, P: int, H: int, pred, meas, off, est, sel=None, dist=None, stream=None):
        """gato_select_hypotheses: pred [P H, nx_max], meas [P, nx_max] float32; off [H, 3] and est
        [P, 3] float64 (est updated in place); sel [P] int32 and dist [P H] float64 optional."""
        import torch
        self._chk(pred, (P * H, self.nx_max))
        self._chk(meas, (P, self.nx_max))
        self._chk(off, (H, 3), torch.float64)
        self._chk(est, (P, 3), torch.float64)
        if sel is not None:
            self._chk(sel, (P,), torch.int32)
        if dist is not None:
            self._chk(dist, (P * H,), torch.float64)
        st = stream.cuda_stream if stream is not None else None
        _check(lib().gato_select_hypotheses(self._h, int(P), int(H), _dptr(pred), _dptr(meas), _dptr(off), _dptr(est),
                                            _dptr(sel), _dptr(dist), C.c_void_p(st) if st else None))

    def reset_warm_start(self):
        _check(lib().gato_reset_warm_start(self._h))

    def get_multipliers(self):
        """gato_get_multipliers: the PCG warm-start multipliers, float64 cuda tensor [M, N_max, nx_max]."""
        import torch
        lam = torch.empty((self.M, self.N_max, self.nx_max), dtype=torch.float64, device="cuda")
        _check(lib().gato_get_multipliers(self._h, _dptr(lam)))
        return lam

    def set_multipliers(self, lam):
        """gato_set_multipliers: lam float64 cuda tensor [M, N_max, nx_max]."""
        import torch
        self._chk(lam, (self.M, self.N_max, self.nx_max), torch.float64)
        _check(lib().gato_set_multipliers(self._h, _dptr(lam)))

    def shift_warm_start(self, slots, stream=None):
        """gato_shift_warm_start: shift the resident plans of slots (int32 cuda tensor) one knot."""
        import torch
        n = int(slots.shape[0])
        self._chk(slots, (n,), torch.int32)
        st = stream.cuda_stream if stream is not None else None
        _check(lib().gato_shift_warm_start(self._h, _dptr(slots), n, C.c_void_p(st) if st else None))


class ServeContext:
    """A gato_serve_ctx: one serving launch's stream, event and pinned staging.

    The staging is exposed as numpy arrays over the pinned memory (slots, xs,
    goal in; x1, u0, stats out), written and read in place.
    """

    def __init__(self, batch: "Batch", capacity: int | None = None, n_iters: int = 1):
        self.batch = batch
        self.capacity = int(capacity or batch.M)
        self.n_iters = int(n_iters)
        h = C.c_void_p()
        _check(lib().gato_serve_ctx_create(batch._h, self.capacity, self.n_iters, C.byref(h)))
        self._h = h
        _live_ctx.add(self)
        p = [C.c_void_p() for _ in range(6)]
        _check(lib().gato_serve_ctx_buffers(self._h, *[C.byref(x) for x in p]))
        cap, nx, nu = self.capacity, batch.nx_max, batch.nu_max

        def view(ptr, ctype, shape, dtype=None):
            a = np.ctypeslib.as_array(C.cast(ptr, C.POINTER(ctype)), shape=shape)
            return a.view(dtype) if dtype is not None else a

        self.slots = view(p[0], C.c_int32, (cap,))
        self.xs = view(p[1], C.c_float, (cap, nx))
        self.goal = view(p[2], C.c_float, (cap, nu))
        self.x1 = view(p[3], C.c_float, (cap, nx))
        self.u0 = view(p[4], C.c_float, (cap, nu))
        nb = cap * self.n_iters * STATS_DTYPE.itemsize
        self.stats = view(p[5], C.c_uint8, (nb,)).view(STATS_DTYPE).reshape(cap, self.n_iters)
        self.n = 0

    def submit(self, n_req: int, shift: int = 1):
        self.n = int(n_req)
        _check(lib().gato_serve_ctx_submit(self._h, self.n, int(shift)))

    def done(self) -> bool:
        return _check(lib().gato_serve_ctx_query(self._h)) == 1

    def trajectories(self):
        b = self.batch
        X = np.zeros((self.n, b.N_max, b.nx_max), np.float32)
        U = np.zeros((self.n, b.N_max - 1, b.nu_max), np.float32)
        _check(lib().gato_serve_ctx_trajectories(self._h, X.ctypes.data_as(C.c_void_p), U.ctypes.data_as(C.c_void_p)))
        return X, U

    def close(self):
        if getattr(self, "_h", None):
            lib().gato_serve_ctx_destroy(self._h)
            self._h = None
        _live_ctx.discard(self)

    def __del__(self, _finalizing=sys.is_finalizing):
        # (The default argument keeps the function reachable: at interpreter
        # shutdown the module's globals, sys included, may already be gone.)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def pack_inputs(solves, device="cuda"):
    """Pads a list of problems into the boundary layout: xs, goal, X, U tensors."""
    import torch
    M = len(solves)
    n_max = max(s.n for s in solves)
    N_max = max(s.N for s in solves)
    nx, nu = 2 * n_max, n_max
    xs = np.zeros((M, nx), np.float32)
    goal = np.zeros((M, nu), np.float32)
    X = np.zeros((M, N_max, nx), np.float32)
    U = np.zeros((M, N_max - 1, nu), np.float32)
    for i, s in enumerate(solves):
        xs[i, :2 * s.n] = s.xs
        goal[i, :s.n] = s.qgoal
        X[i, :s.N, :2 * s.n] = s.X0
        U[i, :s.N - 1, :s.n] = s.U0
    t = lambda a: torch.from_numpy(a).to(device)
    return t(xs), t(goal), t(X), t(U)
