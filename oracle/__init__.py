"""FP64 CPU oracle for the batched SQP path (ctypes binding of gato_oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark. The product library never imports it.

Every function takes a :class:`workload.Solve` (robot, horizon, weights, start
state, goal) plus plain numpy arrays, and returns FP64 numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "gato_oracle.cpp")
LIB = os.path.join(_HERE, "libgato_oracle.so")

MAX_ALPHA = 32
ST_PCG_MAXITER, ST_NONFINITE, ST_NO_DESCENT = 1, 2, 4


def build() -> str:
    """Compile the oracle with g++ (IEEE FP64, no fast-math)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-Wall", "-Wextra", SRC, "-o", LIB + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class _Robot(C.Structure):
    _fields_ = [("model", C.c_int), ("n", C.c_int), ("link", C.POINTER(C.c_double)),
                ("gravity", C.c_double), ("spring_k", C.c_double), ("fext", C.c_double * 3)]


class _Problem(C.Structure):
    _fields_ = [("N", C.c_int), ("dt", C.c_double), ("Qd", C.POINTER(C.c_double)),
                ("Rd", C.POINTER(C.c_double)), ("QNd", C.POINTER(C.c_double)),
                ("Wee", C.POINTER(C.c_double)), ("WeeN", C.POINTER(C.c_double)), ("pref", C.POINTER(C.c_double))]


class _Params(C.Structure):
    _fields_ = [("sqp_iters", C.c_int), ("kkt_mode", C.c_int), ("pcg_tol", C.c_double),
                ("pcg_max_iter", C.c_int), ("warm_lambda", C.c_int), ("mu", C.c_double),
                ("beta", C.c_double), ("n_alpha", C.c_int), ("rho", C.c_double), ("rho_adapt", C.c_int)]


class _IterLog(C.Structure):
    _fields_ = [("merit0", C.c_double), ("merit", C.c_double), ("alpha", C.c_double), ("J", C.c_double),
                ("c1", C.c_double), ("kkt_res", C.c_double), ("pcg_iters", C.c_int), ("status", C.c_int),
                ("argmin", C.c_int), ("pad", C.c_int), ("rho", C.c_double), ("merits", C.c_double * MAX_ALPHA),
                ("pcg_stop", C.c_double), ("pcg_stop_prev", C.c_double)]


@dataclass
class Params:
    """Solver settings (the paper leaves them to its code; see the design notes)."""

    sqp_iters: int = 10
    kkt_mode: int = 0          # 0 dense LU of the KKT matrix, 1 Schur + PCG, 2 Riccati
    pcg_tol: float = 1e-6
    pcg_max_iter: int = 0      # 0: N * nx
    warm_lambda: int = 1
    mu: float = 10.0
    beta: float = 2.0
    n_alpha: int = 8
    rho: float = 0.0           # initial damping on every Q_k
    rho_adapt: int = 0         # 1: rho /= 3 after a descent, rho *= 2 after none


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        rp, pp = C.POINTER(_Robot), C.POINTER(_Problem)
        L.orc_inverse_dynamics.argtypes = [rp, dp, dp, dp, C.c_int, dp]
        L.orc_mass_matrix.argtypes = [rp, dp, dp]
        L.orc_forward_dynamics.argtypes = [rp, dp, dp, dp, dp]
        L.orc_fd_derivatives.argtypes = [rp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_step.argtypes = [rp, C.c_double, dp, dp, dp]
        L.orc_step_jacobians.argtypes = [rp, C.c_double, dp, dp, dp, dp, dp]
        L.orc_plant_rk4.argtypes = [rp, C.c_double, C.c_int, dp, dp, dp]
        L.orc_lq.argtypes = [rp, pp, C.c_double, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_kkt_parts.argtypes = [rp, pp, C.c_double, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_schur.argtypes = [rp, pp, C.c_double, dp, dp, dp, dp, dp, dp, dp]
        L.orc_pcg_dense.argtypes = [C.c_int, dp, dp, dp, dp, C.c_double, C.c_int, C.POINTER(C.c_int)]
        L.orc_qp_step.argtypes = [rp, pp, C.c_double, dp, dp, dp, dp, C.c_int, C.c_double, C.c_int, dp, dp,
                                  C.POINTER(C.c_int), dp]
        L.orc_kkt_from_lq.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, dp, dp, dp, dp, dp, dp, C.c_int, dp, dp,
                                      dp]
        L.orc_kkt_residual.argtypes = [rp, pp, C.c_double, dp, dp, dp, dp, dp, dp]
        L.orc_kkt_residual.restype = C.c_double
        L.orc_merit.argtypes = [rp, pp, dp, dp, dp, dp, C.c_double, dp, dp]
        L.orc_merit.restype = C.c_double
        L.orc_tip.argtypes = [rp, dp, dp, dp]
        L.orc_lq_hessian.argtypes = [rp, pp, C.c_double, dp, dp, dp, dp, dp]
        L.orc_sqp.argtypes = [rp, pp, C.POINTER(_Params), dp, dp, dp, dp, dp, C.POINTER(_IterLog), dp,
                              C.POINTER(C.c_int), C.POINTER(C.c_int)]
        _lib = L
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class _Ctx:
    """Keeps the numpy buffers behind the C structs alive."""

    def __init__(self, s):
        self.link = _f64(s.links).reshape(-1) if s.links is not None else np.zeros(5)
        fe = tuple(float(v) for v in getattr(s, "fext", (0.0, 0.0, 0.0)))
        self.robot = _Robot(int(s.model), int(s.n), _ptr(self.link), float(s.gravity), float(s.spring_k),
                            (C.c_double * 3)(*fe))
        N = getattr(s, "N", 2)
        self.Qd, self.Rd, self.QNd = (_f64(getattr(s, k, np.ones(1))) for k in ("Qd", "Rd", "QNd"))
        self.prob = _Problem(int(N), float(getattr(s, "dt", 0.01)), _ptr(self.Qd), _ptr(self.Rd), _ptr(self.QNd))
        if getattr(s, "Wee", None) is not None:
            # Task-space tracking of the tip (all three or none).
            self.Wee, self.WeeN = _f64(s.Wee).reshape(3), _f64(s.WeeN).reshape(3)
            self.pref = _f64(s.pref).reshape(int(N), 3)
            self.prob.Wee, self.prob.WeeN, self.prob.pref = _ptr(self.Wee), _ptr(self.WeeN), _ptr(self.pref)


def inverse_dynamics(s, q, qd, qdd, gravity: bool = True) -> np.ndarray:
    c = _Ctx(s)
    q, qd, qdd = _f64(q), _f64(qd), _f64(qdd)
    tau = np.zeros(s.n)
    lib().orc_inverse_dynamics(C.byref(c.robot), _ptr(q), _ptr(qd), _ptr(qdd), int(gravity), _ptr(tau))
    return tau


def mass_matrix(s, q) -> np.ndarray:
    c = _Ctx(s)
    q = _f64(q)
    M = np.zeros((s.n, s.n))
    lib().orc_mass_matrix(C.byref(c.robot), _ptr(q), _ptr(M))
    return M


def forward_dynamics(s, q, qd, tau) -> np.ndarray:
    c = _Ctx(s)
    q, qd, tau = _f64(q), _f64(qd), _f64(tau)
    qdd = np.zeros(s.n)
    if lib().orc_forward_dynamics(C.byref(c.robot), _ptr(q), _ptr(qd), _ptr(tau), _ptr(qdd)) != 0:
        raise FloatingPointError("mass matrix not positive definite")
    return qdd


def fd_derivatives(s, q, qd, tau):
    """Returns (qdd, dqdd/dq, dqdd/dqd, M^-1)."""
    c = _Ctx(s)
    q, qd, tau = _f64(q), _f64(qd), _f64(tau)
    n = s.n
    qdd, dq, dqd, Minv = np.zeros(n), np.zeros((n, n)), np.zeros((n, n)), np.zeros((n, n))
    if lib().orc_fd_derivatives(C.byref(c.robot), _ptr(q), _ptr(qd), _ptr(tau), _ptr(qdd), _ptr(dq), _ptr(dqd),
                                _ptr(Minv)) != 0:
        raise FloatingPointError("mass matrix not positive definite")
    return qdd, dq, dqd, Minv


def step(s, x, u, h=None) -> np.ndarray:
    c = _Ctx(s)
    x, u = _f64(x), _f64(u)
    xn = np.zeros(2 * s.n)
    if lib().orc_step(C.byref(c.robot), float(s.dt if h is None else h), _ptr(x), _ptr(u), _ptr(xn)) != 0:
        raise FloatingPointError("mass matrix not positive definite")
    return xn


def plant_rk4(s, x, tau, h: float = 0.01, substeps: int = 10) -> np.ndarray:
    """Closed-loop plant: RK4 on x' = [qd; FD(q, qd, tau)], tau held over h (Sec. IV-E)."""
    c = _Ctx(s)
    x, tau = _f64(x), _f64(tau)
    xn = np.zeros(2 * s.n)
    rc = lib().orc_plant_rk4(C.byref(c.robot), float(h), int(substeps), _ptr(x), _ptr(tau), _ptr(xn))
    if rc != 0:
        raise FloatingPointError("mass matrix not positive definite" if rc == -1 else "substeps must be >= 1")
    return xn


def hypothesis_select(s, x, tau, forces, x_meas, h: float = 0.01, substeps: int = 10):
    """Selection step of the hypothesize-and-test case study (Sec. IV-D), read
    as in the design notes: each hypothesis is an external tip force; its
    one-step prediction is the RK4 plant from x under tau with that force; it
    scores the Euclidean distance of its prediction to the measured state
    x_meas; the smallest distance wins, ties to the smaller index. forces
    [H, 3]; returns (index, distances [H])."""
    import dataclasses
    d = np.zeros(len(forces))
    for j, f in enumerate(np.asarray(forces, np.float64)):
        sj = dataclasses.replace(s, fext=tuple(float(v) for v in f))
        d[j] = np.linalg.norm(plant_rk4(sj, x, tau, h, substeps) - _f64(x_meas))
    best = 0
    for j in range(1, len(d)):
        if d[j] < d[best]:
            best = j
    return best, d


def step_jacobians(s, x, u, h=None):
    """Returns (f(x, u), A, B) of the explicit Euler step."""
    c = _Ctx(s)
    x, u = _f64(x), _f64(u)
    n = s.n
    xn, A, B = np.zeros(2 * n), np.zeros((2 * n, 2 * n)), np.zeros((2 * n, n))
    if lib().orc_step_jacobians(C.byref(c.robot), float(s.dt if h is None else h), _ptr(x), _ptr(u), _ptr(xn),
                                _ptr(A), _ptr(B)) != 0:
        raise FloatingPointError("mass matrix not positive definite")
    return xn, A, B


def lq(s, X, U, rho: float = 0.0) -> dict:
    """LQ data of Eq. (1) at (X, U)."""
    c = _Ctx(s)
    X, U, xs, qg = _f64(X), _f64(U), _f64(s.xs), _f64(s.qgoal)
    n, N = s.n, s.N
    nx, nu = 2 * n, n
    out = dict(A=np.zeros((N - 1, nx, nx)), B=np.zeros((N - 1, nx, nu)), e=np.zeros((N - 1, nx)),
               q=np.zeros((N, nx)), r=np.zeros((max(N - 1, 0), nu)), c0=np.zeros(nx))
    lib().orc_lq(C.byref(c.robot), C.byref(c.prob), float(rho), _ptr(xs), _ptr(qg), _ptr(X), _ptr(U),
                 *(_ptr(out[k]) for k in ("A", "B", "e", "q", "r", "c0")))
    return out


def tip(s, q):
    """Tip position [3] (base frame) and its Jacobian [3, n] at joint angles q."""
    c = _Ctx(s)
    q = _f64(q)
    p, J = np.zeros(3), np.zeros((3, s.n))
    if lib().orc_tip(C.byref(c.robot), _ptr(q), _ptr(p), _ptr(J)) != 0:
        raise ValueError("tip kinematics need the revolute chain model")
    return p, J


def lq_hessian(s, X, U, rho: float = 0.0) -> np.ndarray:
    """State Hessian blocks Q_k [N, nx, nx] of the QP at (X, U)."""
    c = _Ctx(s)
    X, U, xs, qg = _f64(X), _f64(U), _f64(s.xs), _f64(s.qgoal)
    nx, N = 2 * s.n, s.N
    Qf = np.zeros((N, nx, nx))
    lib().orc_lq_hessian(C.byref(c.robot), C.byref(c.prob), float(rho), _ptr(xs), _ptr(qg), _ptr(X), _ptr(U),
                         _ptr(Qf))
    return Qf


def kkt_parts(s, X, U, rho: float = 0.0):
    """Dense G, g, C, c of Eq. (2); dZ is ordered [x_0 u_0 x_1 u_1 ... x_{N-1}]."""
    c = _Ctx(s)
    X, U, xs, qg = _f64(X), _f64(U), _f64(s.xs), _f64(s.qgoal)
    nx, nu, N = 2 * s.n, s.n, s.N
    nz, nc = N * nx + (N - 1) * nu, N * nx
    G, g, Cm, cv = np.zeros((nz, nz)), np.zeros(nz), np.zeros((nc, nz)), np.zeros(nc)
    lib().orc_kkt_parts(C.byref(c.robot), C.byref(c.prob), float(rho), _ptr(xs), _ptr(qg), _ptr(X), _ptr(U),
                        _ptr(G), _ptr(g), _ptr(Cm), _ptr(cv))
    return G, g, Cm, cv


def schur(s, X, U, rho: float = 0.0):
    """Dense S~, gamma~, P (Eqs. (5)-(6), sign readings R2/R3)."""
    c = _Ctx(s)
    X, U, xs, qg = _f64(X), _f64(U), _f64(s.xs), _f64(s.qgoal)
    dim = s.N * 2 * s.n
    S, gam, P = np.zeros((dim, dim)), np.zeros(dim), np.zeros((dim, dim))
    lib().orc_schur(C.byref(c.robot), C.byref(c.prob), float(rho), _ptr(xs), _ptr(qg), _ptr(X), _ptr(U),
                    _ptr(S), _ptr(gam), _ptr(P))
    return S, gam, P


def pcg_dense(S, P, gamma, lam0=None, tol: float = 1e-6, max_iter: int = 0):
    """PCG of Sec. II-B on dense inputs; returns (lambda, iterations, hit_max)."""
    S, P, gamma = _f64(S), _f64(P), _f64(gamma)
    dim = gamma.shape[0]
    lam = _f64(np.zeros(dim) if lam0 is None else lam0).copy()
    hm = C.c_int(0)
    it = lib().orc_pcg_dense(dim, _ptr(S), _ptr(P), _ptr(gamma), _ptr(lam), float(tol),
                             int(max_iter if max_iter > 0 else dim), C.byref(hm))
    return lam, it, bool(hm.value)


def split_dz(s, dZ):
    """dZ [x_0 u_0 ... x_{N-1}] -> (dX [N, nx], dU [N-1, nu])."""
    nx, nu, N = 2 * s.n, s.n, s.N
    dX = np.zeros((N, nx))
    dU = np.zeros((N - 1, nu))
    for k in range(N):
        o = k * (nx + nu)
        dX[k] = dZ[o:o + nx]
        if k < N - 1:
            dU[k] = dZ[o + nx:o + nx + nu]
    return dX, dU


def qp_step(s, X, U, mode: int = 0, rho: float = 0.0, pcg_tol: float = 1e-6, pcg_max_iter: int = 0,
            lam0=None):
    """One linear solve of the SQP step; returns (dX, dU, lambda, pcg_iters, kkt_res)."""
    c = _Ctx(s)
    X, U, xs, qg = _f64(X), _f64(U), _f64(s.xs), _f64(s.qgoal)
    nx, nu, N = 2 * s.n, s.n, s.N
    dZ = np.zeros(N * nx + (N - 1) * nu)
    lam = _f64(np.zeros(N * nx) if lam0 is None else lam0).reshape(-1).copy()
    its, res = C.c_int(0), C.c_double(0.0)
    rc = lib().orc_qp_step(C.byref(c.robot), C.byref(c.prob), float(rho), _ptr(xs), _ptr(qg), _ptr(X), _ptr(U),
                           int(mode), float(pcg_tol), int(pcg_max_iter), _ptr(dZ), _ptr(lam), C.byref(its),
                           C.byref(res))
    if rc != 0:
        raise FloatingPointError("QP step failed")
    dX, dU = split_dz(s, dZ)
    return dX, dU, lam.reshape(N, nx), its.value, res.value


def kkt_residual(s, X, U, dZ, lam, rho: float = 0.0) -> float:
    """inf-norm residual of the KKT system of Eq. (2) at (X, U) for the given
    dZ [x_0 u_0 ... x_{N-1}] and multipliers lambda [N, nx] (the value the SQP
    loop logs as kkt_res)."""
    c = _Ctx(s)
    X, U, xs, qg = _f64(X), _f64(U), _f64(s.xs), _f64(s.qgoal)
    dZ, lam = _f64(dZ).reshape(-1), _f64(lam).reshape(-1)
    nx, nu, N = 2 * s.n, s.n, s.N
    assert dZ.size == N * nx + (N - 1) * nu and lam.size == N * nx
    r = lib().orc_kkt_residual(C.byref(c.robot), C.byref(c.prob), float(rho), _ptr(xs), _ptr(qg), _ptr(X), _ptr(U),
                               _ptr(dZ), _ptr(lam))
    if r < 0:
        raise FloatingPointError("QP data could not be formed")
    return r


def kkt_from_lq(A, B, e, q, r, c0, Qh, Rh, mode: int = 0):
    """KKT solve (Eq. (2)) on given QP data; returns (dX [N, nx], dU [N-1, nu], lambda [N, nx], residual).

    Qh is the [N, nx] Hessian diagonal of the states (Q_k + rho, Q_N + rho at
    the last knot), Rh the [nu] control Hessian diagonal.
    """
    A, B, e, q, r, c0, Qh, Rh = (_f64(v) for v in (A, B, e, q, r, c0, Qh, Rh))
    N, nx = q.shape
    nu = Rh.shape[0]
    dZ = np.zeros(N * nx + (N - 1) * nu)
    lam = np.zeros(N * nx)
    res = C.c_double(0.0)
    rc = lib().orc_kkt_from_lq(nx, nu, N, _ptr(A), _ptr(B), _ptr(e), _ptr(q), _ptr(r), _ptr(c0), _ptr(Qh),
                               _ptr(Rh), int(mode), _ptr(dZ), _ptr(lam), C.byref(res))
    if rc != 0:
        raise FloatingPointError("KKT solve failed")
    dX = np.zeros((N, nx))
    dU = np.zeros((N - 1, nu))
    for k in range(N):
        o = k * (nx + nu)
        dX[k] = dZ[o:o + nx]
        if k < N - 1:
            dU[k] = dZ[o + nx:o + nx + nu]
    return dX, dU, lam.reshape(N, nx), res.value


def merit(s, X, U, mu: float = 10.0):
    """Eq. (3) at (X, U): returns (merit, J, ||c||_1)."""
    c = _Ctx(s)
    X, U, xs, qg = _f64(X), _f64(U), _f64(s.xs), _f64(s.qgoal)
    J, c1 = C.c_double(0.0), C.c_double(0.0)
    m = lib().orc_merit(C.byref(c.robot), C.byref(c.prob), _ptr(xs), _ptr(qg), _ptr(X), _ptr(U), float(mu),
                        C.byref(J), C.byref(c1))
    return m, J.value, c1.value


@dataclass
class SqpResult:
    X: np.ndarray
    U: np.ndarray
    lam: np.ndarray
    logs: list
    rc: int


def sqp(s, params: Params | None = None, X=None, U=None, lam=None, alpha_replay=None,
        descent_replay=None, pcg_replay=None) -> SqpResult:
    """The SQP loop for one solve (Sec. II-A, Algorithm 1). alpha_replay /
    descent_replay / pcg_replay prescribe, per SQP iteration, the accepted
    step, the descent decision of the rho adaptation and (Schur + PCG mode)
    the PCG iteration count; each log entry keeps the oracle's own view of the
    decision (merits, pcg_stop and pcg_stop_prev: the stopping value over its
    threshold after the last PCG iteration and after the one before)."""
    p = params or Params()
    c = _Ctx(s)
    nx, N = 2 * s.n, s.N
    X = _f64(s.X0 if X is None else X).copy()
    U = _f64(s.U0 if U is None else U).copy()
    lamv = _f64(np.zeros((N, nx)) if lam is None else lam).copy()
    xs, qg = _f64(s.xs), _f64(s.qgoal)
    prm = _Params(p.sqp_iters, p.kkt_mode, p.pcg_tol, p.pcg_max_iter, p.warm_lambda, p.mu, p.beta, p.n_alpha,
                  p.rho, p.rho_adapt)
    logs = (_IterLog * max(p.sqp_iters, 1))()
    rep = None
    if alpha_replay is not None:
        rep = _f64(alpha_replay)
    rc = lib().orc_sqp(C.byref(c.robot), C.byref(c.prob), C.byref(prm), _ptr(xs), _ptr(qg), _ptr(X), _ptr(U),
                       _ptr(lamv), logs, _ptr(rep) if rep is not None else None,
                       (C.c_int * len(descent_replay))(*[int(v) for v in descent_replay])
                       if descent_replay is not None else None,
                       (C.c_int * len(pcg_replay))(*[int(v) for v in pcg_replay])
                       if pcg_replay is not None else None)
    out = []
    for i in range(p.sqp_iters):
        L = logs[i]
        out.append(dict(merit0=L.merit0, merit=L.merit, alpha=L.alpha, J=L.J, c1=L.c1, kkt_res=L.kkt_res,
                        pcg_iters=L.pcg_iters, status=L.status, argmin=L.argmin, rho=L.rho,
                        pcg_stop=L.pcg_stop, pcg_stop_prev=L.pcg_stop_prev,
                        merits=np.array(L.merits[:p.n_alpha])))
    return SqpResult(X=X, U=U, lam=lamv, logs=out, rc=rc)


def sqp_batch(solves, params: Params | None = None, threads: int = 1, X=None, U=None):
    """Runs :func:`sqp` over a batch, one solve per thread (ctypes drops the GIL)."""
    lib()
    def one(i):
        return sqp(solves[i], params, X=None if X is None else X[i], U=None if U is None else U[i])
    if threads <= 1:
        return [one(i) for i in range(len(solves))]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(one, range(len(solves))))
