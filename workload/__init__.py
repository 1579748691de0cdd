"""Seeded synthetic workloads for the batched trajectory-optimisation path.

This module only draws random robot chains, start states and goals; it holds
none of the solver's arithmetic. Both the FP64 oracle and the GPU library are
fed from it, so the two sides always see identical inputs.

The robots of the paper (a 6-DoF Indy7 and a 7-DoF KUKA iiwa, Sec. IV) are not
available, so seeded revolute serial chains stand in for them:

* link lengths  U[0.2, 0.4] m, masses U[1, 4] kg,
* diagonal inertias about the centre of mass U[0.01, 0.1] kg m^2,
* joint goals and start angles U[-1, 1] rad, start velocities N(0, 0.1^2),
* diagonal tracking weights Q = 1, R = 1e-3, Q_N = 100, dt = 0.01 s.

Solve ``i`` of seed ``s`` draws from ``PCG64(SeedSequence([s, i]))`` in the
order lengths, masses, inertias, goal, start angles, start velocities.  The
uneven batch first draws the DoF from {3, 6, 7} and then N from
{16, 32, 64, 128} from ``PCG64(SeedSequence([s, i, 1]))``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

DEFAULT_DT = 0.01
Q_DIAG = 1.0
R_DIAG = 1e-3
QN_DIAG = 100.0
GRAVITY = 9.81


@dataclass
class Solve:
    """One trajectory-optimisation problem (FP64, row-major numpy arrays)."""

    n: int                      # degrees of freedom
    N: int                      # knot points (states x_0..x_{N-1}); N-1 controls
    dt: float
    links: np.ndarray           # [n, 5]: length, mass, Ixx, Iyy, Izz
    xs: np.ndarray              # [2n] start state [q; qd]
    qgoal: np.ndarray           # [n] joint goal
    Qd: np.ndarray              # [2n] stage state weights
    Rd: np.ndarray              # [n] control weights
    QNd: np.ndarray             # [2n] terminal state weights
    X0: np.ndarray              # [N, 2n] initial state guess
    U0: np.ndarray              # [N-1, n] initial control guess
    model: int = 0              # 0 revolute chain, 1 linear double-integrator chain
    gravity: float = GRAVITY
    spring_k: float = 0.0
    fext: tuple = (0.0, 0.0, 0.0)   # external force on the tip of the last link (base frame), N
    # Task-space tracking of the tip (None: joint-space costs only).
    Wee: np.ndarray | None = None   # [3] stage weights on the tip position error
    WeeN: np.ndarray | None = None  # [3] terminal weights
    pref: np.ndarray | None = None  # [N, 3] reference tip positions, base frame

    @property
    def nx(self) -> int:
        return 2 * self.n

    @property
    def nu(self) -> int:
        return self.n


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def chain_solve(seed: int, i: int, n: int = 7, N: int = 32, dt: float = DEFAULT_DT,
                zero_init: bool = False) -> Solve:
    """Solve ``i`` of the seeded 7-DoF (or n-DoF) chain family."""
    g = _rng(seed, i)
    length = g.uniform(0.2, 0.4, n)
    mass = g.uniform(1.0, 4.0, n)
    inertia = g.uniform(0.01, 0.1, (n, 3))
    qgoal = g.uniform(-1.0, 1.0, n)
    q0 = g.uniform(-1.0, 1.0, n)
    qd0 = g.normal(0.0, 0.1, n)
    links = np.column_stack([length, mass, inertia])
    xs = np.concatenate([q0, qd0])
    nx = 2 * n
    X0 = np.zeros((N, nx)) if zero_init else np.tile(xs, (N, 1))
    U0 = np.zeros((N - 1, n))
    return Solve(n=n, N=N, dt=dt, links=links, xs=xs, qgoal=qgoal,
                 Qd=np.full(nx, Q_DIAG), Rd=np.full(n, R_DIAG), QNd=np.full(nx, QN_DIAG),
                 X0=X0, U0=U0)


def chain_batch(seed: int, M: int, n: int = 7, N: int = 32, dt: float = DEFAULT_DT) -> list[Solve]:
    """``M`` independent seeded chains of one shape (the uniform batch)."""
    return [chain_solve(seed, i, n=n, N=N, dt=dt) for i in range(M)]


def uneven_batch(seed: int, M: int = 128, dofs=(3, 6, 7), horizons=(16, 32, 64, 128),
                 dt: float = DEFAULT_DT) -> list[Solve]:
    """``M`` chains whose DoF and horizon are drawn uniformly per solve."""
    out = []
    for i in range(M):
        g = _rng(seed, i, 1)
        n = int(g.choice(dofs))
        N = int(g.choice(horizons))
        out.append(chain_solve(seed, i, n=n, N=N, dt=dt))
    return out


# Task-space (figure-8) tracking weights: a light joint-posture and velocity
# regulariser, the tip position weighted per axis.
TS_Q_POS, TS_Q_VEL, TS_QN_VEL = 1e-1, 1e-1, 1.0
TS_W_STAGE, TS_W_TERMINAL = 1e2, 1e3
TS_PERIOD_S = 2.0


def figure8_solve(seed: int, i: int, n: int = 7, N: int = 32, dt: float = DEFAULT_DT, t0: float = 0.0) -> Solve:
    """Solve ``i`` of the chain family tracking a figure-8 with the tip.

    The chain, start state and posture goal are those of :func:`chain_solve`.
    Extra draws from ``PCG64(SeedSequence([seed, i, 4]))``: the azimuth of the
    figure's centre U[-pi, pi] and its phase U[0, 2 pi]. With reach L (the sum
    of the link lengths), the centre sits at horizontal distance 0.35 L and
    height 0.45 L; the figure (a lemniscate of Gerono, amplitude 0.1 L, period
    2 s) lies in the vertical plane through the centre, tangent to the circle
    around the base:  pref(t) = c + 0.1 L (sin th e_t + sin th cos th e_z),
    th = 2 pi t / T + phase, t = t0 + k dt.  Weights: Q = 1e-1 on angles (towards
    the posture goal) and 1e-1 on velocities, Q_N = 1e-1 / 1, R = 1e-3, tip
    weights 1e2 per axis at every stage and 1e3 at the last knot.
    """
    s = chain_solve(seed, i, n=n, N=N, dt=dt)
    g = _rng(seed, i, 4)
    az = g.uniform(-np.pi, np.pi)
    phase = g.uniform(0.0, 2.0 * np.pi)
    L = float(np.sum(s.links[:, 0]))
    c = np.array([0.35 * L * np.cos(az), 0.35 * L * np.sin(az), 0.45 * L])
    e_t = np.array([-np.sin(az), np.cos(az), 0.0])
    e_z = np.array([0.0, 0.0, 1.0])
    th = 2.0 * np.pi * (t0 + dt * np.arange(N)) / TS_PERIOD_S + phase
    a = 0.1 * L
    s.pref = c + a * (np.sin(th)[:, None] * e_t + (np.sin(th) * np.cos(th))[:, None] * e_z)
    s.Qd = np.concatenate([np.full(n, TS_Q_POS), np.full(n, TS_Q_VEL)])
    s.QNd = np.concatenate([np.full(n, TS_Q_POS), np.full(n, TS_QN_VEL)])
    s.Wee = np.full(3, TS_W_STAGE)
    s.WeeN = np.full(3, TS_W_TERMINAL)
    return s


def figure8_batch(seed: int, M: int, n: int = 7, N: int = 32, dt: float = DEFAULT_DT) -> list[Solve]:
    """``M`` seeded chains tracking figure-8s with the tip."""
    return [figure8_solve(seed, i, n=n, N=N, dt=dt) for i in range(M)]


def figure8_uneven_batch(seed: int, M: int = 128, dofs=(3, 6, 7), horizons=(16, 32, 64, 128),
                         dt: float = DEFAULT_DT) -> list[Solve]:
    """The DoF and horizons of :func:`uneven_batch` (the same draws), every
    solve tracking a figure-8 with the tip as in :func:`figure8_solve`."""
    return [figure8_solve(seed, i, n=s.n, N=s.N, dt=dt)
            for i, s in enumerate(uneven_batch(seed, M=M, dofs=dofs, horizons=horizons, dt=dt))]


def double_integrator_solve(seed: int, i: int, n: int = 3, N: int = 8, dt: float = 0.05,
                            spring_k: float = 1.0) -> Solve:
    """A linear chain of unit masses coupled by springs (q'' = u - k T q).

    The start state and goal are seeded; the initial guess is left for the
    caller (tests roll it out to make the constraints feasible).
    """
    g = _rng(seed, i, 2)
    q0 = g.uniform(-1.0, 1.0, n)
    qd0 = g.normal(0.0, 0.1, n)
    qgoal = g.uniform(-1.0, 1.0, n)
    U0 = g.normal(0.0, 0.5, (N - 1, n))
    xs = np.concatenate([q0, qd0])
    nx = 2 * n
    return Solve(n=n, N=N, dt=dt, links=np.zeros((n, 5)), xs=xs, qgoal=qgoal,
                 Qd=np.full(nx, Q_DIAG), Rd=np.full(n, R_DIAG), QNd=np.full(nx, QN_DIAG),
                 X0=np.tile(xs, (N, 1)), U0=U0, model=1, gravity=0.0, spring_k=spring_k)


@dataclass
class MpcRequests:
    """Poisson request stream over a pool of MPC instances."""

    arrival_s: np.ndarray       # [R] arrival times
    instance: np.ndarray        # [R] instance ids
    goal_noise: np.ndarray      # [R, n] goal perturbation, rad
    extra: dict = field(default_factory=dict)


def mpc_requests(seed: int, rate_hz: float, duration_s: float, n_instances: int, n: int = 7,
                 goal_sigma: float = 0.05) -> MpcRequests:
    """Poisson arrivals, uniform instance choice and N(0, sigma^2) goal jitter."""
    g = _rng(seed, 3)
    count = int(g.poisson(rate_hz * duration_s))
    t = np.sort(g.uniform(0.0, duration_s, count))
    inst = g.integers(0, n_instances, count)
    noise = g.normal(0.0, goal_sigma, (count, n))
    return MpcRequests(arrival_s=t, instance=inst, goal_noise=noise)
