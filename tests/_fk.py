"""Independent forward kinematics of the revolute test chain (numpy, FP64).

Used only to pin the oracle: the mass matrix from geometric Jacobians and the
potential energy, from which the Lagrangian form of the dynamics follows. It
shares nothing with the oracle's Newton-Euler recursion.
"""
import numpy as np


def rot(axis_y: bool, q: float) -> np.ndarray:
    c, s = np.cos(q), np.sin(q)
    if axis_y:
        return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def frames(links, q):
    """World rotation R_i, joint origin p_i, joint axis z_i, COM c_i of each link."""
    n = len(q)
    R, p, z, c = [], [], [], []
    Rc, pc = np.eye(3), np.zeros(3)
    for i in range(n):
        if i > 0:
            pc = pc + Rc @ np.array([0, 0, links[i - 1][0]])
        Rc = Rc @ rot(i % 2 == 1, q[i])
        R.append(Rc.copy())
        p.append(pc.copy())
        z.append(Rc @ (np.array([0, 1.0, 0]) if i % 2 else np.array([0, 0, 1.0])))
        c.append(pc + Rc @ np.array([0, 0, 0.5 * links[i][0]]))
    return R, p, z, c


def mass_matrix(links, q) -> np.ndarray:
    """M(q) = sum_i m_i Jv_i^T Jv_i + Jw_i^T R_i Ic_i R_i^T Jw_i."""
    n = len(q)
    R, p, z, c = frames(links, q)
    M = np.zeros((n, n))
    for i in range(n):
        Jv = np.zeros((3, n))
        Jw = np.zeros((3, n))
        for j in range(i + 1):
            Jv[:, j] = np.cross(z[j], c[i] - p[j])
            Jw[:, j] = z[j]
        m = links[i][1]
        Ic = np.diag(links[i][2:5])
        M += m * Jv.T @ Jv + Jw.T @ (R[i] @ Ic @ R[i].T) @ Jw
    return M


def potential(links, q, g=9.81) -> float:
    _, _, _, c = frames(links, q)
    return sum(links[i][1] * g * c[i][2] for i in range(len(q)))


def lagrangian_id(links, q, qd, qdd, g=9.81, h=1e-5) -> np.ndarray:
    """tau = M qdd + Mdot qd - 1/2 d(qd^T M qd)/dq + dV/dq, derivatives by central differences."""
    n = len(q)
    M = mass_matrix(links, q)
    dM = []
    dV = np.zeros(n)
    for j in range(n):
        e = np.zeros(n)
        e[j] = h
        dM.append((mass_matrix(links, q + e) - mass_matrix(links, q - e)) / (2 * h))
        dV[j] = (potential(links, q + e, g) - potential(links, q - e, g)) / (2 * h)
    Mdot = sum(dM[j] * qd[j] for j in range(n))
    quad = np.array([qd @ dM[i] @ qd for i in range(n)])
    return M @ qdd + Mdot @ qd - 0.5 * quad + dV


def tip(links, q) -> np.ndarray:
    """Position of the tip of the last link (its far end along its local +z)."""
    R, p, _, _ = frames(links, q)
    return p[-1] + R[-1] @ np.array([0, 0, links[len(q) - 1][0]])


def tip_jacobian(links, q) -> np.ndarray:
    """Positional Jacobian of the tip: column j = z_j x (p_tip - p_j)."""
    _, p, z, _ = frames(links, q)
    pt = tip(links, q)
    return np.stack([np.cross(z[j], pt - p[j]) for j in range(len(q))], axis=1)
