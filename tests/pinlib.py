"""Independent numpy helpers that pin the oracle: brute-force kinematics,
geometric-Jacobian mass matrix, potential energy, Christoffel terms by
finite differences. Written from the definitions (rigid-body mechanics), not
from the oracle's code."""
import numpy as np


def rot(axis, q):
    a = np.asarray(axis, dtype=float)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(q) * K + (1 - np.cos(q)) * K @ K


def chain_of(robot, e):
    """Per-link dicts for env e."""
    n = int(robot.n_dof[e])
    links = []
    for j in range(n):
        xx, yy, zz, xy, xz, yz = robot.inertia[:, j, e]
        jt = 0 if getattr(robot, "joint_type", None) is None else int(robot.joint_type[j, e])
        links.append(dict(axis=robot.axis[:, j, e], offset=robot.offset[:, j, e], com=robot.com[:, j, e],
                          m=robot.mass[j, e], Ic=np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]]),
                          prismatic=jt == 1))
    return links, robot.tip[:, e], np.asarray(robot.gravity, dtype=float)


def fk(links, tip, q):
    """World (R_j, p_j) of every link frame, world COMs and the tip."""
    R = np.eye(3)
    p = np.zeros(3)
    Rs, ps, coms = [], [], []
    for j, l in enumerate(links):
        if l.get("prismatic"):
            p = p + R @ (l["offset"] + q[j] * np.asarray(l["axis"]))
        else:
            p = p + R @ l["offset"]
            R = R @ rot(l["axis"], q[j])
        Rs.append(R)
        ps.append(p)
        coms.append(p + R @ l["com"])
    return Rs, ps, coms, p + R @ tip


def mass_matrix(links, tip, q):
    """M = sum_k m_k Jv_k^T Jv_k + Jw_k^T (R_k Ic_k R_k^T) Jw_k."""
    n = len(links)
    Rs, ps, coms, _ = fk(links, tip, q)
    z = [Rs[i] @ links[i]["axis"] for i in range(n)]
    M = np.zeros((n, n))
    for k in range(n):
        Jv = np.zeros((3, n))
        Jw = np.zeros((3, n))
        for i in range(k + 1):
            if links[i].get("prismatic"):
                Jv[:, i] = z[i]
            else:
                Jv[:, i] = np.cross(z[i], coms[k] - ps[i])
                Jw[:, i] = z[i]
        Iw = Rs[k] @ links[k]["Ic"] @ Rs[k].T
        M += links[k]["m"] * Jv.T @ Jv + Jw.T @ Iw @ Jw
    return M


def potential(links, tip, q, grav):
    _, _, coms, _ = fk(links, tip, q)
    return -sum(l["m"] * np.dot(grav, c) for l, c in zip(links, coms))


def bias_fd(links, tip, q, qd, grav, eps=1e-6):
    """C(q, qd) qd + G(q) from central differences of M and V."""
    n = len(links)
    dM = np.zeros((n, n, n))  # dM[:, :, k] = dM/dq_k
    G = np.zeros(n)
    for k in range(n):
        dq = np.zeros(n)
        dq[k] = eps
        dM[:, :, k] = (mass_matrix(links, tip, q + dq) - mass_matrix(links, tip, q - dq)) / (2 * eps)
        G[k] = (potential(links, tip, q + dq, grav) - potential(links, tip, q - dq, grav)) / (2 * eps)
    c = np.zeros(n)
    for i in range(n):
        for j in range(n):
            for k in range(n):
                gamma = 0.5 * (dM[i, j, k] + dM[i, k, j] - dM[j, k, i])
                c[i] += gamma * qd[j] * qd[k]
    return c + G


def energy(links, tip, q, qd, grav):
    M = mass_matrix(links, tip, q)
    return 0.5 * qd @ M @ qd + potential(links, tip, q, grav)
