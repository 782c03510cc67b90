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


# ---- expected share of BF16 rounding flips ---------------------------------
def rne_bf16(x):
    """Round float64 values to the nearest BF16 value (ties to even) via the
    float32 bit pattern (values are first rounded to float32)."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _act(kind, z):
    if kind == "tanh":
        return np.tanh(z)
    if kind == "elu":
        return np.where(z > 0, z, np.expm1(np.minimum(z, 0)))
    return z


def flip_share(layers, acts, x, thr, trials=4, seed=0, rel_scale=None, x_err=None):
    """Expected share of the outputs of a BF16-emulating MLP (each layer's
    input and weights rounded to BF16, sums exact) that move by more than thr
    when every hidden unit carries the error of an FP32 evaluation: the
    pre-activation z + e with e ~ N(0, s^2), s = 2^-24 sqrt(K) |w . h|_2 (K
    FP32 additions of the layer's products, K the fan-in), and the
    activation a + f with f ~ N(0, 2^-46) (tanh or ELU formed from the
    hardware exponential and reciprocal, whose absolute error is about one
    FP32 unit of 1, 2^-23). Such errors only matter where they move an
    activation across a BF16 rounding boundary (a flip of one BF16 unit), so
    the share is the flip share to expect from a correct FP32 kernel. layers: [(W, b)]
    with W [out][in]; acts: activation per layer ('tanh', 'elu', None);
    x: [in][B]. x_err (optional, broadcastable to x): the standard deviation
    of the inputs' own FP32 error where the kernel forms them itself.
    rel_scale (per output row, optional) divides the output differences.
    Returns the largest share over `trials` error draws."""
    rng = np.random.default_rng(seed)

    def forward(noise):
        h = rne_bf16(x + x_err * rng.standard_normal(x.shape) if (noise and x_err is not None) else x)
        for (W, b), kind in zip(layers, acts):
            Wb = rne_bf16(W)
            z = Wb @ h + b[:, None]
            if kind is not None and noise:
                s = 2.0 ** -24 * np.sqrt(W.shape[1]) * np.sqrt((Wb ** 2) @ (h ** 2))
                z = z + s * rng.standard_normal(z.shape)
            a = _act(kind, z)
            if kind is not None and noise:
                a = a + 2.0 ** -23 * rng.standard_normal(a.shape)
            h = rne_bf16(a) if kind is not None else a
        return h

    ref = forward(False)
    worst = 0.0
    for _ in range(trials):
        d = np.abs(forward(True) - ref)
        if rel_scale is not None:
            d = d / np.asarray(rel_scale)[:, None]
        worst = max(worst, float((d > thr).mean()))
    return worst


def allowed_count(share, m):
    """Outputs above the threshold allowed among m: twice the expected flip
    share plus four binomial standard deviations (at least one output)."""
    lam = 2.0 * share * m
    return lam + 4.0 * np.sqrt(max(lam, 1.0))
