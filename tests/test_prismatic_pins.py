"""Prismatic joints (the P of the paper's RRPRRR arms) in the oracle: a
rotating telescoping arm in closed form, the RNEA/ABA round trip, ABA =
CRBA + Cholesky, and the brute-force Jacobian mass matrix."""
import numpy as np

import oracle
import pinlib
import synth

G = 9.81


def _telescope(n_env):
    """Joint 0 revolute about y at the origin, joint 1 prismatic along link
    0's z axis (no offset)."""
    r = synth.make_chain(n_env, 2, 5, dt=1 / 120, substeps=1, pattern="RP")
    r.axis[:] = 0.0
    r.axis[1, 0] = 1.0
    r.axis[2, 1] = 1.0
    r.offset[:] = 0.0
    return r


def test_telescoping_arm_closed_form():
    r = _telescope(7)
    o = oracle.Oracle(r)
    rng = np.random.default_rng(3)
    q = np.stack([rng.uniform(-3, 3, 7), rng.uniform(-0.1, 0.1, 7)])
    qd = rng.uniform(-2, 2, (2, 7))
    m1, m2 = r.mass
    c1, c2 = r.com[2]
    I1, I2 = r.inertia[1]
    rho = q[1] + c2
    M11 = I1 + m1 * c1 ** 2 + I2 + m2 * rho ** 2
    H = o.crba(q)
    np.testing.assert_allclose(H[:, 0, 0], M11, rtol=1e-13)
    np.testing.assert_allclose(H[:, 1, 1], m2, rtol=1e-14)
    np.testing.assert_allclose(H[:, 0, 1], 0.0, atol=1e-14)
    C1 = 2 * m2 * rho * qd[0] * qd[1]
    C2 = -m2 * rho * qd[0] ** 2
    G1 = -G * np.sin(q[0]) * (m1 * c1 + m2 * rho)
    G2 = G * m2 * np.cos(q[0])
    bias = o.rnea(q, qd, np.zeros_like(q))
    np.testing.assert_allclose(bias[0], C1 + G1, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(bias[1], C2 + G2, rtol=1e-12, atol=1e-12)
    tau = rng.normal(0, 5, (2, 7))
    qdd = o.aba(q, qd, tau)
    np.testing.assert_allclose(qdd[0], (tau[0] - C1 - G1) / M11, rtol=1e-11)
    np.testing.assert_allclose(qdd[1], (tau[1] - C2 - G2) / m2, rtol=1e-11)
    # the tip rides the prismatic joint: (L sin q0, 0, L cos q0), L = q1 + tip_z
    L = q[1] + r.tip[2]
    np.testing.assert_allclose(o.fk(q), np.stack([L * np.sin(q[0]), 0 * L, L * np.cos(q[0])]), atol=1e-14)


def test_psm_like_invariants():
    w = synth.psm_like(12, dtype=np.float64)
    o = oracle.Oracle(w.robot, w.task)
    q, qd = synth.random_states(9, w.robot)
    tau = np.random.default_rng(4).normal(0, 10, q.shape)
    arm = o.drive_armature()
    qdd = o.aba(q, qd, tau, arm)
    np.testing.assert_allclose(o.rnea(q, qd, qdd) + arm * qdd, tau, rtol=1e-10, atol=1e-10)
    alt, bad = o.fd_crba(q, qd, tau, arm)
    assert bad == 0
    np.testing.assert_allclose(qdd, alt, rtol=1e-9, atol=1e-9)
    H = o.crba(q)
    for e in range(12):
        links, tip, grav = pinlib.chain_of(w.robot, e)
        np.testing.assert_allclose(H[e], pinlib.mass_matrix(links, tip, q[:, e]), rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(o.rnea(q, qd, np.zeros_like(q))[:, e],
                                   pinlib.bias_fd(links, tip, q[:, e], qd[:, e], grav), rtol=1e-6, atol=1e-6)
        np.testing.assert_allclose(o.fk(q)[:, e], pinlib.fk(links, tip, q[:, e])[3], atol=1e-14)
