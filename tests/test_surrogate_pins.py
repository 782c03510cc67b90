"""Pins of the oracle's learned-surrogate pieces: features against their
definition, the network against a numpy forward pass, gradients against
central finite differences, Adam against its closed-form first step, the
residual check against the mass matrix."""
import numpy as np

import oracle
import synth


def _small_net(seed, dims):
    rng = np.random.default_rng(seed)
    W = [rng.uniform(-1, 1, (dims[l + 1], dims[l])) / np.sqrt(dims[l]) for l in range(len(dims) - 1)]
    b = [rng.uniform(-0.2, 0.2, dims[l + 1]) for l in range(len(dims) - 1)]
    norm = (rng.normal(0, 1, dims[0]), rng.uniform(0.5, 2, dims[0]), rng.normal(0, 1, dims[-1]),
            rng.uniform(0.5, 2, dims[-1]))
    return W, b, norm


def _np_forward(W, b, norm, x_raw):
    h = (x_raw - norm[0][:, None]) / norm[1][:, None]
    for l in range(len(W)):
        z = W[l] @ h + b[l][:, None]
        h = z if l == len(W) - 1 else np.where(z > 0, z, np.expm1(z))
    return h * norm[3][:, None] + norm[2][:, None], h


def test_features_are_the_standard_inertial_parameters():
    w = synth.mixed_dof(16)
    o = oracle.Oracle(w.robot, w.task)
    q, qd = synth.random_states(3, w.robot)
    tau = synth.surrogate_torques(4, 16, 9)
    env = np.arange(16)[::-1].copy()
    x = oracle.surrogate_features(o, q[:, env], qd[:, env], tau, env)
    r = w.robot
    J = 9
    for s, e in enumerate(env):
        n = r.n_dof[e]
        for j in range(J):
            blk = x[3 * J + 10 * j:3 * J + 10 * j + 10, s]
            if j >= n:
                assert np.all(blk == 0) and x[j, s] == 0
                continue
            m, c = r.mass[j, e], r.com[:, j, e]
            Ic = np.diag(r.inertia[:3, j, e])
            Ic[0, 1] = Ic[1, 0] = r.inertia[3, j, e]
            Ic[0, 2] = Ic[2, 0] = r.inertia[4, j, e]
            Ic[1, 2] = Ic[2, 1] = r.inertia[5, j, e]
            IO = Ic + m * (c @ c * np.eye(3) - np.outer(c, c))  # parallel-axis theorem
            ref = [m, *(m * c), IO[0, 0], IO[1, 1], IO[2, 2], IO[0, 1], IO[0, 2], IO[1, 2]]
            np.testing.assert_allclose(blk, ref, rtol=1e-14, atol=1e-16)
            assert x[j, s] == q[j, e] and x[J + j, s] == qd[j, e] and x[2 * J + j, s] == tau[j, s]


def test_forward_matches_numpy():
    dims = (13, 9, 8, 5)
    W, b, norm = _small_net(1, dims)
    s = oracle.SurrogateRef(W, b, norm)
    x = np.random.default_rng(2).normal(0, 2, (13, 40))
    out, outn = s.forward(x)
    ref, refn = _np_forward(W, b, norm, x)
    np.testing.assert_allclose(out, ref, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(outn, refn, rtol=1e-13, atol=1e-13)


def test_gradients_match_central_differences():
    dims = (7, 6, 5, 3)
    W, b, norm = _small_net(3, dims)
    rng = np.random.default_rng(4)
    x = rng.normal(0, 1.5, (7, 11))
    t = rng.normal(0, 1, (3, 11))

    def loss(W, b):
        return oracle.SurrogateRef(W, b, norm).grad(x, t)[0]

    L0, gW, gb = oracle.SurrogateRef(W, b, norm).grad(x, t)
    # the loss itself is the mean squared normalised error
    _, yn = _np_forward(W, b, norm, x)
    tn = (t - norm[2][:, None]) / norm[3][:, None]
    np.testing.assert_allclose(L0, ((yn - tn) ** 2).mean(), rtol=1e-13)
    h = 1e-6
    for l in range(len(W)):
        for idx in [(0, 0), (W[l].shape[0] - 1, W[l].shape[1] - 1), (1, 2)]:
            Wp = [w.copy() for w in W]
            Wm = [w.copy() for w in W]
            Wp[l][idx] += h
            Wm[l][idx] -= h
            fd = (loss(Wp, b) - loss(Wm, b)) / (2 * h)
            assert abs(fd - gW[l][idx]) <= 1e-7 * max(1.0, abs(fd)), (l, idx, fd, gW[l][idx])
        for i in range(b[l].size):
            bp = [x_.copy() for x_ in b]
            bm = [x_.copy() for x_ in b]
            bp[l][i] += h
            bm[l][i] -= h
            fd = (loss(W, bp) - loss(W, bm)) / (2 * h)
            assert abs(fd - gb[l][i]) <= 1e-7 * max(1.0, abs(fd))


def test_adam_first_step_and_moments():
    rng = np.random.default_rng(5)
    w0 = rng.normal(0, 1, 50)
    g = rng.normal(0, 1, 50)
    lr, eps = 1e-3, 1e-8
    w1, m1, v1 = oracle.adam(w0, g, np.zeros(50), np.zeros(50), lr, 1, eps=eps)
    # bias-corrected first step: m_hat = g, v_hat = g^2
    np.testing.assert_allclose(w1, w0 - lr * g / (np.abs(g) + eps), rtol=1e-14)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-14)
    # constant gradient: m_hat stays g, v_hat stays g^2 at any step
    w, m, v = w0, np.zeros(50), np.zeros(50)
    for t in range(1, 20):
        w, m, v = oracle.adam(w, g, m, v, lr, t, eps=0.0)
    np.testing.assert_allclose(w, w0 - 19 * lr * np.sign(g), rtol=1e-12)


def test_residual_is_zero_for_the_exact_solve_and_scales_with_H():
    w = synth.path_rollout(20, dtype=np.float64)
    o = oracle.Oracle(w.robot, w.task)
    q, qd = synth.random_states(6, w.robot)
    tau = synth.surrogate_torques(7, 20, 7)
    arm = o.drive_armature()
    qdd = o.aba(q, qd, tau, arm)
    assert oracle.residual(o, q, qd, tau, qdd, arm).max() < 1e-12
    dq = np.random.default_rng(8).normal(0, 0.1, qdd.shape)
    rel = oracle.residual(o, q, qd, tau, qdd + dq, arm)
    H = o.crba(q)
    for e in range(20):
        r = (H[e] + np.diag(arm[:, e])) @ dq[:, e]
        np.testing.assert_allclose(rel[e], np.linalg.norm(r) / np.linalg.norm(tau[:, e]), rtol=1e-9)


def test_elu_hidden_units_and_linear_output():
    # one hidden unit with identity weights: output = elu(x) through a
    # linear last layer, normalisation switched off
    W = [np.array([[1.0]]), np.array([[1.0]])]
    b = [np.array([0.0]), np.array([0.0])]
    norm = (np.zeros(1), np.ones(1), np.zeros(1), np.ones(1))
    s = oracle.SurrogateRef(W, b, norm)
    x = np.array([[-3.0, -0.5, 0.0, 0.25, 2.0]])
    out, _ = s.forward(x)
    np.testing.assert_allclose(out[0], [np.exp(-3) - 1, np.exp(-0.5) - 1, 0.0, 0.25, 2.0], rtol=1e-15)
