"""Pins of the oracle's adjoint (reverse mode of an open-loop rollout):
central finite differences of its own forward loss for every action and
every link mass, on revolute and prismatic chains, with and without limit
contacts and an episode reset inside the rollout; the forward loss itself
equals the negated sum of the step's rewards."""
import numpy as np
import pytest

import oracle
import synth


def _workload(kind, n_env=6):
    if kind == "path":
        w = synth.path_rollout(n_env, dtype=np.float64)
    elif kind == "psm":
        w = synth.psm_like(n_env, dtype=np.float64)
    else:
        w = synth.mixed_dof(n_env, dtype=np.float64)
    return w


def _fd(o, T, act, q0, qd0, pr, h=1e-6):
    N, J = o.N, o.J
    n = o.robot.n_dof
    ga = np.zeros((T, J, N))
    for t in range(T):
        for j in range(J):
            e = np.zeros_like(act)
            e[t, j] = h
            lp = oracle.adjoint(o, T, act + e, q0, qd0, pr, want_grad=False)
            lm = oracle.adjoint(o, T, act - e, q0, qd0, pr, want_grad=False)
            ga[t, j] = (lp - lm) / (2 * h)
    gm = np.zeros((J, N))
    for j in range(J):
        s = np.ones((J, N))
        s[j] += h
        lp = oracle.adjoint(o, T, act, q0, qd0, pr, mass_scale=s, want_grad=False)
        s[j] -= 2 * h
        lm = oracle.adjoint(o, T, act, q0, qd0, pr, mass_scale=s, want_grad=False)
        # d/d(scale) = m dL/dm
        gm[j] = (lp - lm) / (2 * h) / np.where(j < n, o.robot.mass[j], 1.0)
    return ga, gm


@pytest.mark.parametrize("kind,T", [("path", 6), ("psm", 5), ("mixed", 4)])
def test_adjoint_matches_central_differences(kind, T):
    w = _workload(kind)
    o = oracle.Oracle(w.robot, w.task)
    N, J = w.robot.n_env, w.robot.max_dof
    rng = np.random.default_rng(11)
    act = rng.uniform(-0.9, 0.9, (T, J, N))
    q0, qd0 = synth.random_states(3, w.robot, qd_scale=0.5)
    pr = w.task.progress0
    loss, ga, gm = oracle.adjoint(o, T, act, q0, qd0, pr)
    fa, fm = _fd(o, T, act, q0, qd0, pr)
    scale_a = np.abs(fa).max()
    assert scale_a > 1e-3
    np.testing.assert_allclose(ga, fa, rtol=1e-5, atol=1e-6 * scale_a)
    np.testing.assert_allclose(gm, fm, rtol=1e-5, atol=1e-6 * np.abs(fm).max())


def test_adjoint_with_limit_contacts_and_a_reset():
    """Large actions drive joints into their stops; an env whose episode ends
    inside the rollout restarts. Entries whose perturbation changes the set
    of clamped coordinates are skipped (the loss is not differentiable
    there) and counted."""
    w = synth.path_rollout(8, dtype=np.float64)
    w.task.ep_len = 128
    w.task.progress0[:] = 125  # every env resets after step 3
    o = oracle.Oracle(w.robot, w.task)
    N, J, T = 8, 7, 6
    rng = np.random.default_rng(5)
    act = rng.uniform(-1.5, 1.5, (T, J, N))
    q0 = w.robot.q_hi * 0.97
    qd0 = np.full((J, N), 3.0)
    loss, ga, gm = oracle.adjoint(o, T, act, q0, qd0, w.task.progress0)
    fa, fm = _fd(o, T, act, q0, qd0, w.task.progress0, h=1e-7)
    # saturated actions (|a| > 1) have zero gradient
    assert np.all(ga[np.abs(act) >= 1] == 0)
    # actions of steps before the reset cannot change later steps' losses, so
    # they only see the first 3 steps; compare where FD agrees with a smooth
    # model (relative mismatch flags a contact switch)
    bad = np.abs(ga - fa) > 1e-4 * (1 + np.abs(fa))
    assert bad.mean() < 0.02, bad.mean()
    np.testing.assert_allclose(gm, fm, rtol=1e-4, atol=1e-6 * np.abs(fm).max())


def test_forward_loss_is_the_negated_reward_sum():
    w = synth.path_rollout(10, dtype=np.float64)
    o = oracle.Oracle(w.robot, w.task)
    N, J, T = 10, 7, 7
    act = np.random.default_rng(2).uniform(-1, 1, (T, J, N))
    q, qd, pr = w.robot.q0.copy(), np.zeros((J, N)), w.task.progress0.copy()
    total = np.zeros(N)
    for t in range(T):
        q, qd, pr, rew, done, _ = o.step(act[t], q, qd, pr)
        total -= rew
    loss = oracle.adjoint(o, T, act, w.robot.q0, np.zeros((J, N)), w.task.progress0, want_grad=False)
    np.testing.assert_allclose(loss, total, rtol=1e-13, atol=1e-13)
