"""Pins of the oracle's active-tracking task (paper Sec. IV): a noise-free
goal moves linearly and stops at its box wall with the outward velocity
dropped; the velocity increments and new-episode centres have the stated
Gaussian statistics; the reward uses the goal active during the step while
the observation carries the updated goal; the robot part of the step equals
the reaching task's with that goal."""
import dataclasses

import numpy as np

import oracle
import synth


def _track(n, **kw):
    w = synth.tracking(n, dtype=np.float64)
    w.task.track.update(kw)
    return w


def _gs0(w):
    tg = w.task.target
    return np.ascontiguousarray(np.concatenate([tg, np.zeros_like(tg), tg]))


def test_noise_free_goal_moves_linearly_and_stops_at_the_wall():
    w = _track(5, sigma=0.0)
    w.task.ep_len = 0
    o = oracle.Oracle(w.robot, w.task)
    gs = _gs0(w)
    v = np.array([[0.031], [-0.047], [0.071]]) * np.arange(1, 6)[None, :] / 5  # no step lands on a wall
    gs[3:6] = v
    q, qd, pr = w.robot.q0.copy(), np.zeros((7, 5)), w.task.progress0.copy()
    act = np.zeros((7, 5))
    c = w.task.target
    for k in range(1, 12):
        q, qd, pr, rew, done, obs = o.step(act, q, qd, pr, goal_state=gs, seed=w.seed, step=k)
        want = c + np.clip(k * v, -0.2, 0.2)
        np.testing.assert_allclose(gs[0:3], want, rtol=0, atol=1e-15)
        hit = np.abs(k * v) > 0.2
        np.testing.assert_array_equal(gs[3:6], np.where(hit, 0.0, v))
        np.testing.assert_array_equal(gs[6:9], c)
        np.testing.assert_array_equal(obs[2 * 7 + 3:2 * 7 + 6], gs[0:3])


def test_velocity_increments_and_new_centres_have_the_stated_statistics():
    n = 20000
    w = _track(n, sigma=1e-4, reset_std=0.05)
    w.task.progress0[:] = 126  # every env ends its episode at the second step
    o = oracle.Oracle(w.robot, w.task)
    gs = _gs0(w)
    q, qd, pr = w.robot.q0.copy(), np.zeros((7, n)), w.task.progress0.copy()
    act = np.zeros((7, n))
    q, qd, pr, _, done, _ = o.step(act, q, qd, pr, goal_state=gs, seed=w.seed, step=0, threads=8)
    assert not done.any()
    inc = gs[3:6].ravel() / 1e-4
    assert abs(inc.mean()) < 5 / np.sqrt(inc.size)
    assert abs(inc.std() - 1) < 5 / np.sqrt(2 * inc.size)
    # the x, y, z increments are independent
    cc = np.corrcoef(gs[3:6])
    assert np.abs(cc - np.eye(3)).max() < 5 / np.sqrt(n)
    q, qd, pr, _, done, _ = o.step(act, q, qd, pr, goal_state=gs, seed=w.seed, step=1, threads=8)
    assert done.all()
    cen = (gs[6:9] - np.asarray(synth.WORK_CENTRE)[:, None]) / 0.05
    assert np.abs(cen.mean(axis=1)).max() < 5 / np.sqrt(n)
    assert np.abs(cen.std(axis=1) - 1).max() < 5 / np.sqrt(2 * n)
    np.testing.assert_array_equal(gs[0:3], gs[6:9])
    np.testing.assert_array_equal(gs[3:6], 0.0)
    # different steps and envs draw different numbers; the same counter the same
    gs2 = _gs0(w)
    o.step(act, w.robot.q0, np.zeros((7, n)), w.task.progress0, goal_state=gs2, seed=w.seed, step=0, threads=8)
    gs3 = _gs0(w)
    o.step(act, w.robot.q0, np.zeros((7, n)), w.task.progress0, goal_state=gs3, seed=w.seed, step=0, threads=8)
    np.testing.assert_array_equal(gs2, gs3)
    gs4 = _gs0(w)
    o.step(act, w.robot.q0, np.zeros((7, n)), w.task.progress0, goal_state=gs4, seed=w.seed, step=7, threads=8)
    assert not np.any(gs4[3:6] == gs2[3:6])


def test_reward_uses_the_step_goal_and_robot_matches_reaching():
    n = 64
    w = _track(n)
    o = oracle.Oracle(w.robot, w.task)
    gs = _gs0(w)
    gs[3:6] = np.random.default_rng(1).normal(0, 1e-3, (3, n))
    g_before = gs[0:3].copy()
    reach = dataclasses.replace(w.task, task=synth.TASK_REACH, target=g_before.copy(), track=None)
    orr = oracle.Oracle(w.robot, reach)
    q0, qd0 = synth.random_states(2, w.robot)
    act = np.random.default_rng(3).uniform(-1, 1, (7, n))
    pr0 = w.task.progress0.copy()
    q1, qd1, pr1, rew, done, obs = o.step(act, q0, qd0, pr0, goal_state=gs, seed=w.seed, step=3)
    r1, rd1, rp1, rrew, rdone, robs = orr.step(act, q0, qd0, pr0)
    np.testing.assert_array_equal(q1, r1)
    np.testing.assert_array_equal(qd1, rd1)
    np.testing.assert_array_equal(done, rdone)
    np.testing.assert_array_equal(rew, rrew)   # reward against g_t
    ok = done == 0
    np.testing.assert_array_equal(obs[17:20][:, ok], gs[0:3][:, ok])   # obs carries g_{t+1}
    assert np.all(gs[0:3][:, ok] != g_before[:, ok])
