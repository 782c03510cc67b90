"""Pins of the oracle's per-episode re-randomisation (paper Sec. III: resets
start new trajectories; Sec. IV: targets and paths are sampled per task
instance): at a reset the env draws its next goal from Philox block 10 of
(env, step) -- reach: a target uniform in the box centre +- half per axis;
path: one of its host-prepared waypoint sets. Checked against the
known-answer-pinned Philox generator, the box bounds and moments, bank
frequencies, and the episode bookkeeping: the reward of the step that ends an
episode uses the old goal, the post-reset observation the new one, and envs
that do not reset keep theirs."""
import numpy as np

import oracle
import synth


def _words(seed, env, step):
    return oracle.philox4x32_10([env, step & 0xFFFFFFFF, step >> 32, 10], [seed & 0xFFFFFFFF, seed >> 32])


def _u24(x):
    return ((x >> 8) + 0.5) / 16777216.0


def _ending_step(w, n, step):
    """State one step before every env's time-out."""
    q, qd = w.robot.q0.copy(), np.zeros((7, n))
    pr = np.full(n, w.task.ep_len - 1, dtype=np.int32)
    return q, qd, pr


def test_reach_targets_redrawn_at_reset_from_block_10():
    n, step = 257, 41
    w = synth.reach_rerand(n, dtype=np.float64)
    o = oracle.Oracle(w.robot, w.task)
    gs = np.ascontiguousarray(w.task.target.copy())
    old = gs.copy()
    q, qd, pr = _ending_step(w, n, step)
    act = synth.random_actions(3, n, 7)
    q1, qd1, pr1, rew, done, obs = o.step(act, q, qd, pr, goal_state=gs, seed=w.seed, step=step)
    assert np.all(done == 3) and np.all(pr1 == 0)
    c, h = np.array(w.task.rerand["centre"]), w.task.rerand["half"]
    for e in range(n):
        x = _words(w.seed, e, step)
        want = c + h * (2.0 * np.array([_u24(x[k]) for k in range(3)]) - 1.0)
        np.testing.assert_allclose(gs[:, e], want, rtol=0, atol=1e-15)
    # the step's reward used the old target, the observation holds the new one
    ref_q, _, _, ref_rew, _, _ = oracle.Oracle(w.robot, _reach_fixed(w, old)).step(act, q, qd, pr)
    np.testing.assert_allclose(rew, ref_rew, rtol=0, atol=1e-15)
    np.testing.assert_allclose(obs[14 + 3:14 + 6], gs, rtol=0, atol=0)
    tip = obs[14:17]
    np.testing.assert_allclose(obs[14 + 6:14 + 9], gs - tip, rtol=0, atol=1e-15)


def _reach_fixed(w, target):
    import dataclasses
    return dataclasses.replace(w.task, target=target, rerand=None)


def test_reach_redraws_fill_the_box_uniformly():
    n = 4096
    w = synth.reach_rerand(n, dtype=np.float64)
    o = oracle.Oracle(w.robot, w.task)
    c, h = np.array(w.task.rerand["centre"]), w.task.rerand["half"]
    draws = []
    for step in (5, 77, 1000003):
        gs = np.ascontiguousarray(w.task.target.copy())
        q, qd, pr = _ending_step(w, n, step)
        o.step(np.zeros((7, n)), q, qd, pr, goal_state=gs, seed=w.seed, step=step)
        draws.append(gs.copy())
    d = (np.concatenate(draws, axis=1) - c[:, None]) / h   # uniform on [-1, 1]
    assert d.min() > -1 and d.max() < 1
    m = d.shape[1]
    assert np.all(np.abs(d.mean(axis=1)) < 4 * np.sqrt(1 / 3 / m))
    assert np.all(np.abs((d ** 2).mean(axis=1) - 1 / 3) < 4 * np.sqrt(4 / 45 / m))
    # independent draws at different steps
    assert np.abs(np.corrcoef(draws[0][0], draws[1][0])[0, 1]) < 0.06


def test_no_reset_keeps_the_goal():
    n = 64
    w = synth.reach_rerand(n, dtype=np.float64)
    o = oracle.Oracle(w.robot, w.task)
    gs = np.ascontiguousarray(w.task.target.copy())
    g0 = gs.copy()
    q, qd = w.robot.q0.copy(), np.zeros((7, n))
    pr = np.zeros(n, dtype=np.int32)
    _, _, _, rew, done, obs = o.step(np.zeros((7, n)), q, qd, pr, goal_state=gs, seed=w.seed, step=9)
    assert not done.any()
    np.testing.assert_array_equal(gs, g0)
    _, _, _, rew_f, _, obs_f = oracle.Oracle(w.robot, _reach_fixed(w, g0)).step(np.zeros((7, n)), q, qd, pr)
    np.testing.assert_array_equal(rew, rew_f)
    np.testing.assert_array_equal(obs, obs_f)


def test_path_bank_chosen_by_integer_draw_and_used_for_waypoints():
    n, step, B = 300, 1234, 4
    w = synth.path_rerand(n, banks=B, dtype=np.float64)
    o = oracle.Oracle(w.robot, w.task)
    gs = np.zeros((1, n))
    q, qd, pr = _ending_step(w, n, step)
    _, _, pr1, _, done, obs = o.step(np.zeros((7, n)), q, qd, pr, goal_state=gs, seed=w.seed, step=step)
    assert np.all(done == 3)
    K = w.task.n_waypoints
    for e in range(n):
        b = ((_words(w.seed, e, step)[0] >> 8) * B) >> 24
        assert gs[0, e] == b
        # progress 0 after the reset: the first waypoint of the new set
        np.testing.assert_array_equal(obs[17:20, e], w.task.waypoints[b * K, :, e])
    counts = np.bincount(gs[0].astype(int), minlength=B)
    assert counts.min() > n / B - 4 * np.sqrt(n / B)
    # later steps of the episode walk the new set's waypoints
    gsb = gs.copy()
    qs, qds, prs = q.copy(), qd.copy(), np.full(n, 16 * 3 - 1, dtype=np.int32)
    _, _, _, rew, _, obs = o.step(np.zeros((7, n)), qs, qds, prs, goal_state=gsb, seed=w.seed, step=step + 1)
    for e in range(0, n, 37):
        b = int(gs[0, e])
        np.testing.assert_array_equal(obs[17:20, e], w.task.waypoints[b * K + 3, :, e])
