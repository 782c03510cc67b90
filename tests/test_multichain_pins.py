"""Pins of the oracle's multi-chain environments (paper Sec. IV multi-tool
reaching): with C chains per env, each chain moves exactly as a one-chain
reaching env with its own goal; the env reward is the sum of those rewards;
the episode is shared; a non-finite chain ends the episode of all its env's
chains with reward 0; the rollout shares rewards and dones across an env's
chains."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("C", [2, 4])
def test_group_step_equals_single_chains_with_summed_reward(C):
    n_env = 6
    w = synth.multi_arm(n_env, C, dtype=np.float64)
    N = n_env * C
    o = oracle.Oracle(w.robot, w.task)
    single = oracle.Oracle(w.robot, dataclasses.replace(w.task, chains=1))
    q, qd = synth.random_states(4, w.robot)
    pr = w.task.progress0.copy()
    pr[:] = np.repeat(np.arange(n_env) + 120, C)  # some envs time out within the run
    q1, qd1, p1 = q.copy(), qd.copy(), pr.copy()
    ended = 0
    for s in range(10):
        a = np.random.default_rng(s).uniform(-1, 1, (7, N))
        qg, qdg, pg, rg, dg, og = o.step(a, q, qd, pr)
        qs, qds, ps, rs, ds, os_ = single.step(a, q1, qd1, p1)
        np.testing.assert_array_equal(qg, qs)
        np.testing.assert_array_equal(qdg, qds)
        np.testing.assert_array_equal(dg, ds)
        np.testing.assert_array_equal(og, os_)
        ended += int(dg.sum())
        np.testing.assert_allclose(rg, np.repeat(rs.reshape(n_env, C).sum(1), C), rtol=1e-15)
        q, qd, pr = qg, qdg, pg
        q1, qd1, p1 = qs, qds, ps
    assert ended >= C  # an env's chains time out together inside the run


def test_non_finite_chain_resets_its_whole_env():
    n_env, C = 4, 2
    w = synth.multi_arm(n_env, C, dtype=np.float64)
    o = oracle.Oracle(w.robot, w.task)
    q, qd = synth.random_states(5, w.robot)
    qd[2, 3] = np.nan  # env 1, chain 1
    a = np.zeros((7, n_env * C))
    qn, qdn, pn, rew, done, obs = o.step(a, q, qd, w.task.progress0)
    assert done[2] == done[3] == 5 and not done[[0, 1, 4, 5, 6, 7]].any()
    assert rew[2] == rew[3] == 0.0
    np.testing.assert_array_equal(qn[:, 2:4], w.robot.q0[:, 2:4])
    assert pn[2] == pn[3] == 0


def test_rollout_shares_reward_and_done_within_an_env():
    n_env, C, T = 5, 2, 6
    w = synth.multi_arm(n_env, C, dtype=np.float64)
    w.task.progress0[:] = 125
    o = oracle.Oracle(w.robot, w.task, w.policy)
    N = n_env * C
    obs0 = o.observe(w.robot.q0, np.zeros((7, N)), w.task.progress0)
    r = o.rollout(T, w.seed, 0, w.robot.q0, np.zeros((7, N)), w.task.progress0, obs0)
    rew = r["rew"].reshape(T, n_env, C)
    np.testing.assert_array_equal(rew[..., 0], rew[..., 1])
    done = r["done"].reshape(T, n_env, C)
    np.testing.assert_array_equal(done[..., 0], done[..., 1])
    assert done[2].all()  # 125 + 3 = 128: the shared time-out
    # replaying the chains as separate one-chain envs with the rollout's own
    # actions reproduces the summed reward
    single = oracle.Oracle(w.robot, dataclasses.replace(w.task, chains=1))
    q, qd, pr = w.robot.q0.copy(), np.zeros((7, N)), w.task.progress0.copy()
    for t in range(T):
        q, qd, pr, rs, ds, _ = single.step(r["act"][t], q, qd, pr)
        np.testing.assert_allclose(r["rew"][t], np.repeat(rs.reshape(n_env, C).sum(1), C), rtol=1e-12)
