"""Multi-chain environments (paper Sec. IV multi-tool reaching) through the
HIP library against the FP64 oracle: the control step with state hand-off
(rewards summed over an env's chains by wavefront shuffles, shared
episodes), a non-finite chain forced from the host resetting its env, and
the fused rollout replayed step by step. Tolerances as in the step and
rollout tests."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("C,team", [(2, 1), (4, 1), (2, 4), (4, 4)])
def test_step_handoff(sg, C, team):
    import torch
    n_env = 160 // C * 2 + 1   # a partial last wave
    w = synth.multi_arm(n_env, C)
    N = n_env * C
    sim = sg.Sim(w.robot, w.task)
    sim.set_team(team)
    o = oracle.Oracle(w.robot, w.task)
    ended = 0
    for s in range(15):
        q0, qd0, pr0, _ = sim.get_state()
        a = synth.random_actions(800 + s, N, 7, np.float32)
        obs, rew, done = sim.step(torch.from_numpy(a.astype(np.float32)).cuda())
        q1, _, pr1, _ = sim.get_state()
        qn, qdn, prn, rw, dn, ob = o.step(a, host(q0), host(qd0), pr0.cpu().numpy())
        d = done.cpu().numpy()
        ended += int((d != 0).sum())
        assert np.array_equal(d, dn), s
        assert np.array_equal(pr1.cpu().numpy(), prn), s
        assert (np.abs(host(q1) - qn) / (1 + np.abs(qn))).max() <= 2e-5, s
        r = host(rew)
        assert np.abs(r - rw).max() <= 2e-4 * C, s
        assert np.array_equal(r.reshape(n_env, C), np.repeat(r.reshape(n_env, C)[:, :1], C, axis=1))
        assert (np.abs(host(obs) - ob) / np.maximum(1.0, np.abs(ob))).max() <= 2e-3, s
    assert ended > 0


def test_non_finite_chain_resets_its_env(sg):
    import torch
    n_env, C = 70, 2
    w = synth.multi_arm(n_env, C)
    sim = sg.Sim(w.robot, w.task)
    q, qd, pr, rs = sim.get_state()
    qd[3, 5] = float("nan")  # env 2, chain 1
    sim.set_state(q, qd, pr, rs)
    obs, rew, done = sim.step(torch.zeros(7, n_env * C, device="cuda"))
    d = done.cpu().numpy()
    assert d[4] == d[5] == 5
    assert rew[4].item() == rew[5].item() == 0.0
    assert (d[np.arange(n_env * C) // C != 2] & 4).sum() == 0
    q1 = host(sim.get_state()[0])
    np.testing.assert_array_equal(q1[:, 4:6], w.robot.q0[:, 4:6].astype(np.float32))


@pytest.mark.parametrize("team", [1, 4])
def test_rollout_replay(sg, team):
    from test_gpu_rollout import check_policy_outputs
    n_env, C, T = 100, 2, 12
    w = synth.multi_arm(n_env, C)
    w.task.progress0[:40] = 122
    N = n_env * C
    sim = sg.from_workload(w)
    sim.set_team(team)
    o = oracle.Oracle(w.robot, w.task, w.policy)
    b = sim.rollout(T)
    obs, act, rew = host(b["obs"]), host(b["act"]), host(b["rew"])
    done = b["done"].cpu().numpy()
    sigma = np.exp(w.policy.log_std)
    prog = w.task.progress0.astype(np.int32).copy()
    for t in range(T):
        mv = o.mlp(obs[t], emulate=True)
        check_policy_outputs(act[t], mv[:7] + sigma[:, None] * oracle.noise(w.seed, t, 7, N))
        qn, qdn, prn, rw, dn, ob = o.step(act[t], obs[t][:7], obs[t][7:14], prog)
        assert np.array_equal(done[t], dn), t
        assert np.abs(rew[t] - rw).max() <= 4e-4, t
        assert (np.abs(obs[t + 1] - ob) / np.maximum(1.0, np.abs(ob))).max() <= 2e-3, t
        prog = prn
    assert done.any()
    # GAE sees the env's shared reward on every chain
    r = rew.reshape(T, n_env, C)
    np.testing.assert_array_equal(r[..., 0], r[..., 1])


def test_invalid_groupings_rejected(sg):
    w = synth.multi_arm(10, 2)
    w.task.chains = 3
    with pytest.raises(sg.SgError):
        sg.Sim(w.robot, w.task)
    w = synth.multi_arm(10, 2)
    w.task.progress0[1] += 1   # the chains of env 0 disagree
    with pytest.raises(sg.SgError):
        sg.Sim(w.robot, w.task)
    w = synth.multi_arm(10, 2)
    sim = sg.Sim(w.robot, w.task)
    with pytest.raises(sg.SgError):
        sim.set_schedule(sg.SG_SCHED_SORTED)
