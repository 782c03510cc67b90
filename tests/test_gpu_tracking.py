"""Active tracking (moving goal) through the HIP library against the FP64
oracle: the control step with state and goal hand-off, and the fused
rollout replayed step by step. Tolerances as in the step and rollout
tests; the goal state (positions ~0.5 m, velocity increments 1e-4 m) within
1e-6 m."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("team", [1, 4])
def test_step_handoff_with_goal_state(sg, team):
    import torch
    N = 300
    w = synth.tracking(N)
    w.task.progress0[:60] = 122  # a fifth of the envs start a new episode inside the run
    sim = sg.Sim(w.robot, w.task, seed=w.seed)
    sim.set_team(team)
    o = oracle.Oracle(w.robot, w.task)
    resets = 0
    for s in range(12):
        q0, qd0, pr0, rs = sim.get_state()
        gs = np.ascontiguousarray(host(sim.get_goal_state()))
        a = synth.random_actions(500 + s, N, 7, np.float32)
        obs, rew, done = sim.step(torch.from_numpy(a.astype(np.float32)).cuda())
        q1, qd1, pr1, rs1 = sim.get_state()
        assert rs1 == rs + 1
        qn, qdn, prn, rw, dn, ob = o.step(a, host(q0), host(qd0), pr0.cpu().numpy(), goal_state=gs, seed=w.seed,
                                          step=rs)
        d = done.cpu().numpy()
        resets += int((d != 0).sum())
        assert np.array_equal(d, dn), s
        assert np.array_equal(pr1.cpu().numpy(), prn), s
        assert (np.abs(host(q1) - qn) / (1 + np.abs(qn))).max() <= 2e-5, s
        assert np.abs(host(rew) - rw).max() <= 2e-4, s
        assert np.abs(host(sim.get_goal_state()) - gs).max() <= 1e-6, s
        assert (np.abs(host(obs) - ob) / np.maximum(1.0, np.abs(ob))).max() <= 2e-3, s
    assert resets >= 60


@pytest.mark.parametrize("team", [1, 4])
def test_rollout_replay_with_moving_goal(sg, team):
    from test_gpu_rollout import check_policy_outputs
    N, T = 200, 16
    w = synth.tracking(N)
    w.task.progress0[:40] = 120
    sim = sg.from_workload(w)
    sim.set_team(team)
    o = oracle.Oracle(w.robot, w.task, w.policy)
    gs = np.ascontiguousarray(host(sim.get_goal_state()))
    b = sim.rollout(T)
    obs, act, rew = host(b["obs"]), host(b["act"]), host(b["rew"])
    done = b["done"].cpu().numpy()
    sigma = np.exp(w.policy.log_std)
    prog = w.task.progress0.astype(np.int32).copy()
    for t in range(T):
        mv = o.mlp(obs[t], emulate=True)
        check_policy_outputs(act[t], mv[:7] + sigma[:, None] * oracle.noise(w.seed, t, 7, N))
        qn, qdn, prn, rw, dn, ob = o.step(act[t], obs[t][:7], obs[t][7:14], prog, goal_state=gs, seed=w.seed,
                                          step=t)
        assert np.array_equal(done[t], dn), t
        assert np.abs(rew[t] - rw).max() <= 2e-4, t
        assert (np.abs(obs[t + 1] - ob) / np.maximum(1.0, np.abs(ob))).max() <= 2e-3, t
        prog = prn
    assert np.abs(host(sim.get_goal_state()) - gs).max() <= 1e-6
    assert done.any()


def test_goal_state_api_and_reset(sg):
    import torch
    w = synth.tracking(64)
    sim = sg.Sim(w.robot, w.task, seed=w.seed)
    g0 = host(sim.get_goal_state())
    np.testing.assert_allclose(g0[0:3], w.task.target, atol=0)
    np.testing.assert_allclose(g0[6:9], w.task.target, atol=0)
    assert not g0[3:6].any()
    for _ in range(3):
        sim.step(torch.zeros(7, 64, device="cuda"))
    assert not np.array_equal(host(sim.get_goal_state()), g0)
    sim.reset()
    np.testing.assert_array_equal(host(sim.get_goal_state()), g0)
    custom = torch.from_numpy(g0.astype(np.float32) + 0.01).cuda()
    sim.set_goal_state(custom)
    np.testing.assert_array_equal(host(sim.get_goal_state()), host(custom))
    # other tasks have no goal state; the adjoint does not take a moving goal
    p = synth.path_rollout(8)
    sp = sg.Sim(p.robot, p.task)
    with pytest.raises(sg.SgError):
        sp.get_goal_state()
    with pytest.raises(sg.SgError):
        sim.adjoint(torch.zeros(2, 7, 64, device="cuda"), 1)
