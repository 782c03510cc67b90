"""Per-episode re-randomisation through the HIP library against the FP64
oracle: reach targets redrawn in their box and path waypoint sets picked from
each env's bank at every reset (Philox block 10 of (env, step)). The control
step with state and goal hand-off, and the fused rollout replayed step by
step across resets. Tolerances as in the tracking tests: the waypoint-set
index exactly, the reach target within 1e-6 m (FP32 rounding of the
centre + half (2u - 1) draw), rewards 2e-4, observations 2e-3 relative."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("kind,team", [("reach", 1), ("path", 1), ("reach", 4), ("path", 4)])
def test_step_handoff_with_redrawn_goals(sg, kind, team):
    import torch
    N = 300
    w = synth.reach_rerand(N) if kind == "reach" else synth.path_rerand(N)
    w.task.progress0[:60] = 122  # a fifth of the envs start a new episode inside the run
    sim = sg.Sim(w.robot, w.task, seed=w.seed)
    sim.set_team(team)
    o = oracle.Oracle(w.robot, w.task)
    resets = 0
    for s in range(12):
        q0, qd0, pr0, rs = sim.get_state()
        gs = np.ascontiguousarray(host(sim.get_goal_state()))
        a = synth.random_actions(700 + s, N, 7, np.float32)
        obs, rew, done = sim.step(torch.from_numpy(a.astype(np.float32)).cuda())
        q1, qd1, pr1, rs1 = sim.get_state()
        qn, qdn, prn, rw, dn, ob = o.step(a, host(q0), host(qd0), pr0.cpu().numpy(), goal_state=gs, seed=w.seed,
                                          step=rs)
        d = done.cpu().numpy()
        resets += int((d != 0).sum())
        assert np.array_equal(d, dn), s
        assert np.array_equal(pr1.cpu().numpy(), prn), s
        assert (np.abs(host(q1) - qn) / (1 + np.abs(qn))).max() <= 2e-5, s
        assert np.abs(host(rew) - rw).max() <= 2e-4, s
        g1 = host(sim.get_goal_state())
        if kind == "path":
            assert np.array_equal(g1, gs), s
        else:
            assert np.abs(g1 - gs).max() <= 1e-6, s
        assert (np.abs(host(obs) - ob) / np.maximum(1.0, np.abs(ob))).max() <= 2e-3, s
    assert resets >= 60
    g = host(sim.get_goal_state())
    if kind == "path":
        assert len(np.unique(g[0, :60])) > 1  # the resets picked different sets
    else:
        assert not np.allclose(g[:, :60], w.task.target[:, :60])


@pytest.mark.parametrize("kind,N,team", [("reach", 200, 1), ("path", 200, 1), ("path", 1024, 1), ("reach", 200, 4),
                                         ("path", 1024, 4)])
def test_rollout_replay_across_resets(sg, kind, N, team):
    from test_gpu_rollout import check_policy_outputs
    T = 16
    w = synth.reach_rerand(N) if kind == "reach" else synth.path_rerand(N)
    w.task.progress0[: N // 5] = 120
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
                                          step=t, threads=8)
        assert np.array_equal(done[t], dn), t
        assert np.abs(rew[t] - rw).max() <= 2e-4, t
        assert (np.abs(obs[t + 1] - ob) / np.maximum(1.0, np.abs(ob))).max() <= 2e-3, t
        prog = prn
    g = host(sim.get_goal_state())
    if kind == "path":
        assert np.array_equal(g, gs)
    else:
        assert np.abs(g - gs).max() <= 1e-6
    assert done.any()


def test_goal_state_reset_and_validation(sg):
    import torch
    w = synth.path_rerand(64)
    w.task.progress0[:] = 127
    sim = sg.Sim(w.robot, w.task, seed=w.seed)
    g0 = host(sim.get_goal_state())
    assert g0.shape == (1, 64) and not g0.any()
    sim.step(torch.zeros(7, 64, device="cuda"))
    assert host(sim.get_goal_state()).any()
    sim.reset()
    np.testing.assert_array_equal(host(sim.get_goal_state()), g0)
    # several waypoint sets without re-randomisation are rejected
    p = synth.path_rerand(8)
    p.task.rerand = None
    with pytest.raises(sg.SgError):
        sg.Sim(p.robot, p.task)
