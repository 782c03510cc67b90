"""The wave-team mapping of the solve (sg_set_team: four waves per 64-env
block share pass 1 of ABA) against the oracle and against the one-wave
mapping.

Tolerances: the team evaluates the same operations as the one-wave solve,
but in other waves whose code the compiler fuses into FMAs differently, so
the two mappings agree to FP32 rounding, not bit for bit. From the same
state one control step of each is within the hand-off bound of the oracle
(2e-5 (1 + |q|)), so they are compared within twice that; the observation
before the step, the policy outputs and the done bits are equal. Over many
steps rounding differences grow where trajectories hit the joint limits
(reading 20), so longer rollouts of the team mapping are replayed against
the oracle step by step exactly as the one-wave rollout is (test_gpu_rollout.py
and the variant tests, parametrized by mapping).
"""
import numpy as np
import pytest

import synth
from test_gpu_rollout import _replay_rollout

pytestmark = pytest.mark.gpu

_KEYS = ("obs", "act", "logp", "rew", "val", "adv", "ret")


def _mixed_path(n_env, seed=61):
    """Path task on chains of 4, 6 and 7 joints (per-joint guards in the
    solve), with the rollout policy."""
    w = synth.path_rollout(n_env, seed=seed)
    classes = np.array([4, 6, 7], dtype=np.int32)
    n_dof = classes[synth.stream(seed, "team_dof").integers(0, 3, size=n_env)]
    r = synth.make_chain(n_env, n_dof, seed, dt=1.0 / 120.0, substeps=4, max_dof=7, q0_frac=0.25)
    w.robot = synth._round_robot(r, np.float32)
    return w


def _workloads():
    return {
        "path_7dof": lambda: synth.path_rollout(1000),
        "mixed_4_6_7": lambda: _mixed_path(700),
        "prismatic_rrprrr": lambda: _with_policy(synth.psm_like(512), (22, 256, 128, 7)),
        "tracking": lambda: synth.tracking(512),
        "multi_arm_2": lambda: synth.multi_arm(256, 2),
        "path_rerand": lambda: synth.path_rerand(512),
    }


def _with_policy(w, dims):
    w.policy = synth.make_policy(w.seed + 7, dims=dims)
    return w


def _set_policy(w):
    if w.policy is None:
        w.policy = synth.make_policy(w.seed)
    return w


@pytest.mark.parametrize("name", list(_workloads()))
def test_team_step_matches_one_wave_step(sg, name):
    w = _set_policy(_workloads()[name]())
    out = {}
    for team in (1, 4):
        sim = sg.from_workload(w)
        sim.set_team(team)
        assert sim.get_team() == team
        b = sim.rollout(1)
        out[team] = {k: b[k].detach().cpu().numpy().astype(np.float64) for k in _KEYS} | \
            {"done": b["done"].cpu().numpy()}
        sim.close()
    a, b = out[1], out[4]
    assert np.array_equal(a["done"], b["done"]), name
    np.testing.assert_array_equal(a["obs"][0], b["obs"][0])
    for k in ("act", "logp"):
        np.testing.assert_array_equal(a[k], b[k])
    np.testing.assert_array_equal(a["val"][0], b["val"][0])
    # the value of the post-step state: a rounding-level difference of the
    # state can flip one BF16 activation (test_gpu_rollout.py's bound)
    assert np.abs(a["val"][1] - b["val"][1]).max() <= 2e-3, name
    # twice the one-step hand-off bounds of test_gpu_step.py: q 2e-5 (1 + |q|),
    # the rest of the observation 2e-3 max(1, |obs|), reward 2e-4
    J = w.robot.max_dof
    q1, q4 = a["obs"][1][:J], b["obs"][1][:J]
    assert (np.abs(q1 - q4) / (1.0 + np.abs(q1))).max() <= 4e-5, name
    assert np.abs(a["obs"][1] - b["obs"][1]).max() <= 4e-3 * max(1.0, np.abs(a["obs"][1]).max()), name
    assert np.abs(a["rew"] - b["rew"]).max() <= 4e-4, name


def test_team_rollout_replay_ragged(sg):
    # 300 envs: four full blocks and a partial one, two consecutive rollouts
    _replay_rollout(sg, synth.path_rollout(300), 24, n_rollouts=2, team=4)


def test_team_rollout_replay_mixed_dof(sg):
    """Chains of 4, 6 and 7 joints (the per-joint guards of the general
    kernel): the library's actions past an env's joint count are zero, the
    rest follow the policy; every step is replayed by the oracle from the
    stored observation."""
    import oracle
    from test_gpu_rollout import check_policy_outputs, host
    w = _mixed_path(200)
    T = 12
    sim = sg.from_workload(w)
    sim.set_team(4)
    o = oracle.Oracle(w.robot, w.task, w.policy)
    N, J = w.robot.n_env, w.robot.max_dof
    nd = np.asarray(w.robot.n_dof)
    live = np.arange(J)[:, None] < nd[None, :]
    sigma = np.exp(w.policy.log_std)
    prog = w.task.progress0.astype(np.int32).copy()
    b = sim.rollout(T)
    obs, act, rew = host(b["obs"]), host(b["act"]), host(b["rew"])
    done = b["done"].cpu().numpy()
    for t in range(T):
        mv = o.mlp(obs[t], emulate=True)
        eps = oracle.noise(w.seed, t, J, N)
        ref = mv[:J] + sigma[:, None] * eps
        check_policy_outputs(act[t][live], ref[live], w.policy)
        assert not act[t][~live].any()
        qn, qdn, prn, rw, dn, ob = o.step(act[t], obs[t][:J], obs[t][J:2 * J], prog)
        assert np.array_equal(done[t], dn), t
        assert np.abs(rew[t] - rw).max() <= 2e-4, t
        scale = np.maximum(1.0, np.abs(ob))
        assert (np.abs(obs[t + 1] - ob) / scale).max() <= 2e-3, t
        prog = prn
    sim.close()


def test_team_step_handoff_path(sg):
    from test_gpu_step import _run_handoff
    # 300 envs: a partial last block
    _run_handoff(sg, synth.path_rollout(300), 30, 5100, qtol=2e-5, tol_qdd=1e-4, team=4)


def test_team_step_handoff_mixed_dof(sg):
    from test_gpu_step import _run_handoff
    # 4/6/7/9 joints through the 9-joint general kernel
    _run_handoff(sg, synth.mixed_dof(333), 20, 5200, qtol=2e-5, tol_qdd=1e-4, team=4)


def test_team_step_matches_one_wave_step_at_16384(sg):
    """The 7-joint path step at the size the benchmark times: one step of
    each mapping from the same state, every env, within twice the hand-off
    bound (2e-5 (1 + |q|)); done and progress equal."""
    import torch
    from test_gpu_rollout import host
    w = synth.path_rollout(16384)
    a = torch.from_numpy(synth.random_actions(5300, 16384, 7, np.float32)).float().cuda()
    res = {}
    for team in (1, 4):
        sim = sg.from_workload(w)
        sim.set_team(team)
        o, r, d = sim.step(a)
        q, qd, pr, _ = sim.get_state()
        res[team] = (host(q), host(r), d.cpu().numpy(), pr.cpu().numpy())
        sim.close()
    (q1, r1, d1, p1), (q4, r4, d4, p4) = res[1], res[4]
    assert np.array_equal(d1, d4) and np.array_equal(p1, p4)
    assert (np.abs(q1 - q4) / (1.0 + np.abs(q1))).max() <= 4e-5
    assert np.abs(r1 - r4).max() <= 4e-4


@pytest.mark.parametrize("n_env", [1, 63, 65, 301])
def test_team_small_and_ragged_sizes(sg, n_env):
    """Sizes that exercise the staging's partial paths (N not a multiple of
    4, a partial last block, a single env): the team step and a short team
    rollout from the oracle's state, each checked against the oracle."""
    from test_gpu_step import _run_handoff
    w = synth.path_rollout(n_env)
    _run_handoff(sg, w, 6, 5400 + n_env, qtol=2e-5, tol_qdd=1e-4, team=4)
    _replay_rollout(sg, synth.path_rollout(n_env), 6, team=4)


def test_team_argument_checks(sg):
    w = synth.path_rollout(64)
    sim = sg.from_workload(w)
    assert sim.get_team() == 0  # the library's choice by default
    for bad in (-1, 2, 3, 8):
        with pytest.raises(RuntimeError):
            sim.set_team(bad)
    assert sim.get_team() == 0
    for ok in (1, 4, 0):
        sim.set_team(ok)
        assert sim.get_team() == ok
    sim.close()
    w64 = synth.reach_fp64(8)
    sim = sg.from_workload(w64)
    assert sim.get_team() == 0
    with pytest.raises(RuntimeError):
        sim.set_team(4)
    sim.set_team(1)
    sim.close()
