"""Chains with prismatic joints (the RRPRRR joint sequence of the paper's
PSM/ECM arms) through the HIP library: forward and inverse dynamics, tip
kinematics, the control step with state hand-off, and the fused rollout,
against the FP64 oracle. Tolerances are those of the revolute step and
rollout tests."""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_step import _run_handoff, dev, host, rel_qdd_err

pytestmark = pytest.mark.gpu


def _telescope(n_env, dtype):
    """J = 2 (joint 0 revolute about y, joint 1 prismatic along z): runs in a
    kernel sized for more joints than the context has."""
    r = synth.make_chain(n_env, 2, 21, dt=1 / 120, substeps=2, pattern="RP")
    r.axis[:] = 0.0
    r.axis[1, 0] = 1.0
    r.axis[2, 1] = 1.0
    w = synth.psm_like(n_env, dtype=dtype)
    w.robot = synth._round_robot(r, dtype)
    return w


@pytest.mark.parametrize("name,dtype,n_env", [("psm", np.float64, 64), ("psm", np.float32, 300),
                                              ("telescope", np.float64, 65), ("psm", np.float32, 1)])
def test_dynamics_and_tip(sg, name, dtype, n_env):
    import torch
    w = synth.psm_like(n_env, dtype=dtype) if name == "psm" else _telescope(n_env, dtype)
    td = torch.float64 if dtype == np.float64 else torch.float32
    sim = sg.Sim(w.robot, w.task, dtype=dtype)
    o = oracle.Oracle(w.robot, w.task)
    q, qd = synth.random_states(13, w.robot, dtype=dtype)
    tau = synth._as_dtype(np.random.default_rng(5).normal(0, 10, q.shape), dtype)
    tol = 1e-10 if dtype == np.float64 else 1e-4
    g = host(sim.forward_dynamics(dev(q, torch, td), dev(qd, torch, td), dev(tau, torch, td), sg.SG_ARM_DRIVE))
    ref = o.aba(q, qd, tau, o.drive_armature())
    assert rel_qdd_err(g, ref) <= tol, rel_qdd_err(g, ref)
    qdd = synth._as_dtype(np.random.default_rng(6).normal(0, 5, q.shape), dtype)
    g = host(sim.inverse_dynamics(dev(q, torch, td), dev(qd, torch, td), dev(qdd, torch, td)))
    ref = o.rnea(q, qd, qdd)
    scale = np.maximum(np.abs(ref).max(axis=0), 1.0)
    assert (np.abs(g - ref) / scale).max() <= (1e-11 if dtype == np.float64 else 2e-5)
    tip = host(sim.tip_position(dev(q, torch, td)))
    assert np.abs(tip - o.fk(q)).max() <= (1e-13 if dtype == np.float64 else 2e-6)
    sim.synchronize()


def test_step_handoff_fp64(sg):
    _run_handoff(sg, synth.psm_like(64, dtype=np.float64), 40, 4100, qtol=1e-11, tol_qdd=1e-10)


@pytest.mark.parametrize("team", [1, 4])
def test_step_handoff_fp32(sg, team):
    _run_handoff(sg, synth.psm_like(300), 30, 4200, qtol=2e-5, tol_qdd=1e-4, team=team)


def test_prismatic_contexts_keep_padded_schedule_and_refuse_surrogate(sg):
    w = synth.psm_like(128)
    sim = sg.Sim(w.robot, w.task)
    with pytest.raises(sg.SgError):
        sim.set_schedule(sg.SG_SCHED_SORTED)
    assert sim.get_schedule() == sg.SG_SCHED_PADDED
    with pytest.raises(sg.SgError):
        sg.Surrogate(sim, 256)


@pytest.mark.parametrize("team", [1, 4])
def test_rollout_replay(sg, team):
    from test_gpu_rollout import check_policy_outputs
    w = synth.psm_like(200)
    w.policy = synth.make_policy(77, dims=(22, 256, 128, 7))
    sim = sg.from_workload(w)
    sim.set_team(team)
    o = oracle.Oracle(w.robot, w.task, w.policy)
    N, J, T = w.robot.n_env, w.robot.max_dof, 12
    sigma = np.exp(w.policy.log_std)
    prog = w.task.progress0.astype(np.int32).copy()
    b = sim.rollout(T)
    obs, act, rew = host(b["obs"]), host(b["act"]), host(b["rew"])
    done = b["done"].cpu().numpy()
    for t in range(T):
        mv = o.mlp(obs[t], emulate=True)
        eps = oracle.noise(w.seed, t, J, N)
        check_policy_outputs(act[t], mv[:J] + sigma[:, None] * eps)
        qn, qdn, prn, rw, dn, ob = o.step(act[t], obs[t][:J], obs[t][J:2 * J], prog)
        assert np.array_equal(done[t], dn), t
        assert np.abs(rew[t] - rw).max() <= 2e-4, t
        scale = np.maximum(1.0, np.abs(ob))
        assert (np.abs(obs[t + 1] - ob) / scale).max() <= 2e-3, t
        prog = prn
    sim.synchronize()
