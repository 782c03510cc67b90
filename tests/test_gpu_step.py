"""Parity of the HIP environment step against the FP64 oracle.

Tolerances (FP32 ones derived from the arithmetic; FP64 ones from rounding
accumulation over one control step):
* joint accelerations, per substep with state hand-off:
  ||qdd_gpu - qdd_ora||_2 / max(||qdd_ora||_2, 1 rad/s^2) <= 1e-4 (FP32),
  <= 1e-10 (FP64);
* one control step with hand-off: |dq| <= 1e-5 (1 + |q|) rad in FP32;
* 1000-step free run of the 64-env FP64 workload: max |dq| <= 1e-9 rad;
  the same in FP32: max |dq| <= 1e-3 rad and max |d tip| <= 1e-3 m; both
  over the envs whose oracle trajectory is numerically unique (it moves by
  less than a tenth of the bound when the oracle's own start is perturbed at
  the precision's rounding level; limit contacts make the rest sensitive).
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def dev(a, torch, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel_qdd_err(g, o):
    num = np.linalg.norm(g - o, axis=0)
    den = np.maximum(np.linalg.norm(o, axis=0), 1.0)
    return (num / den).max()


@pytest.mark.parametrize("name,n_env", [("reach_fp64", 64), ("path_fp32", 300), ("mixed_fp32", 257),
                                        ("path_fp32", 1)])
def test_forward_inverse_dynamics_and_tip(sg, name, n_env):
    import torch
    if name == "reach_fp64":
        w = synth.reach_fp64(n_env)
    elif name == "path_fp32":
        w = synth.path_rollout(n_env)
    else:
        w = synth.mixed_dof(n_env)
    td = torch.float64 if w.dtype == np.float64 else torch.float32
    sim = sg.Sim(w.robot, w.task, dtype=w.dtype)
    o = oracle.Oracle(w.robot, w.task)
    q, qd = synth.random_states(11, w.robot, dtype=w.dtype)
    tau = synth._as_dtype(np.random.default_rng(1).normal(0, 10, q.shape), w.dtype)
    tau[np.arange(w.robot.max_dof)[:, None] >= w.robot.n_dof[None, :]] = 0
    tol = 1e-10 if w.dtype == np.float64 else 1e-4
    eps = np.finfo(w.dtype).eps
    for mode, arm in ((sg.SG_ARM_NONE, None), (sg.SG_ARM_DRIVE, o.drive_armature())):
        g = host(sim.forward_dynamics(dev(q, torch, td), dev(qd, torch, td), dev(tau, torch, td), mode))
        ref = o.aba(q, qd, tau, arm)
        if mode == sg.SG_ARM_DRIVE:
            # the gated quantity: the implicit-PD step's solve
            assert rel_qdd_err(g, ref) <= tol, (mode, rel_qdd_err(g, ref))
        else:
            # plain forward dynamics: the error scales with the condition
            # number of H, reported separately from the gate
            H = o.crba(q)
            kappa = np.array([np.linalg.cond(H[e, :n, :n]) for e, n in enumerate(w.robot.n_dof)])
            num = np.linalg.norm(g - ref, axis=0)
            den = np.maximum(np.linalg.norm(ref, axis=0), 1.0)
            assert np.all(num / den <= tol + 20 * kappa * eps), (num / den / kappa).max()
    qdd = synth._as_dtype(np.random.default_rng(2).normal(0, 5, q.shape), w.dtype)
    g = host(sim.inverse_dynamics(dev(q, torch, td), dev(qd, torch, td), dev(qdd, torch, td)))
    ref = o.rnea(q, qd, qdd)
    scale = np.maximum(np.abs(ref).max(axis=0), 1.0)
    assert (np.abs(g - ref) / scale).max() <= (1e-11 if w.dtype == np.float64 else 2e-5)
    tip = host(sim.tip_position(dev(q, torch, td)))
    assert np.abs(tip - o.fk(q)).max() <= (1e-13 if w.dtype == np.float64 else 2e-6)
    sim.synchronize()


def _run_handoff(sg, w, steps, act_seed, qtol, tol_qdd, team=1):
    import torch
    td = torch.float64 if w.dtype == np.float64 else torch.float32
    sim = sg.Sim(w.robot, w.task, dtype=w.dtype)
    sim.set_team(team)
    o = oracle.Oracle(w.robot, w.task)
    J, N = w.robot.max_dof, w.robot.n_env
    worst = 0.0
    for s in range(steps):
        q0, qd0, pr0, _ = sim.get_state()
        a = synth.random_actions(act_seed + s, N, J, dtype=w.dtype)
        obs, rew, done = sim.step(dev(a, torch, td))
        q1, qd1, pr1, _ = sim.get_state()
        qn, qdn, prn, rw, dn, ob = o.step(a, host(q0), host(qd0), host(pr0).astype(np.int32))
        assert np.array_equal(host(done).astype(np.uint8), dn), s
        assert np.array_equal(host(pr1).astype(np.int32), prn), s
        dq = np.abs(host(q1) - qn) / (1 + np.abs(qn))
        worst = max(worst, dq.max())
        assert dq.max() <= qtol, (s, dq.max())
        assert np.abs(host(qd1) - qdn).max() <= qtol * 100 * max(1.0, np.abs(qdn).max()), s
        assert np.abs(host(rew) - rw).max() <= qtol * 10, s
        assert np.abs(host(obs) - ob).max() <= qtol * 100 * max(1.0, np.abs(ob).max()), s
        if s % 7 == 0:
            # per-substep accelerations of the first substep at this state
            h = w.robot.dt / w.robot.substeps
            qs = a.clip(-1, 1) * w.robot.q_hi
            tau = w.robot.kp * (qs - host(q0) - h * host(qd0)) - w.robot.kd * host(qd0)
            tau = synth._as_dtype(tau, w.dtype)
            g = host(sim.forward_dynamics(q0, qd0, dev(tau, torch, td), sg.SG_ARM_DRIVE))
            ref = o.aba(host(q0), host(qd0), tau, o.drive_armature())
            assert rel_qdd_err(g, ref) <= tol_qdd, (s, rel_qdd_err(g, ref))
    sim.synchronize()
    return worst


def test_step_handoff_fp64(sg):
    w = synth.reach_fp64(64)
    _run_handoff(sg, w, 60, 900, qtol=1e-11, tol_qdd=1e-10)


def test_step_handoff_fp32_path(sg):
    w = synth.path_rollout(300)
    _run_handoff(sg, w, 40, 1900, qtol=2e-5, tol_qdd=1e-4)


def test_step_handoff_fp32_mixed_dof(sg):
    w = synth.mixed_dof(333)
    _run_handoff(sg, w, 20, 2900, qtol=2e-5, tol_qdd=1e-4)


def _free_run(sg, w, steps, dtype, perturb):
    """Actions resampled every 50 steps, both sides integrate on their own.
    The oracle also runs from q0 + perturb: envs whose oracle trajectory moves
    by more than the checked bound under that perturbation (limit contacts
    make some trajectories sensitive) have no numerically unique answer and
    are reported, not compared."""
    import torch
    td = torch.float64 if dtype == np.float64 else torch.float32
    rob = synth._round_robot(w.robot, dtype)
    tsk = synth._round_task(w.task, dtype)
    sim = sg.Sim(rob, tsk, dtype=dtype)
    o = oracle.Oracle(rob, tsk)
    J, N = rob.max_dof, rob.n_env
    q, qd, pr = rob.q0.copy(), np.zeros((J, N)), tsk.progress0.copy()
    qp, qdp, prp = rob.q0 + perturb, np.zeros((J, N)), tsk.progress0.copy()
    for s in range(steps):
        if s % 50 == 0:
            a = synth.random_actions(5000 + s // 50, N, J, dtype=dtype)
            at = dev(a, torch, td)
        sim.step(at)
        q, qd, pr = o.step(a, q, qd, pr)[:3]
        qp, qdp, prp = o.step(a, qp, qdp, prp)[:3]
    qg = host(sim.get_state()[0])
    tip_g = host(sim.tip_position(sim.get_state()[0]))
    sim.synchronize()
    sens = np.abs(qp - q).max(0)
    return qg, q, tip_g, o.fk(q), sens


def test_free_run_1000_steps_fp64(sg):
    w = synth.reach_fp64(64)
    qg, qo, tg, to, sens = _free_run(sg, w, 1000, np.float64, 1e-13)
    ok = sens <= 1e-10
    print(f"fp64 free run: {ok.sum()}/64 envs with a unique trajectory")
    assert ok.sum() >= 48
    assert np.abs(qg - qo)[:, ok].max() <= 1e-9
    assert np.abs(tg - to)[:, ok].max() <= 1e-9


def test_free_run_1000_steps_fp32_drift(sg):
    w = synth.reach_fp64(64)
    qg, qo, tg, to, sens = _free_run(sg, w, 1000, np.float32, 1e-6)
    ok = sens <= 1e-4
    print(f"fp32 free run: {ok.sum()}/64 envs with a unique trajectory at FP32 resolution")
    assert ok.sum() >= 32
    assert np.abs(qg - qo)[:, ok].max() <= 1e-3
    assert np.abs(tg - to)[:, ok].max() <= 1e-3


def test_observe_reset_and_state_roundtrip(sg):
    import torch
    w = synth.path_rollout(100)
    sim = sg.Sim(w.robot, w.task)
    o = oracle.Oracle(w.robot, w.task)
    obs = host(sim.observe())
    ref = o.observe(w.robot.q0, np.zeros_like(w.robot.q0), w.task.progress0)
    assert np.abs(obs - ref).max() <= 2e-6
    q, qd, pr, rs = sim.get_state()
    a = dev(synth.random_actions(1, 100, 7, np.float32), torch, torch.float32)
    o1 = host(sim.step(a)[0])
    sim.set_state(q, qd, pr, rs)
    o2 = host(sim.step(a)[0])
    assert np.array_equal(o1, o2)  # bit-identical replay after restore
    sim.reset()
    assert np.array_equal(host(sim.get_state()[0]), w.robot.q0.astype(np.float32).astype(np.float64))


def test_nonfinite_state_forced_from_host(sg):
    import torch
    w = synth.path_rollout(64)
    sim = sg.Sim(w.robot, w.task)
    q, qd, pr, _ = sim.get_state()
    q2 = q.clone()
    q2[3, 5] = float("nan")
    qd2 = qd.clone()
    qd2[1, 9] = float("inf")
    sim.set_state(q2, qd2, pr)
    a = torch.zeros(7, 64, device="cuda")
    obs, rew, done = sim.step(a)
    d = host(done).astype(int)
    assert d[5] == 5 and d[9] == 5
    assert np.all(np.isfinite(host(obs)))
    assert host(rew)[5] == 0 and host(rew)[9] == 0
    others = np.setdiff1d(np.arange(64), [5, 9])
    ref = sg.Sim(w.robot, w.task)
    ref.set_state(q, qd, pr)
    obs_r, _, _ = ref.step(a)
    assert np.array_equal(host(obs)[:, others], host(obs_r)[:, others])


def test_gae_parity(sg):
    import torch
    w = synth.path_rollout(8)
    sim = sg.Sim(w.robot, w.task)
    rng = np.random.default_rng(5)
    T, N = 32, 1000
    rew = rng.normal(0, 1, (T, N)).astype(np.float32)
    val = rng.normal(0, 1, (T + 1, N)).astype(np.float32)
    done = (rng.random((T, N)) < 0.1).astype(np.uint8)
    done |= ((rng.random((T, N)) < 0.5) & (done == 1)).astype(np.uint8) << 1
    adv, ret = sim.gae(dev(rew, torch, torch.float32), dev(val, torch, torch.float32),
                       torch.from_numpy(done).cuda())
    ra, rr = oracle.gae(rew.astype(np.float64), val.astype(np.float64), done)
    assert np.abs(host(adv) - ra).max() <= 1e-5 * max(1, np.abs(ra).max())
    assert np.abs(host(ret) - rr).max() <= 1e-5 * max(1, np.abs(rr).max())


def test_bad_arguments_rejected(sg):
    import torch
    w = synth.path_rollout(16)
    sim = sg.Sim(w.robot, w.task)
    a = torch.zeros(7, 16, device="cuda")
    with pytest.raises(sg.SgError) as ei:
        sim._call(sg.lib.sg_step, None, a.data_ptr(), a.data_ptr(), a.data_ptr())
    assert ei.value.status == sg.SG_E_INVAL
    with pytest.raises(sg.SgError) as ei:
        sim.forward_dynamics(a, a, a, arm_mode=7)
    assert ei.value.status == sg.SG_E_INVAL
