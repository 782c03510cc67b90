"""Edge cases through the HIP library: every DOF bucket from 1 to the
maximum of 16 joints (uniform and per-env joint counts, FP32 and FP64)
against the FP64 oracle; invalid sizes rejected at create; the control step
captured in a HIP graph and replayed, each replay checked against the same
step run eagerly; the measured device rates; degenerate dynamics (no drive,
no gravity: exactly at rest) and the joint-limit property at the uneven
batch's full size."""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_step import _run_handoff, dev, host, rel_qdd_err

pytestmark = pytest.mark.gpu


def _chain_workload(N, n_dof, dtype, seed=2024, max_dof=None):
    r = synth.make_chain(N, n_dof, seed, dt=1 / 120, substeps=2, max_dof=max_dof, q0_frac=0.2)
    tgt = (synth.WORK_CENTRE[None, :] + synth.stream(seed, "tg").uniform(-0.25, 0.25, (N, 3))).T.copy()
    t = synth.Task(task=synth.TASK_REACH, target=tgt, waypoints=None, dwell=1, ep_len=64,
                   progress0=synth.stream(seed, "p0").integers(0, 64, N).astype(np.int32))
    return synth.Workload("chain", synth._round_robot(r, dtype), synth._round_task(t, dtype), None, dtype, seed)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("J,mixed", [(1, False), (2, False), (3, False), (4, False), (5, True), (8, False),
                                     (12, True), (16, False)])
def test_every_dof_bucket(sg, J, mixed, dtype):
    import torch
    N = 70
    n_dof = np.array([(k % J) + 1 for k in range(N)]) if mixed else J
    w = _chain_workload(N, n_dof, dtype, max_dof=J)
    td = torch.float64 if dtype == np.float64 else torch.float32
    sim = sg.Sim(w.robot, w.task, dtype=dtype)
    o = oracle.Oracle(w.robot, w.task)
    q, qd = synth.random_states(21, w.robot, dtype=dtype)
    tau = synth._as_dtype(np.random.default_rng(J).normal(0, 5, q.shape), dtype)
    tau[np.arange(J)[:, None] >= w.robot.n_dof[None, :]] = 0
    g = host(sim.forward_dynamics(dev(q, torch, td), dev(qd, torch, td), dev(tau, torch, td), sg.SG_ARM_DRIVE))
    tol = 1e-10 if dtype == np.float64 else 1e-4
    assert rel_qdd_err(g, o.aba(q, qd, tau, o.drive_armature())) <= tol
    tip = host(sim.tip_position(dev(q, torch, td)))
    assert np.abs(tip - o.fk(q)).max() <= (1e-13 if dtype == np.float64 else 3e-6)
    _run_handoff(sg, w, 6, 7000 + J, qtol=1e-11 if dtype == np.float64 else 2e-5,
                 tol_qdd=1e-10 if dtype == np.float64 else 1e-4)


def test_create_rejects_invalid_sizes(sg):
    w = _chain_workload(8, 3, np.float32)
    bad = synth._round_robot(synth.make_chain(8, 17, 1, dt=0.01, substeps=1), np.float32)
    with pytest.raises(sg.SgError):
        sg.Sim(bad, w.task)   # more than 16 joints
    r = synth.make_chain(8, 3, 1, dt=0.01, substeps=1)
    r.n_dof[2] = 4            # above max_dof
    with pytest.raises(sg.SgError):
        sg.Sim(synth._round_robot(r, np.float32), w.task)
    r = synth.make_chain(8, 3, 1, dt=0.01, substeps=1)
    r.mass[1, 3] = 0.0        # massless link
    with pytest.raises(sg.SgError):
        sg.Sim(synth._round_robot(r, np.float32), w.task)
    r = synth.make_chain(8, 3, 1, dt=0.0, substeps=1)
    with pytest.raises(sg.SgError):
        sg.Sim(synth._round_robot(r, np.float32), w.task)


def test_step_replayed_from_a_captured_graph(sg):
    import torch
    N = 512
    w = synth.path_rollout(N)
    sim_g = sg.Sim(w.robot, w.task)
    sim_e = sg.Sim(w.robot, w.task)
    a = torch.from_numpy(synth.random_actions(55, N, 7, np.float32).astype(np.float32)).cuda()
    obs = torch.empty(24, N, device="cuda")
    rew = torch.empty(N, device="cuda")
    done = torch.empty(N, dtype=torch.uint8, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        # warm-up on the capture stream, then rewind both contexts
        sim_g.step(a, obs, rew, done)
    torch.cuda.current_stream().wait_stream(side)
    sim_g.reset()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        sim_g.step(a, obs, rew, done)
    # capture records the launch without running it
    sim_g.reset()
    torch.cuda.synchronize()
    for k in range(4):
        graph.replay()
        oe, re, de = sim_e.step(a)
        torch.cuda.synchronize()
        assert torch.equal(obs, oe) and torch.equal(rew, re) and torch.equal(done, de), k
        qg, qdg, pg, _ = sim_g.get_state()
        qe, qde, pe, _ = sim_e.get_state()
        assert torch.equal(qg, qe) and torch.equal(qdg, qde) and torch.equal(pg, pe), k
        # eager work of the program between replays
        assert torch.equal(sim_g.observe(), sim_e.observe())
        torch.cuda.synchronize()


def test_measured_peaks_are_sane(sg):
    pk = sg.measure_peaks()
    assert all(np.isfinite(v) and v > 0 for v in pk.values())
    # below the datasheet figures (FP32 vector 157.3 TFLOP/s, BF16 dense
    # 2.5 PFLOP/s, HBM 8 TB/s) and a lone wave slower than a full chip
    assert pk["fp32_fma_tflops"] < 157.3 * 1.05
    assert pk["bf16_mfma_tflops"] < 2500 * 1.05
    assert pk["copy_gbps"] < 8000 * 1.05
    assert pk["fp32_fma_wave_gflops"] * 1e-3 < pk["fp32_fma_tflops"]


def test_undriven_chain_without_gravity_stays_at_rest(sg):
    """Degenerate dynamics: no gravity and zero PD gains, at rest. Every bias
    and drive term is exactly zero, so ABA returns exactly zero accelerations
    and the state must not move at all, whatever the actions (ragged 300
    envs, mixed joint counts)."""
    import torch
    N = 300
    n_dof = np.array([(k % 7) + 1 for k in range(N)])
    r = synth.make_chain(N, n_dof, 77, dt=1 / 120, substeps=4, max_dof=7, q0_frac=0.3)
    r.kp[:] = 0.0
    r.kd[:] = 0.0
    r.gravity = (0.0, 0.0, 0.0)
    tgt = (synth.WORK_CENTRE[None, :] + synth.stream(77, "tg").uniform(-0.25, 0.25, (N, 3))).T.copy()
    t = synth.Task(task=synth.TASK_REACH, target=tgt, waypoints=None, dwell=1, ep_len=1000,
                   progress0=np.zeros(N, dtype=np.int32))
    w = synth.Workload("rest", synth._round_robot(r, np.float32), synth._round_task(t, np.float32), None,
                       np.float32, 77)
    sim = sg.Sim(w.robot, w.task)
    q0, qd0, _, _ = sim.get_state()
    for s in range(5):
        a = torch.from_numpy(synth.random_actions(500 + s, N, 7, np.float32).astype(np.float32)).cuda()
        sim.step(a)
    q1, qd1, _, _ = sim.get_state()
    assert torch.equal(q1, q0)
    assert torch.count_nonzero(qd1).item() == 0
    assert torch.count_nonzero(qd0).item() == 0


def test_mixed_batch_stays_within_limits(sg):
    """Property at the uneven batch's full size, any schedule: after every
    step each joint lies within its limits (compared in the context's FP32)
    and every observation is finite."""
    import torch
    w = synth.mixed_dof(16384)
    lo = torch.from_numpy(w.robot.q_lo.astype(np.float32)).cuda()
    hi = torch.from_numpy(w.robot.q_hi.astype(np.float32)).cuda()
    for sched in (sg.SG_SCHED_PADDED, sg.SG_SCHED_SORTED):
        sim = sg.Sim(w.robot, w.task)
        sim.set_schedule(sched)
        for s in range(10):
            a = torch.from_numpy(synth.random_actions(600 + s, 16384, 9, np.float32).astype(np.float32)).cuda()
            obs, _, _ = sim.step(a)
            q, _, _, _ = sim.get_state()
            assert bool(((q >= lo) & (q <= hi)).all()), (sched, s)
            assert bool(torch.isfinite(obs).all()), (sched, s)
        sim.close()
