"""HIP graph capture of the learning-loop calls: the noise counter and the
Adam step count live in device memory and are advanced by the captured
kernels, so replays of a captured call equal the same number of eager
calls (bit for bit: same kernels, same inputs) and consecutive replays draw
fresh noise and take new Adam steps. Each replay is followed by the
program's own synchronization and a copy of its outputs."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

KEYS = ("obs", "act", "logp", "rew", "done", "val", "adv", "ret")


def snap(bufs):
    return {k: bufs[k].detach().cpu().numpy().copy() for k in KEYS}


def test_captured_rollout_replays_match_eager_calls(sg):
    import torch
    w = synth.path_rollout(256)
    T = 8
    eager = sg.from_workload(w)
    ref = [snap(eager.rollout(T)) for _ in range(3)]
    cap = sg.from_workload(w)
    bufs = cap.rollout_buffers(T)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        cap.rollout(T, bufs)
    got = []
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
        got.append(snap(bufs))
        # the program's own eager work between replays
        cap.get_state()
    for r, x in zip(ref, got):
        for k in KEYS:
            np.testing.assert_array_equal(x[k], r[k], err_msg=k)
    assert not np.array_equal(got[0]["act"], got[1]["act"])
    assert not np.array_equal(got[1]["act"], got[2]["act"])
    assert cap.get_state()[3] == 3 * T == eager.get_state()[3]
    # the eager path continues from where the replays left the counter
    a = snap(eager.rollout(T))
    b = snap(cap.rollout(T))
    np.testing.assert_array_equal(a["act"], b["act"])


def test_captured_step_advances_tracking_goal_draws(sg):
    import torch
    w = synth.tracking(128)
    eager = sg.from_workload(w)
    cap = sg.from_workload(w)
    J = w.robot.max_dof
    act = torch.from_numpy(synth.random_actions(5, 128, J, np.float32)).float().cuda()
    ref = []
    for _ in range(3):
        o, r, d = eager.step(act)
        ref.append((o.cpu().numpy().copy(), r.cpu().numpy().copy()))
    o_buf = torch.empty(2 * J + 10, 128, device="cuda")
    r_buf = torch.empty(128, device="cuda")
    d_buf = torch.empty(128, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        cap.step(act, o_buf, r_buf, d_buf)
    for i in range(3):
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(o_buf.cpu().numpy(), ref[i][0])
        np.testing.assert_array_equal(r_buf.cpu().numpy(), ref[i][1])
    gs_e = eager.get_goal_state().cpu().numpy()
    gs_c = cap.get_goal_state().cpu().numpy()
    np.testing.assert_array_equal(gs_c, gs_e)
    assert cap.get_state()[3] == 3


def test_captured_ppo_update_takes_new_adam_steps(sg):
    import torch
    w = synth.path_rollout(256)
    T = 8
    sim = sg.from_workload(w)
    bufs = sim.rollout(T)
    p0 = sg.ppo_flat_params(w.policy)
    pa = sg.Ppo(sim, p0, T * 256)
    pb = sg.Ppo(sim, p0, T * 256)
    st = torch.empty(8, device="cuda")
    pa.update(bufs, T, stats=st)
    a1 = pa.params()
    pa.update(bufs, T, stats=st)
    a2 = pa.params()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pb.update(bufs, T, stats=st)
    g.replay()
    torch.cuda.synchronize()
    b1 = pb.params()
    g.replay()
    torch.cuda.synchronize()
    b2 = pb.params()
    np.testing.assert_array_equal(b1, a1)
    np.testing.assert_array_equal(b2, a2)
    assert not np.array_equal(b1, b2)
