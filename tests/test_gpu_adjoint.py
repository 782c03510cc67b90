"""Adjoint of an open-loop rollout on the GPU (FP32, checkpointed) against
the FP64 oracle's adjoint (full tape), which is itself pinned by central
differences.

Tolerances: gradients over all envs and entries rel L2 <= 1e-3 and cosine
>= 0.9999 (FP32 rounding accumulated over T steps of the forward and
reverse sweeps); the loss within 1e-5 relative. The checkpoint interval
changes only the recomputation schedule: results for different K agree to
FP32 rounding (rel 1e-5)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _rel_cos(g, r):
    g, r = g.ravel(), r.ravel()
    return np.linalg.norm(g - r) / np.linalg.norm(r), (g @ r) / (np.linalg.norm(g) * np.linalg.norm(r))


def _case(sg, w, T, seed, K):
    import torch
    sim = sg.Sim(w.robot, w.task)
    N, J = w.robot.n_env, w.robot.max_dof
    act = synth._as_dtype(np.random.default_rng(seed).uniform(-0.95, 0.95, (T, J, N)), np.float32)
    act[:, np.arange(J)[:, None] >= w.robot.n_dof[None, :]] = 0
    at = torch.from_numpy(act.astype(np.float32)).cuda()
    q, qd, pr, _ = sim.get_state()
    loss, ga, gm = sim.adjoint(at, K)
    o = oracle.Oracle(w.robot, w.task)
    rl, ra, rm = oracle.adjoint(o, T, act, host(q), host(qd), pr.cpu().numpy(), threads=8)
    return sim, at, (host(loss), host(ga), host(gm)), (rl, ra, rm)


@pytest.mark.parametrize("kind,N,T,K", [("path", 300, 16, 4), ("psm", 130, 12, 5), ("mixed", 200, 10, 3),
                                        ("path", 1, 5, 5)])
def test_adjoint_matches_oracle(sg, kind, N, T, K):
    w = {"path": synth.path_rollout, "psm": synth.psm_like, "mixed": synth.mixed_dof}[kind](N)
    if kind == "mixed":
        # the adjoint covers max_dof <= 7
        w = synth.Workload("mixed7", synth._round_robot(synth.make_chain(N, np.array([4, 6, 7, 5] * N)[:N], 1003,
                                                                         dt=1 / 120, substeps=4, gain_jitter=True,
                                                                         q0_frac=0.25), np.float32),
                           synth.path_rollout(N).task, None, np.float32, 1003)
    sim, at, (l, ga, gm), (rl, ra, rm) = _case(sg, w, T, 17, K)
    np.testing.assert_allclose(l, rl, rtol=1e-5, atol=1e-6)
    for g, r in ((ga, ra), (gm, rm)):
        rel, cos = _rel_cos(g, r)
        assert rel <= 1e-3 and cos >= 0.9999, (rel, cos)


def test_checkpoint_interval_does_not_change_results(sg):
    import torch
    w = synth.path_rollout(256)
    sim = sg.Sim(w.robot, w.task)
    T = 12
    gen = torch.Generator(device="cuda").manual_seed(12)
    act = torch.rand(T, 7, 256, device="cuda", generator=gen) * 1.8 - 0.9
    outs = [[host(x) for x in sim.adjoint(act, K)] for K in (1, 4, 12)]
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-6 * np.abs(b).max())
    # the context's state is left unchanged
    q0 = host(sim.get_state()[0])
    sim.adjoint(act, 4)
    np.testing.assert_array_equal(host(sim.get_state()[0]), q0)


def test_full_size_every_env_and_memory(sg):
    """4096 envs x 64 steps x 4 substeps, checkpoints every 8 steps; every
    env checked against the oracle's full-tape adjoint (the same criteria as
    the small cases, over all envs and entries); workspace against the full
    tape the reverse sweep reads (each substep's q, qd and accelerations for
    all T steps)."""
    import torch
    N, T, K = 4096, 64, 8
    w = synth.path_rollout(N)
    w.task.ep_len = 0  # open loop over the whole horizon
    sim = sg.Sim(w.robot, w.task)
    act = synth._as_dtype(np.random.default_rng(3).uniform(-0.9, 0.9, (T, 7, N)), np.float32)
    q, qd, pr, _ = sim.get_state()
    q, qd, pr = host(q), host(qd), pr.cpu().numpy()
    loss, ga, gm = sim.adjoint(torch.from_numpy(act.astype(np.float32)).cuda(), K)
    o = oracle.Oracle(w.robot, w.task)
    rl, ra, rm = oracle.adjoint(o, T, act, q, qd, pr, threads=8)
    np.testing.assert_allclose(host(loss), rl, rtol=1e-4)
    for g, r in ((host(ga), ra), (host(gm), rm)):
        rel, cos = _rel_cos(g, r)
        assert rel <= 1e-3 and cos >= 0.9999, (rel, cos)
    full_tape = T * 4 * 3 * 7 * N * 4
    assert sim.adjoint_workspace_bytes(T, K) < full_tape / 4


def test_gradient_agrees_with_oracle_finite_differences(sg):
    """Central differences (h = 1e-3) of the FP64 oracle's forward loss for a
    few actions and masses against the GPU gradient."""
    import torch
    w = synth.path_rollout(8)
    w.task.ep_len = 0
    sim = sg.Sim(w.robot, w.task)
    T = 8
    act = synth._as_dtype(np.random.default_rng(4).uniform(-0.8, 0.8, (T, 7, 8)), np.float32)
    _, ga, gm = sim.adjoint(torch.from_numpy(act.astype(np.float32)).cuda(), 4)
    ga, gm = host(ga), host(gm)
    o = oracle.Oracle(w.robot, w.task)
    q, qd, pr, _ = sim.get_state()
    q, qd, pr = host(q), host(qd), pr.cpu().numpy()
    h = 1e-3
    for (t, j) in ((0, 1), (3, 3), (7, 6), (5, 0)):
        e = np.zeros_like(act, dtype=np.float64)
        e[t, j] = h
        fd = (oracle.adjoint(o, T, act + e, q, qd, pr, want_grad=False) -
              oracle.adjoint(o, T, act - e, q, qd, pr, want_grad=False)) / (2 * h)
        np.testing.assert_allclose(ga[t, j], fd, rtol=2e-2, atol=1e-3 * np.abs(fd).max())
    for j in (0, 3, 6):
        s = np.ones((7, 8))
        s[j] += h
        lp = oracle.adjoint(o, T, act, q, qd, pr, mass_scale=s, want_grad=False)
        s[j] -= 2 * h
        lm = oracle.adjoint(o, T, act, q, qd, pr, mass_scale=s, want_grad=False)
        fd = (lp - lm) / (2 * h) / w.robot.mass[j]
        np.testing.assert_allclose(gm[j], fd, rtol=2e-2, atol=1e-3 * np.abs(fd).max())


def test_autograd_function_and_mass_update(sg):
    import torch
    w = synth.path_rollout(64)
    w.task.ep_len = 0
    sim = sg.Sim(w.robot, w.task)
    T = 6
    act = (torch.rand(T, 7, 64, device="cuda") * 1.6 - 0.8).requires_grad_()
    m0 = torch.from_numpy(w.robot.mass.astype(np.float32)).cuda()
    m = (m0 * 1.1).requires_grad_()
    loss = sg.rollout_loss(sim, act, m, 3)
    loss.sum().backward()
    l2, ga, gm = sim.adjoint(act.detach(), 3)
    assert torch.equal(loss.detach(), l2)
    assert torch.equal(act.grad, ga) and torch.equal(m.grad, gm)
    # the masses were installed: the oracle with masses x 1.1 agrees
    o = oracle.Oracle(w.robot, w.task)
    q, qd, pr, _ = sim.get_state()
    rl = oracle.adjoint(o, T, host(act), host(q), host(qd), pr.cpu().numpy(), mass_scale=np.full((7, 64), 1.1),
                        want_grad=False)
    np.testing.assert_allclose(host(loss), rl, rtol=1e-4)


def test_bad_arguments_rejected(sg):
    import torch
    w = synth.path_rollout(16)
    sim = sg.Sim(w.robot, w.task)
    act = torch.zeros(4, 7, 16, device="cuda")
    with pytest.raises(sg.SgError):
        sim.adjoint(act, 5)      # K > T
    with pytest.raises(sg.SgError):
        sim.adjoint(act, 0)
    w64 = synth.reach_fp64(8)
    s64 = sg.Sim(w64.robot, w64.task, dtype=np.float64)
    with pytest.raises(sg.SgError):
        s64.adjoint(torch.zeros(2, 7, 8, device="cuda"), 1)
