"""Parity at the sizes and launch configurations bench.py times.

* The fused path-following rollout at 4096 envs (two consecutive T = 32
  rollouts, as the timed loop runs them) and at 16384 envs: the oracle
  replays every env's control step from the stored observations (which hold
  q and qd exactly) and recomputes GAE for every env; the policy outputs
  (action means plus the Philox noise, values, log-densities) are checked on
  512 envs spread over all waves: the first and last 64 and a seeded draw.
* The uneven 4/6/7/9-DOF batch at 16384 envs under every step schedule the
  autotuner times, each step checked for every env against the oracle's
  step from the state the GPU handed over.
* The surrogate step at 65536 envs: the exact-fallback path against the
  oracle's step, and the accept/fallback decisions against the oracle's
  residuals.
* The PPO gradient of a 32,768-sample minibatch of a 4096-env T = 32
  rollout against the oracle's.
* The prismatic, tracking and multi-arm variants through the fused rollout
  at 4096 chains, replayed like the path rollout.

Tolerances are those of the smaller parity tests: see test_gpu_rollout.py
(policy outputs, log-density, GAE, replayed step) and test_gpu_step.py
(hand-off step).
"""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_rollout import check_policy_outputs, host

pytestmark = pytest.mark.gpu

THREADS = 16


def _sample(N, seed=5, k=384):
    rng = np.random.default_rng(seed)
    mid = rng.choice(np.arange(64, N - 64), size=min(k, max(N - 128, 0)), replace=False)
    return np.unique(np.concatenate([np.arange(min(64, N)), np.arange(max(N - 64, 0), N), mid]))


def _replay_full(sg, w, T, n_rollouts, rew_tol=2e-4, track=False):
    sim = sg.from_workload(w)
    # tracking task: the oracle advances its own copy of the goal state
    gs = np.ascontiguousarray(host(sim.get_goal_state())) if track else None
    o = oracle.Oracle(w.robot, w.task, w.policy)
    N, J = w.robot.n_env, w.robot.max_dof
    idx = _sample(N)
    sigma = np.exp(w.policy.log_std)
    bufs = sim.rollout_buffers(T)
    prog = w.task.progress0.astype(np.int32).copy()
    step0 = 0
    for r in range(n_rollouts):
        sim.rollout(T, bufs)
        obs, act, logp = host(bufs["obs"]), host(bufs["act"]), host(bufs["logp"])
        rew, done, val = host(bufs["rew"]), bufs["done"].cpu().numpy(), host(bufs["val"])
        adv, ret = host(bufs["adv"]), host(bufs["ret"])
        for t in range(T + 1):
            mv = o.mlp(obs[t][:, idx], emulate=True)
            check_policy_outputs(val[t][idx][None], mv[J][None])
            if t == T:
                break
            eps = oracle.noise(w.seed, step0 + t, J, N)
            check_policy_outputs(act[t][:, idx], mv[:J] + sigma[:, None] * eps[:, idx])
            lp = (-0.5 * eps ** 2 - w.policy.log_std[:, None] - 0.5 * np.log(2 * np.pi)).sum(0)
            np.testing.assert_allclose(logp[t], lp, rtol=1e-5, atol=1e-4)
            q, qd = obs[t][:J], obs[t][J:2 * J]
            qn, qdn, prn, rw, dn, ob = o.step(act[t], q, qd, prog, threads=THREADS, goal_state=gs, seed=w.seed,
                                              step=step0 + t)
            assert np.array_equal(done[t], dn), (r, t)
            assert np.abs(rew[t] - rw).max() <= rew_tol, (r, t, np.abs(rew[t] - rw).max())
            scale = np.maximum(1.0, np.abs(ob))
            assert (np.abs(obs[t + 1] - ob) / scale).max() <= 2e-3, (r, t)
            prog = prn
        ra, rr = oracle.gae(rew, val, done, 0.99, 0.95)
        np.testing.assert_allclose(adv, ra, rtol=1e-5, atol=1e-4)
        np.testing.assert_allclose(ret, rr, rtol=1e-5, atol=1e-4)
        step0 += T
    q, qd, pr, rs = sim.get_state()
    assert rs == step0
    if track:
        assert np.abs(host(sim.get_goal_state()) - gs).max() <= 2e-6
    np.testing.assert_array_equal(host(q), obs[T][:J])
    np.testing.assert_array_equal(pr.cpu().numpy(), prog)
    sim.close()


def test_path_rollout_4096_two_rollouts(sg):
    _replay_full(sg, synth.path_rollout(4096), 32, 2)


def test_path_rollout_16384(sg):
    _replay_full(sg, synth.path_rollout(16384), 32, 1)


@pytest.mark.parametrize("name", ["prismatic_rrprrr", "tracking", "multi_arm_2", "multi_arm_4"])
def test_variant_rollouts_4096_chains(sg, name):
    """The joint and task variants bench.py times, at its 4096 chains: RRPRRR
    chains, active tracking (two rollouts; the oracle draws the goal walk and
    re-draws from the same counters), and 2 or 4 arms per env whose reward is
    the sum over the env's arms (the reward tolerance scales with the number
    of summed terms)."""
    if name == "prismatic_rrprrr":
        w = synth.psm_like(4096)
        w.policy = synth.make_policy(w.seed + 7, dims=(22, 256, 128, 7))
        _replay_full(sg, w, 32, 1)
    elif name == "tracking":
        _replay_full(sg, synth.tracking(4096), 32, 2, track=True)
    else:
        C = int(name[-1])
        _replay_full(sg, synth.multi_arm(4096 // C, chains=C), 32, 1, rew_tol=2e-4 * C)


@pytest.mark.parametrize("schedule", ["padded", "sorted", "per_class", "persistent"])
def test_mixed_dof_16384_every_schedule(sg, schedule):
    import torch
    w = synth.mixed_dof(16384)
    sim = sg.Sim(w.robot, w.task)
    sim.set_schedule(sg.SCHEDULE_NAMES.index(schedule))
    o = oracle.Oracle(w.robot, w.task)
    J, N = w.robot.max_dof, w.robot.n_env
    qtol = 2e-5
    for s in range(3):
        q0, qd0, pr0, _ = sim.get_state()
        a = synth.random_actions(900 + s, N, J, dtype=np.float32).astype(np.float32)
        obs, rew, done = sim.step(torch.from_numpy(a).cuda())
        q1, qd1, pr1, _ = sim.get_state()
        qn, qdn, prn, rw, dn, ob = o.step(a, host(q0), host(qd0), host(pr0).astype(np.int32), threads=THREADS)
        assert np.array_equal(host(done).astype(np.uint8), dn), s
        assert np.array_equal(host(pr1).astype(np.int32), prn), s
        dq = np.abs(host(q1) - qn) / (1 + np.abs(qn))
        assert dq.max() <= qtol, (s, dq.max())
        assert np.abs(host(qd1) - qdn).max() <= qtol * 100 * max(1.0, np.abs(qdn).max()), s
        assert np.abs(host(rew) - rw).max() <= qtol * 10, s
        assert np.abs(host(obs) - ob).max() <= qtol * 100 * max(1.0, np.abs(ob).max()), s
    sim.close()


def test_surrogate_step_65536_threshold_zero_is_the_oracle_step(sg):
    """The surrogate step at its 65536-env size with threshold 0: every env
    takes the exact solve, so each step matches the oracle's step for every
    env (tolerances of the hand-off step)."""
    import torch
    from test_gpu_surrogate import _setup
    N = 65536
    w, sim, o, T, _ = _setup(sg, n_env=N)
    S = sg.Surrogate(sim, 64)
    W, b = synth.surrogate_init(1)
    S.set_params(W, b)
    S.fit_norm(T["q"], T["qd"], T["tau"], T["env"], T["qdd"])
    nfb = torch.zeros(4, dtype=torch.int32, device="cuda")
    qtol = 2e-5
    for s in range(2):
        q0, qd0, pr0, _ = sim.get_state()
        a = synth.random_actions(60 + s, N, 7, np.float32).astype(np.float32)
        obs, rew, done = S.step(torch.from_numpy(a).cuda(), 0.0, n_fallback=nfb)
        assert np.all(nfb.cpu().numpy() == N)
        q1, qd1, pr1, _ = sim.get_state()
        qn, qdn, prn, rw, dn, ob = o.step(a, host(q0), host(qd0), host(pr0).astype(np.int32), threads=THREADS)
        assert np.array_equal(host(done).astype(np.uint8), dn), s
        assert np.array_equal(host(pr1).astype(np.int32), prn), s
        assert (np.abs(host(q1) - qn) / (1 + np.abs(qn))).max() <= qtol, s
        assert np.abs(host(qd1) - qdn).max() <= qtol * 100 * max(1.0, np.abs(qdn).max()), s
        assert np.abs(host(rew) - rw).max() <= qtol * 10, s
        assert np.abs(host(obs) - ob).max() <= qtol * 100 * max(1.0, np.abs(ob).max()), s
    S.close()


def test_surrogate_step_65536_accepts_predictions_and_counts_fallbacks(sg):
    """One substep at 65536 envs: with an infinite threshold the step
    integrates the network's prediction (the library's predict call, itself
    checked against the FP64 network in test_gpu_surrogate.py); with a
    finite one the fallback count equals the number of envs whose oracle
    residual of that prediction exceeds it, up to envs within 1e-3 of the
    threshold."""
    import torch
    from test_gpu_surrogate import _setup
    N = 65536
    w, sim, o, T, _ = _setup(sg, n_env=N, substeps=1)
    S = sg.Surrogate(sim, 256)
    Wt, bt = synth.surrogate_init(2)
    S.set_params(Wt, bt)
    S.fit_norm(T["q"], T["qd"], T["tau"], T["env"], T["qdd"])
    q0, qd0, pr0, _ = sim.get_state()
    a = synth.random_actions(77, N, 7, np.float32)
    at = torch.from_numpy(a).float().cuda()
    h = w.robot.dt
    tau = w.robot.kp * (a.clip(-1, 1) * w.robot.q_hi - host(q0) - h * host(qd0)) - w.robot.kd * host(qd0)
    tau32 = torch.from_numpy(tau.astype(np.float32)).cuda()
    qh = host(S.predict(q0, qd0, tau32, T["env"]))
    nfb = torch.zeros(1, dtype=torch.int32, device="cuda")
    _, _, done = S.step(at, float("inf"), n_fallback=nfb)
    assert int(nfb.item()) == 0
    q1, qd1, _, _ = sim.get_state()
    qd_ref = host(qd0) + h * qh
    q_ref = np.clip(host(q0) + h * qd_ref, w.robot.q_lo, w.robot.q_hi)
    inside = (q_ref < w.robot.q_hi) & (q_ref > w.robot.q_lo) & (done.cpu().numpy() == 0)[None, :]
    # The step forms tau in FP32 from its own state, the reference in FP64:
    # features differing in the last bits can flip one BF16 rounding of a
    # hidden activation (test_gpu_surrogate.py's bound: ~1e-3 on a
    # normalised output), which moves qd by up to ~1e-3 after the factor h.
    # Over 455 k coordinates a few such flips occur: bound the tail.
    d = np.abs(host(qd1)[inside] - qd_ref[inside]) / np.maximum(1.0, np.abs(qd_ref[inside]))
    assert np.median(d) <= 1e-6, np.median(d)
    assert d.max() <= 1e-2, d.max()
    assert (d > 1e-3).mean() <= 1e-4, (d > 1e-3).mean()
    sim.set_state(q0, qd0, pr0)
    rel = oracle.residual(o, host(q0), host(qd0), tau, qh, o.drive_armature())
    thr = float(np.median(rel))
    S.step(at, thr, n_fallback=nfb)
    lo, hi = (rel > thr * (1 + 1e-3)).sum(), (rel > thr * (1 - 1e-3)).sum()
    assert lo <= int(nfb.item()) <= hi, (lo, int(nfb.item()), hi)
    S.close()


def test_ppo_minibatch_gradient_4096_envs(sg):
    """The PPO gradient at the benchmark's size: a T = 32 rollout of 4096
    envs (advantages normalised over all 131,072 samples) and one minibatch
    of 32,768 sample ids drawn across the whole rollout, the minibatch the
    timed update uses; statistics and each parameter block's gradient
    against the oracle's FP64 gradient of the same samples (tolerances of
    test_gpu_ppo.py)."""
    import torch
    from test_gpu_ppo import DIMS, _blocks, _rows, _setup
    T, N = 32, 4096
    w, sim, ppo, params, bufs = _setup(sg, N, T)
    g = torch.Generator(device="cuda").manual_seed(11)
    bufs["logp"] += 0.3 * torch.randn(bufs["logp"].shape, device="cuda", generator=g)
    idx = torch.randperm(T * N, device="cuda", generator=g)[:32768].to(torch.int32)
    gg, st = ppo.grad(bufs, T, idx)
    h, x, a = _rows(bufs, T, N)
    an = oracle.ppo_normalise(h["adv"]).ravel()
    s = idx.cpu().numpy()
    L, gr, so = oracle.ppo_grad(DIMS, params.astype(np.float64), x[:, s], a[:, s], h["logp"].ravel()[s], an[s],
                                h["ret"].ravel()[s], h["val"][:T].ravel()[s], emulate=True)
    st = host(st)
    for k, name in enumerate(("loss_pi", "loss_v", "entropy", "approx_kl", "clip_frac")):
        assert abs(st[k] - so[name]) <= 1e-3 * max(1.0, abs(so[name])) + 1e-5, (name, st[k], so[name])
    assert 0.05 < so["clip_frac"] < 0.95
    for i, (gb, rb) in enumerate(zip(_blocks(host(gg)), _blocks(gr))):
        rel = np.linalg.norm(gb - rb) / np.linalg.norm(rb)
        cos = (gb @ rb) / (np.linalg.norm(gb) * np.linalg.norm(rb))
        assert rel <= 2e-2 and cos >= 0.999, (i, rel, cos)
    ppo.close()
