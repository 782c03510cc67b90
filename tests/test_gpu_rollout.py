"""Parity of the fused rollout (policy on the matrix cores, noise, env step,
GAE) and of the policy network alone, against the FP64 oracle.

Tolerances:
* policy outputs vs the oracle's BF16-emulating forward pass on the same
  FP32 inputs: the GPU accumulates in FP32 and forms tanh from the hardware
  exponential and reciprocal, so a hidden activation can round to the
  neighbouring BF16 value; one such flip moves an output by at most
  |w| * 2^-8 * |h| with |w| <= 1/sqrt(fan_in), i.e. ~4e-4. The share of
  outputs that such FP32-level errors move by more than 1e-4 is derived
  from the oracle side alone (pinlib.flip_share: the emulating forward pass
  with every hidden unit perturbed by the error model of an FP32 evaluation,
  on observations of the path workload): about 1.5 % for this network. The
  check allows twice that share plus four binomial deviations of outputs
  above 1e-4, |d out| <= 2e-3 everywhere and a median <= 2e-5.
* log-density, GAE: relative 1e-5 (FP32 accumulation).
* env step inside the rollout, replayed by the oracle from the stored
  observation (which holds q and qd exactly): as in the step tests.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


_SHARE = {}


def policy_flip_share(policy=None):
    """Expected share of policy outputs moved by more than 1e-4 by BF16
    flips of a correct FP32 evaluation (see the module docstring), for the
    rollout workload's network or the given one, on observations of the path
    workload."""
    key = None if policy is None else id(policy)
    if key not in _SHARE:
        import pinlib
        w = synth.path_rollout(512, seed=77)
        pol = w.policy if policy is None else policy
        o = oracle.Oracle(w.robot, w.task, w.policy)
        q, qd = synth.random_states(5, w.robot, dtype=np.float32, qd_scale=2.0)
        x = o.observe(q, qd, w.task.progress0)
        L = len(pol.W)
        layers = [(np.asarray(pol.W[l], np.float64), np.asarray(pol.b[l], np.float64)) for l in range(L)]
        act = getattr(pol, "act", "tanh")
        _SHARE[key] = pinlib.flip_share(layers, [act] * (L - 1) + [None], x.astype(np.float32), 1e-4)
    return _SHARE[key]


def check_policy_outputs(g, ref, policy=None):
    import pinlib
    d = np.abs(g - ref)
    share = policy_flip_share(policy)
    assert d.max() <= 2e-3, d.max()
    assert np.median(d) <= 2e-5, np.median(d)
    n = int((d > 1e-4).sum())
    assert n <= pinlib.allowed_count(share, d.size), (n, d.size, share)


@pytest.mark.parametrize("n", [1, 64, 100, 1000])
def test_policy_forward_matches_oracle(sg, n):
    import torch
    w = synth.path_rollout(8)
    sim = sg.from_workload(w)
    o = oracle.Oracle(w.robot, w.task, w.policy)
    rng = np.random.default_rng(n)
    x = rng.normal(0, 1, (24, n)).astype(np.float32)
    x[:7] *= 1.5
    out = host(sim.policy_forward(torch.from_numpy(x).cuda()))
    ref = o.mlp(x.astype(np.float64), emulate=True)
    check_policy_outputs(out, ref)
    # the exact (un-quantised) network is within BF16 quantisation error
    ex = o.mlp(x.astype(np.float64), emulate=False)
    assert np.abs(out - ex).max() < 0.05


def _replay_rollout(sg, w, T, n_rollouts=1, team=1):
    import torch
    sim = sg.from_workload(w)
    sim.set_team(team)
    o = oracle.Oracle(w.robot, w.task, w.policy)
    N, J, W = w.robot.n_env, w.robot.max_dof, 2 * w.robot.max_dof + 10
    sigma = np.exp(w.policy.log_std)
    prog = w.task.progress0.astype(np.int32).copy()
    step0 = 0
    for r in range(n_rollouts):
        b = sim.rollout(T)
        obs, act, logp = host(b["obs"]), host(b["act"]), host(b["logp"])
        rew, done, val = host(b["rew"]), b["done"].cpu().numpy(), host(b["val"])
        adv, ret = host(b["adv"]), host(b["ret"])
        for t in range(T + 1):
            mv = o.mlp(obs[t], emulate=True)
            check_policy_outputs(val[t][None], mv[J][None], w.policy)
            if t == T:
                break
            eps = oracle.noise(w.seed, step0 + t, J, N)
            check_policy_outputs(act[t], mv[:J] + sigma[:, None] * eps, w.policy)
            lp = (-0.5 * eps ** 2 - w.policy.log_std[:, None] - 0.5 * np.log(2 * np.pi)).sum(0)
            np.testing.assert_allclose(logp[t], lp, rtol=1e-5, atol=1e-4)
            q, qd = obs[t][:J], obs[t][J:2 * J]
            qn, qdn, prn, rw, dn, ob = o.step(act[t], q, qd, prog)
            assert np.array_equal(done[t], dn), t
            assert np.abs(rew[t] - rw).max() <= 2e-4, (t, np.abs(rew[t] - rw).max())
            scale = np.maximum(1.0, np.abs(ob))
            assert (np.abs(obs[t + 1] - ob) / scale).max() <= 2e-3, (t, (np.abs(obs[t + 1] - ob) / scale).max())
            prog = prn
        ra, rr = oracle.gae(rew, val, done, 0.99, 0.95)
        np.testing.assert_allclose(adv, ra, rtol=1e-5, atol=1e-4)
        np.testing.assert_allclose(ret, rr, rtol=1e-5, atol=1e-4)
        step0 += T
    # the state left behind continues the last observation
    q, qd, pr, rs = sim.get_state()
    assert rs == step0
    np.testing.assert_array_equal(host(q), obs[T][:J])
    np.testing.assert_array_equal(host(qd), obs[T][J:2 * J])
    np.testing.assert_array_equal(pr.cpu().numpy(), prog)
    sim.synchronize()
    return b


def test_rollout_replay_ragged(sg):
    # 300 envs: four full waves and a partial one
    w = synth.path_rollout(300)
    _replay_rollout(sg, w, 32, n_rollouts=2)


def test_rollout_single_env_and_short(sg):
    w = synth.path_rollout(1)
    _replay_rollout(sg, w, 5)


def test_rollout_episode_ends_inside(sg):
    # progress0 near the episode length: time-outs (bits 0|1) fall inside the rollout
    w = synth.path_rollout(128)
    w.task.progress0[:] = np.arange(128) % 8 + 120
    b = _replay_rollout(sg, w, 16)
    d = b["done"].cpu().numpy()
    assert ((d & 3) == 3).any(axis=0).all()


def test_rollout_deterministic(sg):
    w = synth.path_rollout(200)
    a = sg.from_workload(w).rollout(8)
    b = sg.from_workload(w).rollout(8)
    for k in a:
        assert np.array_equal(a[k].cpu().numpy(), b[k].cpu().numpy()), k


def test_rollout_prefix_stable(sg):
    """Env i's rollout does not depend on how many envs run."""
    small = synth.path_rollout(70)
    big = synth.path_rollout(333)
    a = sg.from_workload(small).rollout(6)
    b = sg.from_workload(big).rollout(6)
    for k in ("act", "rew", "val", "logp"):
        assert np.array_equal(a[k].cpu().numpy(), b[k].cpu().numpy()[..., :70]), k
