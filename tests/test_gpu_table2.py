"""The paper's Table II policy (Sec. IV learning-dynamics benchmark: three
hidden layers of 256, 128 and 64 ELU units) through the HIP library against
the FP64 oracle: the policy network alone, the fused rollout replayed step
by step, the PPO minibatch gradient and a whole update. Tolerances as in
test_gpu_rollout.py and test_gpu_ppo.py (the BF16-flip share derived for
this network on the oracle side; gradients per block rel L2 <= 2e-2, cosine
>= 0.999 and element by element within twice the BF16 quantisation effect
plus 1e-3 of the block's largest entry)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

DIMS3 = (24, 256, 128, 64, 7)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _workload(n_env, seed=51):
    w = synth.path_rollout(n_env)
    w.policy = synth.make_policy(seed, dims=synth.TABLE2_DIMS, act="elu")
    return w


@pytest.mark.parametrize("n", [1, 100, 1000])
def test_policy_forward_matches_oracle(sg, n):
    import torch
    from test_gpu_rollout import check_policy_outputs
    w = _workload(8)
    sim = sg.from_workload(w)
    o = oracle.Oracle(w.robot, w.task, w.policy)
    rng = np.random.default_rng(n)
    x = rng.normal(0, 1, (24, n)).astype(np.float32)
    x[:7] *= 1.5
    out = host(sim.policy_forward(torch.from_numpy(x).cuda()))
    ref = o.mlp(x.astype(np.float64), emulate=True)
    check_policy_outputs(out, ref, w.policy)
    ex = o.mlp(x.astype(np.float64), emulate=False)
    assert np.abs(out - ex).max() < 0.05
    # the tanh network of the same widths differs: the activation is wired through
    tanh = synth.Policy(dims=w.policy.dims, W=w.policy.W, b=w.policy.b, log_std=w.policy.log_std, act="tanh")
    assert np.abs(oracle.Oracle(w.robot, w.task, tanh).mlp(x.astype(np.float64), emulate=True) - ref).max() > 1e-2


@pytest.mark.parametrize("team", [1, 0])
def test_rollout_replay(sg, team):
    """One wave per 64 envs (team 1), and the library's default (0), which
    for this network is the wave team with layer 1's weights read from the
    global image."""
    from test_gpu_rollout import _replay_rollout
    w = _workload(300)
    _replay_rollout(sg, w, 16, team=team)


def test_ppo_minibatch_gradient_matches_oracle(sg):
    import torch
    T, N = 8, 256
    w = _workload(N, seed=52)
    sim = sg.Sim(w.robot, w.task, seed=w.seed)
    sim.set_policy(w.policy)
    params = sg.ppo_flat_params(w.policy)
    ppo = sg.Ppo(sim, params, T * N, dims=synth.TABLE2_DIMS, act="elu")
    bufs = sim.rollout(T)
    idx = torch.randperm(T * N, device="cuda", generator=torch.Generator(device="cuda").manual_seed(1))[:1000]
    idx = idx.to(torch.int32)
    gg, st = ppo.grad(bufs, T, idx)
    h = {k: host(v) for k, v in bufs.items()}
    x = h["obs"][:T].transpose(1, 0, 2).reshape(-1, T * N)
    a = h["act"].transpose(1, 0, 2).reshape(7, T * N)
    an = oracle.ppo_normalise(h["adv"]).ravel()
    s = idx.cpu().numpy()
    args = (x[:, s], a[:, s], h["logp"].ravel()[s], an[s], h["ret"].ravel()[s], h["val"][:T].ravel()[s])
    L, gr, so = oracle.ppo_grad(DIMS3, params.astype(np.float64), *args, emulate=True, act="elu")
    _, gx, _ = oracle.ppo_grad(DIMS3, params.astype(np.float64), *args, emulate=False, act="elu")
    st = host(st)
    for k, name in enumerate(("loss_pi", "loss_v", "entropy", "approx_kl", "clip_frac")):
        assert abs(st[k] - so[name]) <= 1e-3 * max(1.0, abs(so[name])) + 1e-5, (name, st[k], so[name])
    sizes = [24, 256, 128, 64, 8]
    cuts = [0]
    for l in range(4):
        cuts += [cuts[-1] + sizes[l + 1] * sizes[l], cuts[-1] + sizes[l + 1] * sizes[l] + sizes[l + 1]]
    cuts.append(cuts[-1] + 7)
    g = host(gg)
    assert g.size == cuts[-1]
    for i in range(len(cuts) - 1):
        gb, rb, xb = (v[cuts[i]:cuts[i + 1]] for v in (g, gr, gx))
        rel = np.linalg.norm(gb - rb) / np.linalg.norm(rb)
        cos = (gb @ rb) / (np.linalg.norm(gb) * np.linalg.norm(rb))
        assert rel <= 2e-2 and cos >= 0.999, (i, rel, cos)
        bound = 2 * np.abs(rb - xb) + 1e-3 * np.abs(rb).max()
        assert np.all(np.abs(gb - rb) <= bound), (i, np.max(np.abs(gb - rb) / bound))
    ppo.close()


def test_ppo_update_matches_oracle_and_installs_the_policy(sg):
    import torch
    T, N = 4, 256
    w = _workload(N, seed=53)
    sim = sg.Sim(w.robot, w.task, seed=w.seed)
    sim.set_policy(w.policy)
    params = sg.ppo_flat_params(w.policy)
    ppo = sg.Ppo(sim, params, T * N, dims=synth.TABLE2_DIMS, act="elu")
    bufs = sim.rollout(T)
    gen = torch.Generator(device="cuda").manual_seed(7)
    perm = torch.stack([torch.randperm(T * N, device="cuda", generator=gen) for _ in range(2)]).to(torch.int32)
    cfg = dict(epochs=2, minibatches=2)
    st = host(ppo.update(bufs, T, cfg=cfg, perm=perm))
    p1 = ppo.params().astype(np.float64)
    h = {k: host(v) for k, v in bufs.items()}
    p0 = params.astype(np.float64)
    pr, _, _, t, so = oracle.ppo_update(DIMS3, p0, np.zeros_like(p0), np.zeros_like(p0), 0, h, T, N,
                                        perm=perm.cpu().numpy(), epochs=2, n_mb=2, emulate=True, act="elu")
    _, _, _, _, sx = oracle.ppo_update(DIMS3, p0, np.zeros_like(p0), np.zeros_like(p0), 0, h, T, N,
                                       perm=perm.cpu().numpy(), epochs=2, n_mb=2, emulate=False, act="elu")
    assert t == 4
    d, dr = p1 - p0, pr - p0
    cos = (d @ dr) / (np.linalg.norm(d) * np.linalg.norm(dr))
    assert cos >= 0.95, cos
    # statistics averaged over the minibatches: after the first Adam step the
    # parameters differ where the gradient is below its BF16 error (Adam's
    # first steps move every parameter by ~lr with the gradient's sign), so
    # each statistic may differ from the emulating oracle by up to twice the
    # whole BF16 effect on it (emulating minus exact update) plus 1e-3
    for k, name in enumerate(("loss_pi", "loss_v", "entropy", "approx_kl", "clip_frac")):
        bound = 2 * abs(so[name] - sx[name]) + 1e-3 * max(1.0, abs(so[name]))
        assert abs(st[k] - so[name]) <= bound, (name, st[k], so[name], sx[name])
    # the rollout policy is now the updated one
    sizes = [24, 256, 128, 64, 8]
    Ws, bs, o = [], [], 0
    for l in range(4):
        n = sizes[l + 1] * sizes[l]
        Ws.append(oracle.round_bf16(p1[o:o + n].reshape(sizes[l + 1], sizes[l])).astype(np.float32))
        bs.append(p1[o + n:o + n + sizes[l + 1]].astype(np.float32))
        o += n + sizes[l + 1]
    upd = synth.Policy(dims=tuple(sizes), W=Ws, b=bs, log_std=p1[o:o + 7].astype(np.float32), act="elu")
    ref_sim = sg.Sim(w.robot, w.task, seed=w.seed)
    ref_sim.set_policy(upd)
    x = torch.randn(24, 64, device="cuda")
    assert torch.equal(sim.policy_forward(x), ref_sim.policy_forward(x))
    ppo.close()


def test_unsupported_networks_rejected(sg):
    w = synth.path_rollout(8)
    sim = sg.Sim(w.robot, w.task)
    bad = synth.make_policy(1, dims=(24, 256, 128, 32, 8), act="elu")
    with pytest.raises(sg.SgError):
        sim.set_policy(bad)
    bad2 = synth.make_policy(1, dims=synth.TABLE2_DIMS, act="tanh")
    with pytest.raises(sg.SgError):
        sim.set_policy(bad2)
