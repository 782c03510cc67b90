"""PPO update on the GPU against the FP64 oracle.

Tolerances:
* minibatch gradient vs the oracle's BF16-emulating gradient on the same
  rollout buffers: per parameter block rel L2 <= 2e-2 and cosine >= 0.999
  (the GPU's tanh and FP32 accumulation move a BF16-rounded activation or
  layer gradient to the neighbouring value now and then, as in the
  surrogate's gradient test); element by element, |g - g_emul| <=
  2 |g_emul - g_exact| + 1e-3 max|g_emul| per block: a flip changes one
  rounded operand by one BF16 unit, the size of the rounding itself, and
  flips touch a small fraction of the operands, so the kernel's distance
  from the emulating gradient stays below twice the whole quantisation
  effect (the emulating minus the exact FP64 gradient), which the oracle
  gives alone; loss statistics within 1e-3 relative.
* one Adam step: the GPU's own gradient, clipped and stepped by the
  oracle's Adam, matches the GPU update to FP32 rounding (rtol 1e-5).
* several steps: Adam's first steps move every parameter by about the
  learning rate with the sign of its gradient, so parameters whose gradient
  is below the gradient's error can flip; the update direction is compared
  by cosine >= 0.95 and the averaged statistics within 2e-2 relative. That
  a longer update is exactly the single step repeated is checked bit for
  bit (two one-epoch updates against one two-epoch update).
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

DIMS = (24, 256, 128, 7)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _setup(sg, n_env=256, T=8, seed=31):
    w = synth.path_rollout(n_env)
    w.policy = synth.make_policy(seed)
    sim = sg.Sim(w.robot, w.task, seed=w.seed)
    params = sg.ppo_flat_params(w.policy)
    ppo = sg.Ppo(sim, params, T * n_env)
    bufs = sim.rollout(T)
    return w, sim, ppo, params, bufs


def _rows(bufs, T, N, J=7):
    """Host arrays in sample order s = t N + e."""
    h = {k: host(v) for k, v in bufs.items()}
    x = h["obs"][:T].transpose(1, 0, 2).reshape(-1, T * N)
    a = h["act"].transpose(1, 0, 2).reshape(J, T * N)
    return h, x, a


def _blocks(p):
    n_in, h1, h2, J = DIMS
    sz = [h1 * n_in, h1, h2 * h1, h2, (J + 1) * h2, J + 1, J]
    o = np.cumsum([0] + sz)
    return [p[o[i]:o[i + 1]] for i in range(7)]


def test_trainer_installs_the_same_policy_as_set_policy(sg):
    import torch
    w = synth.path_rollout(300)
    w.policy = synth.make_policy(5)
    a = sg.Sim(w.robot, w.task, seed=w.seed)
    a.set_policy(w.policy)
    b = sg.Sim(w.robot, w.task, seed=w.seed)
    ppo = sg.Ppo(b, sg.ppo_flat_params(w.policy), 300 * 4)
    x = torch.randn(24, 500, device="cuda")
    assert torch.equal(a.policy_forward(x), b.policy_forward(x))
    ra, rb = a.rollout(4), b.rollout(4)
    for k in ra:
        assert torch.equal(ra[k], rb[k]), k
    ppo.close()


@pytest.mark.parametrize("perturb", [False, True])
def test_minibatch_gradient_matches_oracle(sg, perturb):
    import torch
    T, N = 8, 256
    w, sim, ppo, params, bufs = _setup(sg, N, T)
    if perturb:
        # move the behaviour log-densities so that a share of the ratios leaves
        # the clip interval on both sides
        g = torch.Generator(device="cuda").manual_seed(3)
        bufs["logp"] += 0.3 * torch.randn(bufs["logp"].shape, device="cuda", generator=g)
    idx = torch.randperm(T * N, device="cuda", generator=torch.Generator(device="cuda").manual_seed(1))[:1000]
    idx = idx.to(torch.int32)
    gg, st = ppo.grad(bufs, T, idx)
    h, x, a = _rows(bufs, T, N)
    an = oracle.ppo_normalise(h["adv"]).ravel()
    s = idx.cpu().numpy()
    L, gr, so = oracle.ppo_grad(DIMS, params.astype(np.float64), x[:, s], a[:, s], h["logp"].ravel()[s], an[s],
                                h["ret"].ravel()[s], h["val"][:T].ravel()[s], emulate=True)
    st = host(st)
    for k, name in enumerate(("loss_pi", "loss_v", "entropy", "approx_kl", "clip_frac")):
        assert abs(st[k] - so[name]) <= 1e-3 * max(1.0, abs(so[name])) + 1e-5, (name, st[k], so[name])
    if perturb:
        assert 0.05 < so["clip_frac"] < 0.95
    _, gx, _ = oracle.ppo_grad(DIMS, params.astype(np.float64), x[:, s], a[:, s], h["logp"].ravel()[s], an[s],
                               h["ret"].ravel()[s], h["val"][:T].ravel()[s], emulate=False)
    for i, (gb, rb, xb) in enumerate(zip(_blocks(host(gg)), _blocks(gr), _blocks(gx))):
        rel = np.linalg.norm(gb - rb) / np.linalg.norm(rb)
        cos = (gb @ rb) / (np.linalg.norm(gb) * np.linalg.norm(rb))
        assert rel <= 2e-2 and cos >= 0.999, (i, rel, cos)
        bound = 2 * np.abs(rb - xb) + 1e-3 * np.abs(rb).max()
        assert np.all(np.abs(gb - rb) <= bound), (i, np.max(np.abs(gb - rb) / bound))
    assert abs(st[5] - np.linalg.norm(gr)) <= 2e-2 * np.linalg.norm(gr)
    ppo.close()


def test_minibatch_gradient_six_dof_chain(sg):
    """A 6-DOF RRPRRR reaching workload (22 inputs, 7 outputs): the
    narrower input and output layers, with a minibatch of 777 rows (six
    whole 128-row chunks of the fused front and a ragged one); the same
    criteria as the 7-DOF gradient test."""
    import torch
    T, N, J = 8, 256, 6
    dims = (2 * J + 10, 256, 128, J)
    w = synth.psm_like(N)
    w.policy = synth.make_policy(35, dims=(dims[0], 256, 128, J + 1))
    sim = sg.Sim(w.robot, w.task, seed=w.seed)
    params = sg.ppo_flat_params(w.policy)
    ppo = sg.Ppo(sim, params, T * N)
    bufs = sim.rollout(T)
    idx = torch.randperm(T * N, device="cuda", generator=torch.Generator(device="cuda").manual_seed(2))[:777]
    idx = idx.to(torch.int32)
    gg, st = ppo.grad(bufs, T, idx)
    h, x, a = _rows(bufs, T, N, J)
    an = oracle.ppo_normalise(h["adv"]).ravel()
    s = idx.cpu().numpy()
    args = (x[:, s], a[:, s], h["logp"].ravel()[s], an[s], h["ret"].ravel()[s], h["val"][:T].ravel()[s])
    _, gr, so = oracle.ppo_grad(dims, params.astype(np.float64), *args, emulate=True)
    _, gx, _ = oracle.ppo_grad(dims, params.astype(np.float64), *args, emulate=False)
    st = host(st)
    for k, name in enumerate(("loss_pi", "loss_v", "entropy", "approx_kl", "clip_frac")):
        assert abs(st[k] - so[name]) <= 1e-3 * max(1.0, abs(so[name])) + 1e-5, (name, st[k], so[name])
    n_in, h1, h2, _ = dims
    sz = [h1 * n_in, h1, h2 * h1, h2, (J + 1) * h2, J + 1, J]
    o = np.cumsum([0] + sz)
    for i in range(7):
        gb, rb, xb = host(gg)[o[i]:o[i + 1]], gr[o[i]:o[i + 1]], gx[o[i]:o[i + 1]]
        rel = np.linalg.norm(gb - rb) / np.linalg.norm(rb)
        cos = (gb @ rb) / (np.linalg.norm(gb) * np.linalg.norm(rb))
        assert rel <= 2e-2 and cos >= 0.999, (i, rel, cos)
        bound = 2 * np.abs(rb - xb) + 1e-3 * np.abs(rb).max()
        assert np.all(np.abs(gb - rb) <= bound), (i, np.max(np.abs(gb - rb) / bound))
    ppo.close()


def test_one_update_step_is_clip_and_adam_of_the_gradient(sg):
    T, N = 4, 256
    w, sim, ppo, params, bufs = _setup(sg, N, T, seed=32)
    cfg = dict(epochs=1, minibatches=1, max_grad_norm=0.5)
    g, _ = ppo.grad(bufs, T, cfg=cfg)
    ppo.update(bufs, T, cfg=cfg)
    p1 = ppo.params().astype(np.float64)
    gc, _ = oracle.clip_grad_norm(host(g), 0.5)
    ref, _, _ = oracle.adam(params.astype(np.float64), gc, np.zeros(params.size), np.zeros(params.size), 1e-3, 1)
    np.testing.assert_allclose(p1, ref, rtol=1e-5, atol=1e-7)
    # the rollout policy now is the updated one
    import torch
    x = torch.randn(24, 64, device="cuda")
    upd = synth.Policy(dims=(24, 256, 128, 8), W=[b.reshape(s) for b, s in zip(_blocks(p1)[0:6:2],
                                                                               [(256, 24), (128, 256), (8, 128)])],
                       b=[_blocks(p1)[k] for k in (1, 3, 5)], log_std=_blocks(p1)[6])
    ref_sim = sg.Sim(w.robot, w.task, seed=w.seed)
    upd.W = [oracle.round_bf16(W).astype(np.float32) for W in upd.W]
    upd.b = [b.astype(np.float32) for b in upd.b]
    upd.log_std = upd.log_std.astype(np.float32)
    ref_sim.set_policy(upd)
    assert torch.equal(sim.policy_forward(x), ref_sim.policy_forward(x))
    ppo.close()


def test_epochs_compose_exactly(sg):
    """An update of two epochs (one minibatch each) equals two one-epoch
    updates bit for bit (the Adam step count, the advantage statistics and
    the gathered rows carry over): with the single step pinned above to clip
    + Adam of the GPU's own gradient, every step of a longer update is that
    step."""
    T, N = 4, 128
    outs = []
    for split in (False, True):
        w, sim, ppo, params, bufs = _setup(sg, N, T, seed=36)
        if split:
            ppo.update(bufs, T, cfg=dict(epochs=1, minibatches=1))
            ppo.update(bufs, T, cfg=dict(epochs=1, minibatches=1))
        else:
            ppo.update(bufs, T, cfg=dict(epochs=2, minibatches=1))
        outs.append(ppo.params())
        ppo.close()
    np.testing.assert_array_equal(outs[0], outs[1])
    assert not np.array_equal(outs[0], params)


def test_update_matches_oracle(sg):
    import torch
    T, N = 4, 256
    w, sim, ppo, params, bufs = _setup(sg, N, T, seed=33)
    gen = torch.Generator(device="cuda").manual_seed(7)
    perm = torch.stack([torch.randperm(T * N, device="cuda", generator=gen) for _ in range(2)]).to(torch.int32)
    cfg = dict(epochs=2, minibatches=2)
    st = host(ppo.update(bufs, T, cfg=cfg, perm=perm))
    p1 = ppo.params().astype(np.float64)
    h = {k: host(v) for k, v in bufs.items()}
    p0 = params.astype(np.float64)
    pr, _, _, t, so = oracle.ppo_update(DIMS, p0, np.zeros_like(p0), np.zeros_like(p0), 0, h, T, N,
                                        perm=perm.cpu().numpy(), epochs=2, n_mb=2, emulate=True)
    assert t == 4
    d, dr = p1 - p0, pr - p0
    cos = (d @ dr) / (np.linalg.norm(d) * np.linalg.norm(dr))
    assert cos >= 0.95, cos
    for k, name in enumerate(("loss_pi", "loss_v", "entropy", "approx_kl", "clip_frac")):
        assert abs(st[k] - so[name]) <= 2e-2 * max(abs(so[name]), 1e-2), (name, st[k], so[name])
    ppo.close()


def test_in_order_update_equals_identity_permutation(sg):
    import torch
    T, N = 4, 128
    outs = []
    for use_perm in (False, True):
        w, sim, ppo, params, bufs = _setup(sg, N, T, seed=34)
        perm = None
        if use_perm:
            perm = torch.arange(T * N, device="cuda", dtype=torch.int32).repeat(2)
        ppo.update(bufs, T, cfg=dict(epochs=2, minibatches=4), perm=perm)
        outs.append(ppo.params())
        ppo.close()
    np.testing.assert_array_equal(outs[0], outs[1])


def test_training_raises_the_return(sg):
    """Rollout + update iterations on the path task: the mean reward of the
    last iterations beats that of the first ones."""
    import torch
    T, N = 32, 1024
    w = synth.path_rollout(N)
    w.policy = synth.make_policy(40)
    sim = sg.Sim(w.robot, w.task, seed=w.seed)
    ppo = sg.Ppo(sim, sg.ppo_flat_params(w.policy), T * N)
    bufs = sim.rollout_buffers(T)
    gen = torch.Generator(device="cuda").manual_seed(0)
    rews = []
    for it in range(40):
        sim.rollout(T, bufs)
        rews.append(float(bufs["rew"].mean()))
        perm = torch.stack([torch.randperm(T * N, device="cuda", generator=gen) for _ in range(5)]).to(torch.int32)
        ppo.update(bufs, T, perm=perm)
    first, last = np.mean(rews[:5]), np.mean(rews[-5:])
    assert last > first + 0.1 * abs(first), (first, last)
    ppo.close()


def test_bad_arguments_rejected(sg):
    T, N = 4, 100
    w, sim, ppo, params, bufs = _setup(sg, N, T, seed=35)
    with pytest.raises(sg.SgError):
        ppo.update(bufs, T, cfg=dict(minibatches=7))   # 400 % 7 != 0
    with pytest.raises(sg.SgError):
        ppo.update(bufs, 8, cfg=dict(minibatches=1))   # T N above max_samples
    with pytest.raises(sg.SgError):
        ppo.update(bufs, T, cfg=dict(clip=0.0))
    with pytest.raises(ValueError):
        sg.Ppo(sim, params[:-1], T * N)
    ppo.close()
