"""Pins of the PPO-update oracle: the Gaussian log-density and entropy against
scipy, hand-computed cases of the clipped policy and value objectives,
central finite differences of the loss for every parameter, advantage
normalisation against numpy, the gradient-norm clip and the first Adam step
in closed form."""
import numpy as np
import pytest
from scipy import stats

import oracle
import synth

DIMS = (5, 6, 4, 2)  # n_in, h1, h2, J


def _net(seed, dims=DIMS, scale=0.7):
    n_in, h1, h2, J = dims
    rng = np.random.default_rng(seed)
    W = [rng.normal(0, scale, (h1, n_in)), rng.normal(0, scale, (h2, h1)), rng.normal(0, scale, (J + 1, h2))]
    b = [rng.normal(0, 0.3, h1), rng.normal(0, 0.3, h2), rng.normal(0, 0.3, J + 1)]
    ls = rng.normal(-0.5, 0.2, J)
    return synth.Policy(dims=(n_in, h1, h2, J + 1), W=W, b=b, log_std=ls)


def _forward(pol, x):
    """mu, V through the oracle's policy MLP (pinned against brute force
    elsewhere)."""
    o = oracle.Oracle(synth.make_chain(1, 1, 0, dt=0.01, substeps=1), policy=pol)
    out = o.mlp(x, emulate=False)
    return out[:-1], out[-1]


def test_log_density_and_value_match_forward_and_scipy():
    pol = _net(1)
    p = oracle.ppo_flat(pol)
    rng = np.random.default_rng(2)
    for _ in range(5):
        x = rng.normal(0, 1, (5, 1))
        a = rng.normal(0, 1, (2, 1))
        mu, V = _forward(pol, x)
        # logp_old = 0 makes approx_kl = -logp for one sample
        _, _, st = oracle.ppo_grad(DIMS, p, x, a, [0.0], [0.3], [0.0], [0.0], cfg=dict(clip=1e9), emulate=False)
        ref = stats.norm.logpdf(a[:, 0], mu[:, 0], np.exp(pol.log_std)).sum()
        assert st["approx_kl"] == pytest.approx(-ref, rel=1e-12, abs=1e-12)
        # ret = v_old = 0 and an open clip: loss_v = V^2
        assert st["loss_v"] == pytest.approx(V[0] ** 2, rel=1e-12)
        assert st["entropy"] == pytest.approx(stats.norm.entropy(scale=np.exp(pol.log_std)).sum(), rel=1e-12)


def _bias_only(mu, V, ls):
    """J = 1 net whose outputs are its output bias: mu = b3[0], V = b3[1]."""
    dims = (3, 4, 4, 1)
    W = [np.zeros((4, 3)), np.zeros((4, 4)), np.zeros((2, 4))]
    b = [np.zeros(4), np.zeros(4), np.array([mu, V])]
    return dims, oracle.ppo_flat(synth.Policy(dims=(3, 4, 4, 2), W=W, b=b, log_std=np.array([ls])))


@pytest.mark.parametrize("r,A,live", [(1.5, 1.0, False), (1.5, -1.0, True), (0.5, 1.0, True),
                                      (0.5, -1.0, False), (1.1, 2.0, True), (0.9, -2.0, True)])
def test_clipped_policy_objective_hand_cases(r, A, live):
    mu, ls, a = 0.3, -0.2, 0.8
    dims, p = _bias_only(mu, 0.0, ls)
    logp = stats.norm.logpdf(a, mu, np.exp(ls))
    x = np.zeros((3, 1))
    loss, g, st = oracle.ppo_grad(dims, p, x, [[a]], [logp - np.log(r)], [A], [0.0], [0.0],
                                  cfg=dict(clip=0.2, c_v=0.0, c_e=0.0), emulate=False)
    rc = min(max(r, 0.8), 1.2)
    assert st["loss_pi"] == pytest.approx(-min(r * A, rc * A), rel=1e-12)
    assert st["clip_frac"] == (1.0 if abs(r - 1) > 0.2 else 0.0)
    # d loss / d mu = -A r (a - mu) / sigma^2 when the unclipped term is live
    off_b3 = p.size - 1 - 2
    sig2 = np.exp(2 * ls)
    want = -A * r * (a - mu) / sig2 if live else 0.0
    assert g[off_b3] == pytest.approx(want, rel=1e-12, abs=1e-15)
    # d loss / d log_std = -A r (u^2 - 1)
    u2 = (a - mu) ** 2 / sig2
    assert g[-1] == pytest.approx(-A * r * (u2 - 1) if live else 0.0, rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("V,Vold,R,loss,grad", [(2.0, 1.0, 0.0, 4.0, 4.0), (0.5, 1.0, 2.0, 2.25, -3.0),
                                                (1.5, 1.0, 3.0, 3.24, 0.0), (1.1, 1.0, 0.0, 1.21, 2.2)])
def test_clipped_value_loss_hand_cases(V, Vold, R, loss, grad):
    dims, p = _bias_only(0.0, V, 0.0)
    logp = stats.norm.logpdf(0.0, 0.0, 1.0)
    _, g, st = oracle.ppo_grad(dims, p, np.zeros((3, 1)), [[0.0]], [logp], [0.0], [R], [Vold],
                               cfg=dict(clip=0.2, c_v=0.5, c_e=0.0), emulate=False)
    assert st["loss_v"] == pytest.approx(loss, rel=1e-12)
    assert g[p.size - 2] == pytest.approx(0.5 * grad, rel=1e-12, abs=1e-15)


def test_entropy_gradient_is_minus_coefficient():
    dims, p = _bias_only(0.0, 0.0, 0.4)
    _, g, _ = oracle.ppo_grad(dims, p, np.zeros((3, 1)), [[0.0]], [0.0], [0.0], [0.0], [0.0],
                              cfg=dict(clip=0.2, c_v=0.0, c_e=0.25), emulate=False)
    # with A = 0 the policy term vanishes; only the entropy bonus is left
    assert g[-1] == pytest.approx(-0.25, rel=1e-14)


def test_gradient_matches_central_differences():
    pol = _net(3)
    p = oracle.ppo_flat(pol)
    B = 9
    rng = np.random.default_rng(4)
    x = rng.normal(0, 1, (5, B))
    a = rng.normal(0, 1, (2, B))
    mu, _ = _forward(pol, x)
    logp = stats.norm.logpdf(a, mu, np.exp(pol.log_std)[:, None]).sum(0)
    logp_old = logp - np.log(rng.uniform(0.6, 1.4, B))  # a mix of clipped and live ratios
    adv = rng.normal(0, 1, B)
    ret = rng.normal(0, 1, B)
    vold = rng.normal(0, 1, B)
    cfg = dict(clip=0.2, c_v=0.7, c_e=0.05)
    L0, g, st = oracle.ppo_grad(DIMS, p, x, a, logp_old, adv, ret, vold, cfg=cfg, emulate=False)
    assert 0 < st["clip_frac"] < 1
    h = 1e-6
    fd = np.zeros_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (oracle.ppo_grad(DIMS, p + e, x, a, logp_old, adv, ret, vold, cfg=cfg, emulate=False)[0] -
                 oracle.ppo_grad(DIMS, p - e, x, a, logp_old, adv, ret, vold, cfg=cfg, emulate=False)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-8)


def test_bf16_emulation_stays_close_to_exact():
    pol = _net(5, dims=(24, 256, 128, 7), scale=0.1)
    p = oracle.ppo_flat(pol)
    rng = np.random.default_rng(6)
    B = 16
    args = (rng.normal(0, 1, (24, B)), rng.normal(0, 1, (7, B)), rng.normal(-8, 1, B), rng.normal(0, 1, B),
            rng.normal(0, 1, B), rng.normal(0, 1, B))
    _, ge, _ = oracle.ppo_grad((24, 256, 128, 7), p, *args, emulate=True)
    _, gx, _ = oracle.ppo_grad((24, 256, 128, 7), p, *args, emulate=False)
    assert np.linalg.norm(ge - gx) <= 0.05 * np.linalg.norm(gx)


def test_advantage_normalisation_matches_numpy():
    a = np.random.default_rng(7).normal(3, 2, (4, 33))
    ref = (a - a.mean()) / (a.std(ddof=1) + 1e-8)
    np.testing.assert_allclose(oracle.ppo_normalise(a), ref, rtol=1e-13, atol=1e-13)


def test_grad_norm_clip_and_first_adam_step():
    g, n = oracle.clip_grad_norm(np.array([3.0, 4.0]), 1.0)
    assert n == 5.0
    np.testing.assert_allclose(g, np.array([0.6, 0.8]) * 5 / (5 + 1e-6), rtol=1e-15)
    g2, _ = oracle.clip_grad_norm(np.array([0.3, 0.4]), 1.0)
    np.testing.assert_array_equal(g2, [0.3, 0.4])
    # first Adam step: m_hat = g, v_hat = g^2, so w moves by -lr g / (|g| + eps)
    w0 = np.array([1.0, -2.0, 0.5])
    gg = np.array([0.1, -3.0, 1e-3])
    w1, _, _ = oracle.adam(w0, gg, np.zeros(3), np.zeros(3), 1e-3, 1)
    np.testing.assert_allclose(w1, w0 - 1e-3 * gg / (np.abs(gg) + 1e-8), rtol=1e-12)


def test_update_is_minibatch_gradient_clip_and_adam():
    """One epoch, one minibatch: the update equals gradient -> clip -> Adam on
    the normalised advantages."""
    pol = _net(8)
    p = oracle.ppo_flat(pol)
    T, N = 3, 4
    rng = np.random.default_rng(9)
    bufs = dict(obs=rng.normal(0, 1, (T + 1, 5, N)), act=rng.normal(0, 1, (T, 2, N)),
                logp=rng.normal(-2.5, 0.3, (T, N)), adv=rng.normal(0.5, 2, (T, N)), ret=rng.normal(0, 1, (T, N)),
                val=rng.normal(0, 1, (T + 1, N)))
    p1, m1, v1, t1, _ = oracle.ppo_update(DIMS, p, np.zeros_like(p), np.zeros_like(p), 0, bufs, T, N, epochs=1,
                                          n_mb=1, emulate=False)
    assert t1 == 1
    x = bufs["obs"][:T].transpose(1, 0, 2).reshape(5, T * N)
    a = bufs["act"].transpose(1, 0, 2).reshape(2, T * N)
    an = oracle.ppo_normalise(bufs["adv"]).ravel()
    _, g, _ = oracle.ppo_grad(DIMS, p, x, a, bufs["logp"].ravel(), an, bufs["ret"].ravel(), bufs["val"][:T].ravel(),
                              emulate=False)
    g, _ = oracle.clip_grad_norm(g, 1.0)
    ref, _, _ = oracle.adam(p, g, np.zeros_like(p), np.zeros_like(p), 1e-3, 1)
    np.testing.assert_allclose(p1, ref, rtol=1e-12, atol=1e-14)


# ---- the paper's Table II network: three hidden layers, ELU units -----------
DIMS3 = (5, 6, 5, 4, 2)  # n_in, h1, h2, h3, J


def _net3(seed, dims=DIMS3, scale=0.7):
    rng = np.random.default_rng(seed)
    sizes = list(dims[:-1]) + [dims[-1] + 1]
    W = [rng.normal(0, scale, (sizes[l + 1], sizes[l])) for l in range(len(sizes) - 1)]
    b = [rng.normal(0, 0.3, sizes[l + 1]) for l in range(len(sizes) - 1)]
    return synth.Policy(dims=tuple(sizes), W=W, b=b, log_std=rng.normal(-0.5, 0.2, dims[-1]), act="elu")


def _elu(z):
    return np.where(z > 0, z, np.expm1(np.minimum(z, 0)))


def test_elu3_forward_matches_brute_force():
    pol = _net3(11, dims=(24, 256, 128, 64, 7), scale=0.1)
    o = oracle.Oracle(synth.make_chain(1, 1, 0, dt=0.01, substeps=1), policy=pol)
    x = np.random.default_rng(12).normal(0, 1, (24, 40))
    h = x
    for l in range(3):
        h = _elu(pol.W[l] @ h + pol.b[l][:, None])
    out = pol.W[3] @ h + pol.b[3][:, None]
    np.testing.assert_allclose(o.mlp(x, emulate=False), out, rtol=1e-12, atol=1e-12)
    # ELU is the identity above zero and e^z - 1 below: a layer of positive
    # pre-activations passes them unchanged
    z = np.array([[0.5, -0.5, 2.0, -3.0]])
    np.testing.assert_allclose(_elu(z), [[0.5, np.exp(-0.5) - 1, 2.0, np.exp(-3.0) - 1]], rtol=1e-15)


def test_elu3_gradient_matches_central_differences_for_every_parameter():
    pol = _net3(13)
    p = oracle.ppo_flat(pol)
    n_in, J = DIMS3[0], DIMS3[-1]
    B = 9
    rng = np.random.default_rng(14)
    x = rng.normal(0, 1, (n_in, B))
    a = rng.normal(0, 1, (J, B))
    o = oracle.Oracle(synth.make_chain(1, 1, 0, dt=0.01, substeps=1), policy=pol)
    mu = o.mlp(x, emulate=False)[:J]
    logp = stats.norm.logpdf(a, mu, np.exp(pol.log_std)[:, None]).sum(0)
    logp_old = logp - np.log(rng.uniform(0.6, 1.4, B))
    adv, ret, vold = rng.normal(0, 1, B), rng.normal(0, 1, B), rng.normal(0, 1, B)
    cfg = dict(clip=0.2, c_v=0.7, c_e=0.05)
    L0, g, st = oracle.ppo_grad(DIMS3, p, x, a, logp_old, adv, ret, vold, cfg=cfg, emulate=False, act="elu")
    assert 0 < st["clip_frac"] < 1
    # the ELU's kink at 0 is not crossed by the differences (|z| >> h)
    assert p.size == 6 * 5 + 6 + 5 * 6 + 5 + 4 * 5 + 4 + 3 * 4 + 3 + 2
    h = 1e-6
    fd = np.zeros_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (oracle.ppo_grad(DIMS3, p + e, x, a, logp_old, adv, ret, vold, cfg=cfg, emulate=False, act="elu")[0]
                 - oracle.ppo_grad(DIMS3, p - e, x, a, logp_old, adv, ret, vold, cfg=cfg, emulate=False,
                                   act="elu")[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-8)
    # the same network with tanh units has a different gradient: the
    # activation is wired through
    _, gt, _ = oracle.ppo_grad(DIMS3, p, x, a, logp_old, adv, ret, vold, cfg=cfg, emulate=False, act="tanh")
    assert np.abs(gt - g).max() > 1e-3
