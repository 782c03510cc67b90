"""Pins of the oracle's BF16-emulating paths (the surrogate MLP's forward and
backward, the PPO minibatch gradient): the matrix cores take BF16 operands
and accumulate in FP32, and the oracle's "emulate" mode rounds exactly those
operands to BF16 (round to nearest, ties to even) and keeps everything else
in FP64. What is pinned is where the roundings sit:

* hand cases with one operand off the BF16 grid at a time, whose emulated
  results follow from the BF16 grid alone (1 + 2^-9 rounds to 1, 1 + 3 2^-9
  to 1 + 2^-7, biases and activation derivatives are not rounded);
* random networks against a numpy pass written here, which rounds with an
  integer bit trick on the float64 pattern (itself checked against torch's
  float32 -> bfloat16 conversion) at the operand positions the definition
  names, forward and backward.
"""
import numpy as np
import pytest

import oracle
import synth

U = 2.0 ** -9  # a quarter of BF16's spacing above 1 (2^-7)


def bf16(x):
    """Round float64 values to the nearest BF16 value (8 significant bits),
    ties to even, by integer arithmetic on the float64 bit pattern: add
    half of the dropped range (minus one, plus the kept least significant
    bit) and clear the 45 dropped mantissa bits."""
    a = np.ascontiguousarray(x, dtype=np.float64)
    bits = a.view(np.uint64)
    drop = np.uint64(45)
    lsb = (bits >> drop) & np.uint64(1)
    r = (bits + (np.uint64((1 << 44) - 1) + lsb)) & ~np.uint64((1 << 45) - 1)
    out = r.view(np.float64)
    return np.where(np.isfinite(a) & (a != 0), out, a)


def test_bit_trick_rounding_matches_torch_on_float32_values():
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 3, 20000), rng.uniform(-1e-3, 1e-3, 5000),
                        np.array([1 + U, 1 + 2 * U, 1 + 3 * U, 1 - U / 2, -(1 + 2 * U), 3 * 2.0 ** -8])])
    x = x.astype(np.float32)
    # ties: values exactly halfway between BF16 neighbours, both parities
    ties = (np.arange(1, 200, dtype=np.float32) * np.float32(2 ** -7) + np.float32(1)) + np.float32(2 ** -8)
    x = np.concatenate([x, ties, -ties])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(bf16(x.astype(np.float64)), ref)
    np.testing.assert_array_equal(oracle.round_bf16(x.astype(np.float64)), ref)


# ---- surrogate: hand cases -------------------------------------------------------
def _net(W, b, mu_x=0.0, sd_x=1.0):
    W = [np.array(w, dtype=np.float64) for w in W]
    b = [np.array(x, dtype=np.float64) for x in b]
    F, O = W[0].shape[1], W[-1].shape[0]
    norm = (np.full(F, mu_x), np.full(F, sd_x), np.zeros(O), np.ones(O))
    return oracle.SurrogateRef(W, b, norm)


def test_surrogate_emulate_rounds_weights_and_inputs_not_biases():
    x = np.array([[1.0]])
    # weight off the grid: 1 + 2^-9 -> 1
    out, _ = _net([[[1 + U]]], [[0.0]]).forward(x, emulate=True)
    assert out[0, 0] == 1.0
    out, _ = _net([[[1 + U]]], [[0.0]]).forward(x, emulate=False)
    assert out[0, 0] == 1 + U
    # normalised input off the grid: (x - 0.5) / 0.25 = 1 + 3 2^-9 -> 1 + 2^-7
    xr = np.array([[0.5 + 0.25 * (1 + 3 * U)]])
    out, _ = _net([[[1.0]]], [[0.0]], mu_x=0.5, sd_x=0.25).forward(xr, emulate=True)
    assert out[0, 0] == 1 + 2 ** -7
    # the bias is added unrounded
    out, _ = _net([[[1.0]]], [[U / 4]]).forward(x, emulate=True)
    assert out[0, 0] == 1 + U / 4


def test_surrogate_emulate_rounds_hidden_activations():
    # z1 = 1 + 2^-9 (weight 1, input 1, unrounded bias 2^-9), elu(z1) = z1 is
    # rounded to 1 as the second layer's input; the output layer is linear
    net = _net([[[1.0]], [[3.0]]], [[U], [0.25]])
    out, _ = net.forward(np.array([[1.0]]), emulate=True)
    assert out[0, 0] == 3.0 + 0.25
    out, _ = net.forward(np.array([[1.0]]), emulate=False)
    assert out[0, 0] == 3.0 * (1 + U) + 0.25
    # a negative pre-activation: elu(z) = e^z - 1 is rounded too
    net = _net([[[1.0]], [[1.0]]], [[-1.5], [0.0]])
    out, _ = net.forward(np.array([[1.0]]), emulate=True)
    assert out[0, 0] == bf16(np.expm1(-0.5))


def test_surrogate_emulate_backward_rounds_the_output_gradient_for_products_only():
    # one sample, one output: L = (y - t)^2, dL/dy = 2 (y - t). With
    # y = 1 (W = 1, x = 1, b = 0) and t = 1 - (1 + U) / 2: dL/dy = 1 + 2^-9,
    # which the weight gradient sees rounded (to 1) and the bias gradient
    # exact
    t = np.array([[1 - (1 + U) / 2]])
    L, gW, gb = _net([[[1.0]]], [[0.0]]).grad(np.array([[1.0]]), t, emulate=True)
    assert gW[0][0, 0] == 1.0 * 1.0
    assert gb[0][0] == 1 + U
    # two layers: hidden z1 = 0.5 (elu' = 1), output weight W2 = 1 + 2^-9
    # (rounded to 1 in the product that carries the gradient back), output
    # gradient 2 (y - t) with y = round(W2) round(0.5) = 0.5
    net = _net([[[0.5]], [[1 + U]]], [[0.0], [0.0]])
    t = np.array([[0.5 - 1.5]])  # dL/dy = 3 (on the BF16 grid)
    L, gW, gb = net.grad(np.array([[1.0]]), t, emulate=True)
    assert gb[1][0] == 3.0 and gW[1][0, 0] == 3.0 * 0.5
    assert gb[0][0] == 3.0 * 1.0 * 1.0      # round(W2) * round(g) * elu'(0.5)
    assert gW[0][0, 0] == 3.0 * 1.0          # round(g1) * round(x)
    # a negative hidden pre-activation: elu'(z) = e^z, applied unrounded
    net = _net([[[1.0]], [[1.0]]], [[-1.5], [0.0]])
    y = bf16(np.expm1(-0.5))
    t = np.array([[y - 0.5]])  # dL/dy = 1
    L, gW, gb = net.grad(np.array([[1.0]]), t, emulate=True)
    assert gb[0][0] == np.exp(-0.5)
    assert gW[0][0, 0] == bf16(np.exp(-0.5)) * 1.0


# ---- surrogate: random networks against the numpy pass ----------------------------
def _np_surrogate(W, b, norm, x_raw, t_raw):
    """Emulated forward, MSE loss and backward written from the definition:
    every matrix-product operand (weights, layer inputs, the layer gradient
    carried into a product) rounded to BF16; biases, pre-activations, the
    ELU derivative and the accumulations in float64."""
    B = x_raw.shape[1]
    h = (x_raw - norm[0][:, None]) / norm[1][:, None]
    acts, pres = [], []
    for l in range(len(W)):
        a = bf16(h)
        z = bf16(W[l]) @ a + b[l][:, None]
        acts.append(a)
        pres.append(z)
        h = z if l == len(W) - 1 else np.where(z > 0, z, np.expm1(z))
    y = h
    tn = (t_raw - norm[2][:, None]) / norm[3][:, None]
    O = y.shape[0]
    loss = ((y - tn) ** 2).sum() / (B * O)
    g = 2.0 * (y - tn) / (B * O)
    gW, gb = [None] * len(W), [None] * len(W)
    for l in range(len(W) - 1, -1, -1):
        gr = bf16(g)
        gb[l] = g.sum(1)
        gW[l] = gr @ acts[l].T
        if l == 0:
            break
        z = pres[l - 1]
        g = (bf16(W[l]).T @ gr) * np.where(z > 0, 1.0, np.exp(z))
    return y, loss, gW, gb


@pytest.mark.parametrize("dims,seed", [((13, 9, 8, 5), 1), ((91, 32, 32, 32, 7), 2)])
def test_surrogate_emulate_matches_numpy_pass(dims, seed):
    rng = np.random.default_rng(seed)
    W = [rng.uniform(-1, 1, (dims[l + 1], dims[l])) / np.sqrt(dims[l]) for l in range(len(dims) - 1)]
    b = [rng.uniform(-0.2, 0.2, dims[l + 1]) for l in range(len(dims) - 1)]
    norm = (rng.normal(0, 1, dims[0]), rng.uniform(0.5, 2, dims[0]), rng.normal(0, 1, dims[-1]),
            rng.uniform(0.5, 2, dims[-1]))
    x = rng.normal(0, 2, (dims[0], 37))
    t = rng.normal(0, 2, (dims[-1], 37))
    ref = oracle.SurrogateRef(W, b, norm)
    _, outn = ref.forward(x, emulate=True)
    y, L, gW, gb = _np_surrogate(W, b, norm, x, t)
    np.testing.assert_allclose(outn, y, rtol=1e-12, atol=1e-13)
    L0, rW, rb = ref.grad(x, t, emulate=True)
    assert L0 == pytest.approx(L, rel=1e-12)
    for l in range(len(W)):
        np.testing.assert_allclose(rW[l], gW[l], rtol=1e-11, atol=1e-14)
        np.testing.assert_allclose(rb[l], gb[l], rtol=1e-11, atol=1e-14)
    # and the emulated network differs from the exact one (the roundings act)
    _, exn = ref.forward(x, emulate=False)
    assert np.abs(exn - outn).max() > 1e-4


# ---- PPO: random networks against the numpy pass -----------------------------------
def _np_ppo(dims, pol, x, a, logp_old, adv, ret, v_old, cfg):
    """Emulated PPO minibatch gradient from the definition (operands of every
    product in BF16: observations, weights, hidden activations, and the
    layer gradients carried into products; losses, tanh derivatives, biases
    and accumulations float64)."""
    n_in, h1, h2, J = dims
    W1, W2, W3 = pol.W
    b1, b2, b3 = pol.b
    ls = pol.log_std
    B = x.shape[1]
    xr = bf16(x)
    z1 = bf16(W1) @ xr + b1[:, None]
    a1 = bf16(np.tanh(z1))
    z2 = bf16(W2) @ a1 + b2[:, None]
    a2 = bf16(np.tanh(z2))
    out = bf16(W3) @ a2 + b3[:, None]
    mu, V = out[:J], out[J]
    sig = np.exp(ls)[:, None]
    u = (a - mu) / sig
    logp = (-0.5 * u * u - ls[:, None] - 0.5 * np.log(2 * np.pi)).sum(0)
    r = np.exp(logp - logp_old)
    eps = cfg["clip"]
    live = np.where(adv >= 0, r <= 1 + eps, r >= 1 - eps)
    dlogp = np.where(live, -adv * r / B, 0.0)
    g_ls = (dlogp[None, :] * (u * u - 1)).sum(1) - cfg["c_e"]
    d3 = np.zeros((J + 1, B))
    d3[:J] = dlogp[None, :] * u / sig
    dv = V - v_old
    Vc = v_old + np.clip(dv, -eps, eps)
    e1, e2 = (V - ret) ** 2, (Vc - ret) ** 2
    dV = np.where(e1 >= e2, 2 * (V - ret), np.where(np.abs(dv) <= eps, 2 * (Vc - ret), 0.0))
    d3[J] = cfg["c_v"] * dV / B
    g3 = bf16(d3)
    gW3, gb3 = g3 @ a2.T, d3.sum(1)
    d2 = (bf16(W3).T @ g3) * (1 - np.tanh(z2) ** 2)
    g2 = bf16(d2)
    gW2, gb2 = g2 @ a1.T, d2.sum(1)
    d1 = (bf16(W2).T @ g2) * (1 - np.tanh(z1) ** 2)
    g1 = bf16(d1)
    gW1, gb1 = g1 @ xr.T, d1.sum(1)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3, g_ls])


@pytest.mark.parametrize("dims,seed", [((5, 6, 4, 2), 3), ((24, 64, 32, 7), 4)])
def test_ppo_emulate_gradient_matches_numpy_pass(dims, seed):
    n_in, h1, h2, J = dims
    rng = np.random.default_rng(seed)
    W = [rng.normal(0, 0.7, (h1, n_in)), rng.normal(0, 0.7, (h2, h1)), rng.normal(0, 0.7, (J + 1, h2))]
    b = [rng.normal(0, 0.3, h1), rng.normal(0, 0.3, h2), rng.normal(0, 0.3, J + 1)]
    pol = synth.Policy(dims=(n_in, h1, h2, J + 1), W=W, b=b, log_std=rng.normal(-0.5, 0.2, J))
    p = oracle.ppo_flat(pol)
    B = 64
    x = rng.normal(0, 1, (n_in, B))
    a = rng.normal(0, 1, (J, B))
    logp_old = rng.normal(-J, 1.0, B)
    adv = rng.normal(0, 1, B)
    ret = rng.normal(0, 1, B)
    v_old = rng.normal(0, 1, B)
    cfg = dict(oracle.PPO_DEFAULTS)
    _, g, _ = oracle.ppo_grad(dims, p, x, a, logp_old, adv, ret, v_old, emulate=True)
    ref = _np_ppo(dims, pol, x, a, logp_old, adv, ret, v_old, cfg)
    np.testing.assert_allclose(g, ref, rtol=1e-10, atol=1e-13)
    _, gx, _ = oracle.ppo_grad(dims, p, x, a, logp_old, adv, ret, v_old, emulate=False)
    assert np.abs(gx - g).max() > 1e-6


def _np_ppo_deep(sizes, pol, x, a, logp_old, adv, ret, v_old, cfg, act):
    """The same emulated minibatch gradient for any depth and activation."""
    f = (lambda z: np.tanh(z)) if act == "tanh" else (lambda z: np.where(z > 0, z, np.expm1(np.minimum(z, 0))))
    df = (lambda z: 1 - np.tanh(z) ** 2) if act == "tanh" else (lambda z: np.where(z > 0, 1.0, np.exp(np.minimum(z, 0))))
    L = len(pol.W)
    J = sizes[-1] - 1
    B = x.shape[1]
    acts, zs = [bf16(x)], []
    for l in range(L):
        z = bf16(pol.W[l]) @ acts[-1] + pol.b[l][:, None]
        zs.append(z)
        acts.append(bf16(f(z)) if l + 1 < L else z)
    out = acts[-1]
    mu, V = out[:J], out[J]
    ls = pol.log_std
    sig = np.exp(ls)[:, None]
    u = (a - mu) / sig
    logp = (-0.5 * u * u - ls[:, None] - 0.5 * np.log(2 * np.pi)).sum(0)
    r = np.exp(logp - logp_old)
    eps = cfg["clip"]
    live = np.where(adv >= 0, r <= 1 + eps, r >= 1 - eps)
    dlogp = np.where(live, -adv * r / B, 0.0)
    g_ls = (dlogp[None, :] * (u * u - 1)).sum(1) - cfg["c_e"]
    d = np.zeros((J + 1, B))
    d[:J] = dlogp[None, :] * u / sig
    dv = V - v_old
    Vc = v_old + np.clip(dv, -eps, eps)
    e1, e2 = (V - ret) ** 2, (Vc - ret) ** 2
    dV = np.where(e1 >= e2, 2 * (V - ret), np.where(np.abs(dv) <= eps, 2 * (Vc - ret), 0.0))
    d[J] = cfg["c_v"] * dV / B
    parts = []
    for l in range(L - 1, -1, -1):
        gd = bf16(d)
        parts.append((gd @ acts[l].T, d.sum(1)))
        if l > 0:
            d = (bf16(pol.W[l]).T @ gd) * df(zs[l - 1])
    out = []
    for gW, gb in reversed(parts):
        out += [gW.ravel(), gb]
    return np.concatenate(out + [g_ls])


@pytest.mark.parametrize("dims,seed,act", [((5, 6, 5, 4, 2), 5, "elu"), ((24, 64, 32, 16, 7), 6, "elu"),
                                           ((5, 6, 4, 2), 7, "elu"), ((5, 6, 5, 4, 2), 8, "tanh")])
def test_ppo_emulate_gradient_matches_numpy_pass_any_depth(dims, seed, act):
    rng = np.random.default_rng(seed)
    sizes = list(dims[:-1]) + [dims[-1] + 1]
    W = [rng.normal(0, 0.7, (sizes[l + 1], sizes[l])) for l in range(len(sizes) - 1)]
    b = [rng.normal(0, 0.3, sizes[l + 1]) for l in range(len(sizes) - 1)]
    J = dims[-1]
    pol = synth.Policy(dims=tuple(sizes), W=W, b=b, log_std=rng.normal(-0.5, 0.2, J), act=act)
    p = oracle.ppo_flat(pol)
    B = 64
    x = rng.normal(0, 1, (dims[0], B))
    a = rng.normal(0, 1, (J, B))
    logp_old = rng.normal(-J, 1.0, B)
    adv, ret, v_old = rng.normal(0, 1, B), rng.normal(0, 1, B), rng.normal(0, 1, B)
    cfg = dict(oracle.PPO_DEFAULTS)
    _, g, _ = oracle.ppo_grad(dims, p, x, a, logp_old, adv, ret, v_old, emulate=True, act=act)
    ref = _np_ppo_deep(sizes, pol, x, a, logp_old, adv, ret, v_old, cfg, act)
    np.testing.assert_allclose(g, ref, rtol=1e-10, atol=1e-13)
