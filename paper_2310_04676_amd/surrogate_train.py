"""Data generation and training loop for the learned surrogate.

Orchestration only: the states come from the library's own environment step
(random PD targets, the paper's random-action protocol), the labels from its
forward-dynamics kernel with the drive armature, the gradient steps from its
BF16 matrix-core training kernels. Torch supplies device memory and the
random inputs (actions, torques, minibatch indices).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import SG_ARM_DRIVE, Surrogate


@dataclasses.dataclass
class Dataset:
    q: object      # [J][n] float32 device
    qd: object
    tau: object
    env: object    # [n] int32
    qdd: object    # [J][n] labels (FP32 ABA with the drive armature)

    @property
    def n(self):
        return self.q.shape[1]

    def split(self, n_val):
        a = Dataset(*[x[..., :-n_val].contiguous() for x in (self.q, self.qd, self.tau, self.env, self.qdd)])
        b = Dataset(*[x[..., -n_val:].contiguous() for x in (self.q, self.qd, self.tau, self.env, self.qdd)])
        return a, b


def generate(sim, n_samples, every=4, tau_sigma=20.0, seed=0):
    """States visited under random actions a ~ U(-1, 1) (held for `every`
    steps between snapshots), torques tau ~ N(0, tau_sigma^2) i.i.d., labels
    qdd = (H + diag(arm))^-1 (tau - C)."""
    torch = sim.torch
    dev = sim.device
    J, N = sim.J, sim.N
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    n_snap = (n_samples + N - 1) // N
    q = torch.empty(J, n_snap * N, device=dev)
    qd = torch.empty_like(q)
    tau = torch.empty_like(q)
    qdd = torch.empty_like(q)
    env = torch.arange(N, device=dev, dtype=torch.int32).repeat(n_snap)
    for k in range(n_snap):
        a = torch.rand(J, N, device=dev, generator=g) * 2 - 1
        for _ in range(every):
            sim.step(a)
        qs, qds, _, _ = sim.get_state()
        t = torch.randn(J, N, device=dev, generator=g) * tau_sigma
        sl = slice(k * N, (k + 1) * N)
        q[:, sl] = qs
        qd[:, sl] = qds
        tau[:, sl] = t
        qdd[:, sl] = sim.forward_dynamics(qs, qds, t.contiguous(), SG_ARM_DRIVE)
    sl = slice(0, n_samples)
    return Dataset(q[:, sl].contiguous(), qd[:, sl].contiguous(), tau[:, sl].contiguous(), env[sl].contiguous(),
                   qdd[:, sl].contiguous())


def train(surr: Surrogate, data: Dataset, epochs=3, batch=4096, lr=1e-3, lr_final=1e-4, seed=0, log=None):
    """Adam over shuffled minibatches with a geometric learning-rate decay
    from lr to lr_final. Returns the per-epoch mean training loss."""
    torch = surr.sim.torch
    dev = surr.sim.device
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    n = data.n
    steps = epochs * (n // batch)
    loss = torch.zeros(1, device=dev)
    hist = []
    it = 0
    for ep in range(epochs):
        perm = torch.randperm(n, device=dev, generator=g).to(torch.int32)
        acc = torch.zeros(1, device=dev)
        for b in range(n // batch):
            rate = lr * (lr_final / lr) ** (it / max(steps - 1, 1))
            idx = perm[b * batch:(b + 1) * batch]
            surr.train_step(data.q, data.qd, data.tau, data.env, data.qdd, idx, rate, loss)
            acc += loss
            it += 1
        hist.append(float(acc.item()) / (n // batch))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.5f}")
    return hist


def qdd_error(pred, ref):
    """Relative error per sample: |pred - ref|_2 / max(|ref|_2, 1)."""
    num = np.linalg.norm(pred - ref, axis=0)
    den = np.maximum(np.linalg.norm(ref, axis=0), 1.0)
    return num / den
