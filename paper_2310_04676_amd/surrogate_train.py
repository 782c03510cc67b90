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


def drive_torques(robot, q, qd, a, h, torch):
    """The implicit-PD drive torque the control step forms for action a:
    tau = kp (q* - q - h qd) - kd qd, q* = mid + half clamp(a, -1, 1), per
    env column (robot arrays [J][N]); q, qd, a [J][n] device tensors whose
    column c belongs to env c % N."""
    dev = q.device
    N = robot.n_env
    f = lambda x: torch.as_tensor(np.asarray(x, np.float32), device=dev)
    kp, kd, lo, hi = f(robot.kp), f(robot.kd), f(robot.q_lo), f(robot.q_hi)
    n = q.shape[1]
    rep = lambda x: x.repeat(1, (n + N - 1) // N)[:, :n]
    kp, kd, lo, hi = rep(kp), rep(kd), rep(lo), rep(hi)
    qs = 0.5 * (hi + lo) + 0.5 * (hi - lo) * a.clamp(-1, 1)
    return kp * (qs - q - h * qd) - kd * qd


def generate(sim, n_samples, every=4, tau_sigma=20.0, seed=0, robot=None, pd_share=0.0):
    """States visited under random actions a ~ U(-1, 1) (held for `every`
    steps between snapshots); torques tau ~ N(0, tau_sigma^2) i.i.d., or --
    for a pd_share of each snapshot's columns (needs robot) -- the drive
    torque the step forms at that state for a fresh random action (the
    inputs the surrogate sees when it replaces the solve inside the step);
    labels qdd = (H + diag(arm))^-1 (tau - C)."""
    torch = sim.torch
    dev = sim.device
    J, N = sim.J, sim.N
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    h = float(robot.dt) / robot.substeps if robot is not None else 0.0
    n_pd = int(round(pd_share * N)) if robot is not None else 0
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
        if n_pd:
            # a random n_pd of the envs take the drive torque of a fresh
            # action (a different subset every snapshot)
            a2 = torch.rand(J, N, device=dev, generator=g) * 2 - 1
            pd = drive_torques(robot, qs, qds, a2, h, torch)
            perm = torch.randperm(N, device=dev, generator=g)[:n_pd]
            t[:, perm] = pd[:, perm]
        sl = slice(k * N, (k + 1) * N)
        q[:, sl] = qs
        qd[:, sl] = qds
        tau[:, sl] = t
        qdd[:, sl] = sim.forward_dynamics(qs, qds, t.contiguous(), SG_ARM_DRIVE)
    sl = slice(0, n_samples)
    return Dataset(q[:, sl].contiguous(), qd[:, sl].contiguous(), tau[:, sl].contiguous(), env[sl].contiguous(),
                   qdd[:, sl].contiguous())


def train(surr: Surrogate, data: Dataset, epochs=3, batch=4096, lr=1e-3, lr_final=1e-4, seed=0, log=None,
          val: Dataset = None, val_hist=None):
    """Adam over shuffled minibatches with a geometric learning-rate decay
    from lr to lr_final. Returns the per-epoch mean training loss; with val,
    appends each epoch's median relative qdd error on it to val_hist."""
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
        if val is not None and val_hist is not None:
            m = min(val.n, 16384)
            pred = surr.predict(val.q[:, :m].contiguous(), val.qd[:, :m].contiguous(), val.tau[:, :m].contiguous(),
                                val.env[:m].contiguous())
            err = qdd_error(pred.detach().cpu().numpy().astype(np.float64),
                            val.qdd[:, :m].detach().cpu().numpy().astype(np.float64))
            val_hist.append(float(np.median(err)))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.5f}")
    return hist


def qdd_error(pred, ref):
    """Relative error per sample: |pred - ref|_2 / max(|ref|_2, 1)."""
    num = np.linalg.norm(pred - ref, axis=0)
    den = np.maximum(np.linalg.norm(ref, axis=0), 1.0)
    return num / den


def fp64_report(sim64, surr, data: Dataset, thresholds=(1e-2, 3e-2, 1e-1, 3e-1)):
    """The surrogate against the exact FP64 solve of the library's FP64
    context sim64 (the same robot), on data whose columns are one snapshot
    of all sim64.N envs (env ids distinct): the relative qdd error, and the
    residual check the step applies, |RNEA(q, qd, qdd_hat) + arm qdd_hat -
    tau| / max(|tau|, 1e-3), evaluated in FP64: the accepted fraction at
    each threshold and the error of the accepted predictions."""
    torch = surr.sim.torch
    N = sim64.N
    m = min(data.n, N)
    env = data.env[:m].long()
    assert torch.unique(env).numel() == m
    pred = surr.predict(data.q[:, :m].contiguous(), data.qd[:, :m].contiguous(), data.tau[:, :m].contiguous(),
                        data.env[:m].contiguous())

    def scat(x):
        z = torch.zeros(sim64.J, N, dtype=torch.float64, device=x.device)
        z[:, env] = x[:, :m].double()
        return z

    q, qd, tau, ph = scat(data.q), scat(data.qd), scat(data.tau), scat(pred)
    exact = sim64.forward_dynamics(q, qd, tau, SG_ARM_DRIVE)[:, env]
    idn = sim64.inverse_dynamics(q, qd, ph)[:, env]
    rob = sim64.robot
    h = float(rob.dt) / rob.substeps
    arm = torch.as_tensor(h * np.asarray(rob.kd) + h * h * np.asarray(rob.kp), device=q.device)[:, env]
    res = idn + arm * ph[:, env] - tau[:, env]
    rel = (res.norm(dim=0) / tau[:, env].norm(dim=0).clamp_min(1e-3)).cpu().numpy()
    err = qdd_error(pred.detach().cpu().numpy().astype(np.float64), exact.cpu().numpy())
    out = {"samples": m, "qdd_rel_err_vs_fp64": {"median": float(np.median(err)), "p99": float(np.quantile(err, 0.99)),
                                                 "max": float(err.max())},
           "residual_median": float(np.median(rel)), "accepted": []}
    for t in thresholds:
        ok = rel <= t
        out["accepted"].append({"threshold": t, "fraction": float(ok.mean()),
                                "accepted_qdd_rel_err_median": float(np.median(err[ok])) if ok.any() else None,
                                "accepted_qdd_rel_err_max": float(err[ok].max()) if ok.any() else None})
    return out
