"""FP64 CPU oracle -- test infrastructure.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. The product path (the HIP library and
its binding) never does, and shares no code with it. Every function here
calls the plain C++ implementation in this directory (``oracle.cpp`` and the
headers it includes), which follows Featherstone's textbook for the dynamics
and the paper for the task, observation, reward, time-out and GAE rules.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_u8p = C.POINTER(C.c_uint8)


class _Robot(C.Structure):
    _fields_ = [("n_env", C.c_int32), ("max_dof", C.c_int32), ("n_dof", _ip),
                ("axis", _dp), ("offset", _dp), ("com", _dp), ("mass", _dp), ("inertia", _dp),
                ("kp", _dp), ("kd", _dp), ("q_lo", _dp), ("q_hi", _dp), ("q0", _dp), ("tip", _dp),
                ("dt", C.c_double), ("substeps", C.c_int32), ("gravity", C.c_double * 3), ("joint_type", _ip)]


class _Task(C.Structure):
    _fields_ = [("task", C.c_int32), ("n_waypoints", C.c_int32), ("dwell", C.c_int32),
                ("ep_len", C.c_int32), ("target", _dp), ("waypoints", _dp), ("trk_sigma", C.c_double),
                ("trk_offset", C.c_double), ("trk_reset_std", C.c_double), ("trk_centre", C.c_double * 3),
                ("chains", C.c_int32), ("rerand", C.c_int32), ("n_banks", C.c_int32),
                ("rand_centre", C.c_double * 3), ("rand_half", C.c_double)]


TASK_TRACK = 2


def _track_params(task):
    tr = getattr(task, "track", None) or {}
    return (float(tr.get("sigma", 0.0)), float(tr.get("offset", 0.0)), float(tr.get("reset_std", 0.0)),
            (C.c_double * 3)(*tr.get("centre", (0.0, 0.0, 0.0))))


def _rerand_params(task):
    rr = getattr(task, "rerand", None)
    if rr is None:
        return (0, 1, (C.c_double * 3)(0.0, 0.0, 0.0), 0.0)
    return (1, int(getattr(task, "n_banks", 1) or 1), (C.c_double * 3)(*rr.get("centre", (0.0, 0.0, 0.0))),
            float(rr.get("half", 0.0)))


class _Policy(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("dims", C.c_int32 * 5), ("W", _dp * 4), ("b", _dp * 4),
                ("log_std", _dp), ("act", C.c_int32)]


ACTS = {"tanh": 0, "elu": 1}


def _arch(dims, act):
    """PPO network code of the oracle: dims = (n_in, hidden sizes..., J)."""
    L = len(dims) - 2
    return (C.c_int * (L + 4))(L, dims[0], *dims[1:-1], dims[-1], ACTS[act])


def lib():
    global _lib
    if _lib is None:
        path = _build.build()
        _lib = C.CDLL(path)
        _lib.ora_round_bf16.restype = C.c_double
        _lib.ora_round_bf16.argtypes = [C.c_double]
        _lib.ora_noise.argtypes = [C.c_uint64, C.c_uint64, C.c_int, C.c_int, _dp]
        _lib.ora_rollout.argtypes = None
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=_dp):
    return None if a is None else a.ctypes.data_as(t)


class Oracle:
    """Holds contiguous float64 copies of a workload's robot and task arrays."""

    def __init__(self, robot, task=None, policy=None):
        self.robot = robot
        self.N, self.J = robot.n_env, robot.max_dof
        self.W = 2 * self.J + 10
        self._keep = []
        k = self._keep
        arr = {}
        for name in ("axis", "offset", "com", "mass", "inertia", "kp", "kd", "q_lo", "q_hi", "q0", "tip"):
            arr[name] = _f64(getattr(robot, name))
            k.append(arr[name])
        nd = np.ascontiguousarray(robot.n_dof, dtype=np.int32)
        jt = None if getattr(robot, "joint_type", None) is None else np.ascontiguousarray(robot.joint_type, np.int32)
        k.extend([nd, jt])
        self.r = _Robot(self.N, self.J, _ptr(nd, _ip), *[_ptr(arr[n]) for n in
                        ("axis", "offset", "com", "mass", "inertia", "kp", "kd", "q_lo", "q_hi", "q0", "tip")],
                        float(robot.dt), int(robot.substeps), (C.c_double * 3)(*robot.gravity), _ptr(jt, _ip))
        if task is not None:
            tgt = None if task.target is None else _f64(task.target)
            wps = None if task.waypoints is None else _f64(task.waypoints)
            k.extend([tgt, wps])
            self.t = _Task(task.task, task.n_waypoints, task.dwell, task.ep_len, _ptr(tgt), _ptr(wps),
                           *_track_params(task), int(getattr(task, "chains", 1) or 1), *_rerand_params(task))
        else:
            self.t = _Task(0, 0, 1, 0, None, None, 0.0, 0.0, 0.0, (C.c_double * 3)(0.0, 0.0, 0.0), 1, 0, 1,
                           (C.c_double * 3)(0.0, 0.0, 0.0), 0.0)
        self.seed = int(getattr(task, "seed", 0) or 0) if task is not None else 0
        self.p = None
        if policy is not None:
            Ws = [_f64(w) for w in policy.W]
            bs = [_f64(b) for b in policy.b]
            ls = _f64(policy.log_std)
            k.extend(Ws + bs + [ls])
            nl = len(policy.dims) - 1
            dims = list(policy.dims) + [0] * (5 - len(policy.dims))
            self.p = _Policy(nl, (C.c_int32 * 5)(*dims), (_dp * 4)(*([_ptr(w) for w in Ws] + [None] * (4 - nl))),
                             (_dp * 4)(*([_ptr(b) for b in bs] + [None] * (4 - nl))), _ptr(ls),
                             ACTS[getattr(policy, "act", "tanh")])

    # ---- dynamics -------------------------------------------------------
    def fk(self, q):
        out = np.zeros((3, self.N))
        lib().ora_fk(C.byref(self.r), _ptr(_f64(q)), _ptr(out))
        return out

    def fk_links(self, q):
        com = np.zeros((3, self.J, self.N))
        jw = np.zeros((3, self.J, self.N))
        R = np.zeros((9, self.J, self.N))
        lib().ora_fk_links(C.byref(self.r), _ptr(_f64(q)), _ptr(com), _ptr(jw), _ptr(R))
        return com, jw, R

    def rnea(self, q, qd, qdd):
        out = np.zeros((self.J, self.N))
        lib().ora_rnea(C.byref(self.r), _ptr(_f64(q)), _ptr(_f64(qd)), _ptr(_f64(qdd)), _ptr(out))
        return out

    def crba(self, q):
        out = np.zeros((self.N, self.J, self.J))
        lib().ora_crba(C.byref(self.r), _ptr(_f64(q)), _ptr(out))
        return out

    def aba(self, q, qd, tau, arm=None):
        out = np.zeros((self.J, self.N))
        a = None if arm is None else _f64(arm)
        lib().ora_aba(C.byref(self.r), _ptr(_f64(q)), _ptr(_f64(qd)), _ptr(_f64(tau)), _ptr(a), _ptr(out))
        return out

    def fd_crba(self, q, qd, tau, arm=None):
        out = np.zeros((self.J, self.N))
        a = None if arm is None else _f64(arm)
        bad = lib().ora_fd_crba(C.byref(self.r), _ptr(_f64(q)), _ptr(_f64(qd)), _ptr(_f64(tau)), _ptr(a),
                                _ptr(out))
        return out, bad

    def drive_armature(self):
        """arm = h kd + h^2 kp per joint [J][N] (the implicit-PD armature)."""
        h = self.robot.dt / self.robot.substeps
        return h * _f64(self.robot.kd) + h * h * _f64(self.robot.kp)

    # ---- environment -----------------------------------------------------
    def observe(self, q, qd, progress, goal_state=None):
        """goal_state [9][N] (tracking task): goal, goal velocity, centre."""
        obs = np.zeros((self.W, self.N))
        pr = np.ascontiguousarray(progress, dtype=np.int32)
        gs = None if goal_state is None else _f64(goal_state)
        lib().ora_observe(C.byref(self.r), C.byref(self.t), _ptr(_f64(q)), _ptr(_f64(qd)), _ptr(pr, _ip),
                          _ptr(obs), _ptr(gs))
        return obs

    def step(self, action, q, qd, progress, log_qdd=False, envs=None, threads=1, goal_state=None, seed=0, step=0):
        """One control step. Returns (q, qd, progress, reward, done, obs[, qdd_log]).
        Tracking task: goal_state [9][N] is updated in place with the draws of
        Philox counter (seed; env, step)."""
        q = _f64(q).copy()
        qd = _f64(qd).copy()
        pr = np.ascontiguousarray(progress, dtype=np.int32).copy()
        rew = np.zeros(self.N)
        done = np.zeros(self.N, dtype=np.uint8)
        obs = np.zeros((self.W, self.N))
        qlog = np.zeros((self.robot.substeps, self.J, self.N)) if log_qdd else None
        e0, e1 = (0, self.N) if envs is None else envs
        gs = None
        if goal_state is not None:
            assert goal_state.dtype == np.float64 and goal_state.flags.c_contiguous
            gs = goal_state
        lib().ora_step(C.byref(self.r), C.byref(self.t), _ptr(_f64(action)), _ptr(q), _ptr(qd), _ptr(pr, _ip),
                       _ptr(rew), _ptr(done, _u8p), _ptr(obs), _ptr(qlog), C.c_int(e0), C.c_int(e1),
                       C.c_int(threads), _ptr(gs), C.c_uint64(seed), C.c_uint64(step))
        out = (q, qd, pr, rew, done, obs)
        return out + (qlog,) if log_qdd else out

    def opcount_step(self, action, env=0):
        counts = (C.c_longlong * 10)()
        lib().ora_opcount_step(C.byref(self.r), C.byref(self.t), C.c_int(env), _ptr(_f64(action)), counts)
        names = ["add", "mul", "div", "sqrt", "trans"]
        step = dict(zip(names, counts[:5]))
        phys = dict(zip(names, counts[5:]))
        return step, phys

    # ---- learning side ---------------------------------------------------
    def mlp(self, x, emulate=True):
        B = x.shape[1]
        out = np.zeros((self.p.dims[self.p.n_layers], B))
        lib().ora_mlp_forward(C.byref(self.p), _ptr(_f64(x)), _ptr(out), C.c_int(B), C.c_int(int(emulate)))
        return out

    def rollout(self, T, seed, step0, q, qd, progress, obs0, gamma=0.99, lam=0.95, emulate=True, envs=None,
                threads=1, goal_state=None):
        N, J, W = self.N, self.J, self.W
        q = _f64(q).copy()
        qd = _f64(qd).copy()
        pr = np.ascontiguousarray(progress, dtype=np.int32).copy()
        obs = np.zeros((T + 1, W, N))
        obs[0] = obs0
        act = np.zeros((T, J, N))
        logp = np.zeros((T, N))
        rew = np.zeros((T, N))
        done = np.zeros((T, N), dtype=np.uint8)
        val = np.zeros((T + 1, N))
        adv = np.zeros((T, N))
        ret = np.zeros((T, N))
        e0, e1 = (0, N) if envs is None else envs
        lib().ora_rollout(C.byref(self.r), C.byref(self.t), C.byref(self.p), C.c_int(T), C.c_uint64(seed),
                          C.c_uint64(step0), C.c_double(gamma), C.c_double(lam), C.c_int(int(emulate)), _ptr(q),
                          _ptr(qd), _ptr(pr, _ip), _ptr(obs), _ptr(act), _ptr(logp), _ptr(rew), _ptr(done, _u8p),
                          _ptr(val), _ptr(adv), _ptr(ret), C.c_int(e0), C.c_int(e1), C.c_int(threads),
                          _ptr(goal_state))
        return dict(q=q, qd=qd, progress=pr, obs=obs, act=act, logp=logp, rew=rew, done=done, val=val, adv=adv,
                    ret=ret)


class _Surrogate(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("dims", _ip), ("W", C.POINTER(_dp)), ("b", C.POINTER(_dp)),
                ("mu_x", _dp), ("sd_x", _dp), ("mu_y", _dp), ("sd_y", _dp)]


class SurrogateRef:
    """FP64 reference of the learned forward-dynamics surrogate: ELU MLP on
    z-scored features, MSE loss on z-scored targets, chain-rule gradients,
    Adam. W[l] is [out][in], b[l] [out]; norm = (mu_x, sd_x, mu_y, sd_y)."""

    def __init__(self, W, b, norm):
        self.set(W, b, norm)

    def set(self, W, b, norm):
        self.Ws = [_f64(w) for w in W]
        self.bs = [_f64(x) for x in b]
        self.norm = [_f64(x) for x in norm]
        self.dims = np.array([self.Ws[0].shape[1]] + [w.shape[0] for w in self.Ws], dtype=np.int32)
        L = len(self.Ws)
        self._Wp = (_dp * L)(*[_ptr(w) for w in self.Ws])
        self._bp = (_dp * L)(*[_ptr(x) for x in self.bs])
        self.s = _Surrogate(L, _ptr(self.dims, _ip), C.cast(self._Wp, C.POINTER(_dp)), C.cast(self._bp, C.POINTER(_dp)),
                            *[_ptr(x) for x in self.norm])

    def forward(self, x_raw, emulate=False):
        B = x_raw.shape[1]
        out = np.zeros((self.dims[-1], B))
        outn = np.zeros((self.dims[-1], B))
        lib().ora_surrogate_forward(C.byref(self.s), _ptr(_f64(x_raw)), C.c_int(B), C.c_int(int(emulate)), _ptr(out),
                                    _ptr(outn))
        return out, outn

    def grad(self, x_raw, target, emulate=False):
        B = x_raw.shape[1]
        gW = np.zeros(sum(w.size for w in self.Ws))
        gb = np.zeros(sum(x.size for x in self.bs))
        f = lib().ora_surrogate_grad
        f.restype = C.c_double
        loss = f(C.byref(self.s), _ptr(_f64(x_raw)), _ptr(_f64(target)), C.c_int(B), C.c_int(int(emulate)), _ptr(gW),
                 _ptr(gb))
        outW, outb, ow, ob = [], [], 0, 0
        for w, x in zip(self.Ws, self.bs):
            outW.append(gW[ow:ow + w.size].reshape(w.shape))
            outb.append(gb[ob:ob + x.size])
            ow += w.size
            ob += x.size
        return loss, outW, outb


def surrogate_features(orc, q, qd, tau, env):
    """Raw features [13 J][B] of samples (q, qd, tau [J][B]) of envs env[B]."""
    B = q.shape[1]
    x = np.zeros((13 * orc.J, B))
    e = np.ascontiguousarray(env, dtype=np.int32)
    lib().ora_surrogate_features(C.byref(orc.r), _ptr(_f64(q)), _ptr(_f64(qd)), _ptr(_f64(tau)), _ptr(e, _ip),
                                 C.c_int(B), _ptr(x))
    return x


def adam(w, g, m, v, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
    w, m, v = _f64(w).copy(), _f64(m).copy(), _f64(v).copy()
    lib().ora_adam(C.c_int(w.size), _ptr(w), _ptr(_f64(g)), _ptr(m), _ptr(v), C.c_double(lr), C.c_double(beta1),
                   C.c_double(beta2), C.c_double(eps), C.c_int(t))
    return w, m, v


def residual(orc, q, qd, tau, qdd_hat, arm=None):
    rel = np.zeros(orc.N)
    a = None if arm is None else _f64(arm)
    lib().ora_residual(C.byref(orc.r), _ptr(_f64(q)), _ptr(_f64(qd)), _ptr(_f64(tau)), _ptr(_f64(qdd_hat)), _ptr(a),
                       _ptr(rel))
    return rel


OPCOUNT_PRIMITIVES = ("dot", "cross", "m3v3", "m3m3", "xform_motion", "xform_force_T", "crm", "crf", "si_mul",
                      "sdot", "congruence", "si_add", "axis_rotation")


def opcount_primitives():
    """Operation tallies of single spatial-algebra primitives on the op
    counter: {name: {add, mul, div, sqrt, trans}}."""
    out = np.zeros((len(OPCOUNT_PRIMITIVES), 5), dtype=np.int64)
    k = lib().ora_opcount_primitives(out.ctypes.data_as(C.POINTER(C.c_longlong)))
    assert k == len(OPCOUNT_PRIMITIVES)
    keys = ("add", "mul", "div", "sqrt", "trans")
    return {n: dict(zip(keys, map(int, out[i]))) for i, n in enumerate(OPCOUNT_PRIMITIVES)}


def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().ora_philox4x32_10(c, k, o)
    return [o[i] for i in range(4)]


def noise(seed, step, n, N):
    eps = np.zeros((n, N))
    lib().ora_noise(C.c_uint64(seed), C.c_uint64(step), C.c_int(n), C.c_int(N), _ptr(eps))
    return eps


def round_bf16(x):
    f = lib().ora_round_bf16
    return np.vectorize(lambda v: f(float(v)))(np.asarray(x, dtype=np.float64))


def gae(rew, val, done, gamma=0.99, lam=0.95):
    T, N = rew.shape
    adv = np.zeros((T, N))
    ret = np.zeros((T, N))
    lib().ora_gae(C.c_int(T), C.c_int(N), _ptr(_f64(rew)), _ptr(_f64(val)),
                  _ptr(np.ascontiguousarray(done, dtype=np.uint8), _u8p), C.c_double(gamma), C.c_double(lam),
                  _ptr(adv), _ptr(ret))
    return adv, ret


# ---- PPO update -------------------------------------------------------------
PPO_DEFAULTS = dict(clip=0.2, c_v=1.0, c_e=0.01, max_norm=1.0, lr=1e-3, beta1=0.9, beta2=0.999, adam_eps=1e-8)


def _ppo_cfg(cfg):
    c = dict(PPO_DEFAULTS)
    c.update(cfg or {})
    return (C.c_double * 8)(*[float(c[k]) for k in ("clip", "c_v", "c_e", "max_norm", "lr", "beta1", "beta2",
                                                       "adam_eps")])


def ppo_flat(policy):
    """Flat parameter vector W1, b1, W2, b2, W3, b3, log_std."""
    parts = []
    for W, b in zip(policy.W, policy.b):
        parts += [np.ravel(W), np.ravel(b)]
    parts.append(np.ravel(policy.log_std))
    return np.concatenate([_f64(p) for p in parts])


def ppo_grad(dims, p, x, a, logp_old, adv, ret, v_old, cfg=None, emulate=True, act="tanh"):
    """One minibatch: (loss, gradient [P], stats dict). dims = (n_in, hidden
    sizes..., J); x [n_in][B], a [J][B]."""
    B = x.shape[1]
    g = np.zeros(p.size)
    st = np.zeros(5)
    d = _arch(dims, act)
    f = lib().ora_ppo_grad
    f.restype = C.c_double
    loss = f(d, _ptr(_f64(p)), _ptr(_f64(x)), _ptr(_f64(a)), _ptr(_f64(logp_old)), _ptr(_f64(adv)), _ptr(_f64(ret)),
             _ptr(_f64(v_old)), C.c_int(B), _ppo_cfg(cfg), C.c_int(int(emulate)), _ptr(g), _ptr(st))
    return loss, g, dict(zip(("loss_pi", "loss_v", "entropy", "approx_kl", "clip_frac"), st))


def ppo_normalise(adv):
    a = _f64(adv).ravel()
    out = np.zeros_like(a)
    lib().ora_ppo_normalise(C.c_int(a.size), _ptr(a), _ptr(out))
    return out.reshape(np.shape(adv))


def clip_grad_norm(g, max_norm):
    g = _f64(g).copy()
    f = lib().ora_clip_grad_norm
    f.restype = C.c_double
    n = f(C.c_int(g.size), _ptr(g), C.c_double(max_norm))
    return g, n


def ppo_update(dims, p, m, v, t, bufs, T, N, perm=None, epochs=5, n_mb=4, cfg=None, emulate=True, act="tanh"):
    """Whole update on rollout buffers (dict of obs, act, logp, adv, ret, val
    arrays in the rollout layouts). Returns (p, m, v, t, stats)."""
    p, m, v = _f64(p).copy(), _f64(m).copy(), _f64(v).copy()
    tt = C.c_int(t)
    st = np.zeros(5)
    pm = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32)
    rc = lib().ora_ppo_update(_arch(dims, act), _ptr(p), _ptr(m), _ptr(v), C.byref(tt),
                              *[_ptr(_f64(bufs[k])) for k in ("obs", "act", "logp", "adv", "ret", "val")],
                              C.c_int(T), C.c_int(N), _ptr(pm, _ip), C.c_int(epochs), C.c_int(n_mb), _ppo_cfg(cfg),
                              C.c_int(int(emulate)), _ptr(st))
    if rc != 0:
        raise ValueError("ppo_update: T*N must be a multiple of n_mb")
    return p, m, v, tt.value, dict(zip(("loss_pi", "loss_v", "entropy", "approx_kl", "clip_frac"), st))


# ---- adjoint of an open-loop rollout -------------------------------------------
def adjoint(orc, T, act, q0, qd0, progress0=None, mass_scale=None, want_grad=True, threads=1):
    """Loss L [N] = sum_t |tip(q_{t+1}) - goal_t| of an open-loop rollout with
    actions act [T][J][N]; with want_grad also dL/da [T][J][N] and dL/dm
    [J][N]. mass_scale [J][N] multiplies link masses and inertias."""
    N, J = orc.N, orc.J
    loss = np.zeros(N)
    ga = np.zeros((T, J, N)) if want_grad else None
    gm = np.zeros((J, N)) if want_grad else None
    pr = None if progress0 is None else np.ascontiguousarray(progress0, dtype=np.int32)
    ms = None if mass_scale is None else _f64(mass_scale)
    lib().ora_adjoint(C.byref(orc.r), C.byref(orc.t), C.c_int(T), _ptr(_f64(act)), _ptr(_f64(q0)), _ptr(_f64(qd0)),
                      _ptr(pr, _ip), _ptr(ms), C.c_int(int(want_grad)), _ptr(loss), _ptr(ga), _ptr(gm),
                      C.c_int(threads))
    return (loss, ga, gm) if want_grad else loss
