"""Python binding of the MI355X serial-chain simulator (``libsurgym.so``).

Argument marshalling only: every step of the method runs in the HIP
kernels behind the C interface declared in ``include/surgym.h``. PyTorch
provides device memory (tensors) and the current HIP stream. There is no
CPU fallback: importing this package raises if the library is not built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsurgym.so")

SG_OK, SG_E_INVAL, SG_E_UNSUPPORTED, SG_E_HIP, SG_E_STATE, SG_E_NOMEM = 0, -1, -2, -3, -4, -5
SG_F32, SG_F64 = 0, 1
SG_TASK_REACH, SG_TASK_PATH = 0, 1
SG_ARM_NONE, SG_ARM_DRIVE = 0, 1
DONE_ENDED, DONE_TIMEOUT, DONE_NONFINITE = 1, 2, 4

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_vp = C.c_void_p


class RobotDesc(C.Structure):
    _fields_ = [("n_env", C.c_int32), ("max_dof", C.c_int32), ("n_dof", _ip), ("dtype", C.c_int32),
                ("axis", _dp), ("offset", _dp), ("com", _dp), ("mass", _dp), ("inertia", _dp), ("kp", _dp),
                ("kd", _dp), ("q_lo", _dp), ("q_hi", _dp), ("q0", _dp), ("tip", _dp), ("dt", C.c_double),
                ("substeps", C.c_int32), ("gravity", C.c_double * 3), ("joint_type", _ip)]


class TaskDesc(C.Structure):
    _fields_ = [("task", C.c_int32), ("n_waypoints", C.c_int32), ("dwell", C.c_int32), ("ep_len", C.c_int32),
                ("target", _dp), ("waypoints", _dp), ("progress0", _ip), ("seed", C.c_uint64),
                ("track_sigma", C.c_double), ("track_offset", C.c_double), ("track_reset_std", C.c_double),
                ("track_centre", C.c_double * 3), ("chains_per_env", C.c_int32), ("rerandomize", C.c_int32),
                ("n_banks", C.c_int32), ("rand_centre", C.c_double * 3), ("rand_half_width", C.c_double)]


class PolicyArch(C.Structure):
    _fields_ = [("n_hidden", C.c_int32), ("hidden", C.c_int32 * 3), ("act", C.c_int32)]


SG_ACT_TANH, SG_ACT_ELU = 0, 1


def policy_arch(dims, act="tanh"):
    """sg_policy_arch of a network dims = (n_in, hidden sizes..., n_out)."""
    hidden = list(dims[1:-1])
    return PolicyArch(len(hidden), (C.c_int32 * 3)(*(hidden + [0] * (3 - len(hidden)))),
                      SG_ACT_ELU if act == "elu" else SG_ACT_TANH)


class RolloutBufs(C.Structure):
    _fields_ = [("obs", _vp), ("act", _vp), ("logp", _vp), ("rew", _vp), ("done", _vp), ("val", _vp),
                ("adv", _vp), ("ret", _vp), ("gamma", C.c_float), ("lam", C.c_float)]


lib = C.CDLL(LIB_PATH)
lib.sg_version.restype = C.c_char_p
lib.sg_last_error.restype = C.c_char_p
lib.sg_last_error.argtypes = [_vp]
lib.sg_create.argtypes = [C.POINTER(RobotDesc), C.POINTER(TaskDesc), C.POINTER(_vp)]
lib.sg_destroy.argtypes = [_vp]
lib.sg_destroy.restype = None
lib.sg_set_stream.argtypes = [_vp, _vp]
lib.sg_synchronize.argtypes = [_vp]
lib.sg_reset.argtypes = [_vp]
lib.sg_step.argtypes = [_vp, _vp, _vp, _vp, _vp]
lib.sg_observe.argtypes = [_vp, _vp]
lib.sg_get_state.argtypes = [_vp, _vp, _vp, _vp, C.POINTER(C.c_uint64)]
lib.sg_set_state.argtypes = [_vp, _vp, _vp, _vp, C.c_uint64]
lib.sg_forward_dynamics.argtypes = [_vp, _vp, _vp, _vp, C.c_int32, _vp]
lib.sg_inverse_dynamics.argtypes = [_vp, _vp, _vp, _vp, _vp]
lib.sg_tip_position.argtypes = [_vp, _vp, _vp]
lib.sg_set_policy.argtypes = [_vp, C.POINTER(PolicyArch), _vp, _vp, _vp]
lib.sg_policy_forward.argtypes = [_vp, _vp, C.c_int32, _vp]
lib.sg_rollout.argtypes = [_vp, C.c_int32, C.POINTER(RolloutBufs)]
lib.sg_gae.argtypes = [_vp, C.c_int32, C.c_int32, _vp, _vp, _vp, C.c_float, C.c_float, _vp, _vp]


lib.sg_surrogate_create.argtypes = [_vp, C.c_int32, C.POINTER(_vp)]
lib.sg_surrogate_destroy.argtypes = [_vp]
lib.sg_surrogate_destroy.restype = None
lib.sg_surrogate_set_params.argtypes = [_vp, _vp, _vp]
lib.sg_surrogate_get_params.argtypes = [_vp, _vp, _vp]
lib.sg_surrogate_fit_norm.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, C.c_int32]
lib.sg_surrogate_grad.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, C.c_int32, _vp, C.c_int32, _vp, _vp]
lib.sg_surrogate_train_step.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, C.c_int32, _vp, C.c_int32, C.c_float, _vp]
lib.sg_surrogate_predict.argtypes = [_vp, _vp, _vp, _vp, _vp, C.c_int32, _vp]
lib.sg_surrogate_step.argtypes = [_vp, _vp, _vp, _vp, _vp, C.c_float, _vp]


class SgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"status {status}: {msg}")
        self.status = status


def version() -> str:
    return lib.sg_version().decode()


def _check(st):
    if st != SG_OK:
        raise SgError(st, lib.sg_last_error(None).decode())


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=_dp):
    return None if a is None else a.ctypes.data_as(t)


def _dptr(t, dtype=None):
    """Device pointer of a contiguous torch tensor (None passes through);
    with dtype given, the tensor must have exactly that element type."""
    if t is None:
        return None
    if not (t.is_cuda and t.is_contiguous()):
        raise TypeError("expected a contiguous device tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected a {dtype} tensor, got {t.dtype}")
    return t.data_ptr()


def make_descs(robot, task, dtype, seed=0):
    """ctypes descriptions (and the arrays they point at) from numpy arrays."""
    keep = []
    arrs = {}
    for name in ("axis", "offset", "com", "mass", "inertia", "kp", "kd", "q_lo", "q_hi", "q0", "tip"):
        arrs[name] = _f64(getattr(robot, name))
        keep.append(arrs[name])
    nd = np.ascontiguousarray(robot.n_dof, dtype=np.int32)
    jt = getattr(robot, "joint_type", None)
    jt = None if jt is None else np.ascontiguousarray(jt, dtype=np.int32)
    keep.extend([nd, jt])
    rd = RobotDesc(robot.n_env, robot.max_dof, _ptr(nd, _ip), dtype,
                   *[_ptr(arrs[n]) for n in ("axis", "offset", "com", "mass", "inertia", "kp", "kd", "q_lo",
                                             "q_hi", "q0", "tip")],
                   float(robot.dt), int(robot.substeps), (C.c_double * 3)(*robot.gravity), _ptr(jt, _ip))
    tgt = None if task.target is None else _f64(task.target)
    wps = None if task.waypoints is None else _f64(task.waypoints)
    p0 = None if task.progress0 is None else np.ascontiguousarray(task.progress0, dtype=np.int32)
    keep.extend([tgt, wps, p0])
    tr = getattr(task, "track", None) or {}
    td = TaskDesc(task.task, task.n_waypoints, task.dwell, task.ep_len, _ptr(tgt), _ptr(wps), _ptr(p0, _ip),
                  seed & 0xFFFFFFFFFFFFFFFF, float(tr.get("sigma", 0.0)), float(tr.get("offset", 0.0)),
                  float(tr.get("reset_std", 0.0)), (C.c_double * 3)(*tr.get("centre", (0.0, 0.0, 0.0))),
                  int(getattr(task, "chains", 1) or 1))
    td.n_banks = int(getattr(task, "n_banks", 1) or 1)
    rr = getattr(task, "rerand", None)
    if rr is not None:
        td.rerandomize = 1
        td.rand_centre = (C.c_double * 3)(*rr.get("centre", (0.0, 0.0, 0.0)))
        td.rand_half_width = float(rr.get("half", 0.0))
    return rd, td, keep


class Sim:
    """N environments on the current GPU (one ``sg_ctx``)."""

    def __init__(self, robot, task, dtype=np.float32, seed=0, device=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.N, self.J = robot.n_env, robot.max_dof
        self.W = 2 * self.J + 10
        self.tdtype = torch.float64 if dtype == np.float64 else torch.float32
        sgd = SG_F64 if dtype == np.float64 else SG_F32
        rd, td, keep = make_descs(robot, task, sgd, seed)
        ctx = _vp()
        with torch.cuda.device(self.device):
            st = lib.sg_create(C.byref(rd), C.byref(td), C.byref(ctx))
        if st != SG_OK:
            raise SgError(st, lib.sg_last_error(None).decode())
        self.ctx = ctx
        self.task = task
        self.robot = robot
        self.policy_dims = None

    def close(self):
        if getattr(self, "ctx", None):
            lib.sg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- plumbing ------------------------------------------------------------
    def _call(self, fn, *args):
        lib.sg_set_stream(self.ctx, self.torch.cuda.current_stream(self.device).cuda_stream)
        st = fn(self.ctx, *args)
        if st != SG_OK:
            raise SgError(st, lib.sg_last_error(self.ctx).decode())

    def _empty(self, *shape, dtype=None):
        return self.torch.empty(*shape, dtype=dtype or self.tdtype, device=self.device)

    def synchronize(self):
        self._call(lib.sg_synchronize)

    # -- environment ---------------------------------------------------------
    def reset(self):
        self._call(lib.sg_reset)

    def step(self, actions, obs=None, reward=None, done=None):
        """actions [J][N] -> (obs [W][N], reward [N], done [N] uint8)."""
        obs = self._empty(self.W, self.N) if obs is None else obs
        reward = self._empty(self.N) if reward is None else reward
        done = self._empty(self.N, dtype=self.torch.uint8) if done is None else done
        td, u8 = self.tdtype, self.torch.uint8
        self._call(lib.sg_step, _dptr(actions, td), _dptr(obs, td), _dptr(reward, td), _dptr(done, u8))
        return obs, reward, done

    def observe(self, obs=None):
        obs = self._empty(self.W, self.N) if obs is None else obs
        self._call(lib.sg_observe, _dptr(obs, self.tdtype))
        return obs

    def get_state(self):
        q = self._empty(self.J, self.N)
        qd = self._empty(self.J, self.N)
        pr = self._empty(self.N, dtype=self.torch.int32)
        rs = C.c_uint64()
        self._call(lib.sg_get_state, _dptr(q), _dptr(qd), _dptr(pr), C.byref(rs))
        return q, qd, pr, rs.value

    def set_state(self, q=None, qd=None, progress=None, rng_step=0):
        td = self.tdtype
        self._call(lib.sg_set_state, _dptr(q, td), _dptr(qd, td), _dptr(progress, self.torch.int32),
                   C.c_uint64(rng_step))

    def forward_dynamics(self, q, qd, tau, arm_mode=SG_ARM_DRIVE, out=None):
        out = self._empty(self.J, self.N) if out is None else out
        td = self.tdtype
        self._call(lib.sg_forward_dynamics, _dptr(q, td), _dptr(qd, td), _dptr(tau, td), C.c_int32(arm_mode),
                   _dptr(out, td))
        return out

    def inverse_dynamics(self, q, qd, qdd, out=None):
        out = self._empty(self.J, self.N) if out is None else out
        td = self.tdtype
        self._call(lib.sg_inverse_dynamics, _dptr(q, td), _dptr(qd, td), _dptr(qdd, td), _dptr(out, td))
        return out

    def tip_position(self, q, out=None):
        out = self._empty(3, self.N) if out is None else out
        self._call(lib.sg_tip_position, _dptr(q, self.tdtype), _dptr(out, self.tdtype))
        return out

    # -- learning side ----------------------------------------------------------
    def set_policy(self, policy):
        w = np.ascontiguousarray(policy.w_bf16_bits())
        b = np.ascontiguousarray(policy.b_f32())
        ls = np.ascontiguousarray(policy.log_std.astype(np.float32))
        arch = policy_arch(policy.dims, getattr(policy, "act", "tanh"))
        self._call(lib.sg_set_policy, C.byref(arch), w.ctypes.data_as(_vp), b.ctypes.data_as(_vp),
                   ls.ctypes.data_as(_vp))
        self.policy_dims = tuple(policy.dims)

    def policy_forward(self, x, out=None):
        n = x.shape[1]
        out = self._empty(self.J + 1, n, dtype=self.torch.float32) if out is None else out
        f32 = self.torch.float32
        self._call(lib.sg_policy_forward, _dptr(x, f32), C.c_int32(n), _dptr(out, f32))
        return out

    def rollout_buffers(self, T):
        t, f = self.torch, self.torch.float32
        return dict(obs=self._empty(T + 1, self.W, self.N, dtype=f), act=self._empty(T, self.J, self.N, dtype=f),
                    logp=self._empty(T, self.N, dtype=f), rew=self._empty(T, self.N, dtype=f),
                    done=self._empty(T, self.N, dtype=t.uint8), val=self._empty(T + 1, self.N, dtype=f),
                    adv=self._empty(T, self.N, dtype=f), ret=self._empty(T, self.N, dtype=f))

    def rollout(self, T, bufs=None, gamma=0.99, lam=0.95):
        bufs = self.rollout_buffers(T) if bufs is None else bufs
        f32, u8 = self.torch.float32, self.torch.uint8
        rb = RolloutBufs(*[_dptr(bufs[k], u8 if k == "done" else f32)
                           for k in ("obs", "act", "logp", "rew", "done", "val", "adv", "ret")],
                         gamma, lam)
        self._call(lib.sg_rollout, C.c_int32(T), C.byref(rb))
        return bufs

    def gae(self, rew, val, done, gamma=0.99, lam=0.95):
        T, n = rew.shape
        adv = self._empty(T, n, dtype=self.torch.float32)
        ret = self._empty(T, n, dtype=self.torch.float32)
        f32, u8 = self.torch.float32, self.torch.uint8
        self._call(lib.sg_gae, C.c_int32(T), C.c_int32(n), _dptr(rew, f32), _dptr(val, f32), _dptr(done, u8),
                   C.c_float(gamma), C.c_float(lam), _dptr(adv, f32), _dptr(ret, f32))
        return adv, ret


def surrogate_dims(J):
    return (13 * J, 256, 256, 256, J)


def pack_params(W, b):
    """Per layer W [out][in] then b [out], float32."""
    return np.concatenate([np.concatenate([np.asarray(w, np.float32).ravel(), np.asarray(x, np.float32).ravel()])
                           for w, x in zip(W, b)])


def unpack_params(flat, dims):
    W, b, o = [], [], 0
    for l in range(len(dims) - 1):
        n = dims[l + 1] * dims[l]
        W.append(flat[o:o + n].reshape(dims[l + 1], dims[l]))
        o += n
        b.append(flat[o:o + dims[l + 1]])
        o += dims[l + 1]
    return W, b


class Surrogate:
    """Learned forward-dynamics surrogate bound to a Sim (``sg_surrogate``)."""

    def __init__(self, sim: Sim, max_batch: int):
        self.sim = sim
        self.J = sim.J
        self.dims = surrogate_dims(self.J)
        h = _vp()
        sim._call(lib.sg_surrogate_create, C.c_int32(max_batch), C.byref(h))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib.sg_surrogate_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call(self, fn, *args):
        lib.sg_set_stream(self.sim.ctx, self.sim.torch.cuda.current_stream(self.sim.device).cuda_stream)
        st = fn(self.h, *args)
        if st != SG_OK:
            raise SgError(st, lib.sg_last_error(self.sim.ctx).decode())

    def set_params(self, W, b, norm=None):
        p = np.ascontiguousarray(pack_params(W, b))
        n = None if norm is None else np.ascontiguousarray(np.concatenate([np.asarray(x, np.float32) for x in norm]))
        self._call(lib.sg_surrogate_set_params, p.ctypes.data_as(_vp), None if n is None else n.ctypes.data_as(_vp))

    def get_params(self):
        nparam = sum(self.dims[l + 1] * self.dims[l] + self.dims[l + 1] for l in range(4))
        p = np.zeros(nparam, np.float32)
        F, J = self.dims[0], self.J
        n = np.zeros(2 * F + 2 * J, np.float32)
        self._call(lib.sg_surrogate_get_params, p.ctypes.data_as(_vp), n.ctypes.data_as(_vp))
        W, b = unpack_params(p, self.dims)
        return W, b, (n[:F], n[F:2 * F], n[2 * F:2 * F + J], n[2 * F + J:])

    def fit_norm(self, q, qd, tau, env, qdd):
        f, i = self.sim.torch.float32, self.sim.torch.int32
        self._call(lib.sg_surrogate_fit_norm, _dptr(q, f), _dptr(qd, f), _dptr(tau, f), _dptr(env, i), _dptr(qdd, f),
                   C.c_int32(q.shape[1]))

    def grad(self, q, qd, tau, env, qdd, idx=None, batch=None):
        torch = self.sim.torch
        nparam = sum(self.dims[l + 1] * self.dims[l] + self.dims[l + 1] for l in range(4))
        g = torch.empty(nparam, dtype=torch.float32, device=self.sim.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.sim.device)
        batch = q.shape[1] if batch is None else batch
        f, i = torch.float32, torch.int32
        self._call(lib.sg_surrogate_grad, _dptr(q, f), _dptr(qd, f), _dptr(tau, f), _dptr(env, i), _dptr(qdd, f),
                   C.c_int32(q.shape[1]), _dptr(idx, i), C.c_int32(batch), _dptr(g, f), _dptr(loss, f))
        return g, loss

    def train_step(self, q, qd, tau, env, qdd, idx, lr, loss=None):
        f, i = self.sim.torch.float32, self.sim.torch.int32
        self._call(lib.sg_surrogate_train_step, _dptr(q, f), _dptr(qd, f), _dptr(tau, f), _dptr(env, i),
                   _dptr(qdd, f), C.c_int32(q.shape[1]), _dptr(idx, i), C.c_int32(idx.shape[0]), C.c_float(lr),
                   _dptr(loss, f))

    def predict(self, q, qd, tau, env, out=None):
        n = q.shape[1]
        out = self.sim._empty(self.J, n, dtype=self.sim.torch.float32) if out is None else out
        f, i = self.sim.torch.float32, self.sim.torch.int32
        self._call(lib.sg_surrogate_predict, _dptr(q, f), _dptr(qd, f), _dptr(tau, f), _dptr(env, i), C.c_int32(n),
                   _dptr(out, f))
        return out

    def step(self, actions, threshold, obs=None, reward=None, done=None, n_fallback=None):
        s = self.sim
        obs = s._empty(s.W, s.N) if obs is None else obs
        reward = s._empty(s.N) if reward is None else reward
        done = s._empty(s.N, dtype=s.torch.uint8) if done is None else done
        f, u8 = s.torch.float32, s.torch.uint8
        self._call(lib.sg_surrogate_step, _dptr(actions, f), _dptr(obs, f), _dptr(reward, f), _dptr(done, u8),
                   C.c_float(threshold), _dptr(n_fallback, s.torch.int32))
        return obs, reward, done


def from_workload(w, device=None) -> Sim:
    sim = Sim(w.robot, w.task, dtype=w.dtype, seed=w.seed, device=device)
    if w.policy is not None and w.dtype == np.float32 and w.robot.max_dof <= 7:
        sim.set_policy(w.policy)
    return sim


SG_SCHED_PADDED, SG_SCHED_SORTED, SG_SCHED_PER_CLASS, SG_SCHED_PERSISTENT = 0, 1, 2, 3
SCHEDULE_NAMES = ("padded", "sorted", "per_class", "persistent")
lib.sg_set_schedule.argtypes = [_vp, C.c_int32]
lib.sg_get_schedule.argtypes = [_vp, C.POINTER(C.c_int32)]
lib.sg_set_team.argtypes = [_vp, C.c_int32]
lib.sg_get_team.argtypes = [_vp, C.POINTER(C.c_int32)]
lib.sg_autotune_step.argtypes = [_vp, _vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                 C.POINTER(C.c_float)]
lib.sg_tuning_export.argtypes = [C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]
lib.sg_tuning_import.argtypes = [C.c_char_p]


def _set_schedule(self, schedule):
    self._call(lib.sg_set_schedule, C.c_int32(schedule))


def _get_schedule(self):
    s = C.c_int32()
    self._call(lib.sg_get_schedule, C.byref(s))
    return s.value


CANDIDATE_NAMES = SCHEDULE_NAMES + ("padded_team",)


def _autotune_step(self, actions, trials=5):
    """Time every step schedule and mapping on these actions (state restored
    after each); the fastest becomes the context's schedule and mapping.
    Returns (schedule, waves per block, {candidate name: ms per step})."""
    best, team = C.c_int32(), C.c_int32()
    ms = (C.c_float * 5)()
    self._call(lib.sg_autotune_step, _dptr(actions, self.tdtype), C.c_int32(trials), C.byref(best),
               C.byref(team), ms)
    return best.value, team.value, {CANDIDATE_NAMES[i]: ms[i] for i in range(5) if ms[i] >= 0}


def tuning_export():
    """The autotuner's remembered choices of this process as text."""
    n = C.c_size_t()
    _check(lib.sg_tuning_export(None, 0, C.byref(n)))
    buf = C.create_string_buffer(n.value)
    _check(lib.sg_tuning_export(buf, n.value, C.byref(n)))
    return buf.value.decode()


def tuning_import(text):
    """Merge choices from tuning_export() of an earlier process."""
    _check(lib.sg_tuning_import(text.encode()))


def save_tuning(path):
    with open(path, "w") as f:
        f.write(tuning_export())


def load_tuning(path):
    with open(path) as f:
        tuning_import(f.read())


def _set_team(self, waves):
    self._call(lib.sg_set_team, C.c_int32(waves))


def _get_team(self):
    w = C.c_int32()
    self._call(lib.sg_get_team, C.byref(w))
    return w.value


Sim.set_schedule = _set_schedule
Sim.get_schedule = _get_schedule
Sim.set_team = _set_team
Sim.get_team = _get_team
Sim.autotune_step = _autotune_step


# ---- PPO update ---------------------------------------------------------------
class PpoConfig(C.Structure):
    _fields_ = [("clip", C.c_float), ("value_coef", C.c_float), ("entropy_coef", C.c_float),
                ("max_grad_norm", C.c_float), ("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("adam_eps", C.c_float), ("epochs", C.c_int32), ("minibatches", C.c_int32)]


PPO_DEFAULTS = dict(clip=0.2, value_coef=1.0, entropy_coef=0.01, max_grad_norm=1.0, lr=1e-3, beta1=0.9,
                    beta2=0.999, adam_eps=1e-8, epochs=5, minibatches=4)
PPO_STATS = ("loss_pi", "loss_v", "entropy", "approx_kl", "clip_frac", "grad_norm")

lib.sg_ppo_create.argtypes = [_vp, C.POINTER(PolicyArch), _vp, C.c_int32, C.POINTER(_vp)]
lib.sg_ppo_destroy.argtypes = [_vp]
lib.sg_ppo_destroy.restype = None
lib.sg_ppo_param_count.argtypes = [_vp]
lib.sg_ppo_param_count.restype = C.c_int32
lib.sg_ppo_get_params.argtypes = [_vp, _vp]
lib.sg_ppo_grad.argtypes = [_vp, _vp, C.c_int32, _vp, C.c_int32, _vp, _vp, _vp]
lib.sg_ppo_update.argtypes = [_vp, _vp, C.c_int32, _vp, _vp, _vp]


def ppo_flat_params(policy):
    """Flat FP32 parameter vector W1, b1, W2, b2, W3, b3, log_std."""
    parts = []
    for W, b in zip(policy.W, policy.b):
        parts += [np.asarray(W, np.float32).ravel(), np.asarray(b, np.float32).ravel()]
    parts.append(np.asarray(policy.log_std, np.float32).ravel())
    return np.ascontiguousarray(np.concatenate(parts), dtype=np.float32)


def _ppo_cfg(cfg):
    c = dict(PPO_DEFAULTS)
    c.update(cfg or {})
    return PpoConfig(*[c[k] for k, _ in PpoConfig._fields_])


class Ppo:
    """PPO trainer of a Sim's rollout policy (``sg_ppo``)."""

    def __init__(self, sim: Sim, params, max_samples: int, dims=None, act="tanh"):
        """dims = (n_in, hidden sizes..., J + 1) of the policy (default: the
        rollout's 256-128 tanh network); act its hidden activation."""
        self.sim = sim
        p = np.ascontiguousarray(params, dtype=np.float32)
        W, J = 2 * sim.J + 10, sim.J
        dims = tuple(dims) if dims is not None else (W, 256, 128, J + 1)
        want = sum(dims[l + 1] * dims[l] + dims[l + 1] for l in range(len(dims) - 1)) + J
        if p.size != want:
            raise ValueError(f"expected {want} parameters, got {p.size}")
        h = _vp()
        arch = policy_arch(dims, act)
        sim._call(lib.sg_ppo_create, C.byref(arch), p.ctypes.data_as(_vp), C.c_int32(max_samples), C.byref(h))
        self.h = h
        self.P = lib.sg_ppo_param_count(h)
        self.dims, self.act = dims, act
        sim.policy_dims = dims

    def close(self):
        if getattr(self, "h", None):
            lib.sg_ppo_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call(self, fn, *args):
        s = self.sim
        lib.sg_set_stream(s.ctx, s.torch.cuda.current_stream(s.device).cuda_stream)
        st = fn(self.h, *args)
        if st != SG_OK:
            raise SgError(st, lib.sg_last_error(s.ctx).decode())

    def params(self):
        out = np.zeros(self.P, dtype=np.float32)
        self._call(lib.sg_ppo_get_params, out.ctypes.data_as(_vp))
        return out

    def _bufs(self, bufs):
        f32, u8 = self.sim.torch.float32, self.sim.torch.uint8
        return RolloutBufs(*[_dptr(bufs[k], u8 if k == "done" else f32)
                             for k in ("obs", "act", "logp", "rew", "done", "val", "adv", "ret")], 0.99, 0.95)

    def grad(self, bufs, T, idx=None, rows=None, cfg=None):
        """Gradient of one minibatch: (grad [P], stats dict of device scalars)."""
        t = self.sim.torch
        rows = (idx.numel() if idx is not None else T * self.sim.N) if rows is None else rows
        g = t.empty(self.P, dtype=t.float32, device=self.sim.device)
        st = t.empty(8, dtype=t.float32, device=self.sim.device)
        rb = self._bufs(bufs)
        c = _ppo_cfg(cfg)
        self._call(lib.sg_ppo_grad, C.byref(rb), C.c_int32(T), None if idx is None else _dptr(idx, t.int32),
                   C.c_int32(rows), C.byref(c), _dptr(g, t.float32), _dptr(st, t.float32))
        return g, st

    def update(self, bufs, T, cfg=None, perm=None, stats=None):
        """One PPO update; returns the device stats tensor [8]."""
        t = self.sim.torch
        st = t.empty(8, dtype=t.float32, device=self.sim.device) if stats is None else stats
        rb = self._bufs(bufs)
        c = _ppo_cfg(cfg)
        self._call(lib.sg_ppo_update, C.byref(rb), C.c_int32(T), C.byref(c),
                   None if perm is None else _dptr(perm, t.int32), _dptr(st, t.float32))
        return st


# ---- differentiation ------------------------------------------------------------
lib.sg_adjoint.argtypes = [_vp, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp]
lib.sg_adjoint_static.argtypes = [_vp, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp]
lib.sg_adjoint_workspace_bytes.argtypes = [_vp, C.c_int32, C.c_int32]
lib.sg_adjoint_workspace_bytes.restype = C.c_int64
lib.sg_set_link_masses.argtypes = [_vp, _vp]


def _adjoint(self, actions, K=8, static=False):
    """Loss [N] and its gradients (g_act [T][J][N], g_mass [J][N]) of an
    open-loop rollout with actions [T][J][N] from the current state.
    static=True calls sg_adjoint_static (the library's fixed workspace, no
    device allocation; outputs are still allocated here)."""
    T = actions.shape[0]
    f32 = self.torch.float32
    loss = self._empty(self.N, dtype=f32)
    g_act = self._empty(T, self.J, self.N, dtype=f32)
    g_mass = self._empty(self.J, self.N, dtype=f32)
    self._call(lib.sg_adjoint_static if static else lib.sg_adjoint, C.c_int32(T), C.c_int32(K), _dptr(actions, f32), _dptr(loss, f32), _dptr(g_act, f32),
               _dptr(g_mass, f32))
    return loss, g_act, g_mass


def _adjoint_workspace_bytes(self, T, K):
    return int(lib.sg_adjoint_workspace_bytes(self.ctx, C.c_int32(T), C.c_int32(K)))


def _set_link_masses(self, masses):
    self._call(lib.sg_set_link_masses, _dptr(masses, self.tdtype))


Sim.adjoint = _adjoint
Sim.adjoint_workspace_bytes = _adjoint_workspace_bytes
Sim.set_link_masses = _set_link_masses

_RolloutLoss = None


def rollout_loss(sim, actions, masses, K=8):
    """Differentiable loss [N] of an open-loop rollout: a
    torch.autograd.Function whose inputs are the actions [T][J][N] and the
    link masses [J][N] (installed into the context by the forward pass);
    the backward pass returns the adjoint's gradients."""
    global _RolloutLoss
    if _RolloutLoss is None:
        import torch

        class RolloutLossFn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, act, m, sim_, k):
                sim_.set_link_masses(m.detach().contiguous())
                loss, ga, gm = sim_.adjoint(act.detach().contiguous(), k)
                ctx.save_for_backward(ga, gm)
                return loss

            @staticmethod
            def backward(ctx, gl):
                ga, gm = ctx.saved_tensors
                return ga * gl[None, None, :], gm * gl[None, :], None, None

        _RolloutLoss = RolloutLossFn
    return _RolloutLoss.apply(actions, masses, sim, K)


# ---- tracking task ------------------------------------------------------------------
SG_TASK_REACH, SG_TASK_PATH, SG_TASK_TRACK = 0, 1, 2
lib.sg_get_goal_state.argtypes = [_vp, _vp]
lib.sg_set_goal_state.argtypes = [_vp, _vp]


def _goal_rows(task):
    if task.task == SG_TASK_TRACK:
        return 9
    if getattr(task, "rerand", None) is not None:
        return 3 if task.task == SG_TASK_REACH else 1
    return 0


def _get_goal_state(self):
    """The envs' goal state: tracking [9][N] (goal, goal velocity, episode
    centre); re-randomised reach [3][N] (target); re-randomised path [1][N]
    (waypoint-set index)."""
    gs = self._empty(max(_goal_rows(self.task), 1), self.N)
    self._call(lib.sg_get_goal_state, _dptr(gs))
    return gs


def _set_goal_state(self, gs):
    self._call(lib.sg_set_goal_state, _dptr(gs, self.tdtype))


Sim.get_goal_state = _get_goal_state
Sim.set_goal_state = _set_goal_state


# ---- measured device peaks -----------------------------------------------------------
lib.sg_measure_peaks.argtypes = [C.POINTER(C.c_double)] * 4


def measure_peaks():
    """Measured rates of the current device: FP32 FMA without packed FP32
    (whole chip, TFLOP/s; one wave alone on its SIMD, GFLOP/s per wave),
    BF16 MFMA (TFLOP/s) and a device copy (GB/s)."""
    f, fw, m, c = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    st = lib.sg_measure_peaks(C.byref(f), C.byref(fw), C.byref(m), C.byref(c))
    if st != 0:
        raise SgError(st, lib.sg_last_error(None).decode())
    return {"fp32_fma_tflops": f.value, "fp32_fma_wave_gflops": fw.value, "bf16_mfma_tflops": m.value,
            "copy_gbps": c.value}
