"""Seeded synthetic inputs shared by the oracle and the HIP library.

This module only draws inputs; it computes none of the method's steps.
Every array is prefix-stable in the env index: env i's values do not depend
on how many envs are generated, because each array is drawn from its own
Philox stream in env-major order and then laid out structure-of-arrays
([field][joint][env]).

Workloads (the paper's robots and task assets are not available, so seeded
revolute chains stand in for them; paper Sec. III "Robot Descriptions" lists
7- and 8-DoF all-revolute arms):

* ``reach_fp64`` -- 64 envs x 7-DOF, FP64, dt = 1/120 s, 2 substeps,
  target-reaching task (paper Sec. IV "Target Reaching") with the target
  uniform in a 0.5 m cube.
* ``path_rollout`` -- N envs x 7-DOF, FP32, 4 substeps, path-following task
  (paper Sec. IV "Path following"): 8 waypoints at equal arc length on a
  natural cubic spline through 4 seeded knots in a 0.3 m box; 128-step
  episodes with staggered start progress; policy 24-256-128-8.
* ``mixed_dof`` -- 4/6/7/9-DOF chains mixed 25 % each, per-env gains.

Chain recipe (all per env and per joint, i.i.d.): link mass U[0.5, 3] kg,
length U[0.1, 0.4] m, solid cylinder of radius 0.05 m along the link's +z
with its centre of mass at L/2, joint axes alternating z, y, z, y, ...,
joint j+1 at (0, 0, L_j) in link j's frame, symmetric limits +-U[1.5, 3] rad,
kp = 100, kd = 10, gravity (0, 0, -9.81).
"""
from __future__ import annotations

import dataclasses
import zlib

import numpy as np

__all__ = [
    "Robot", "Task", "Policy", "Workload", "stream", "make_chain", "reach_fp64", "path_rollout",
    "mixed_dof", "tracking", "psm_like", "multi_arm", "make_policy", "random_actions", "random_states",
]

TASK_REACH = 0
TASK_PATH = 1
TASK_TRACK = 2
WORK_CENTRE = np.array([0.4, 0.0, 0.6])


def stream(seed: int, tag: str) -> np.random.Generator:
    """Independent Philox stream for (seed, array tag)."""
    key = np.array([seed & 0xFFFFFFFFFFFFFFFF, zlib.crc32(tag.encode())], dtype=np.uint64)
    return np.random.Generator(np.random.Philox(key=key))


def _per_env(seed, tag, n_env, n_col, lo, hi):
    """Uniform draws [n_env][n_col], env-major so rows are prefix-stable."""
    return stream(seed, tag).uniform(lo, hi, size=(n_env, n_col))


@dataclasses.dataclass
class Robot:
    n_env: int
    max_dof: int
    n_dof: np.ndarray      # int32 [N]
    axis: np.ndarray       # [3][J][N]
    offset: np.ndarray     # [3][J][N]
    com: np.ndarray        # [3][J][N]
    mass: np.ndarray       # [J][N]
    inertia: np.ndarray    # [6][J][N] xx yy zz xy xz yz about the COM
    kp: np.ndarray         # [J][N]
    kd: np.ndarray
    q_lo: np.ndarray
    q_hi: np.ndarray
    q0: np.ndarray
    tip: np.ndarray        # [3][N]
    dt: float
    substeps: int
    gravity: tuple = (0.0, 0.0, -9.81)
    joint_type: np.ndarray | None = None  # int32 [J][N]: 0 revolute, 1 prismatic (None: all revolute)


@dataclasses.dataclass
class Task:
    task: int
    target: np.ndarray | None      # [3][N]
    waypoints: np.ndarray | None   # [K][3][N]
    dwell: int
    ep_len: int
    progress0: np.ndarray          # int32 [N]
    track: dict | None = None      # tracking task: sigma, offset, reset_std, centre
    chains: int = 1                # chains per env (consecutive env indices)
    rerand: dict | None = None     # per-episode re-randomisation: reach {centre, half}; path {} (banks)
    n_banks: int = 1               # path: waypoint sets, waypoints [n_banks K][3][N]

    @property
    def n_waypoints(self):
        return 0 if self.waypoints is None else self.waypoints.shape[0] // max(self.n_banks, 1)


@dataclasses.dataclass
class Policy:
    dims: tuple                    # (n_in, hidden sizes..., n_out)
    W: list                        # per layer [n_out][n_in], values exactly representable in BF16
    b: list                        # per layer [n_out], FP32 values
    log_std: np.ndarray            # [n_out - 1], FP32 values
    act: str = "tanh"              # hidden activation: "tanh" or "elu"

    def w_bf16_bits(self) -> np.ndarray:
        """Concatenated layer weights as BF16 bit patterns (uint16)."""
        flat = np.concatenate([w.astype(np.float32).ravel() for w in self.W])
        return (flat.view(np.uint32) >> 16).astype(np.uint16)

    def b_f32(self) -> np.ndarray:
        return np.concatenate([b.astype(np.float32) for b in self.b])


@dataclasses.dataclass
class Workload:
    name: str
    robot: Robot
    task: Task
    policy: Policy | None
    dtype: type
    seed: int
    extra: dict = dataclasses.field(default_factory=dict)


def _axis_pattern(j):
    return (0.0, 0.0, 1.0) if j % 2 == 0 else (0.0, 1.0, 0.0)


def make_chain(n_env: int, n_dof, seed: int, *, dt: float, substeps: int, max_dof: int | None = None,
               q0_frac: float = 0.0, gain_jitter: bool = False, radius: float = 0.05,
               pattern: str | None = None) -> Robot:
    """Seeded serial chains. ``n_dof`` is an int or an int array [N].
    ``pattern`` (e.g. "RRPRRR") marks prismatic joints: they slide along the
    link axis (+z), limits +-U[0.05, 0.15] m, gains kp 400 N/m, kd 40 N s/m."""
    n_dof = np.broadcast_to(np.asarray(n_dof, dtype=np.int32), (n_env,)).copy()
    J = int(max_dof if max_dof is not None else n_dof.max())
    mass = _per_env(seed, "mass", n_env, J, 0.5, 3.0)
    length = _per_env(seed, "length", n_env, J, 0.1, 0.4)
    hi = _per_env(seed, "limit", n_env, J, 1.5, 3.0)
    q0u = _per_env(seed, "q0", n_env, J, -1.0, 1.0) * q0_frac
    if gain_jitter:
        kp = 100.0 * np.exp2(_per_env(seed, "kp", n_env, J, -1.0, 1.0))
        kd = 10.0 * np.exp2(_per_env(seed, "kd", n_env, J, -1.0, 1.0))
    else:
        kp = np.full((n_env, J), 100.0)
        kd = np.full((n_env, J), 10.0)
    axis = np.zeros((3, J, n_env))
    offset = np.zeros((3, J, n_env))
    com = np.zeros((3, J, n_env))
    inertia = np.zeros((6, J, n_env))
    tip = np.zeros((3, n_env))
    mask = (np.arange(J)[None, :] < n_dof[:, None])  # [N][J]
    for j in range(J):
        ax = _axis_pattern(j)
        for c in range(3):
            axis[c, j, :] = ax[c]
    offset[2, 1:, :] = length[:, :-1].T
    com[2] = 0.5 * length.T
    m = mass.T
    L = length.T
    inertia[0] = m * (3 * radius ** 2 + L ** 2) / 12.0
    inertia[1] = inertia[0]
    inertia[2] = m * radius ** 2 / 2.0
    idx = n_dof - 1
    tip[2] = length[np.arange(n_env), idx]
    z = ~mask.T  # [J][N] padded slots
    for arr in (axis, offset, com, inertia):
        arr[:, z] = 0.0
    q_hi = hi.T.copy()
    q_lo = -q_hi
    q0 = (q0u.T * q_hi)
    m = m.copy()
    m[z] = 0.0
    for arr in (q_hi, q_lo, q0):
        arr[z] = 0.0
    kpT = kp.T.copy(); kpT[z] = 0.0
    kdT = kd.T.copy(); kdT[z] = 0.0
    jt = None
    if pattern is not None:
        jt = np.zeros((J, n_env), dtype=np.int32)
        ph = _per_env(seed, "plimit", n_env, J, 0.05, 0.15).T
        for j in range(J):
            if pattern[j % len(pattern)] == "P":
                jt[j] = 1
                axis[:, j, :] = 0.0
                axis[2, j, :] = 1.0
                q_hi[j] = ph[j]
                q_lo[j] = -ph[j]
                q0[j] = 0.0
                kpT[j] = 400.0
                kdT[j] = 40.0
        jt[z] = 0
        for arr in (q_hi, q_lo, q0, kpT, kdT):
            arr[z] = 0.0
    return Robot(n_env=n_env, max_dof=J, n_dof=n_dof, axis=axis, offset=offset, com=com, mass=m,
                 inertia=inertia, kp=kpT, kd=kdT, q_lo=q_lo, q_hi=q_hi, q0=q0, tip=tip, dt=dt,
                 substeps=substeps, joint_type=jt)


def _natural_cubic_coeffs(u, y):
    """Natural cubic spline through (u_i, y_i): second derivatives at the knots."""
    n = len(u)
    h = np.diff(u)
    A = np.zeros((n, n))
    rhs = np.zeros(n)
    A[0, 0] = A[-1, -1] = 1.0
    for i in range(1, n - 1):
        A[i, i - 1] = h[i - 1]
        A[i, i] = 2 * (h[i - 1] + h[i])
        A[i, i + 1] = h[i]
        rhs[i] = 6 * ((y[i + 1] - y[i]) / h[i] - (y[i] - y[i - 1]) / h[i - 1])
    return np.linalg.solve(A, rhs)


def _spline_eval(u, y, M, t):
    i = np.clip(np.searchsorted(u, t, side="right") - 1, 0, len(u) - 2)
    h = u[i + 1] - u[i]
    a = (u[i + 1] - t) / h
    b = (t - u[i]) / h
    return a * y[i] + b * y[i + 1] + ((a ** 3 - a) * M[i] + (b ** 3 - b) * M[i + 1]) * h * h / 6.0


def spline_waypoints(knots: np.ndarray, n_waypoints: int = 8, n_seg: int = 1024) -> np.ndarray:
    """Waypoints at equal arc length along the natural cubic spline through
    ``knots`` [n_knots][3] (knot parameters uniform in [0, 1]); endpoints
    included. Arc length from an ``n_seg``-segment polyline."""
    nk = knots.shape[0]
    u = np.linspace(0.0, 1.0, nk)
    t = np.linspace(0.0, 1.0, n_seg + 1)
    curve = np.stack([_spline_eval(u, knots[:, c], _natural_cubic_coeffs(u, knots[:, c]), t)
                      for c in range(3)], axis=1)
    seg = np.linalg.norm(np.diff(curve, axis=0), axis=1)
    s = np.concatenate([[0.0], np.cumsum(seg)])
    targets = np.linspace(0.0, s[-1], n_waypoints)
    out = np.empty((n_waypoints, 3))
    for c in range(3):
        out[:, c] = np.interp(targets, s, curve[:, c])
    return out


def _as_dtype(arr, dtype):
    """Round to ``dtype`` and hand back float64 holding exactly those values."""
    if arr is None:
        return None
    if arr.dtype.kind == "f":
        return arr.astype(dtype).astype(np.float64)
    return arr


def _round_robot(r: Robot, dtype) -> Robot:
    fields = {f.name: getattr(r, f.name) for f in dataclasses.fields(r)}
    for k, v in fields.items():
        if isinstance(v, np.ndarray) and v.dtype.kind == "f":
            fields[k] = _as_dtype(v, dtype)
    fields["dt"] = float(np.asarray(r.dt, dtype=dtype))
    fields["gravity"] = tuple(float(np.asarray(g, dtype=dtype)) for g in r.gravity)
    return Robot(**fields)


def _round_task(t: Task, dtype) -> Task:
    tr = None
    if t.track is not None:
        f = lambda v: float(np.asarray(v, dtype=dtype))
        tr = dict(sigma=f(t.track["sigma"]), offset=f(t.track["offset"]), reset_std=f(t.track["reset_std"]),
                  centre=tuple(f(c) for c in t.track["centre"]))
    rr = None
    if t.rerand is not None:
        f = lambda v: float(np.asarray(v, dtype=dtype))
        rr = {k: (tuple(f(c) for c in v) if k == "centre" else f(v)) for k, v in t.rerand.items()}
    return Task(task=t.task, target=_as_dtype(t.target, dtype), waypoints=_as_dtype(t.waypoints, dtype),
                dwell=t.dwell, ep_len=t.ep_len, progress0=t.progress0, track=tr, chains=t.chains, rerand=rr,
                n_banks=t.n_banks)


TABLE2_DIMS = (24, 256, 128, 64, 8)  # the paper's Table II network: 256-128-64 ELU (+ J = 7 means and a value)


def make_policy(seed: int, dims=(24, 256, 128, 8), log_std: float = np.log(0.5), act: str = "tanh") -> Policy:
    """Seeded policy: weights U(+-1/sqrt(fan_in)) truncated to BF16-representable
    values (low 16 bits of the FP32 pattern cleared), FP32 biases; dims =
    (n_in, hidden sizes..., J + 1)."""
    Ws, bs = [], []
    for l in range(len(dims) - 1):
        n_in, n_out = dims[l], dims[l + 1]
        bound = 1.0 / np.sqrt(n_in)
        w = stream(seed, f"W{l}").uniform(-bound, bound, size=(n_out, n_in)).astype(np.float32)
        w = (w.view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32)
        b = stream(seed, f"b{l}").uniform(-bound, bound, size=n_out).astype(np.float32)
        Ws.append(w.astype(np.float64))
        bs.append(b.astype(np.float64))
    ls = np.full(dims[-1] - 1, np.float32(log_std), dtype=np.float32).astype(np.float64)
    return Policy(dims=tuple(dims), W=Ws, b=bs, log_std=ls, act=act)


def reach_fp64(n_env: int = 64, seed: int = 1001) -> Workload:
    """Tiny FP64 parity workload: 7-DOF chains, target reaching, dt = 1/120 s,
    2 substeps, q0 = 0, no time-outs."""
    r = make_chain(n_env, 7, seed, dt=1.0 / 120.0, substeps=2, q0_frac=0.0)
    tgt = (WORK_CENTRE[None, :] + _per_env(seed, "target", n_env, 3, -0.25, 0.25)).T.copy()
    t = Task(task=TASK_REACH, target=tgt, waypoints=None, dwell=1, ep_len=0,
             progress0=np.zeros(n_env, dtype=np.int32))
    return Workload("reach_fp64", r, t, None, np.float64, seed)


def path_rollout(n_env: int = 4096, seed: int = 1002, dtype=np.float32, substeps: int = 4) -> Workload:
    """Path-following rollout workload: 7-DOF FP32 chains, 4 substeps,
    q0 ~ U(-0.25, 0.25) * hi, 8 waypoints on a spline, dwell 16, episodes of
    128 steps with staggered start progress, policy 24-256-128-8."""
    r = make_chain(n_env, 7, seed, dt=1.0 / 120.0, substeps=substeps, q0_frac=0.25)
    knots = (WORK_CENTRE[None, None, :] +
             _per_env(seed, "knots", n_env, 12, -0.15, 0.15).reshape(n_env, 4, 3))
    wps = np.stack([spline_waypoints(knots[e]) for e in range(n_env)], axis=2)  # [K][3][N]
    prog = stream(seed, "progress0").integers(0, 128, size=n_env).astype(np.int32)
    t = Task(task=TASK_PATH, target=None, waypoints=wps, dwell=16, ep_len=128, progress0=prog)
    pol = make_policy(seed)
    return Workload("path_rollout", _round_robot(r, dtype), _round_task(t, dtype), pol, dtype, seed,
                    extra={"knots": knots})


def psm_like(n_env: int = 4096, seed: int = 1004, dtype=np.float32) -> Workload:
    """6-DOF RRPRRR chains (the joint sequence of the paper's PSM/ECM arms,
    Sec. III "Robot Descriptions"), FP32, 4 substeps, target reaching."""
    r = make_chain(n_env, 6, seed, dt=1.0 / 120.0, substeps=4, q0_frac=0.25, pattern="RRPRRR")
    tgt = (WORK_CENTRE[None, :] + _per_env(seed, "target", n_env, 3, -0.25, 0.25)).T.copy()
    t = Task(task=TASK_REACH, target=tgt, waypoints=None, dwell=1, ep_len=128,
             progress0=stream(seed, "progress0").integers(0, 128, size=n_env).astype(np.int32))
    return Workload("psm_like", _round_robot(r, dtype), _round_task(t, dtype), None, dtype, seed)


def tracking(n_env: int = 4096, seed: int = 1005, dtype=np.float32) -> Workload:
    """Active tracking (paper Sec. IV): 7-DOF FP32 chains, 4 substeps; the
    first episode's goal centre is W + N(0, 0.05^2) per axis, then a random
    walk with velocity increments of std 1e-4 m per step inside a +-0.2 m
    box; new centres drawn on the device at each reset; 128-step episodes
    with staggered start progress; policy 24-256-128-8."""
    r = make_chain(n_env, 7, seed, dt=1.0 / 120.0, substeps=4, q0_frac=0.25)
    tgt = (WORK_CENTRE[None, :] + 0.05 * stream(seed, "centre").standard_normal((n_env, 3))).T.copy()
    t = Task(task=TASK_TRACK, target=tgt, waypoints=None, dwell=1, ep_len=128,
             progress0=stream(seed, "progress0").integers(0, 128, size=n_env).astype(np.int32),
             track=dict(sigma=1e-4, offset=0.2, reset_std=0.05, centre=tuple(WORK_CENTRE)))
    return Workload("tracking", _round_robot(r, dtype), _round_task(t, dtype), make_policy(seed + 7), dtype, seed)


def reach_rerand(n_env: int = 4096, seed: int = 1007, dtype=np.float32) -> Workload:
    """Target reaching with per-episode re-randomisation: 7-DOF FP32 chains,
    4 substeps, 128-step episodes with staggered start progress; the first
    target is W + U[-0.25, 0.25]^3, and each reset draws the next one in the
    same box on the device; policy 24-256-128-8."""
    r = make_chain(n_env, 7, seed, dt=1.0 / 120.0, substeps=4, q0_frac=0.25)
    tgt = (WORK_CENTRE[None, :] + _per_env(seed, "target", n_env, 3, -0.25, 0.25)).T.copy()
    t = Task(task=TASK_REACH, target=tgt, waypoints=None, dwell=1, ep_len=128,
             progress0=stream(seed, "progress0").integers(0, 128, size=n_env).astype(np.int32),
             rerand=dict(centre=tuple(WORK_CENTRE), half=0.25))
    return Workload("reach_rerand", _round_robot(r, dtype), _round_task(t, dtype), make_policy(seed + 7), dtype, seed)


def path_rerand(n_env: int = 4096, seed: int = 1008, banks: int = 4, dtype=np.float32) -> Workload:
    """Path following with per-episode re-randomisation: every env holds
    `banks` waypoint sets (each 8 waypoints on its own natural cubic spline
    through 4 knots in the 0.3 m box, as in path_rollout); the first
    episode follows set 0 and each reset picks a set on the device."""
    r = make_chain(n_env, 7, seed, dt=1.0 / 120.0, substeps=4, q0_frac=0.25)
    sets = []
    for b in range(banks):
        knots = (WORK_CENTRE[None, None, :] +
                 _per_env(seed, f"knots{b}", n_env, 12, -0.15, 0.15).reshape(n_env, 4, 3))
        sets.append(np.stack([spline_waypoints(knots[e]) for e in range(n_env)], axis=2))  # [K][3][N]
    wps = np.concatenate(sets, axis=0)  # [banks K][3][N]
    prog = stream(seed, "progress0").integers(0, 128, size=n_env).astype(np.int32)
    t = Task(task=TASK_PATH, target=None, waypoints=wps, dwell=16, ep_len=128, progress0=prog, rerand={},
             n_banks=banks)
    return Workload("path_rerand", _round_robot(r, dtype), _round_task(t, dtype), make_policy(seed + 7), dtype,
                    seed)


def multi_arm(n_env: int = 2048, chains: int = 2, seed: int = 1006, dtype=np.float32) -> Workload:
    """Multi-tool reaching (paper Sec. IV): `chains` 7-DOF arms per env
    (env k owns chains k*C .. k*C + C - 1), bases spread along y (0.6 m
    apart), each arm with its own target U[-0.15, 0.15]^3 around the point
    0.4 m in front of and 0.6 m above its base; FP32, 4 substeps, 128-step
    episodes with a start progress shared by an env's arms."""
    N = n_env * chains
    r = make_chain(N, 7, seed, dt=1.0 / 120.0, substeps=4, q0_frac=0.25)
    base_y = (np.arange(N) % chains - 0.5 * (chains - 1)) * 0.6
    r.offset[1, 0, :] = base_y
    centre = np.stack([np.full(N, 0.4), base_y, np.full(N, 0.6)], axis=1)
    tgt = (centre + _per_env(seed, "target", N, 3, -0.15, 0.15)).T.copy()
    p0 = np.repeat(stream(seed, "progress0").integers(0, 128, size=n_env).astype(np.int32), chains)
    t = Task(task=TASK_REACH, target=tgt, waypoints=None, dwell=1, ep_len=128, progress0=p0, chains=chains)
    return Workload("multi_arm", _round_robot(r, dtype), _round_task(t, dtype), make_policy(seed + 7), dtype, seed)


def mixed_dof(n_env: int = 16384, seed: int = 1003, dtype=np.float32) -> Workload:
    """Uneven batch: 4-, 6-, 7- and 9-DOF chains, 25 % each in a seeded
    permutation, per-env jittered gains, reach task."""
    classes = np.repeat(np.array([4, 6, 7, 9], dtype=np.int32), (n_env + 3) // 4)[:n_env]
    perm = stream(seed, "dof_perm").permutation(n_env)
    n_dof = classes[perm]
    r = make_chain(n_env, n_dof, seed, dt=1.0 / 120.0, substeps=4, max_dof=9, q0_frac=0.25,
                   gain_jitter=True)
    tgt = (WORK_CENTRE[None, :] + _per_env(seed, "target", n_env, 3, -0.25, 0.25)).T.copy()
    t = Task(task=TASK_REACH, target=tgt, waypoints=None, dwell=1, ep_len=128,
             progress0=stream(seed, "progress0").integers(0, 128, size=n_env).astype(np.int32))
    return Workload("mixed_dof", _round_robot(r, dtype), _round_task(t, dtype), None, dtype, seed)


def surrogate_init(seed: int, dims=(91, 256, 256, 256, 7)):
    """Initial FP32 master weights of the surrogate network:
    W U(+-1/sqrt(fan_in)) [out][in], b zero."""
    Ws, bs = [], []
    for l in range(len(dims) - 1):
        bound = 1.0 / np.sqrt(dims[l])
        Ws.append(stream(seed, f"sW{l}").uniform(-bound, bound, size=(dims[l + 1], dims[l])).astype(np.float32))
        bs.append(np.zeros(dims[l + 1], dtype=np.float32))
    return Ws, bs


def surrogate_torques(seed: int, n: int, J: int, sigma: float = 20.0, tag: str = "tau") -> np.ndarray:
    """Joint torques tau ~ N(0, sigma^2) [J][n], FP32 values."""
    t = stream(seed, tag).normal(0.0, sigma, size=(n, J)).T.copy()
    return t.astype(np.float32).astype(np.float64)


def random_actions(seed: int, n_env: int, J: int, dtype=np.float64, tag: str = "actions") -> np.ndarray:
    """Actions a ~ U(-1, 1) [J][N] (the paper's random-action benchmark input)."""
    a = _per_env(seed, tag, n_env, J, -1.0, 1.0).T.copy()
    return _as_dtype(a, dtype)


def random_states(seed: int, robot: Robot, dtype=np.float64, qd_scale: float = 2.0, tag: str = "state"):
    """Random joint states inside the limits: q ~ U(lo, hi) * 0.9, qd ~ U(+-qd_scale)."""
    N, J = robot.n_env, robot.max_dof
    u = _per_env(seed, tag + "_q", N, J, -0.9, 0.9).T
    q = u * robot.q_hi
    qd = _per_env(seed, tag + "_qd", N, J, -qd_scale, qd_scale).T.copy()
    pad = np.arange(J)[:, None] >= robot.n_dof[None, :]
    q[pad] = 0.0
    qd[pad] = 0.0
    return _as_dtype(q, dtype), _as_dtype(qd, dtype)
