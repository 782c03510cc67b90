"""Pins of the FP64 oracle against closed forms, invariants, brute force and
published known answers. None of these re-call the oracle's own formulas."""
import os

import numpy as np
import pytest

import oracle
import pinlib
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
G = 9.81


def _planar(n_env, n, masses, lengths, radius=0.05):
    """n-link chain with every joint about y (a planar arm in x-z)."""
    r = synth.make_chain(n_env, n, 7, dt=1 / 120, substeps=2)
    r.axis[:] = 0.0
    r.axis[1] = 1.0
    for j in range(n):
        m, L = masses[j], lengths[j]
        r.mass[j] = m
        r.offset[:, j] = 0.0
        if j > 0:
            r.offset[2, j] = lengths[j - 1]
        r.com[:, j] = 0.0
        r.com[2, j] = L / 2
        r.inertia[:, j] = 0.0
        r.inertia[0, j] = r.inertia[1, j] = m * (3 * radius ** 2 + L ** 2) / 12
        r.inertia[2, j] = m * radius ** 2 / 2
    r.tip[:] = 0.0
    r.tip[2] = lengths[n - 1]
    return r


# ---- closed forms -----------------------------------------------------------

def test_single_pendulum_closed_form():
    """(I + m c^2) qdd = tau + m g c sin q for a link swinging about y."""
    m, L = 1.7, 0.33
    r = _planar(5, 1, [m], [L])
    o = oracle.Oracle(r)
    rng = np.random.default_rng(1)
    q = rng.uniform(-3, 3, (1, 5))
    qd = rng.uniform(-4, 4, (1, 5))
    tau = rng.uniform(-5, 5, (1, 5))
    c = L / 2
    I = m * (3 * 0.05 ** 2 + L ** 2) / 12
    expect = (tau + m * G * c * np.sin(q)) / (I + m * c * c)
    np.testing.assert_allclose(o.aba(q, qd, tau), expect, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(o.fd_crba(q, qd, tau)[0], expect, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(o.crba(q)[:, 0, 0], I + m * c * c, rtol=1e-14)


def test_two_link_planar_closed_form():
    m1, m2, L1, L2 = 2.1, 0.9, 0.37, 0.21
    r = _planar(6, 2, [m1, m2], [L1, L2])
    o = oracle.Oracle(r)
    rng = np.random.default_rng(2)
    q = rng.uniform(-3, 3, (2, 6))
    qd = rng.uniform(-4, 4, (2, 6))
    c1, c2 = L1 / 2, L2 / 2
    I1 = m1 * (3 * 0.05 ** 2 + L1 ** 2) / 12
    I2 = m2 * (3 * 0.05 ** 2 + L2 ** 2) / 12
    q1, q2 = q
    M11 = I1 + I2 + m1 * c1 ** 2 + m2 * (L1 ** 2 + c2 ** 2 + 2 * L1 * c2 * np.cos(q2))
    M12 = I2 + m2 * (c2 ** 2 + L1 * c2 * np.cos(q2))
    M22 = I2 + m2 * c2 ** 2 + 0 * q2
    H = o.crba(q)
    np.testing.assert_allclose(H[:, 0, 0], M11, rtol=1e-13)
    np.testing.assert_allclose(H[:, 0, 1], M12, rtol=1e-13)
    np.testing.assert_allclose(H[:, 1, 0], M12, rtol=1e-13)
    np.testing.assert_allclose(H[:, 1, 1], M22, rtol=1e-13)
    C1 = -m2 * L1 * c2 * np.sin(q2) * (2 * qd[0] * qd[1] + qd[1] ** 2)
    C2 = m2 * L1 * c2 * np.sin(q2) * qd[0] ** 2
    # V = g [m1 c1 cos q1 + m2 (L1 cos q1 + c2 cos(q1 + q2))], G = dV/dq
    G1 = -G * (m1 * c1 * np.sin(q1) + m2 * (L1 * np.sin(q1) + c2 * np.sin(q1 + q2)))
    G2 = -G * m2 * c2 * np.sin(q1 + q2)
    bias = o.rnea(q, qd, np.zeros_like(q))
    np.testing.assert_allclose(bias[0], C1 + G1, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(bias[1], C2 + G2, rtol=1e-12, atol=1e-12)
    tip = o.fk(q)
    np.testing.assert_allclose(tip[0], L1 * np.sin(q1) + L2 * np.sin(q1 + q2), atol=1e-14)
    np.testing.assert_allclose(tip[1], 0.0, atol=1e-14)
    np.testing.assert_allclose(tip[2], L1 * np.cos(q1) + L2 * np.cos(q1 + q2), atol=1e-14)
    tau = rng.uniform(-5, 5, (2, 6))
    Mm = np.stack([np.stack([M11, M12]), np.stack([M12, M22])])  # [2][2][N]
    for e in range(6):
        expect = np.linalg.solve(Mm[:, :, e], tau[:, e] - np.array([C1[e] + G1[e], C2[e] + G2[e]]))
        np.testing.assert_allclose(o.aba(q, qd, tau)[:, e], expect, rtol=1e-11, atol=1e-11)


# ---- invariants and brute force on 7-DOF chains ---------------------------

@pytest.fixture(scope="module")
def chain7():
    w = synth.reach_fp64(16, seed=4242)
    o = oracle.Oracle(w.robot, w.task)
    q, qd = synth.random_states(77, w.robot)
    return w, o, q, qd


def test_rnea_aba_round_trip(chain7):
    w, o, q, qd = chain7
    tau = np.random.default_rng(3).normal(0, 10, q.shape)
    for arm in (None, o.drive_armature()):
        qdd = o.aba(q, qd, tau, arm)
        back = o.rnea(q, qd, qdd) + (0 if arm is None else arm * qdd)
        np.testing.assert_allclose(back, tau, rtol=1e-11, atol=1e-11)


def test_aba_equals_crba_cholesky(chain7):
    w, o, q, qd = chain7
    tau = np.random.default_rng(4).normal(0, 10, q.shape)
    for arm in (None, o.drive_armature()):
        a1 = o.aba(q, qd, tau, arm)
        a2, bad = o.fd_crba(q, qd, tau, arm)
        assert bad == 0
        np.testing.assert_allclose(a1, a2, rtol=1e-10, atol=1e-10)


def test_mass_matrix_spd_and_bruteforce(chain7):
    w, o, q, qd = chain7
    H = o.crba(q)
    for e in range(w.robot.n_env):
        M = H[e]
        np.testing.assert_allclose(M, M.T, atol=1e-14)
        assert np.linalg.eigvalsh(M).min() > 0
        links, tip, _ = pinlib.chain_of(w.robot, e)
        np.testing.assert_allclose(M, pinlib.mass_matrix(links, tip, q[:, e]), rtol=1e-11, atol=1e-12)


def test_bias_equals_christoffel_plus_gravity(chain7):
    w, o, q, qd = chain7
    bias = o.rnea(q, qd, np.zeros_like(q))
    for e in range(4):
        links, tip, grav = pinlib.chain_of(w.robot, e)
        ref = pinlib.bias_fd(links, tip, q[:, e], qd[:, e], grav)
        np.testing.assert_allclose(bias[:, e], ref, rtol=1e-6, atol=1e-6)


def test_tip_bruteforce(chain7):
    w, o, q, qd = chain7
    tip = o.fk(q)
    for e in range(w.robot.n_env):
        links, tp, _ = pinlib.chain_of(w.robot, e)
        np.testing.assert_allclose(tip[:, e], pinlib.fk(links, tp, q[:, e])[3], atol=1e-14)


def _rk4(o, q, qd, tau, h, steps):
    def f(q, qd):
        return qd, o.aba(q, qd, tau)
    for _ in range(steps):
        k1 = f(q, qd)
        k2 = f(q + 0.5 * h * k1[0], qd + 0.5 * h * k1[1])
        k3 = f(q + 0.5 * h * k2[0], qd + 0.5 * h * k2[1])
        k4 = f(q + h * k3[0], qd + h * k3[1])
        q = q + h / 6 * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0])
        qd = qd + h / 6 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1])
    return q, qd


def test_energy_conserved_rk4():
    """tau = 0, no drive, no limits: RK4 at h = 1e-4 keeps E to 1e-9 over 0.5 s."""
    w = synth.reach_fp64(3, seed=99)
    o = oracle.Oracle(w.robot)
    q, qd = synth.random_states(5, w.robot, qd_scale=0.5)
    E0 = [pinlib.energy(*pinlib.chain_of(w.robot, e)[:2], q[:, e], qd[:, e], np.array(w.robot.gravity))
          for e in range(3)]
    q1, qd1 = _rk4(o, q, qd, np.zeros_like(q), 1e-4, 5000)
    for e in range(3):
        links, tip, grav = pinlib.chain_of(w.robot, e)
        E1 = pinlib.energy(links, tip, q1[:, e], qd1[:, e], grav)
        scale = max(abs(E0[e]), 1.0)
        assert abs(E1 - E0[e]) / scale < 1e-9


def test_power_balance():
    """dE/dt = qd . tau for a driven chain (no drive armature)."""
    w = synth.reach_fp64(3, seed=5)
    o = oracle.Oracle(w.robot)
    q, qd = synth.random_states(6, w.robot, qd_scale=0.5)
    tau = np.random.default_rng(7).normal(0, 3, q.shape)
    h = 1e-5
    q1, qd1 = _rk4(o, q, qd, tau, h, 1)
    for e in range(3):
        links, tip, grav = pinlib.chain_of(w.robot, e)
        dE = (pinlib.energy(links, tip, q1[:, e], qd1[:, e], grav) -
              pinlib.energy(links, tip, q[:, e], qd[:, e], grav)) / h
        p_mid = 0.5 * (qd[:, e] + qd1[:, e]) @ tau[:, e]
        assert abs(dE - p_mid) < 1e-5 * max(1.0, abs(p_mid))


def test_vertical_axis_momentum_conserved():
    """Joint 0 turns about world z and gravity is along z: with tau_0 = 0 the
    generalized momentum (M qd)_0 is conserved whatever the other joints do."""
    w = synth.reach_fp64(3, seed=11)
    o = oracle.Oracle(w.robot)
    q, qd = synth.random_states(12, w.robot, qd_scale=0.5)
    tau = np.random.default_rng(8).normal(0, 3, q.shape)
    tau[0] = 0.0
    p0 = np.einsum("eij,je->ei", o.crba(q), qd)[:, 0]
    q1, qd1 = _rk4(o, q, qd, tau, 1e-4, 2000)
    p1 = np.einsum("eij,je->ei", o.crba(q1), qd1)[:, 0]
    np.testing.assert_allclose(p1, p0, rtol=1e-9, atol=1e-10)


def test_symplectic_euler_energy_bounded():
    """Free chain (3 links) under the env's own integrator (semi-implicit
    Euler at h = 1/240), drive off: energy error stays small with no drift."""
    r = synth.make_chain(2, 3, 21, dt=1 / 240, substeps=1)
    r.kp[:] = 0.0
    r.kd[:] = 0.0
    r.q_hi[:] = 1e9
    r.q_lo[:] = -1e9
    t = synth.Task(task=0, target=np.zeros((3, 2)), waypoints=None, dwell=1, ep_len=0,
                   progress0=np.zeros(2, np.int32))
    o = oracle.Oracle(r, t)
    q, qd = synth.random_states(13, r, qd_scale=0.3)
    grav = np.array(r.gravity)
    E = lambda q, qd, e: pinlib.energy(*pinlib.chain_of(r, e)[:2], q[:, e], qd[:, e], grav)
    E0 = [E(q, qd, e) for e in range(2)]
    pr = np.zeros(2, np.int32)
    errs = []
    for s in range(1000):
        q, qd, pr = o.step(np.zeros_like(q), q, qd, pr)[:3]
        if s % 50 == 49:
            errs.append([abs(E(q, qd, e) - E0[e]) for e in range(2)])
    errs = np.array(errs)
    links_m = [r.mass[:, e].sum() for e in range(2)]
    scale = np.array([G * m * 0.5 for m in links_m])  # a typical potential energy swing
    assert (errs / scale).max() < 2e-2
    # no secular drift: the last quarter is not systematically worse than the first
    assert errs[-5:].mean() < 5 * errs[:5].mean() + 1e-3


# ---- implicit PD and limits -----------------------------------------------

def _rotor(n_env=1, kp=100.0, kd=10.0, S=4, dt=1 / 120):
    r = synth.make_chain(n_env, 1, 3, dt=dt, substeps=S)
    r.axis[:] = 0.0
    r.axis[2] = 1.0  # about z: no gravity torque
    r.kp[:] = kp
    r.kd[:] = kd
    t = synth.Task(task=0, target=np.zeros((3, n_env)), waypoints=None, dwell=1, ep_len=0,
                   progress0=np.zeros(n_env, np.int32))
    return r, t


def test_implicit_pd_rotor_matrix_power():
    r, t = _rotor()
    o = oracle.Oracle(r, t)
    I = r.inertia[2, 0, 0]  # axial inertia, COM on the axis
    kp, kd = 100.0, 10.0
    h = r.dt / r.substeps
    arm = h * kd + h * h * kp
    k = h / (I + arm)
    A = np.array([[1 - h * k * kp, h * (1 - k * (kp * h + kd))], [-k * kp, 1 - k * (kp * h + kd)]])
    qstar = 0.3 * r.q_hi[0, 0]
    b = np.array([h * k * kp * qstar, k * kp * qstar])
    x = np.array([0.0, 0.0])
    q, qd, pr = np.zeros((1, 1)), np.zeros((1, 1)), np.zeros(1, np.int32)
    a = np.full((1, 1), 0.3)
    for step in range(40):
        q, qd, pr = o.step(a, q, qd, pr)[:3]
        for _ in range(r.substeps):
            x = A @ x + b
        np.testing.assert_allclose([q[0, 0], qd[0, 0]], x, rtol=1e-12, atol=1e-13)
    # fixed point is the target
    for _ in range(400):
        q, qd, pr = o.step(a, q, qd, pr)[:3]
    assert abs(q[0, 0] - qstar) < 1e-9 and abs(qd[0, 0]) < 1e-8


def test_implicit_pd_matches_end_of_substep_law():
    """tau = kp (q* - q') - kd qd' holds on the end-of-substep state."""
    w = synth.reach_fp64(4, seed=31)
    o = oracle.Oracle(w.robot, w.task)
    q, qd = synth.random_states(32, w.robot, qd_scale=0.2)
    q *= 0.3
    a = synth.random_actions(33, 4, 7) * 0.3
    q1, qd1, _, _, _, _, qlog = o.step(a, q, qd, np.zeros(4, np.int32), log_qdd=True)
    # one substep replayed: with S = 2 check the first substep through RNEA
    h = w.robot.dt / w.robot.substeps
    qstar = a * w.robot.q_hi
    qdd = qlog[0]
    qd_n = qd + h * qdd
    q_n = q + h * qd_n
    tau = w.robot.kp * (qstar - q_n) - w.robot.kd * qd_n
    np.testing.assert_allclose(o.rnea(q, qd, qdd), tau, rtol=1e-10, atol=1e-10)


def test_limit_projection_cases():
    r, t = _rotor(n_env=3, S=1, kp=0.0, kd=0.0)
    r.q_hi[:] = 1.0
    r.q_lo[:] = -1.0
    o = oracle.Oracle(r, t)
    h = r.dt
    q = np.array([[1.0 - 1e-3, 1.0, -1.0 + 1e-4]])
    qd = np.array([[10.0, -0.5, -5.0]])
    q1, qd1 = o.step(np.zeros((1, 3)), q, qd, np.zeros(3, np.int32))[:2]
    # crossing outward: clamped, outward velocity zeroed
    assert q1[0, 0] == 1.0 and qd1[0, 0] == 0.0
    # exactly at the limit moving inward: inward velocity kept
    assert qd1[0, 1] == -0.5 and q1[0, 1] == 1.0 + h * -0.5
    # crossing the lower limit
    assert q1[0, 2] == -1.0 and qd1[0, 2] == 0.0


def test_limit_tie_counts_as_inside():
    r, t = _rotor(n_env=1, S=1, kp=0.0, kd=0.0)
    r.q_hi[:] = 1.0
    r.q_lo[:] = -1.0
    o = oracle.Oracle(r, t)
    q = np.array([[1.0 - 0.25 * r.dt]])
    qd = np.array([[0.25]])
    q1, qd1 = o.step(np.zeros((1, 1)), q, qd, np.zeros(1, np.int32))[:2]
    assert q1[0, 0] == 1.0 and qd1[0, 0] == 0.25


# ---- observation, reward, episodes ----------------------------------------

def test_path_obs_reward_timeout():
    w = synth.path_rollout(32, seed=77, dtype=np.float64)
    o = oracle.Oracle(w.robot, w.task)
    rb, tk = w.robot, w.task
    q = rb.q0.copy()
    qd = np.zeros_like(q)
    pr = tk.progress0.copy()
    J, N = rb.max_dof, rb.n_env
    for s in range(200):
        a = synth.random_actions(500 + s, N, J)
        pre = pr.copy()
        q1, qd1, pr1, rew, done, obs = o.step(a, q, qd, pr)
        # physics-only state for the reward: replay the step without reset
        tip_post = o.fk(o.step(a, q, qd, np.zeros(N, np.int32))[0])
        k = np.minimum(pre // tk.dwell, tk.n_waypoints - 1)
        goal = tk.waypoints[k, :, np.arange(N)].T
        np.testing.assert_allclose(rew, -np.linalg.norm(tip_post - goal, axis=0), atol=1e-12)
        ended = pre + 1 >= tk.ep_len
        assert np.array_equal(done != 0, ended)
        assert np.all(done[ended] == 3)
        assert np.array_equal(pr1, np.where(ended, 0, pre + 1))
        np.testing.assert_array_equal(q1[:, ended], rb.q0[:, ended])
        assert np.all(qd1[:, ended] == 0)
        # observation of the post-reset state
        tip = o.fk(q1)
        kn = np.minimum(pr1 // tk.dwell, tk.n_waypoints - 1)
        gn = tk.waypoints[kn, :, np.arange(N)].T
        np.testing.assert_array_equal(obs[:J], q1)
        np.testing.assert_array_equal(obs[J:2 * J], qd1)
        np.testing.assert_allclose(obs[2 * J:2 * J + 3], tip, atol=1e-15)
        np.testing.assert_array_equal(obs[2 * J + 3:2 * J + 6], gn)
        np.testing.assert_allclose(obs[2 * J + 6:2 * J + 9], gn - tip, atol=1e-15)
        np.testing.assert_allclose(obs[2 * J + 9], np.linalg.norm(gn - tip, axis=0), atol=1e-15)
        q, qd, pr = q1, qd1, pr1


def test_nonfinite_state_resets():
    w = synth.reach_fp64(4, seed=8)
    o = oracle.Oracle(w.robot, w.task)
    q = np.zeros((7, 4))
    qd = np.zeros((7, 4))
    q[3, 1] = np.nan
    qd[2, 2] = np.inf
    q1, qd1, pr1, rew, done, obs = o.step(np.zeros((7, 4)), q, qd, np.array([5, 5, 5, 5], np.int32))
    assert list(done) == [0, 5, 5, 0]
    assert rew[1] == 0 and rew[2] == 0 and np.all(np.isfinite(obs))
    assert list(pr1) == [6, 0, 0, 6]


# ---- spline waypoints (input synthesis) -----------------------------------

def test_spline_collinear_knots_give_equal_spacing():
    knots = np.array([[0.0, 0, 0], [1.0, 2, 3], [2.0, 4, 6], [3.0, 6, 9]])
    wp = synth.spline_waypoints(knots)
    d = np.linalg.norm(np.diff(wp, axis=0), axis=1)
    np.testing.assert_allclose(d, d[0], rtol=1e-6)
    np.testing.assert_allclose(wp[0], knots[0], atol=1e-12)
    np.testing.assert_allclose(wp[-1], knots[-1], atol=1e-12)
    cr = np.cross(wp - knots[0], knots[-1] - knots[0])
    assert np.abs(cr).max() < 1e-9


# ---- learning side --------------------------------------------------------

def test_philox_known_answers():
    for line in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        f = [int(x, 16) for x in line.split()]
        assert oracle.philox4x32_10(f[0:4], f[4:6]) == f[6:10]


def test_box_muller_moments():
    eps = oracle.noise(seed=123456789, step=7, n=8, N=125000).ravel()  # 1e6 samples
    assert abs(eps.mean()) < 5e-3
    assert abs(eps.var() - 1) < 5e-3
    assert abs((eps ** 4).mean() - 3) < 3e-2
    assert abs((np.abs(eps) < 1).mean() - 0.682689492) < 2e-3


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 20000), rng.normal(0, 1e-3, 5000), rng.normal(0, 1e3, 5000)])
    x = x.astype(np.float32)
    # exact ties: values halfway between two BF16 neighbours
    # (built from normal-range values: the oracle's rounding covers BF16's
    # normal range, which holds every value the method produces)
    base = (x[:4000].view(np.uint32) & np.uint32(0xFFFF0000))
    ties = (base | np.uint32(0x8000)).view(np.float32)
    x = np.concatenate([x, ties])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(oracle.round_bf16(x.astype(np.float64)), ref)


def test_mlp_bruteforce():
    w = synth.path_rollout(8, seed=3)
    o = oracle.Oracle(w.robot, w.task, w.policy)
    x = np.random.default_rng(1).normal(0, 1, (24, 50)).astype(np.float32).astype(np.float64)
    P = w.policy
    h = np.tanh(P.W[0] @ x + P.b[0][:, None])
    h = np.tanh(P.W[1] @ h + P.b[1][:, None])
    out = P.W[2] @ h + P.b[2][:, None]
    np.testing.assert_allclose(o.mlp(x, emulate=False), out, rtol=1e-12, atol=1e-12)
    # emulate mode: inputs to every layer pass through BF16 first
    torch = pytest.importorskip("torch")
    bf = lambda a: torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).double().numpy()
    xe = o.mlp(x, emulate=True)
    h = np.tanh(P.W[0] @ bf(x) + P.b[0][:, None])
    # BF16 rounding of FP64 hidden values: compare with a tolerance that
    # admits the rare double-rounding difference of the FP32 hop used here
    h = np.tanh(P.W[1] @ bf(h) + P.b[1][:, None])
    out = P.W[2] @ bf(h) + P.b[2][:, None]
    assert np.abs(xe - out).max() < 2e-3
    assert np.median(np.abs(xe - out)) < 1e-12


def test_mlp_integer_inputs_exact():
    """Integer-valued weights, inputs and biases with tanh removed by a
    linear check of the last layer: exact arithmetic gives exact outputs."""
    w = synth.path_rollout(4, seed=5)
    P = w.policy
    P2 = synth.Policy(dims=P.dims, W=[np.round(wi * 8) for wi in P.W], b=[np.round(bi * 8) for bi in P.b],
                      log_std=P.log_std)
    o = oracle.Oracle(w.robot, w.task, P2)
    x = np.random.default_rng(2).integers(-3, 4, (24, 20)).astype(np.float64)
    h1 = np.tanh(P2.W[0] @ x + P2.b[0][:, None])
    h2 = np.tanh(P2.W[1] @ h1 + P2.b[1][:, None])
    out = P2.W[2] @ h2 + P2.b[2][:, None]
    np.testing.assert_allclose(o.mlp(x, emulate=False), out, rtol=1e-12)
    pre1 = P2.W[0] @ x + P2.b[0][:, None]
    assert np.all(pre1 == np.round(pre1))  # the first layer's sums are exact integers


def _gae_bruteforce(rew, val, done, gamma, lam):
    T, N = rew.shape
    nd = 1.0 - (done & 1)
    r = rew + gamma * val[:-1] * ((done & 2) != 0)
    delta = r + gamma * val[1:] * nd - val[:-1]
    adv = np.zeros((T, N))
    for t in range(T):
        coef = np.ones(N)
        for l in range(t, T):
            adv[t] += coef * delta[l]
            coef = coef * gamma * lam * nd[l]
    return adv


def test_gae_pins():
    rng = np.random.default_rng(9)
    T, N = 32, 50
    rew = rng.normal(0, 1, (T, N))
    val = rng.normal(0, 1, (T + 1, N))
    done = np.zeros((T, N), np.uint8)
    # lambda = 0: A = delta
    adv, ret = oracle.gae(rew, val, done, 0.99, 0.0)
    np.testing.assert_allclose(adv, rew + 0.99 * val[1:] - val[:-1], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(ret, adv + val[:-1], rtol=1e-13, atol=1e-13)
    # lambda = 1, no dones: discounted return minus baseline
    adv, _ = oracle.gae(rew, val, done, 0.99, 1.0)
    for t in range(T):
        g = sum(0.99 ** k * rew[t + k] for k in range(T - t)) + 0.99 ** (T - t) * val[T]
        np.testing.assert_allclose(adv[t], g - val[t], rtol=1e-11, atol=1e-11)
    # episode ends and time-outs: brute force
    done = (rng.random((T, N)) < 0.1).astype(np.uint8)
    done |= ((rng.random((T, N)) < 0.5) & (done == 1)).astype(np.uint8) << 1
    adv, _ = oracle.gae(rew, val, done, 0.99, 0.95)
    np.testing.assert_allclose(adv, _gae_bruteforce(rew, val, done, 0.99, 0.95), rtol=1e-11, atol=1e-11)


def test_opcount_deterministic_and_scales_with_substeps():
    w2 = synth.reach_fp64(2, seed=1)
    o2 = oracle.Oracle(w2.robot, w2.task)
    a = synth.random_actions(1, 2, 7)
    s2, p2 = o2.opcount_step(a)
    assert o2.opcount_step(a) == (s2, p2)
    w4 = synth.path_rollout(2, seed=1, dtype=np.float64)
    o4 = oracle.Oracle(w4.robot, w4.task)
    s4, p4 = o4.opcount_step(a)
    f2 = sum(p2[k] for k in ("add", "mul", "div", "sqrt"))
    f4 = sum(p4[k] for k in ("add", "mul", "div", "sqrt"))
    # 4 substeps cost twice the substep work of 2 substeps, up to the per-step setup
    assert abs((f4 - f2) - f2) < 0.02 * f2
    assert p4["trans"] == 2 * 7 * 4
