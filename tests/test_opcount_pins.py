"""Pins of the op-counting oracle, whose exact count of one control step is
the algorithmic work the benchmark divides by time.

Two levels, neither of which re-runs the counter against itself:
* every spatial-algebra primitive's tally against a hand count from its
  definition (a 3x3 matrix-vector product is 9 multiplications and 6
  additions, a cross product 6 and 3, ...);
* the whole control step against the count assembled from those hand counts
  and the structure of the method: the three ABA passes of Featherstone's
  Table 7.1 per joint and substep, the implicit-PD torque and the
  semi-implicit Euler update per joint and substep, the per-step PD targets
  and armatures, and the kinematics, reward and observation after the
  substeps, for several chain lengths and substep counts. A dropped or
  doubled term anywhere in the oracle's step moves the total off the formula.
"""
import numpy as np
import pytest

import oracle
import synth

# Hand counts (add, mul) from the definitions; no divisions, square roots or
# transcendental calls unless listed.
DOT = (2, 3)                      # a.b
CROSS = (3, 6)                    # a x b
M3V3 = (6, 9)                     # A v
M3M3 = (18, 27)                   # A B
XM = (M3V3[0] + CROSS[0] + 3 + M3V3[0], M3V3[1] + CROSS[1] + M3V3[1])  # (E w; E (v - r x w))
XFT = (2 * M3V3[0] + CROSS[0] + 3, 2 * M3V3[1] + CROSS[1])            # (E^T n + r x E^T f; E^T f)
CRM = (3 * CROSS[0] + 3, 3 * CROSS[1])   # (w1 x w2; w1 x v2 + v1 x w2)
CRF = (3 * CROSS[0] + 3, 3 * CROSS[1])   # (w x n + v x f; w x f)
SIMUL = (4 * M3V3[0] + 6, 4 * M3V3[1])   # [[A, B], [B^T, C]] m
SDOT = (2 * DOT[0] + 1, 2 * DOT[1])
# congruence X^T I X: E^T A E and E^T C E (full A E, then the 6 upper
# entries, 3 mul + 2 add each), E^T (B E) (two full products), B2 = B1 + rx C1
# (3 cross products + 9 adds), rx B1^T and B2 rx (3 cross products each),
# A2 = A1 + Y - Z on the 6 upper entries (2 adds each)
SYMC = (M3M3[0] + 6 * 2, M3M3[1] + 6 * 3)
CONG = (2 * SYMC[0] + 2 * M3M3[0] + 3 * CROSS[0] + 9 + 2 * 3 * CROSS[0] + 6 * 2,
        2 * SYMC[1] + 2 * M3M3[1] + 3 * CROSS[1] + 2 * 3 * CROSS[1])
SIADD = (27, 0)
# Rodrigues: t = 1 - c; diagonal c + t a_i a_i (2 mul, 1 add); off-diagonal
# t a_i a_j -/+ s a_k (3 mul, 1 add); sin and cos
AXROT = (1 + 3 * 1 + 6 * 1, 3 * 2 + 6 * 3)

EXPECTED = {"dot": DOT, "cross": CROSS, "m3v3": M3V3, "m3m3": M3M3, "xform_motion": XM, "xform_force_T": XFT,
            "crm": CRM, "crf": CRF, "si_mul": SIMUL, "sdot": SDOT, "congruence": CONG, "si_add": SIADD,
            "axis_rotation": AXROT}


def test_primitive_tallies_match_hand_counts():
    got = oracle.opcount_primitives()
    for name, (a, m) in EXPECTED.items():
        t = got[name]
        assert (t["add"], t["mul"], t["div"], t["sqrt"]) == (a, m, 0, 0), (name, t)
        assert t["trans"] == (2 if name == "axis_rotation" else 0), (name, t)
    # the literal totals of the two biggest pieces, for the record
    assert sum(XM) == 42 and sum(CONG) == 342


def flops(c):
    return c[0] + c[1]


def aba_count(n):
    """(add, mul, div) of one ABA solve of an n-joint revolute chain, as the
    oracle states it (Featherstone Table 7.1, dense 6-vector operations)."""
    add = mul = div = 0
    # pass 1 per joint: joint transform (axis rotation), vJ = S qd (6 mul),
    # v = X v_parent + vJ (6 add), c = v x vJ, p = v x* (I v)
    a1 = AXROT[0] + XM[0] + 6 + CRM[0] + SIMUL[0] + CRF[0]
    m1 = AXROT[1] + 6 + XM[1] + CRM[1] + SIMUL[1] + CRF[1]
    add += n * a1
    mul += n * m1
    # pass 2 per joint: U = IA S, D = S.U + arm, u = tau - S.pA
    a2 = SIMUL[0] + SDOT[0] + 1 + SDOT[0] + 1
    m2 = SIMUL[1] + 2 * SDOT[1]
    add += n * a2
    mul += n * m2
    # ... and for every joint with a parent: 1/D, U/D (6 mul), Ia = IA - U (U/D)^T
    # (21 distinct entries, 1 mul + 1 add each), pa = pA + Ia c + U (u/D)
    # (1 + 6 mul, 2 vector adds), congruence into the parent plus the sum,
    # X^T pa plus the sum
    ap = 21 + SIMUL[0] + 12 + CONG[0] + SIADD[0] + XFT[0] + 6
    mp = 6 + 21 + SIMUL[1] + 1 + 6 + CONG[1] + XFT[1]
    add += (n - 1) * ap
    mul += (n - 1) * mp
    div += n - 1
    # pass 3 per joint: a1 = X a_parent + c (6 add), qdd = (u - a1.U) / D,
    # a = a1 + S qdd (6 mul, 6 add)
    add += n * (XM[0] + 6 + SDOT[0] + 1 + 6)
    mul += n * (XM[1] + SDOT[1] + 6)
    div += n
    return add, mul, div


def physics_count(n, S):
    add, mul, div = aba_count(n)
    # per substep and joint: tau = kp (q* - q - h qd) - kd qd (3 mul, 3 add),
    # qd += h qdd, q += h qd (2 mul, 2 add)
    add, mul, div = S * (add + 5 * n), S * (mul + 5 * n), S * div
    # per step: h = dt / S (1 div); per joint mid, half, q* (3 mul, 3 add) and
    # arm = h kd + h^2 kp (3 mul, 1 add)
    return add + 4 * n, mul + 6 * n, div + 1


def fk_count(n):
    # per joint p += R o (9 mul, 9 add), R = R Rot(axis, q); then tip = p + R t
    return n * (9 + M3M3[0] + AXROT[0]) + 9, n * (9 + M3M3[1] + AXROT[1]) + 9


@pytest.mark.parametrize("n,S", [(1, 1), (2, 3), (4, 2), (7, 4), (9, 1)])
def test_step_count_matches_the_method_structure(n, S):
    robot = synth.make_chain(3, n, 11, dt=1 / 120, substeps=S)
    task = synth.path_rollout(3, dtype=np.float64).task
    o = oracle.Oracle(robot, task)
    a = synth.random_actions(3, 3, n)
    step, phys = o.opcount_step(a, env=1)
    pa, pm, pd = physics_count(n, S)
    assert (phys["add"], phys["mul"], phys["div"], phys["sqrt"]) == (pa, pm, pd, 0), (phys, (pa, pm, pd))
    assert phys["trans"] == 2 * n * S
    # after the substeps: kinematics for the reward, reward = -|tip - goal|
    # (3 + 3 mul + 2 add + sqrt), then the observation's kinematics of the
    # (possibly reset) state and goal - tip, |goal - tip| (the same 9 flops)
    fa, fm = fk_count(n)
    assert step["add"] - phys["add"] == 2 * fa + 2 * (3 + 2)
    assert step["mul"] - phys["mul"] == 2 * fm + 2 * 3
    assert step["sqrt"] == 2 and step["div"] == pd
    assert step["trans"] - phys["trans"] == 2 * 2 * n


def test_benchmark_figures_follow_from_the_formula():
    import bench
    pa, pm, pd = physics_count(7, 4)
    assert pa + pm + pd == bench.PHYS_FLOPS_7DOF_S4
    fa, fm = fk_count(7)
    # the step kernel evaluates the kinematics once per step (again only
    # after a reset); the oracle's second evaluation for the observation is
    # not counted as algorithmic work
    assert pa + pm + pd + fa + fm + 2 * 9 == bench.STEP_FLOPS_7DOF_S4
