"""The algorithmic work figures bench.py divides by time are the exact
operation counts of the op-counting oracle for the benchmark workload."""
import numpy as np

import bench
import oracle
import synth


def test_algorithmic_flop_constants_match_the_op_counter():
    w = synth.path_rollout(4, dtype=np.float64)
    o = oracle.Oracle(w.robot, w.task)
    a = synth.random_actions(0, 4, 7)
    flops = lambda c: c["add"] + c["mul"] + c["div"] + c["sqrt"]
    for e in range(4):
        step, phys = o.opcount_step(a, env=e)
        # the counter's step evaluates the kinematics twice (reward, then the
        # observation); the benchmark counts one evaluation
        post = flops(step) - flops(phys)
        assert (post + 2 * 9) % 2 == 0
        assert flops(phys) + (post + 2 * 9) // 2 == bench.STEP_FLOPS_7DOF_S4
        assert flops(phys) == bench.PHYS_FLOPS_7DOF_S4
        assert step["trans"] == bench.TRANS_7DOF_S4 + 2 * 7
    d = w.policy.dims
    assert bench.POLICY_FLOPS == 2 * (d[0] * d[1] + d[1] * d[2] + d[2] * d[3])
