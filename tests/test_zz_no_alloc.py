"""The allocation-free adjoint (sg_adjoint_static, fixed 16 MiB workspace)
against sg_adjoint (library-allocated workspace) through the C ABI: two
calls in a row, the second with fewer envs and steps, each compared with
sg_adjoint on the same inputs. Both run the same kernels on the same inputs,
so the results agree to FP32 rounding (they are expected to be identical;
the check allows 1e-6 relative). Too large a (T, K) is rejected on the host
with SG_E_INVAL before any work is enqueued."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _actions(torch, seed, T, J, N):
    act = np.random.default_rng(seed).uniform(-0.95, 0.95, (T, J, N)).astype(np.float32)
    return torch.from_numpy(act).cuda()


@pytest.mark.parametrize("first,second", [((1024, 24, 8), (300, 10, 5))])
def test_static_workspace_matches_allocating_adjoint(sg, first, second):
    import torch
    for seed, (N, T, K) in enumerate((first, second)):
        w = synth.path_rollout(N)
        sim = sg.Sim(w.robot, w.task)
        act = _actions(torch, 40 + seed, T, w.robot.max_dof, N)
        assert sim.adjoint_workspace_bytes(T, K) <= 16 << 20
        ref = [host(x) for x in sim.adjoint(act, K)]
        got = [host(x) for x in sim.adjoint(act, K, static=True)]
        for g, r in zip(got, ref):
            assert np.all(np.isfinite(g))
            np.testing.assert_allclose(g, r, rtol=1e-6, atol=1e-6 * max(1.0, np.abs(r).max()))
        sim.synchronize()


def test_static_workspace_rejects_too_large_sizes(sg):
    import torch
    w = synth.path_rollout(4096)
    sim = sg.Sim(w.robot, w.task)
    T, K = 64, 32  # 32 steps of tape at 4096 envs: about 48 MB
    assert sim.adjoint_workspace_bytes(T, K) > 16 << 20
    act = torch.zeros(T, 7, 4096, device="cuda")
    with pytest.raises(RuntimeError, match="exceeds the fixed"):
        sim.adjoint(act, K, static=True)
    sim.synchronize()
