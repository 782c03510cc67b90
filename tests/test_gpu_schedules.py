"""Uneven-DOF batches: every step schedule gives the same results as the
padded one (and the oracle), and the autotuner picks one of them without
disturbing the state."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("n_env", [333, 2000])
def test_schedules_agree(sg, n_env):
    import torch
    w = synth.mixed_dof(n_env)
    ref = sg.Sim(w.robot, w.task)
    outs = {}
    for sched in (sg.SG_SCHED_PADDED, sg.SG_SCHED_SORTED, sg.SG_SCHED_PER_CLASS, sg.SG_SCHED_PERSISTENT):
        sim = sg.Sim(w.robot, w.task)
        sim.set_schedule(sched)
        assert sim.get_schedule() == sched
        res = []
        for s in range(3):
            a = torch.from_numpy(synth.random_actions(70 + s, n_env, 9, np.float32)).float().cuda()
            o, r, d = sim.step(a)
            q, qd, pr, _ = sim.get_state()
            res.append((host(o), host(r), d.cpu().numpy(), host(q), host(qd), pr.cpu().numpy()))
        outs[sched] = res
    base = outs[sg.SG_SCHED_PADDED]
    for sched, res in outs.items():
        for (o, r, d, q, qd, pr), (o0, r0, d0, q0, qd0, pr0) in zip(res, base):
            assert np.array_equal(d, d0) and np.array_equal(pr, pr0), sched
            np.testing.assert_allclose(q, q0, rtol=1e-5, atol=1e-6)
            np.testing.assert_allclose(qd, qd0, rtol=1e-4, atol=1e-4)
            np.testing.assert_allclose(o, o0, rtol=1e-4, atol=1e-4)
            np.testing.assert_allclose(r, r0, rtol=1e-5, atol=1e-6)


def test_sorted_schedule_matches_oracle_with_handoff(sg):
    import torch
    w = synth.mixed_dof(500)
    sim = sg.Sim(w.robot, w.task)
    sim.set_schedule(sg.SG_SCHED_SORTED)
    o = oracle.Oracle(w.robot, w.task)
    for s in range(10):
        q0, qd0, pr0, _ = sim.get_state()
        a = synth.random_actions(300 + s, 500, 9, np.float32)
        obs, rew, done = sim.step(torch.from_numpy(a).float().cuda())
        q1, _, pr1, _ = sim.get_state()
        qn, _, prn, rw, dn, ob = o.step(a, host(q0), host(qd0), pr0.cpu().numpy())
        assert np.array_equal(done.cpu().numpy(), dn)
        assert np.array_equal(pr1.cpu().numpy(), prn)
        assert (np.abs(host(q1) - qn) / (1 + np.abs(qn))).max() <= 2e-5
        assert np.abs(host(rew) - rw).max() <= 2e-4


def test_autotune_restores_state_and_picks_a_schedule(sg):
    import torch
    w = synth.mixed_dof(4096)
    sim = sg.Sim(w.robot, w.task)
    q0, qd0, pr0, _ = sim.get_state()
    a = torch.rand(9, 4096, device="cuda") * 2 - 1
    best, team, ms = sim.autotune_step(a, trials=3)
    assert best in (0, 1, 2, 3) and team in (1, 4)
    assert set(ms) == {"padded", "sorted", "per_class", "persistent", "padded_team"}
    chosen = "padded_team" if team == 4 else sg.SCHEDULE_NAMES[best]
    assert team == 1 or best == sg.SG_SCHED_PADDED
    assert ms[chosen] == min(ms.values())
    q1, qd1, pr1, _ = sim.get_state()
    assert np.array_equal(host(q0), host(q1)) and np.array_equal(host(qd0), host(qd1))
    assert np.array_equal(pr0.cpu().numpy(), pr1.cpu().numpy())
    assert sim.get_schedule() == best and sim.get_team() == team
    # the choice is remembered: a new context of the same mix starts from it,
    # and it survives an export / import round trip
    sim2 = sg.Sim(w.robot, w.task)
    assert (sim2.get_schedule(), sim2.get_team()) == (best, team)
    text = sg.tuning_export()
    line = [l for l in text.splitlines() if "|n=4096|f32|j=9|" in l]
    assert len(line) == 1 and line[0].split()[1:] == [str(best), str(team)], text
    key = line[0].split()[0]
    other = 1 if best != 1 else 0
    sg.tuning_import(f"{key} {other} 1\n")
    sim3 = sg.Sim(w.robot, w.task)
    assert (sim3.get_schedule(), sim3.get_team()) == (other, 1)
    sg.tuning_import(f"{key} {best} {team}\n")
    with pytest.raises(sg.SgError):
        sg.tuning_import("key-without-values\n")
    with pytest.raises(sg.SgError):
        sg.tuning_import(f"{key} 7 1\n")
    for s_ in (sim, sim2, sim3):
        s_.close()
    # FP64 contexts keep the padded schedule
    w64 = synth.reach_fp64(64)
    s64 = sg.Sim(w64.robot, w64.task, dtype=np.float64)
    with pytest.raises(sg.SgError):
        s64.set_schedule(sg.SG_SCHED_SORTED)
