"""The C-ABI library loads and exports every function include/surgym.h
declares; host-side argument checks reject bad input before any GPU work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "surgym.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sg_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    import paper_2310_04676_amd as sg
    names = declared_functions()
    assert "sg_create" in names and "sg_rollout" in names and len(names) >= 18
    for n in names:
        assert hasattr(sg.lib, n), n
    assert "gfx950" in sg.version()


def test_create_rejects_bad_descriptions_without_gpu_work():
    import paper_2310_04676_amd as sg
    import synth
    w = synth.path_rollout(4)
    rd, td, keep = sg.make_descs(w.robot, w.task, sg.SG_F32)
    ctx = C.c_void_p()
    bad = sg.RobotDesc.from_buffer_copy(rd)
    bad.n_env = 0
    assert sg.lib.sg_create(C.byref(bad), C.byref(td), C.byref(ctx)) == sg.SG_E_INVAL
    assert b"n_env" in sg.lib.sg_last_error(None)
    bad = sg.RobotDesc.from_buffer_copy(rd)
    bad.max_dof = 17
    assert sg.lib.sg_create(C.byref(bad), C.byref(td), C.byref(ctx)) == sg.SG_E_UNSUPPORTED
    bad = sg.RobotDesc.from_buffer_copy(rd)
    bad.substeps = 0
    assert sg.lib.sg_create(C.byref(bad), C.byref(td), C.byref(ctx)) == sg.SG_E_INVAL
    axis = w.robot.axis.copy()
    axis[:, 2, 1] = [1.0, 1.0, 0.0]
    bad = sg.RobotDesc.from_buffer_copy(rd)
    a2 = np.ascontiguousarray(axis)
    bad.axis = a2.ctypes.data_as(C.POINTER(C.c_double))
    assert sg.lib.sg_create(C.byref(bad), C.byref(td), C.byref(ctx)) == sg.SG_E_INVAL
    assert b"unit" in sg.lib.sg_last_error(None)
    tb = sg.TaskDesc.from_buffer_copy(td)
    tb.n_waypoints = 33
    assert sg.lib.sg_create(C.byref(rd), C.byref(tb), C.byref(ctx)) == sg.SG_E_INVAL
    # calls on a null context fail cleanly
    assert sg.lib.sg_step(None, None, None, None, None) == sg.SG_E_INVAL
    assert sg.lib.sg_rollout(None, 1, None) == sg.SG_E_INVAL


def test_tuning_text_round_trip_and_errors_without_gpu():
    """The autotuner's remembered choices as text (host code only): lines
    merge, later lines win, export lists every key once, malformed lines and
    out-of-range values are rejected, a short buffer is truncated with its
    full length reported."""
    import paper_2310_04676_amd as sg
    # env counts no test creates, so no later context in this process matches
    key_a = "gfx950|n=100003|f32|j=7|pr=0|c=1|task=1|dof=7x100003"
    key_b = "gfx950|n=100019|f32|j=9|pr=0|c=1|task=0|dof=4x50000,9x50019"
    sg.tuning_import(f"{key_a} 1 1\n{key_b} 0 4\n\n{key_a} 3 1\n")
    lines = {l.split()[0]: l.split()[1:] for l in sg.tuning_export().splitlines()}
    assert lines[key_a] == ["3", "1"] and lines[key_b] == ["0", "4"]
    for bad in ("lonely-key\n", f"{key_a} 4 1\n", f"{key_a} 0 2\n", f"{key_a} 0 1 extra\n", f"{key_a} x 1\n"):
        with pytest.raises(sg.SgError):
            sg.tuning_import(bad)
    # lines before a malformed one stay merged
    with pytest.raises(sg.SgError):
        sg.tuning_import(f"{key_b} 2 1\nbroken\n")
    assert {l.split()[0]: l.split()[1:] for l in sg.tuning_export().splitlines()}[key_b] == ["2", "1"]
    n = C.c_size_t()
    assert sg.lib.sg_tuning_export(None, 0, C.byref(n)) == sg.SG_OK
    full = n.value
    buf = C.create_string_buffer(8)
    assert sg.lib.sg_tuning_export(buf, 8, C.byref(n)) == sg.SG_OK
    assert n.value == full and len(buf.value) == 7
    assert sg.lib.sg_tuning_export(None, 8, C.byref(n)) == sg.SG_E_INVAL
    assert sg.lib.sg_tuning_import(None) == sg.SG_E_INVAL
