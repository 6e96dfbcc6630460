"""GPU checks of the C-ABI contract: error codes, latched numeric faults,
resume, and the read-side hazard field."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_1908_05232_amd import fps, inputs as I
from tests.gpu_util import say, snapshot

pytestmark = pytest.mark.gpu


def test_numeric_fault_is_latched_and_cleared():
    sc = I.cfg1_dam_break()
    sim = fps.Sim(sc)
    sim.step(3)
    sim.h[10, 20] = float("nan")
    sim.step(2)
    d = sim.diag(check=False)
    say("diag after NaN:", d["rc"], d["status"])
    assert d["rc"] == fps.FPS_E_NUMERIC
    with pytest.raises(fps.FpsError) as e:
        sim.step(1)
    assert e.value.code == fps.FPS_E_STATE
    # reads stay available
    hz = sim.hazard()
    torch.cuda.synchronize()
    assert hz.shape == sim.h.shape
    # a clean state bound again steps normally
    sim.h.copy_(torch.tensor(sc.h, dtype=torch.float32))
    sim.qx.zero_()
    sim.qy.zero_()
    sim.rebind_fields()
    sim.step(5)
    assert sim.diag()["rc"] == fps.FPS_OK


def test_invalid_arguments_and_capacity():
    sc = I.cfg1_dam_break()
    sim = fps.Sim(sc)
    L = fps.lib()
    assert L.fps_step(sim.h_, -1) == fps.FPS_E_INVALID
    t = np.array([0.0, 10.0, 5.0])
    q = np.zeros(3)
    assert L.fps_set_hydrograph(sim.h_, t.ctypes.data_as(C.POINTER(C.c_double)),
                                q.ctypes.data_as(C.POINTER(C.c_double)), 3) == fps.FPS_E_INVALID
    t = np.arange(70, dtype=np.float64)
    q = np.zeros(70)
    assert L.fps_set_hydrograph(sim.h_, t.ctypes.data_as(C.POINTER(C.c_double)),
                                q.ctypes.data_as(C.POINTER(C.c_double)), 70) == fps.FPS_E_INVALID
    cells = np.zeros(2 * (64 + 64) + 1, np.int32)
    assert L.fps_set_barrier(sim.h_, cells.ctypes.data_as(C.POINTER(C.c_int32)), len(cells), 0, 0, 1,
                             0.2, 0.2, 1) == fps.FPS_E_CAPACITY
    cells = np.array([64 * 64], np.int32)
    assert L.fps_set_barrier(sim.h_, cells.ctypes.data_as(C.POINTER(C.c_int32)), 1, 0, 0, 1,
                             0.2, 0.2, 1) == fps.FPS_E_INVALID
    a = sim.agents_t
    args = [fps._ptr(a[k]) for k in ("x", "y", "vx", "vy", "v_base", "role", "state", "hr_class",
                                      "dest", "timer")]
    assert L.fps_bind_agents(sim.h_, sim.max_agents + 1, *args) == fps.FPS_E_CAPACITY
    a["x"][3] = 1000.0                                    # outside the 32 m box
    assert L.fps_bind_agents(sim.h_, sim.na, *args) == fps.FPS_E_INVALID
    assert b"outside" in L.fps_last_error(sim.h_)
    a["x"][3] = 1.0
    a["dest"][4] = 7                                      # only one destination exists
    assert L.fps_bind_agents(sim.h_, sim.na, *args) == fps.FPS_E_INVALID
    a["dest"][4] = -1
    assert L.fps_bind_agents(sim.h_, sim.na, *args) == fps.FPS_OK


def test_step_before_binding_is_a_state_error():
    d = fps.grid_desc_c(I.GridDesc(nx=16, ny=16, dx=1, dy=1))
    L = fps.lib()
    n = L.fps_workspace_bytes(C.byref(d), 0)
    ws = torch.empty(n + 256, dtype=torch.uint8, device="cuda")
    p = ws.data_ptr() + (-ws.data_ptr()) % 256
    h = C.c_void_p()
    assert L.fps_create(C.byref(d), None, 0, C.c_void_p(p), n, None, C.byref(h)) == fps.FPS_OK
    assert L.fps_step(h, 1) == fps.FPS_E_STATE
    L.fps_destroy(h)


def test_resume_is_bit_identical():
    sc = I.cfg1_dam_break(n_ped=200)
    full = fps.Sim(sc)
    full.step(150)
    part = fps.Sim(sc)
    part.step(100)
    chk, d = snapshot(part, sc)
    resumed = fps.Sim(chk)
    resumed.set_time(d["t"], d["step"])
    resumed.step(50)
    for x, y in zip(full.fields(), resumed.fields()):
        assert np.array_equal(x, y)
    A, B = full.agents(), resumed.agents()
    for k in A:
        assert np.array_equal(A[k], B[k]), k
    assert full.diag()["t"] == resumed.diag()["t"]


def test_hazard_field_definition():
    sc = I.cfg1_dam_break()
    sim = fps.Sim(sc)
    sim.step(100)
    hz = sim.hazard().cpu().numpy()
    h, qx, qy, _ = sim.fields()
    with np.errstate(divide="ignore", invalid="ignore"):
        ref = np.where(h > 1e-5, (np.maximum(np.abs(qx / h), np.abs(qy / h)) + 0.5) * h, 0.0)
    assert np.allclose(hz, ref, rtol=1e-6, atol=1e-7)


def test_time_flood_leaves_the_state_unchanged():
    sc = I.shopping_centre(n=128, dx=0.5, seed=9, n_evac=300)
    a, b = fps.Sim(sc), fps.Sim(sc)
    a.step(40)
    b.step(40)
    before = a.fields()
    ms = a.time_flood(25)
    say(f"flood update 128^2: {ms * 1e3:.1f} us per launch")
    assert ms > 0
    for x, y in zip(before, a.fields()):
        assert np.array_equal(x, y)
    assert a.diag()["dt_next"] == b.diag()["dt_next"]
    a.step(30)
    b.step(30)
    for x, y in zip(a.fields(), b.fields()):
        assert np.array_equal(x, y)
    A, B = a.agents(), b.agents()
    for k in A:
        assert np.array_equal(A[k], B[k])
