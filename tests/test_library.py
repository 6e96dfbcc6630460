"""Host-side checks of the HIP library: it loads and exports every symbol its
header declares, and the pure host entry points validate their inputs.  No
compute call is made here (this runs without a GPU)."""
import ctypes as C
import os
import re

import pytest

from paper_1908_05232_amd import fps, inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "fps.h")).read()
    return sorted(set(re.findall(r"\b(fps_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(fps.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = fps.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_struct_layouts_match_header(tmp_path):
    """Compile a probe against include/fps.h and compare sizes and offsets with ctypes."""
    import subprocess
    structs = {"fps_grid_desc": fps.GridDescC, "fps_ped_params": fps.PedParamsC,
               "fps_diag": fps.DiagC}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fps.h"', "int main(void){"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, cls in structs.items():
        assert got[(cname, "size")] == C.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_workspace_query_validates():
    L = fps.lib()
    d = fps.grid_desc_c(I.GridDesc(nx=64, ny=32, dx=0.5, dy=0.5))
    n0 = L.fps_workspace_bytes(C.byref(d), 0)
    n1 = L.fps_workspace_bytes(C.byref(d), 1000)
    assert 0 < n0 < n1
    # three FP32 ping-pong fields + counts at least
    assert n0 >= 64 * 32 * 16
    bad = fps.grid_desc_c(I.GridDesc(nx=0, ny=32, dx=0.5, dy=0.5))
    assert L.fps_workspace_bytes(C.byref(bad), 0) == 0
    bad = fps.grid_desc_c(I.GridDesc(nx=4, ny=4, dx=0.5, dy=0.5, cfl=1.5))
    assert L.fps_workspace_bytes(C.byref(bad), 0) == 0
    assert L.fps_workspace_bytes(C.byref(d), -1) == 0
    # the flood kernels address a grid by 32-bit byte offsets: 2^30 cells is the
    # largest grid taken, one row more is refused
    big = fps.grid_desc_c(I.GridDesc(nx=32768, ny=32768, dx=0.25, dy=0.25))
    assert L.fps_workspace_bytes(C.byref(big), 0) >= 32768 * 32768 * 16
    over = fps.grid_desc_c(I.GridDesc(nx=32768, ny=32769, dx=0.25, dy=0.25))
    assert L.fps_workspace_bytes(C.byref(over), 0) == 0


def test_create_rejects_bad_arguments_without_touching_the_device():
    L = fps.lib()
    d = fps.grid_desc_c(I.GridDesc(nx=8, ny=8, dx=1, dy=1))
    out = C.c_void_p()
    # NULL workspace and misaligned workspace are rejected before any HIP call
    assert L.fps_create(C.byref(d), None, 0, None, 1 << 20, None, C.byref(out)) == fps.FPS_E_INVALID
    assert L.fps_create(C.byref(d), None, 0, C.c_void_p(4096 + 8), 1 << 20, None,
                        C.byref(out)) == fps.FPS_E_INVALID
    assert L.fps_create(C.byref(d), None, 0, C.c_void_p(4096), 16, None,
                        C.byref(out)) == fps.FPS_E_CAPACITY
    assert b"workspace" in L.fps_last_error(None)
    assert L.fps_status_string(fps.FPS_E_NUMERIC) == b"numeric fault"
    p = fps.PedParamsC()
    L.fps_ped_params_default(C.byref(p))
    assert list(p.v_class) == [0.0, 1.8, 0.9, 0.45, 0.0] and list(p.hr_t) == [0.75, 1.5, 2.5]
    assert p.pick_s == 30.0 and p.drop_s == 30.0


def test_agent_sample_calls_reject_null_arrays_without_touching_the_device():
    L = fps.lib()
    buf = C.c_void_p(4096)          # never dereferenced: every call below fails its checks first
    thr = (C.c_double * 3)(0.75, 1.5, 2.5)
    flood = [buf] * 6
    # judge: NULL agent or flood arrays are rejected when there are agents to sample
    nosel = (None, None, None, 0.0, 0.0)
    assert L.fps_sur_judge(4, 1, None, buf, buf, 8, 8, 1.0, 1.0, *flood, 0.05, 1e-5, thr, *nosel, buf,
                           None) == fps.FPS_E_INVALID
    assert L.fps_sur_judge(4, 1, buf, buf, buf, 8, 8, 1.0, 1.0, buf, None, *flood[2:], 0.05, 1e-5, thr, *nosel,
                           buf, None) == fps.FPS_E_INVALID
    assert L.fps_sur_judge(4, 0, buf, buf, buf, 8, 8, 1.0, 1.0, *flood, 0.05, 1e-5, thr, *nosel, buf,
                           None) == fps.FPS_E_INVALID
    # a selection state with a missing plane, or a negative margin
    assert L.fps_sur_judge(4, 1, buf, buf, buf, 8, 8, 1.0, 1.0, *flood, 0.05, 1e-5, thr, buf, None, buf, 0.1,
                           0.01, buf, None) == fps.FPS_E_INVALID
    assert L.fps_sur_judge(4, 1, buf, buf, buf, 8, 8, 1.0, 1.0, *flood, 0.05, 1e-5, thr, buf, buf, buf, -0.1,
                           0.01, buf, None) == fps.FPS_E_INVALID
    assert L.fps_sur_judge_mask(4, 1, buf, buf, None, 8, 8, 1.0, 1.0, None, None, None, 1e-5, None, 0.0, 0.0,
                                1, 4, buf, None) == fps.FPS_E_INVALID
    assert L.fps_sur_judge_mask(4, 1, buf, buf, buf, 8, 8, 1.0, 1.0, None, None, None, 1e-5, None, 0.0, 0.0,
                                1, 0, buf, None) == fps.FPS_E_INVALID
    assert L.fps_sur_judge_mask(4, 1, buf, buf, buf, 8, 8, 1.0, 1.0, buf, buf, buf, 1e-5, None, 0.1, 0.0,
                                1, 4, buf, None) == fps.FPS_E_INVALID
    assert L.fps_sur_occupancy(4, buf, buf, None, buf, 8, 8, 1.0, 1.0, buf, None) == fps.FPS_E_INVALID
    assert L.fps_sur_occupancy(-1, buf, buf, buf, buf, 8, 8, 1.0, 1.0, buf, None) == fps.FPS_E_INVALID
    assert b"fps_sur_occupancy" in L.fps_sur_last_error(None)
