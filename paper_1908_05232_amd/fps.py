"""ctypes binding of libfps.so (C-ABI in include/fps.h).

Argument marshalling only: every step of the simulation runs in the HIP
kernels of libfps.  PyTorch provides device memory and the stream.  Importing
this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfps.so")

FPS_OK, FPS_E_INVALID, FPS_E_DEVICE, FPS_E_STATE, FPS_E_CAPACITY, FPS_E_NUMERIC = 0, -1, -2, -3, -4, -5
FPS_FLUX_HLLC, FPS_FLUX_HLL = 0, 1

_vp = C.c_void_p


class GridDescC(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("dx", C.c_double), ("dy", C.c_double),
        ("g", C.c_double), ("cfl", C.c_double), ("h_dry", C.c_double), ("dt_max", C.c_double),
        ("bc", C.c_int32 * 4),
        ("inflow_side", C.c_int32), ("inflow_c0", C.c_int32), ("inflow_c1", C.c_int32),
        ("n_base", C.c_double), ("np_cap", C.c_int32),
    ]


class PedParamsC(C.Structure):
    _fields_ = [
        ("tau", C.c_double), ("a_over_m", C.c_double), ("b_range", C.c_double),
        ("radius", C.c_double), ("r_cut", C.c_double), ("r_arrive", C.c_double),
        ("v_class", C.c_double * 5), ("hr_t", C.c_double * 3),
        ("pick_s", C.c_double), ("drop_s", C.c_double),
        ("stability", C.c_int32),
        ("c_drag", C.c_double), ("mu_f", C.c_double), ("rho_w", C.c_double), ("rho_body", C.c_double),
        ("body_h0", C.c_double), ("body_m0", C.c_double),
        ("wading", C.c_int32), ("wade_k", C.c_double),
    ]


class DiagC(C.Structure):
    _fields_ = [
        ("t", C.c_double), ("step", C.c_int64), ("ped_steps", C.c_int64),
        ("dt_last", C.c_double), ("dt_next", C.c_double),
        ("mass", C.c_double), ("v_in", C.c_double), ("v_out", C.c_double), ("v_clip", C.c_double),
        ("any_wet", C.c_int32), ("n_agents", C.c_int32),
        ("class_count", C.c_int32 * 6), ("state_count", C.c_int32 * 8),
        ("barrier_layers_done", C.c_int32), ("barrier_active_cell", C.c_int32),
        ("barrier_bags", C.c_int32), ("barrier_done", C.c_int32),
        ("drops_total", C.c_int32), ("status", C.c_int32),
        ("active", C.c_int32), ("flood_steps", C.c_int32),
        ("doors_closed", C.c_int32), ("door_entries", C.c_int64), ("door_leaves", C.c_int64),
    ]


EXPORTS = {
    "fps_ped_params_default": (None, [C.POINTER(PedParamsC)]),
    "fps_workspace_bytes": (C.c_size_t, [C.POINTER(GridDescC), C.c_int32]),
    "fps_create": (C.c_int, [C.POINTER(GridDescC), C.POINTER(PedParamsC), C.c_int32, _vp, C.c_size_t,
                             _vp, C.POINTER(_vp)]),
    "fps_destroy": (None, [_vp]),
    "fps_bind_fields": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "fps_set_hydrograph": (C.c_int, [_vp, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int32]),
    "fps_set_navigation": (C.c_int, [_vp, C.c_int32, C.c_int32, _vp, _vp]),
    "fps_bind_agents": (C.c_int, [_vp, C.c_int32] + [_vp] * 10),
    "fps_set_barrier": (C.c_int, [_vp, C.POINTER(C.c_int32), C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                  C.c_float, C.c_float, C.c_int32]),
    "fps_set_time": (C.c_int, [_vp, C.c_double, C.c_int64]),
    "fps_set_bodies": (C.c_int, [_vp, _vp, _vp]),
    "fps_set_doors": (C.c_int, [_vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int32,
                                C.c_uint64]),
    "fps_step": (C.c_int, [_vp, C.c_int32]),
    "fps_get_diag": (C.c_int, [_vp, C.POINTER(DiagC)]),
    "fps_get_time": (C.c_int, [_vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "fps_hazard_field": (C.c_int, [_vp, _vp]),
    "fps_get_counts": (C.c_int, [_vp, _vp]),
    "fps_get_bins": (C.c_int, [_vp, _vp, _vp, C.POINTER(C.c_int32)]),
    "fps_step_profiled": (C.c_int, [_vp, C.c_int32, C.POINTER(C.c_double)]),
    "fps_set_end_time": (C.c_int, [_vp, C.c_double]),
    "fps_set_graph": (C.c_int, [_vp, C.c_int32]),
    "fps_set_flux": (C.c_int, [_vp, C.c_int32]),
    "fps_set_order": (C.c_int, [_vp, C.c_int32]),
    "fps_ens_set_order": (C.c_int, [_vp, C.c_int32]),
    "fps_ens_workspace_bytes": (C.c_size_t, [C.c_int32, C.POINTER(GridDescC), C.POINTER(C.c_int32)]),
    "fps_ens_create": (C.c_int, [C.c_int32, C.POINTER(GridDescC), C.POINTER(PedParamsC),
                                 C.POINTER(C.c_int32), _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    "fps_ens_destroy": (None, [_vp]),
    "fps_ens_member": (_vp, [_vp, C.c_int32]),
    "fps_ens_step": (C.c_int, [_vp, C.c_int32]),
    "fps_ens_set_flux": (C.c_int, [_vp, C.c_int32]),
    "fps_ens_step_profiled": (C.c_int, [_vp, C.c_int32, C.POINTER(C.c_double)]),
    "fps_ens_set_graph": (C.c_int, [_vp, C.c_int32]),
    "fps_ens_autotune": (C.c_int, [_vp, C.c_char_p]),
    "fps_ens_active": (C.c_int, [_vp, C.POINTER(C.c_int32)]),
    "fps_ens_time_flood": (C.c_int, [_vp, C.c_int32, C.POINTER(C.c_double)]),
    "fps_ens_last_error": (C.c_char_p, [_vp]),
    "fps_sur_param_count": (C.c_int32, []),
    "fps_sur_workspace_bytes": (C.c_size_t, [C.c_int32, C.c_int32, C.c_int32]),
    "fps_sur_set_blocks": (C.c_int, [_vp, C.c_int32, C.c_int32]),
    "fps_sur_forward_noalloc": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32, _vp, _vp, _vp]),
    "fps_sur_create": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    "fps_sur_destroy": (None, [_vp]),
    "fps_sur_set_params": (C.c_int, [_vp, _vp]),
    "fps_sur_get_params": (C.c_int, [_vp, _vp]),
    "fps_sur_forward": (C.c_int, [_vp, C.c_int32, _vp, _vp]),
    "fps_sur_gradients": (C.c_int, [_vp, C.c_int32, _vp, _vp, _vp, _vp]),
    "fps_sur_adam": (C.c_int, [_vp, C.c_float]),
    "fps_sur_train_step": (C.c_int, [_vp, C.c_int32, _vp, _vp, C.c_float, _vp]),
    "fps_set_judge_region": (C.c_int, [_vp, _vp, C.c_int32]),
    "fps_inflow_depth": (C.c_int, [_vp, C.c_double, C.c_double, C.POINTER(C.c_double)]),
    "fps_time_flood": (C.c_int, [_vp, C.c_int32, C.POINTER(C.c_double)]),
    "fps_set_occupancy": (C.c_int, [_vp, _vp]),
    "fps_set_flood_frozen": (C.c_int, [_vp, C.c_int32]),
    "fps_sur_pack": (C.c_int, [C.c_int32, C.c_int32, _vp, _vp, _vp, _vp, _vp, C.c_int32, C.c_int32, C.c_int32,
                               C.c_double, _vp, _vp]),
    "fps_sur_make_target": (C.c_int, [C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "fps_sur_apply": (C.c_int, [C.c_int64, _vp, _vp, _vp, _vp, C.c_float, C.c_float, _vp]),
    "fps_sur_judge": (C.c_int, [C.c_int32, C.c_int32, _vp, _vp, _vp, C.c_int32, C.c_int32, C.c_double,
                                C.c_double, _vp, _vp, _vp, _vp, _vp, _vp, C.c_double, C.c_double,
                                C.POINTER(C.c_double), _vp, _vp, _vp, C.c_double, C.c_double, _vp, _vp]),
    "fps_sur_judge_mask": (C.c_int, [C.c_int32, C.c_int32, _vp, _vp, _vp, C.c_int32, C.c_int32, C.c_double,
                                     C.c_double, _vp, _vp, _vp, C.c_double, C.POINTER(C.c_double), C.c_double,
                                     C.c_double, C.c_int32, C.c_int32, _vp, _vp]),
    "fps_sur_occupancy": (C.c_int, [C.c_int32, _vp, _vp, _vp, _vp, C.c_int32, C.c_int32, C.c_double,
                                    C.c_double, _vp, _vp]),
    "fps_sur_copy_state": (C.c_int, [C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "fps_sur_last_error": (C.c_char_p, [_vp]),
    "fps_set_rows_per_wave": (C.c_int, [_vp, C.c_int32]),
    "fps_get_rows_per_wave": (C.c_int, [_vp, C.POINTER(C.c_int32)]),
    "fps_autotune": (C.c_int, [_vp, C.c_char_p, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "fps_stream_probe": (C.c_int, [_vp, C.c_int64, C.c_int64, C.c_int32, C.c_int32, C.c_int32, _vp,
                                   C.POINTER(C.c_double)]),
    "fps_status_string": (C.c_char_p, [C.c_int]),
    "fps_last_error": (C.c_char_p, [_vp]),
}

_lib = None


def lib():
    """Load libfps.so; raise if it is missing (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not built: run python -m paper_1908_05232_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class FpsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


def grid_desc_c(d) -> GridDescC:
    g = GridDescC()
    g.nx, g.ny, g.dx, g.dy = d.nx, d.ny, d.dx, d.dy
    g.g, g.cfl, g.h_dry, g.dt_max = d.g, d.cfl, d.h_dry, d.dt_max
    for k in range(4):
        g.bc[k] = d.bc[k]
    g.inflow_side, g.inflow_c0, g.inflow_c1 = d.inflow_side, d.inflow_c0, d.inflow_c1
    g.n_base, g.np_cap = d.n_base, d.np_cap
    return g


def ped_params_c(p) -> PedParamsC:
    c = PedParamsC()
    c.tau, c.a_over_m, c.b_range, c.radius, c.r_cut, c.r_arrive = (
        p.tau, p.a_over_m, p.b_range, p.radius, p.r_cut, p.r_arrive)
    for k in range(5):
        c.v_class[k] = p.v_class[k]
    for k in range(3):
        c.hr_t[k] = p.hr_t[k]
    c.pick_s, c.drop_s = p.pick_s, p.drop_s
    c.stability = int(getattr(p, "stability", 0))
    c.c_drag, c.mu_f = getattr(p, "c_drag", 1.1), getattr(p, "mu_f", 0.45)
    c.rho_w, c.rho_body = getattr(p, "rho_w", 1000.0), getattr(p, "rho_body", 1000.0)
    c.body_h0, c.body_m0 = getattr(p, "body_h0", 1.71), getattr(p, "body_m0", 70.0)
    c.wading, c.wade_k = int(getattr(p, "wading", 0)), getattr(p, "wade_k", 0.1)
    return c


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Member:
    """One scenario's device tensors bound to a libfps handle (standalone or
    ensemble member).  Argument marshalling only."""

    def _bind(self, h, sc, device):
        import torch
        self.torch = torch
        self.sc = sc
        self.device = torch.device(device)
        self.h_ = h
        L = self._lib
        f32 = dict(dtype=torch.float32, device=self.device)
        self.h = torch.tensor(np.asarray(sc.h, np.float32), **f32).contiguous()
        self.qx = torch.tensor(np.asarray(sc.qx, np.float32), **f32).contiguous()
        self.qy = torch.tensor(np.asarray(sc.qy, np.float32), **f32).contiguous()
        self.z = torch.tensor(np.asarray(sc.z, np.float32), **f32).contiguous()
        self._check(L.fps_bind_fields(h, _ptr(self.h), _ptr(self.qx), _ptr(self.qy), _ptr(self.z)))
        if sc.hydro_t is not None and len(sc.hydro_t):
            t = np.ascontiguousarray(sc.hydro_t, np.float64)
            q = np.ascontiguousarray(sc.hydro_q, np.float64)
            self._check(L.fps_set_hydrograph(h, t.ctypes.data_as(C.POINTER(C.c_double)),
                                             q.ctypes.data_as(C.POINTER(C.c_double)), len(t)))
        if sc.dist is not None:
            self.dist = torch.tensor(np.asarray(sc.dist, np.float32), **f32).contiguous()
            self.walk = torch.tensor(np.asarray(sc.walk, np.uint8), dtype=torch.uint8,
                                     device=self.device).contiguous()
            self._check(L.fps_set_navigation(h, self.dist.shape[0], sc.n_exit, _ptr(self.dist),
                                             _ptr(self.walk)))
        if sc.barrier is not None:
            b = sc.barrier
            cells = np.ascontiguousarray(b["cells"], np.int32)
            self._check(L.fps_set_barrier(h, cells.ctypes.data_as(C.POINTER(C.c_int32)), len(cells),
                                          b["storage_dest"], b["barrier_dest"], b["n_layers"],
                                          float(b["t_bag"]), float(b["t_last"]), b["bags_per"]))
        if getattr(sc, "doors", None) is not None:
            self.set_doors(sc.doors)
        self.na = 0 if sc.agents is None else len(sc.agents["x"])
        if self.na:
            A = sc.agents
            self.agents_t = {
                k: torch.tensor(np.asarray(A[k]), device=self.device).contiguous()
                for k in ("x", "y", "vx", "vy", "v_base", "role", "state", "hr_class", "dest", "timer")}
            a = self.agents_t
            self._check(L.fps_bind_agents(h, self.na, *[_ptr(a[k]) for k in (
                "x", "y", "vx", "vy", "v_base", "role", "state", "hr_class", "dest", "timer")]))
            if "height" in A and "mass" in A:
                self.body_t = {k: torch.tensor(np.asarray(A[k], np.float32), device=self.device).contiguous()
                               for k in ("height", "mass")}
                self._check(L.fps_set_bodies(h, _ptr(self.body_t["height"]), _ptr(self.body_t["mass"])))
        if sc.t0:
            self.set_time(sc.t0, 0)

    def _check(self, rc, h=0):
        if rc != FPS_OK:
            msg = self._lib.fps_last_error(self.h_ if h == 0 else h)
            raise FpsError(rc, (msg or b"").decode())
        return rc

    def set_time(self, t, step=0):
        return self._check(self._lib.fps_set_time(self.h_, float(t), int(step)))

    def set_doors(self, doors):
        """Pre-flood door flow: doors = dict(cells, dests, per_step, seed) or None (off)."""
        if doors is None:
            return self._check(self._lib.fps_set_doors(self.h_, 0, None, None, 0, 0))
        cells = np.ascontiguousarray(doors["cells"], np.int32)
        dests = np.ascontiguousarray(doors["dests"], np.int32)
        return self._check(self._lib.fps_set_doors(
            self.h_, len(cells), cells.ctypes.data_as(C.POINTER(C.c_int32)),
            dests.ctypes.data_as(C.POINTER(C.c_int32)), int(doors["per_step"]), int(doors["seed"])))

    def set_end_time(self, t_end):
        return self._check(self._lib.fps_set_end_time(self.h_, float(t_end)))

    def set_flux(self, flux):
        """Face flux of the flood update: FPS_FLUX_HLLC or FPS_FLUX_HLL
        (a standalone simulation; an ensemble sets it for all its members)."""
        return self._check(self._lib.fps_set_flux(self.h_, int(flux)))

    def set_order(self, order):
        """Order of the flood update: 1 (first order) or 2 (the MUSCL variant);
        a standalone simulation (an ensemble sets it for all its members)."""
        return self._check(self._lib.fps_set_order(self.h_, int(order)))

    def rebind_fields(self):
        return self._check(self._lib.fps_bind_fields(self.h_, _ptr(self.h), _ptr(self.qx), _ptr(self.qy),
                                                     _ptr(self.z)))

    def inflow_depth(self, t0, t1):
        """Depth the inflow adds to each inflow cell over [t0, t1] (host float)."""
        d = C.c_double()
        self._check(self._lib.fps_inflow_depth(self.h_, float(t0), float(t1), C.byref(d)))
        return d.value

    def inflow_feature(self, t0, t1):
        """(side, c0, c1, depth) for sur_pack."""
        g = self.sc.desc
        return (g.inflow_side, g.inflow_c0, g.inflow_c1, self.inflow_depth(t0, t1))

    def set_judge_region(self, mask, block):
        """mask: device uint8 [ceil(ny/block), ceil(nx/block)] tensor or None."""
        self._jmask = mask
        ptr = _ptr(mask) if mask is not None else None
        return self._check(self._lib.fps_set_judge_region(self.h_, ptr, int(block)))

    def set_flood_frozen(self, frozen):
        """Hold the flood (steps of dt_max move only the pedestrians) or resume."""
        return self._check(self._lib.fps_set_flood_frozen(self.h_, int(bool(frozen))))

    def set_occupancy(self, counts):
        self._occ = counts
        return self._check(self._lib.fps_set_occupancy(self.h_, _ptr(counts) if counts is not None else None))

    def autotune(self, cache_path=None):
        rows, ms = C.c_int32(), C.c_double()
        cp = None if cache_path is None else str(cache_path).encode()
        self._check(self._lib.fps_autotune(self.h_, cp, C.byref(rows), C.byref(ms)))
        return rows.value, ms.value

    def time_flood(self, reps=200):
        """Average ms per flood-update launch (back-to-back launches, state unchanged)."""
        ms = C.c_double()
        self._check(self._lib.fps_time_flood(self.h_, int(reps), C.byref(ms)))
        return ms.value

    def set_rows_per_wave(self, rows):
        return self._check(self._lib.fps_set_rows_per_wave(self.h_, int(rows)))

    def rows_per_wave(self):
        r = C.c_int32()
        self._check(self._lib.fps_get_rows_per_wave(self.h_, C.byref(r)))
        return r.value

    def diag(self, check=True):
        d = DiagC()
        rc = self._lib.fps_get_diag(self.h_, C.byref(d))
        if check:
            self._check(rc)
        out = {k: getattr(d, k) for k, _ in DiagC._fields_}
        out["class_count"] = list(d.class_count)
        out["state_count"] = list(d.state_count)
        out["rc"] = rc
        return out

    def time(self):
        """(simulated time, length of the next step) without a pass over the agents."""
        t, dt = C.c_double(), C.c_double()
        self._check(self._lib.fps_get_time(self.h_, C.byref(t), C.byref(dt)))
        return t.value, dt.value

    def fields(self):
        self.torch.cuda.synchronize(self.device)
        return tuple(t.cpu().numpy() for t in (self.h, self.qx, self.qy, self.z))

    def agents(self):
        self.torch.cuda.synchronize(self.device)
        return {k: v.cpu().numpy() for k, v in self.agents_t.items()}

    def hazard(self):
        out = self.torch.empty_like(self.h)
        self._check(self._lib.fps_hazard_field(self.h_, _ptr(out)))
        return out

    def counts(self):
        out = self.torch.empty(self.h.shape, dtype=self.torch.int32, device=self.device)
        self._check(self._lib.fps_get_counts(self.h_, _ptr(out)))
        return out

    def bins(self):
        nb = C.c_int32()
        self._check(self._lib.fps_get_bins(self.h_, None, None, C.byref(nb)))
        bs = self.torch.empty(nb.value + 1, dtype=self.torch.int32, device=self.device)
        perm = self.torch.empty(max(self.na, 1), dtype=self.torch.int32, device=self.device)
        self._check(self._lib.fps_get_bins(self.h_, _ptr(bs), _ptr(perm), C.byref(nb)))
        self.torch.cuda.synchronize(self.device)
        bs = bs.cpu().numpy()
        return bs, perm.cpu().numpy()[: bs[-1]]


def _workspace(torch, nbytes, device):
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws, C.c_void_p(ws.data_ptr() + off)


class Sim(Member):
    """One scenario on one GPU: device tensors + a standalone libfps handle."""

    def __init__(self, sc, device="cuda", stream=None, max_agents=None):
        import torch
        self._lib = L = lib()
        d = sc.desc
        self.desc_c = grid_desc_c(d)
        self.ped_c = ped_params_c(sc.ped)
        na = 0 if sc.agents is None else len(sc.agents["x"])
        self.max_agents = na if max_agents is None else max_agents
        nbytes = L.fps_workspace_bytes(C.byref(self.desc_c), self.max_agents)
        if nbytes == 0:
            raise FpsError(FPS_E_INVALID, "fps_workspace_bytes rejected the grid description")
        dev = torch.device(device)
        self.ws, self.ws_ptr = _workspace(torch, nbytes, dev)
        self.ws_bytes = nbytes
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = C.c_void_p()
        self.h_ = h
        self._check(L.fps_create(C.byref(self.desc_c), C.byref(self.ped_c), self.max_agents, self.ws_ptr,
                                 nbytes, C.c_void_p(self.stream.cuda_stream), C.byref(h)), None)
        self._bind(h, sc, device)
        if getattr(d, "flux", FPS_FLUX_HLLC) != FPS_FLUX_HLLC:
            self.set_flux(d.flux)
        if getattr(d, "order", 1) != 1:
            self.set_order(d.order)

    def close(self):
        if getattr(self, "h_", None) and self.h_.value:
            self._lib.fps_destroy(self.h_)
            self.h_ = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        return self._check(self._lib.fps_step(self.h_, int(n)))

    def step_profiled(self, n):
        ms = (C.c_double * 5)()
        self._check(self._lib.fps_step_profiled(self.h_, int(n), ms))
        return list(ms)

    def set_graph(self, steps_per_graph):
        return self._check(self._lib.fps_set_graph(self.h_, int(steps_per_graph)))



class _EnsMember(Member):
    def __init__(self, lib_, handle, sc, device):
        self._lib = lib_
        self._bind(handle, sc, device)


class Ensemble:
    """S scenarios of uneven grids stepped together by one set of launches per step."""

    def __init__(self, scenarios, device="cuda", stream=None):
        import torch
        self.torch = torch
        self._lib = L = lib()
        S = len(scenarios)
        self.descs = (GridDescC * S)(*[grid_desc_c(sc.desc) for sc in scenarios])
        self.peds = (PedParamsC * S)(*[ped_params_c(sc.ped) for sc in scenarios])
        na = [0 if sc.agents is None else len(sc.agents["x"]) for sc in scenarios]
        self.max_agents = (C.c_int32 * S)(*na)
        nbytes = L.fps_ens_workspace_bytes(S, self.descs, self.max_agents)
        if nbytes == 0:
            raise FpsError(FPS_E_INVALID, "fps_ens_workspace_bytes rejected the scenarios")
        dev = torch.device(device)
        self.ws, ws_ptr = _workspace(torch, nbytes, dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.e_ = C.c_void_p()
        rc = L.fps_ens_create(S, self.descs, self.peds, self.max_agents, ws_ptr, nbytes,
                              C.c_void_p(self.stream.cuda_stream), C.byref(self.e_))
        if rc != FPS_OK:
            raise FpsError(rc, (L.fps_last_error(None) or b"").decode())
        self.members = [_EnsMember(L, C.c_void_p(L.fps_ens_member(self.e_, k)), sc, device)
                        for k, sc in enumerate(scenarios)]
        fluxes = {getattr(sc.desc, "flux", FPS_FLUX_HLLC) for sc in scenarios}
        if len(fluxes) > 1:
            raise FpsError(FPS_E_INVALID, "the scenarios of an ensemble share one face flux")
        if fluxes != {FPS_FLUX_HLLC}:
            self.set_flux(fluxes.pop())
        orders = {getattr(sc.desc, "order", 1) for sc in scenarios}
        if len(orders) > 1:
            raise FpsError(FPS_E_INVALID, "the scenarios of an ensemble share one order")
        if orders != {1}:
            self.set_order(orders.pop())

    def _check(self, rc):
        if rc != FPS_OK:
            raise FpsError(rc, (self._lib.fps_ens_last_error(self.e_) or b"").decode())
        return rc

    def __len__(self):
        return len(self.members)

    def __getitem__(self, k):
        return self.members[k]

    def step(self, n=1):
        return self._check(self._lib.fps_ens_step(self.e_, int(n)))

    def step_profiled(self, n):
        ms = (C.c_double * 5)()
        self._check(self._lib.fps_ens_step_profiled(self.e_, int(n), ms))
        return list(ms)

    def set_graph(self, steps_per_graph):
        return self._check(self._lib.fps_ens_set_graph(self.e_, int(steps_per_graph)))

    def set_flux(self, flux):
        return self._check(self._lib.fps_ens_set_flux(self.e_, int(flux)))

    def set_order(self, order):
        return self._check(self._lib.fps_ens_set_order(self.e_, int(order)))

    def autotune(self, cache_path=None):
        cp = None if cache_path is None else str(cache_path).encode()
        return self._check(self._lib.fps_ens_autotune(self.e_, cp))

    def time_flood(self, reps=50):
        """Average ms per flood-update launch over every member (back-to-back
        launches, states unchanged)."""
        ms = C.c_double()
        self._check(self._lib.fps_ens_time_flood(self.e_, int(reps), C.byref(ms)))
        return ms.value

    def active(self):
        n = C.c_int32()
        self._check(self._lib.fps_ens_active(self.e_, C.byref(n)))
        return n.value

    def close(self):
        if getattr(self, "e_", None) and self.e_.value:
            self.torch.cuda.synchronize()
            self._lib.fps_ens_destroy(self.e_)
            self.e_ = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Surrogate:
    """BF16 MFMA convolutional surrogate (training and inference in libfps).
    Inputs/outputs are torch device tensors: x bf16 [n, H, W, 16], y / target
    fp32 [n, H, W, 4]."""

    def __init__(self, max_batch, H, W, device="cuda", stream=None):
        import torch
        self.torch = torch
        self._lib = L = lib()
        self.H, self.W, self.max_batch = H, W, max_batch
        nbytes = L.fps_sur_workspace_bytes(max_batch, H, W)
        if nbytes == 0:
            raise FpsError(FPS_E_INVALID, "surrogate shape rejected (H % 16, W % 32)")
        dev = torch.device(device)
        self.device = dev
        self.ws, ws_ptr = _workspace(torch, nbytes, dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.s_ = C.c_void_p()
        rc = L.fps_sur_create(max_batch, H, W, ws_ptr, nbytes, C.c_void_p(self.stream.cuda_stream),
                              C.byref(self.s_))
        if rc != FPS_OK:
            raise FpsError(rc, (L.fps_sur_last_error(None) or b"").decode())
        self.n_params = L.fps_sur_param_count()
        self.loss_t = torch.zeros(1, dtype=torch.float32, device=dev)

    def _check(self, rc):
        if rc != FPS_OK:
            raise FpsError(rc, (self._lib.fps_sur_last_error(self.s_) or b"").decode())
        return rc

    def set_blocks(self, conv_blocks=0, wgrad_blocks=0):
        """Cap the blocks of the convolution / weight-gradient kernels (0 = default)."""
        return self._check(self._lib.fps_sur_set_blocks(self.s_, int(conv_blocks), int(wgrad_blocks)))

    def set_params(self, params):
        p = params.to(self.device, self.torch.float32).contiguous()
        assert p.numel() == self.n_params
        self._keep = p
        return self._check(self._lib.fps_sur_set_params(self.s_, _ptr(p)))

    def get_params(self):
        p = self.torch.empty(self.n_params, dtype=self.torch.float32, device=self.device)
        self._check(self._lib.fps_sur_get_params(self.s_, _ptr(p)))
        return p

    def _check_x(self, x):
        n = x.shape[0]
        if (tuple(x.shape[1:]) != (self.H, self.W, 16) or x.dtype != self.torch.bfloat16 or not x.is_contiguous()
                or not 1 <= n <= self.max_batch):
            raise FpsError(FPS_E_INVALID, f"surrogate input {tuple(x.shape)} {x.dtype}: expected contiguous bf16 "
                                          f"[1..{self.max_batch}, {self.H}, {self.W}, 16]")
        return n

    def _check_y(self, y, n):
        if tuple(y.shape) != (n, self.H, self.W, 4) or y.dtype != self.torch.float32 or not y.is_contiguous():
            raise FpsError(FPS_E_INVALID, f"surrogate output/target {tuple(y.shape)}: expected contiguous fp32 "
                                          f"[{n}, {self.H}, {self.W}, 4]")

    def forward(self, x, y=None):
        n = self._check_x(x)
        if y is None:
            y = self.torch.empty((n, self.H, self.W, 4), dtype=self.torch.float32, device=self.device)
        self._check_y(y, n)
        self._check(self._lib.fps_sur_forward(self.s_, n, _ptr(x), _ptr(y)))
        return y

    def gradients(self, x, target):
        self._check_y(target, self._check_x(x))
        g = self.torch.empty(self.n_params, dtype=self.torch.float32, device=self.device)
        self._check(self._lib.fps_sur_gradients(self.s_, x.shape[0], _ptr(x), _ptr(target), _ptr(g),
                                                _ptr(self.loss_t)))
        return self.loss_t, g

    def train_step(self, x, target, lr):
        self._check_y(target, self._check_x(x))
        self._check(self._lib.fps_sur_train_step(self.s_, x.shape[0], _ptr(x), _ptr(target), float(lr),
                                                 _ptr(self.loss_t)))
        return self.loss_t

    def close(self):
        if getattr(self, "s_", None) and self.s_.value:
            self.torch.cuda.synchronize()
            self._lib.fps_sur_destroy(self.s_)
            self.s_ = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream_ptr(torch, t, stream):
    st = stream if stream is not None else torch.cuda.current_stream(t.device)
    return C.c_void_p(st.cuda_stream)


def sur_pack(h, hu, hv, z, occupancy=None, inflow=None, out=None, stream=None):
    """Surrogate input bf16 [ny, nx, 16] from float32 device planes [ny, nx]
    (occupancy: int32 evacuee counts per cell or None; inflow: (side, c0, c1,
    depth over the block) or None)."""
    import torch
    ny, nx = h.shape
    if out is None:
        out = torch.empty((ny, nx, 16), dtype=torch.bfloat16, device=h.device)
    assert out.shape == (ny, nx, 16) and out.dtype == torch.bfloat16 and out.is_contiguous()
    occ = _ptr(occupancy) if occupancy is not None else None
    side, c0, c1, depth = inflow if inflow is not None else (-1, 0, 0, 0.0)
    rc = lib().fps_sur_pack(nx, ny, _ptr(h), _ptr(hu), _ptr(hv), _ptr(z), occ, int(side), int(c0), int(c1),
                            float(depth), _ptr(out), _stream_ptr(torch, h, stream))
    if rc != FPS_OK:
        raise FpsError(rc, (lib().fps_sur_last_error(None) or b"").decode())
    return out


def sur_forward_noalloc(params, x, y, stream=None):
    """fps_sur_forward_noalloc: y = net(x) with packed FP32 params (device),
    x bf16 [n, H, W, 16] and a caller-provided y fp32 [n, H, W, 4]; the library
    allocates nothing (its scratch is a static device array)."""
    import torch
    n, H, W = x.shape[0], x.shape[1], x.shape[2]
    if x.dtype != torch.bfloat16 or x.shape[3] != 16 or not x.is_contiguous():
        raise FpsError(FPS_E_INVALID, "x: contiguous bf16 [n, H, W, 16] expected")
    if tuple(y.shape) != (n, H, W, 4) or y.dtype != torch.float32 or not y.is_contiguous():
        raise FpsError(FPS_E_INVALID, "y: contiguous fp32 [n, H, W, 4] expected")
    if params.dtype != torch.float32 or not params.is_contiguous():
        raise FpsError(FPS_E_INVALID, "params: contiguous fp32 expected")
    _sur_rc(lib().fps_sur_forward_noalloc(_ptr(params), n, H, W, _ptr(x), _ptr(y), _stream_ptr(torch, x, stream)))
    return y


def sur_make_target(s0, s1, out=None, stream=None):
    """Training target fp32 [H, W, 4] from two flood states (h, hu, hv)."""
    import torch
    h0 = s0[0]
    if out is None:
        out = torch.empty(h0.shape + (4,), dtype=torch.float32, device=h0.device)
    rc = lib().fps_sur_make_target(h0.numel(), *[_ptr(a) for a in (*s0, *s1)], _ptr(out),
                                   _stream_ptr(torch, h0, stream))
    if rc != FPS_OK:
        raise FpsError(rc, (lib().fps_sur_last_error(None) or b"").decode())
    return out


def sur_apply(y, h, hu, hv, h_dry=1e-5, h_snap=1e-3, stream=None):
    """Apply a surrogate output fp32 [ny, nx, 4] to (h, hu, hv) in place."""
    import torch
    assert y.shape == h.shape + (4,)
    rc = lib().fps_sur_apply(h.numel(), _ptr(y), _ptr(h), _ptr(hu), _ptr(hv), float(h_dry), float(h_snap),
                             _stream_ptr(torch, h, stream))
    if rc != FPS_OK:
        raise FpsError(rc, (lib().fps_sur_last_error(None) or b"").decode())


def _sur_rc(rc):
    if rc != FPS_OK:
        raise FpsError(rc, (lib().fps_sur_last_error(None) or b"").decode())


def sur_judge(x, y, state, nx, ny, dx, dy, a, b, tol=0.01, h_dry=1e-5,
              hr_thresholds=(0.75, 1.5, 2.5), stride=1, select=None, hr_margin=0.0, h_margin=0.0,
              out=None, stream=None):
    """Judge a surrogate state a = (h, qx, qy) against a finite-volume state b
    at the cells of every stride-th agent and, with a selection state
    select = (h, qx, qy), every agent there within hr_margin of a hazard
    threshold or h_margin of the dry threshold; returns the device int32[3]
    result (count of judged agents with |dh| > tol or another hazard class,
    max |dh| as float bits, judged agents)."""
    import torch
    if out is None:
        out = torch.empty(3, dtype=torch.int32, device=a[0].device)
    thr = (C.c_double * 3)(*hr_thresholds)
    sel = [None, None, None] if select is None else [_ptr(t) for t in select]
    _sur_rc(lib().fps_sur_judge(int(x.numel()), int(stride), _ptr(x), _ptr(y), _ptr(state), int(nx), int(ny),
                                float(dx), float(dy), *[_ptr(t) for t in (*a, *b)], float(tol), float(h_dry),
                                thr, *sel, float(hr_margin), float(h_margin), _ptr(out),
                                _stream_ptr(torch, a[0], stream)))
    return out


def sur_judge_mask(x, y, state, nx, ny, dx, dy, halo, block, stride=1, select=None, h_dry=1e-5,
                   hr_thresholds=(0.75, 1.5, 2.5), hr_margin=0.0, h_margin=0.0, out=None, stream=None):
    """Judge-region mask (uint8 [ceil(ny/block), ceil(nx/block)]) around the
    judged agents' cells (the same people as sur_judge with the same
    selection arguments)."""
    import torch
    if out is None:
        out = torch.empty(((ny + block - 1) // block, (nx + block - 1) // block), dtype=torch.uint8,
                          device=x.device)
    thr = (C.c_double * 3)(*hr_thresholds)
    sel = [None, None, None] if select is None else [_ptr(t) for t in select]
    _sur_rc(lib().fps_sur_judge_mask(int(x.numel()), int(stride), _ptr(x), _ptr(y), _ptr(state), int(nx),
                                     int(ny), float(dx), float(dy), *sel, float(h_dry), thr, float(hr_margin),
                                     float(h_margin), int(halo), int(block), _ptr(out),
                                     _stream_ptr(torch, x, stream)))
    return out


def sur_occupancy(x, y, role, state, nx, ny, dx, dy, out=None, stream=None):
    """Per-cell counts of evacuees still evacuating (int32 [ny, nx])."""
    import torch
    if out is None:
        out = torch.empty((ny, nx), dtype=torch.int32, device=x.device)
    _sur_rc(lib().fps_sur_occupancy(int(x.numel()), _ptr(x), _ptr(y), _ptr(role), _ptr(state), int(nx),
                                    int(ny), float(dx), float(dy), _ptr(out), _stream_ptr(torch, x, stream)))
    return out


def sur_copy_state(src, dst, stream=None):
    """Copy a flood state (h, hu, hv) into dst (three tensors of the same size)."""
    import torch
    _sur_rc(lib().fps_sur_copy_state(src[0].numel(), *[_ptr(t) for t in (*src, *dst)],
                                     _stream_ptr(torch, src[0], stream)))


def judge_result(out):
    """(count, max |dh|, judged) from a sur_judge result tensor."""
    import numpy as np
    v = out.cpu().numpy().astype(np.int32)
    return int(v[0]), float(v[1:2].view(np.float32)[0]), int(v[2])



def stream_probe(n, n_in, n_out, reps=20, skew=0, device="cuda", stream=None):
    """fps_stream_probe on a fresh buffer holding n_in + n_out arrays of n floats,
    each array skew floats after the end of the one before: mean ms per pass
    and the bytes it moves (read + written)."""
    import torch
    stride = n + skew
    buf = torch.ones((n_in + n_out) * stride, dtype=torch.float32, device=device)
    ms = C.c_double()
    _sur_rc_generic(lib().fps_stream_probe(_ptr(buf), int(n), int(stride), int(n_in), int(n_out), int(reps),
                                           _stream_ptr(torch, buf, stream), C.byref(ms)))
    del buf
    return ms.value, 4 * (n_in + n_out) * n


def _sur_rc_generic(rc):
    if rc != FPS_OK:
        raise FpsError(rc, (lib().fps_last_error(None) or b"").decode())
