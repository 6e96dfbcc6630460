"""ctypes binding of the FP64 CPU oracle (``oracle/fps_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The product package never imports
it.  The oracle shares no code with the GPU library; both are fed the same
seeded inputs from ``paper_1908_05232_amd.inputs``, which holds no arithmetic
of the method.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_LIB_OMP_PATH = os.path.join(_HERE, "liboracle_omp.so")

_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)
_ip = C.POINTER(C.c_int32)
_up = C.POINTER(C.c_uint8)

WALL, TRANSMISSIVE = 0, 1
ROLE_EVACUEE, ROLE_RESPONDER = 0, 1
ST_EVAC, ST_EXITED, ST_TO_STORAGE, ST_PICKING, ST_TO_BARRIER, ST_DROPPING, ST_SHOPPING, ST_OUTSIDE = range(8)
CLS_DRY, CLS_LOW, CLS_MEDIUM, CLS_HIGH, CLS_HIGHEST, CLS_UNSTABLE = range(6)
FLUX_HLLC, FLUX_HLL = 0, 1


class OrParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("dx", C.c_double), ("dy", C.c_double),
        ("g", C.c_double), ("cfl", C.c_double), ("h_dry", C.c_double), ("dt_max", C.c_double),
        ("bc", C.c_int32 * 4),
        ("inflow_side", C.c_int32), ("inflow_c0", C.c_int32), ("inflow_c1", C.c_int32),
        ("n_base", C.c_double), ("np_cap", C.c_int32),
        ("tau", C.c_double), ("a_over_m", C.c_double), ("b_range", C.c_double),
        ("radius", C.c_double), ("r_cut", C.c_double), ("r_arrive", C.c_double),
        ("v_class", C.c_double * 5), ("hr_t", C.c_double * 3),
        ("pick_s", C.c_double), ("drop_s", C.c_double),
        ("flux", C.c_int32),
        ("order", C.c_int32),
        ("stability", C.c_int32),
        ("c_drag", C.c_double), ("mu_f", C.c_double), ("rho_w", C.c_double), ("rho_body", C.c_double),
        ("body_h0", C.c_double), ("body_m0", C.c_double),
        ("wading", C.c_int32), ("wade_k", C.c_double),
    ]


class OrSim(C.Structure):
    _fields_ = [
        ("P", OrParams),
        ("h", _dp), ("qx", _dp), ("qy", _dp), ("z", _dp), ("np", _ip),
        ("t", C.c_double), ("step", C.c_int64),
        ("nh", C.c_int32), ("ht", _dp), ("hq", _dp),
        ("v_in", C.c_double), ("v_out", C.c_double), ("v_clip", C.c_double),
        ("any_wet", C.c_int32),
        ("n_dest", C.c_int32), ("n_exit", C.c_int32), ("dist", _fp), ("walk", _up),
        ("na", C.c_int32),
        ("x", _dp), ("y", _dp), ("vx", _dp), ("vy", _dp), ("vbase", _dp), ("timer", _dp),
        ("role", _up), ("state", _up), ("cls", _up), ("dest", _ip),
        ("nline", C.c_int32), ("line", _ip),
        ("storage_dest", C.c_int32), ("barrier_dest", C.c_int32), ("n_layers", C.c_int32),
        ("bags_per", C.c_int32),
        ("t_bag", C.c_double), ("t_last", C.c_double),
        ("active", C.c_int32), ("layers_done", C.c_int32), ("bags", C.c_int32),
        ("done", C.c_int32), ("drops_total", C.c_int32),
        ("bin_start", _ip), ("perm", _ip),
        ("n_door", C.c_int32), ("door_rate", C.c_int32),
        ("door_cell", _ip), ("door_dest", _ip),
        ("door_seed", C.c_uint64),
        ("doors_closed", C.c_int32),
        ("door_in", C.c_int64), ("door_out", C.c_int64),
        ("body_h", _dp), ("body_m", _dp),
    ]


def build(force: bool = False, omp: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no FMA contraction, no
    fast-math).  omp=True builds the same source with OpenMP (loops over grid
    rows and over agents; every result identical to the serial build) for
    timing on all host cores."""
    src = os.path.join(_HERE, "fps_oracle.c")
    path = _LIB_OMP_PATH if omp else _LIB_PATH
    if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
        tmp = path + f".tmp{os.getpid()}"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
            "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas", *(["-fopenmp"] if omp else []),
            "-o", tmp, src, "-lm"])
        os.replace(tmp, path)
    return path


_libs = {}


def lib(omp: bool = False):
    """The loaded oracle (serial, or the OpenMP build with omp=True)."""
    if omp not in _libs:
        L = _libs[omp] = C.CDLL(build(omp=omp))
        L.or_hllc.argtypes = [C.c_double] * 7 + [_dp]
        L.or_hll.argtypes = [C.c_double] * 7 + [_dp]
        L.or_face.argtypes = [C.POINTER(OrParams)] + [C.c_double] * 8 + [C.c_int, _dp, _dp, _dp]
        L.or_hydro_integral.argtypes = [C.c_int32, _dp, _dp, C.c_double, C.c_double]
        L.or_hydro_integral.restype = C.c_double
        L.or_hr_class.argtypes = [C.POINTER(OrParams), C.c_double, C.c_double, C.c_double, _dp]
        L.or_hr_class.restype = C.c_int32
        L.or_unstable.argtypes = [C.POINTER(OrParams)] + [C.c_double] * 5 + [_dp]
        L.or_unstable.restype = C.c_int32
        L.or_wade_speed.argtypes = [C.POINTER(OrParams)] + [C.c_double] * 3
        L.or_wade_speed.restype = C.c_double
        L.or_n_eff.argtypes = [C.POINTER(OrParams), C.c_int32]
        L.or_n_eff.restype = C.c_double
        L.or_friction.argtypes = [C.POINTER(OrParams), C.c_double, C.c_double, C.c_double, _dp, _dp]
        L.or_cell_index.argtypes = [C.c_double, C.c_double, C.c_int32]
        L.or_cell_index.restype = C.c_int32
        L.or_bins_dims.argtypes = [C.POINTER(OrParams), _ip, _ip, _ip, _ip]
        L.or_build_bins.argtypes = [C.POINTER(OrParams), C.c_int32, _fp, _fp, _up, _ip, _ip]
        L.or_compute_dt.argtypes = [C.POINTER(OrSim)]
        L.or_compute_dt.restype = C.c_double
        L.or_fv_step.argtypes = [C.POINTER(OrSim), C.c_double]
        L.or_count_evacuees.argtypes = [C.POINTER(OrSim)]
        L.or_ped_step.argtypes = [C.POINTER(OrSim), C.c_double]
        L.or_coupled_step.argtypes = [C.POINTER(OrSim), C.c_double]
        L.or_coupled_step.restype = C.c_double
        L.or_run.argtypes = [C.POINTER(OrSim), C.c_int32, _dp, _dp, C.c_int32]
        L.or_mass.argtypes = [C.POINTER(OrSim)]
        L.or_mass.restype = C.c_double
        L.or_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        L.or_splitmix64.restype = C.c_uint64
        L.or_doors.argtypes = [C.POINTER(OrSim)]
    return _libs[omp]


def _ptr(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def make_params(desc, ped=None) -> OrParams:
    """Fill the oracle's parameter block from an ``inputs.GridDesc`` / ``inputs.PedParams``."""
    from paper_1908_05232_amd.inputs import PedParams
    ped = ped or PedParams()
    P = OrParams()
    P.nx, P.ny, P.dx, P.dy = desc.nx, desc.ny, desc.dx, desc.dy
    P.g, P.cfl, P.h_dry, P.dt_max = desc.g, desc.cfl, desc.h_dry, desc.dt_max
    for k in range(4):
        P.bc[k] = desc.bc[k]
    P.inflow_side, P.inflow_c0, P.inflow_c1 = desc.inflow_side, desc.inflow_c0, desc.inflow_c1
    P.n_base, P.np_cap = desc.n_base, desc.np_cap
    P.tau, P.a_over_m, P.b_range = ped.tau, ped.a_over_m, ped.b_range
    P.radius, P.r_cut, P.r_arrive = ped.radius, ped.r_cut, ped.r_arrive
    for k in range(5):
        P.v_class[k] = ped.v_class[k]
    for k in range(3):
        P.hr_t[k] = ped.hr_t[k]
    P.pick_s, P.drop_s = ped.pick_s, ped.drop_s
    P.flux = getattr(desc, "flux", FLUX_HLLC)
    P.order = getattr(desc, "order", 1)
    P.stability = int(getattr(ped, "stability", 0))
    P.c_drag, P.mu_f = getattr(ped, "c_drag", 1.1), getattr(ped, "mu_f", 0.45)
    P.rho_w, P.rho_body = getattr(ped, "rho_w", 1000.0), getattr(ped, "rho_body", 1000.0)
    P.body_h0, P.body_m0 = getattr(ped, "body_h0", 1.71), getattr(ped, "body_m0", 70.0)
    P.wading, P.wade_k = int(getattr(ped, "wading", 0)), getattr(ped, "wade_k", 0.1)
    return P


class OracleSim:
    """FP64 oracle state built from a ``inputs.Scenario``; arrays are numpy, kept alive here."""

    def __init__(self, sc, omp: bool = False):
        self.L = L = lib(omp)
        self.sc = sc
        d = sc.desc
        self.S = OrSim()
        self.S.P = make_params(d, sc.ped)
        nc = d.nx * d.ny
        self.h = np.ascontiguousarray(sc.h, dtype=np.float64).reshape(nc).copy()
        self.qx = np.ascontiguousarray(sc.qx, dtype=np.float64).reshape(nc).copy()
        self.qy = np.ascontiguousarray(sc.qy, dtype=np.float64).reshape(nc).copy()
        self.z = np.ascontiguousarray(sc.z, dtype=np.float64).reshape(nc).copy()
        self.np_ = np.zeros(nc, dtype=np.int32)
        self.ht = np.asarray(sc.hydro_t if sc.hydro_t is not None else [], dtype=np.float64).copy()
        self.hq = np.asarray(sc.hydro_q if sc.hydro_q is not None else [], dtype=np.float64).copy()
        S = self.S
        S.h, S.qx, S.qy, S.z = (_ptr(a, _dp) for a in (self.h, self.qx, self.qy, self.z))
        S.np = _ptr(self.np_, _ip)
        S.t, S.step = float(sc.t0), 0
        S.nh = len(self.ht)
        S.ht = _ptr(self.ht, _dp) if len(self.ht) else None
        S.hq = _ptr(self.hq, _dp) if len(self.hq) else None
        # navigation
        if sc.dist is not None:
            self.dist = np.ascontiguousarray(sc.dist, dtype=np.float32)
            self.walk = np.ascontiguousarray(sc.walk, dtype=np.uint8).reshape(nc)
            S.n_dest, S.n_exit = self.dist.shape[0], sc.n_exit
            S.dist, S.walk = _ptr(self.dist, _fp), _ptr(self.walk, _up)
        else:
            self.dist = self.walk = None
            S.n_dest = S.n_exit = 0
        # agents
        na = 0 if sc.agents is None else len(sc.agents["x"])
        S.na = na
        if na:
            A = sc.agents
            self.x = np.asarray(A["x"], dtype=np.float64).copy()
            self.y = np.asarray(A["y"], dtype=np.float64).copy()
            self.vx = np.asarray(A["vx"], dtype=np.float64).copy()
            self.vy = np.asarray(A["vy"], dtype=np.float64).copy()
            self.vbase = np.asarray(A["v_base"], dtype=np.float64).copy()
            self.timer = np.asarray(A["timer"], dtype=np.float64).copy()
            self.role = np.asarray(A["role"], dtype=np.uint8).copy()
            self.state = np.asarray(A["state"], dtype=np.uint8).copy()
            self.cls = np.asarray(A["hr_class"], dtype=np.uint8).copy()
            self.dest = np.asarray(A["dest"], dtype=np.int32).copy()
            for nm in ("x", "y", "vx", "vy", "vbase", "timer"):
                setattr(S, nm, _ptr(getattr(self, nm), _dp))
            for nm in ("role", "state", "cls"):
                setattr(S, nm, _ptr(getattr(self, nm), _up))
            S.dest = _ptr(self.dest, _ip)
            if "height" in A and "mass" in A:
                self.body_h = np.asarray(A["height"], dtype=np.float64).copy()
                self.body_m = np.asarray(A["mass"], dtype=np.float64).copy()
                S.body_h, S.body_m = _ptr(self.body_h, _dp), _ptr(self.body_m, _dp)
            bsx, bsy, nbx, nby = self.bins_dims()
            self.bin_start = np.zeros(nbx * nby + 1, dtype=np.int32)
            self.perm = np.zeros(na, dtype=np.int32)
            S.bin_start, S.perm = _ptr(self.bin_start, _ip), _ptr(self.perm, _ip)
        # barrier
        b = sc.barrier
        if b is not None:
            self.line = np.asarray(b["cells"], dtype=np.int32).copy()
            S.nline, S.line = len(self.line), _ptr(self.line, _ip)
            S.storage_dest, S.barrier_dest = b["storage_dest"], b["barrier_dest"]
            S.n_layers, S.bags_per = b["n_layers"], b["bags_per"]
            S.t_bag, S.t_last = b["t_bag"], b["t_last"]
        else:
            S.nline = 0
            S.storage_dest = S.barrier_dest = -1
        # pre-flood door flow
        dr = getattr(sc, "doors", None)
        if dr is not None and na:
            self.door_cell = np.ascontiguousarray(dr["cells"], dtype=np.int32).copy()
            self.door_dest = np.ascontiguousarray(dr["dests"], dtype=np.int32).copy()
            S.n_door, S.door_rate = len(self.door_cell), int(dr["per_step"])
            S.door_cell, S.door_dest = _ptr(self.door_cell, _ip), _ptr(self.door_dest, _ip)
            S.door_seed = int(dr["seed"])
        else:
            S.n_door = 0
        S.any_wet = int(np.any(self.h > d.h_dry))
        if na:
            L.or_count_evacuees(C.byref(S))

    # -- views -----------------------------------------------------------
    def bins_dims(self):
        a = [C.c_int32() for _ in range(4)]
        self.L.or_bins_dims(C.byref(self.S.P), *[C.byref(v) for v in a])
        return tuple(v.value for v in a)

    @property
    def t(self):
        return self.S.t

    def fields(self):
        d = self.sc.desc
        return (self.h.reshape(d.ny, d.nx), self.qx.reshape(d.ny, d.nx),
                self.qy.reshape(d.ny, d.nx), self.z.reshape(d.ny, d.nx))

    def mass(self):
        return self.L.or_mass(C.byref(self.S))

    def set_fields(self, h, qx, qy, z=None):
        self.h[:] = np.asarray(h, dtype=np.float64).reshape(-1)
        self.qx[:] = np.asarray(qx, dtype=np.float64).reshape(-1)
        self.qy[:] = np.asarray(qy, dtype=np.float64).reshape(-1)
        if z is not None:
            self.z[:] = np.asarray(z, dtype=np.float64).reshape(-1)
        self.S.any_wet = int(np.any(self.h > self.sc.desc.h_dry))

    # -- stepping --------------------------------------------------------
    def compute_dt(self):
        return self.L.or_compute_dt(C.byref(self.S))

    def fv_step(self, dt):
        self.L.or_fv_step(C.byref(self.S), float(dt))
        self.S.t += float(dt)
        self.S.step += 1

    def run(self, n, dts=None, with_peds=True):
        dt_used = np.zeros(n, dtype=np.float64)
        d = None if dts is None else np.ascontiguousarray(dts, dtype=np.float64)
        self.L.or_run(C.byref(self.S), int(n), _ptr(d, _dp) if d is not None else None,
                     _ptr(dt_used, _dp), int(bool(with_peds) and self.S.na > 0))
        return dt_used

    def coupled_step(self, dt=0.0):
        return self.L.or_coupled_step(C.byref(self.S), float(dt))


# -- free functions used by the pins ------------------------------------------
def hllc(g, hL, uL, vL, hR, uR, vR):
    F = (C.c_double * 3)()
    lib().or_hllc(g, hL, uL, vL, hR, uR, vR, F)
    return np.array(F[:])


def hll(g, hL, uL, vL, hR, uR, vR):
    F = (C.c_double * 3)()
    lib().or_hll(g, hL, uL, vL, hR, uR, vR, F)
    return np.array(F[:])


def face(params, hL, qnL, qtL, zL, hR, qnR, qtR, zR, wall=0):
    F = (C.c_double * 3)()
    a, b = C.c_double(), C.c_double()
    lib().or_face(C.byref(params), hL, qnL, qtL, zL, hR, qnR, qtR, zR, int(wall), F,
                  C.byref(a), C.byref(b))
    return np.array(F[:]), a.value, b.value


def hydro_integral(t, q, a, b):
    t = np.ascontiguousarray(t, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    return lib().or_hydro_integral(len(t), _ptr(t, _dp), _ptr(q, _dp), float(a), float(b))


def hr_class(params, h, qx, qy):
    hr = C.c_double()
    c = lib().or_hr_class(C.byref(params), float(h), float(qx), float(qy), C.byref(hr))
    return c, hr.value


def unstable(params, h, qx, qy, height, mass):
    """(1 if a person of that body cannot stand in the cell, relative margin)."""
    m = C.c_double()
    r = lib().or_unstable(C.byref(params), float(h), float(qx), float(qy), float(height), float(mass), C.byref(m))
    return r, m.value


def wade_speed(params, h, height, mass):
    """The wading speed cap of a person of that body in still water of depth h (W1, W2)."""
    return lib().or_wade_speed(C.byref(params), float(h), float(height), float(mass))


def n_eff(params, np_count):
    return lib().or_n_eff(C.byref(params), int(np_count))


def friction(params, dt, h, n, qx, qy):
    a, b = C.c_double(qx), C.c_double(qy)
    lib().or_friction(C.byref(params), float(dt), float(h), float(n), C.byref(a), C.byref(b))
    return a.value, b.value


def splitmix64(seed, c):
    """Output c + 1 of SplitMix64 started from seed."""
    return int(lib().or_splitmix64(int(seed), int(c)))


def cell_index(x, d, n):
    return lib().or_cell_index(float(x), float(d), int(n))


def build_bins(params, x, y, state):
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    state = np.ascontiguousarray(state, dtype=np.uint8)
    a = [C.c_int32() for _ in range(4)]
    lib().or_bins_dims(C.byref(params), *[C.byref(v) for v in a])
    nb = a[2].value * a[3].value
    bin_start = np.zeros(nb + 1, dtype=np.int32)
    perm = np.zeros(max(len(x), 1), dtype=np.int32)
    lib().or_build_bins(C.byref(params), len(x), _ptr(x, _fp), _ptr(y, _fp), _ptr(state, _up),
                        _ptr(bin_start, _ip), _ptr(perm, _ip))
    return bin_start, perm[: bin_start[-1]]
