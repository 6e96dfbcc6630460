"""Helpers shared by the GPU parity tests (GPU state -> oracle restarts)."""
import copy
import sys

import numpy as np

from paper_1908_05232_amd import inputs as I


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def snapshot(sim, sc):
    """A scenario holding the GPU's current flood state (and agents, if any)."""
    d = sim.diag()
    h, qx, qy, z = sim.fields()
    s2 = copy.copy(sc)
    s2.h, s2.qx, s2.qy, s2.z = h.astype(np.float64), qx.astype(np.float64), qy.astype(np.float64), \
        z.astype(np.float64)
    s2.t0 = d["t"]
    if sim.na:
        A = sim.agents()
        s2.agents = {k: v.copy() for k, v in A.items()}
        for k in ("height", "mass"):          # bodies do not change: the scenario's own
            if k in sc.agents:
                s2.agents[k] = np.asarray(sc.agents[k]).copy()
    return s2, d


def flood_window(O, sim, sc, nsteps, dt_rtol=1e-5):
    """Run nsteps on the GPU one at a time, then the oracle from the same start
    replaying the GPU's time steps.  Returns (max|dh|, max|dq|, rel mass err,
    max rel dt mismatch of the oracle's own dt)."""
    start, d0 = snapshot(sim, sc)
    dts = []
    for _ in range(nsteps):
        sim.step(1)
        dts.append(sim.diag()["dt_last"])
    ref = O.OracleSim(start)
    ref.S.t = d0["t"]
    worst_dt = 0.0
    for k in range(nsteps):
        own = ref.compute_dt()
        worst_dt = max(worst_dt, abs(own - dts[k]) / dts[k])
        ref.fv_step(dts[k])
    h, qx, qy, _ = sim.fields()
    hr, qxr, qyr, _ = ref.fields()
    dh = float(np.abs(h - hr).max())
    dq = float(max(np.abs(qx - qxr).max(), np.abs(qy - qyr).max()))
    m_gpu = sim.diag()["mass"]
    m_ref = ref.mass()
    rel = abs(m_gpu - m_ref) / max(m_ref, 1e-30)
    return dh, dq, rel, worst_dt, ref


def random_wet_dry(nx, ny, dx, seed, bc=(0, 0, 0, 0), inflow=None):
    rng = I.rng_of(seed)
    z = rng.uniform(0.0, 0.3, (ny, nx))
    z[rng.random((ny, nx)) < 0.05] = 2.0
    h = np.maximum(rng.uniform(-0.3, 1.0, (ny, nx)) - z, 0.0)
    qx = rng.uniform(-0.4, 0.4, (ny, nx)) * (h > 0.01)
    qy = rng.uniform(-0.4, 0.4, (ny, nx)) * (h > 0.01)
    kw = {}
    ht = hq = None
    if inflow is not None:
        side, c0, c1 = inflow
        kw = dict(inflow_side=side, inflow_c0=c0, inflow_c1=c1)
        ht, hq = I.triangular_hydrograph(1.5, 40.0)
    d = I.GridDesc(nx=nx, ny=ny, dx=dx, dy=dx, bc=bc, n_base=0.03, **kw)
    return I.Scenario(desc=d, h=h, qx=qx, qy=qy, z=z, hydro_t=ht, hydro_q=hq,
                      name=f"random_{nx}x{ny}")
