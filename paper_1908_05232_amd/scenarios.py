"""Drivers of the paper's two experiments on the synthetic shopping centre.

Scenario 1 (sec. 3.2): the evacuation run twice, with and without the
people's effect on the flood (the roughness rule of sec. 2.4 switched off by a
zero evacuee cap), at several breach discharges, since on this layout the
crowd only meets the water once the breach carries more than a few m^2/s.
As in the paper the run starts 5 minutes before the breach with the
pre-flood flow of walkers entering and leaving by 7 doors (10 per door and
step, up to 1,000 inside); the first wet step closes the doors and makes the
walkers inside evacuees.  Scenario 2 (sec. 3.3): the pre-flood deployment sweep, six
responder group sizes (5 % to 50 % of the population) times one to six sandbag
layers, each run until its barrier is complete or 12 hours have passed, then
the flood over each finished barrier height.

Host-side orchestration only: scenarios are built by ``inputs`` and every step
runs in the library's kernels (one ensemble launch set per step).  The site is
the paper's 128 x 128 grid over 332 m; its layout is the synthetic random
tiling of ``inputs.shopping_centre`` (the paper's own geometry is only in a
figure), so the numbers are this layout's, not the paper's.

    python -m paper_1908_05232_amd.scenarios [--quick]
"""
from __future__ import annotations

import argparse
import copy
import dataclasses
import json
import time

import numpy as np

from . import fps, inputs as I

SITE_N = 128
SITE_DX = 332.0 / 128          # 2.59 m cells over the 332 m site (sec. 3)
GROUPS = (0.05, 0.10, 0.20, 0.30, 0.40, 0.50)
LAYERS = (1, 2, 3, 4, 5, 6)
LAYER_M = 0.25                 # sandbag thickness per layer (sec. 3.3: three layers reach 0.75 m)
DEPLOY_WINDOW_S = 12 * 3600.0  # the 12-hour deployment window (sec. 3.3)
BREACH_Q = (2.0, 5.0, 10.0, 20.0)  # peak unit discharges of the evacuation runs (m^2/s)
NO_FLOOD = 1.0e9               # hydrograph start of the dry deployment runs
ST_EVAC, ST_EXITED, ST_SHOPPING = 0, 1, 6     # agent states (include/fps.h)


def _site(population, seed, n, dx, **kw):
    return I.shopping_centre(n=n, dx=dx, seed=seed, n_evac=population, n_exits=1, **kw)


def evacuation_pair(population=1000, seed=5232, n=SITE_N, dx=SITE_DX, q_peak=2.0, duration=1800.0, doors=True,
                    bodies=False, wading=False):
    """Scenario 1 with and without the people's effect on the flood.  doors:
    the pre-flood flow (sec. 3.2) fills the site from 7 doors during a
    5-minute spin-up; else the population starts spread uniformly, standing.
    bodies: varied heights and masses and the stability rule (people who
    cannot stand in the flow stop); wading: with bodies, also the wading rule
    (walking speed capped by the drag of wading)."""
    with_people = _site(population, seed, n, dx, q_peak=q_peak, duration=duration)
    if doors:
        with_people = I.add_doors(with_people, seed=seed)
    tag = ""
    if bodies:
        with_people = I.add_bodies(with_people, seed=seed)
        tag = "_bodies"
        if wading:
            with_people.ped = dataclasses.replace(with_people.ped, wading=1)
            tag = "_bodies_wading"
    with_people.name = "evacuation_coupled" + tag
    without = copy.deepcopy(with_people)
    without.desc.np_cap = 0
    without.name = "evacuation_uncoupled" + tag
    return [with_people, without]


def run_evacuation(scs, t_max=3600.0, poll_steps=10):
    """Step an ensemble until every evacuee has left or ``t_max``; per member the
    evacuation time, the people inside when the flood reached the site (the
    evacuees), and the largest number of people seen at once in each hazard
    class (Table 1), polled every ``poll_steps`` steps."""
    ens = fps.Ensemble(scs)
    ens.autotune()
    q = [float(np.max(sc.hydro_q)) if sc.hydro_q is not None and len(sc.hydro_q) else 0.0 for sc in scs]
    out = [dict(name=sc.name, evacuees=None, q_peak=qp, t_evacuated=None, peak_class_count=[0] * 6,
                door_entries=0, door_leaves=0) for sc, qp in zip(scs, q)]
    t = -np.inf
    while t < t_max and any(o["t_evacuated"] is None for o in out):
        ens.step(poll_steps)
        for k, m in enumerate(ens.members):
            d = m.diag()
            t = d["t"]
            o = out[k]
            sc_ = d["state_count"]
            if d["any_wet"] or d["doors_closed"]:
                o["peak_class_count"] = [max(a, b) for a, b in zip(o["peak_class_count"], d["class_count"])]
            if o["evacuees"] is None and (d["doors_closed"] or (d["any_wet"] and sc_[ST_SHOPPING] == 0)):
                o["evacuees"] = sc_[ST_EVAC] + sc_[ST_EXITED]
                o["door_entries"], o["door_leaves"] = d["door_entries"], d["door_leaves"]
            if o["t_evacuated"] is None and o["evacuees"] is not None and sc_[ST_EVAC] + sc_[ST_SHOPPING] == 0:
                o["t_evacuated"] = d["t"]
    for k, m in enumerate(ens.members):
        d = m.diag()
        out[k].update(t_end=d["t"], flood_mass_m3=d["mass"], v_in_m3=d["v_in"])
    return out


def deployment_sweep(population=1000, seed=5232, n=SITE_N, dx=SITE_DX, groups=GROUPS, layers=LAYERS):
    """Scenario 2: one dry scenario per (group size, layer count)."""
    scs = []
    for f in groups:
        n_resp = max(1, int(round(f * population)))
        for L in layers:
            sc = _site(population - n_resp, seed, n, dx, t_flood=NO_FLOOD)
            sc = I.add_barrier(sc, seed=seed, n_resp=n_resp, height=L * LAYER_M, t_bag=LAYER_M)
            sc.name = f"deploy_{int(round(100 * f))}pct_{L}layers"
            sc.group, sc.layers = f, L
            scs.append(sc)
    return scs


def run_deployment(scs, t_max=DEPLOY_WINDOW_S, poll_steps=60):
    """Step until every barrier is complete or ``t_max``; the completion time of
    each member to the polling interval (60 dry steps of 1 s = one minute)."""
    ens = fps.Ensemble(scs)
    out = [dict(name=sc.name, group=sc.group, layers=sc.layers,
                responders=int(np.sum(sc.agents["role"] == I.ROLE_RESPONDER)),
                line_cells=len(sc.barrier["cells"]), bags_per_cell_layer=int(sc.barrier["bags_per"]),
                t_complete=None) for sc in scs]
    t = 0.0
    while t < t_max and any(o["t_complete"] is None for o in out):
        ens.step(poll_steps)
        for k, m in enumerate(ens.members):
            if out[k]["t_complete"] is not None:
                continue
            d = m.diag()
            t = d["t"]
            if d["barrier_done"]:
                out[k]["t_complete"] = d["t"]
    for k, m in enumerate(ens.members):
        d = m.diag()
        out[k].update(layers_done=d["barrier_layers_done"], drops=d["drops_total"], t_end=d["t"])
    return out


def barrier_floods(population=1000, seed=5232, n=SITE_N, dx=SITE_DX, layers=(0,) + LAYERS, q_peak=2.0,
                   duration=1800.0, t_run=1800.0):
    """The flood over each finished barrier (0 = none): the barrier line raised by
    layers x 0.25 m, the same hydrograph, no people.  Returns per layer count the
    largest depth and hazard rate seen downstream (north) of the line, and the
    time water (1 cm) first reaches the cells right behind the line."""
    base = _site(population, seed, n, dx, q_peak=q_peak, duration=duration)
    probe = I.add_barrier(copy.deepcopy(base), seed=seed, n_resp=1, height=LAYER_M, t_bag=LAYER_M)
    cells = probe.barrier["cells"]
    jb = int(cells[0]) // n
    scs = []
    for L in layers:
        sc = copy.deepcopy(base)
        sc.agents = None
        z = sc.z.copy().reshape(-1)
        z[cells] += L * LAYER_M
        sc.z = z.reshape(n, n)
        sc.name = f"flood_{L}layers"
        scs.append(sc)
    ens = fps.Ensemble(scs)
    ens.autotune()
    behind = np.asarray(cells) % n                      # columns of the line, one row north of it
    arrival = [None] * len(scs)
    hmax = [np.zeros((n - jb - 1, n), np.float32) for _ in scs]
    hrmax = [np.zeros((n - jb - 1, n), np.float32) for _ in scs]
    t = 0.0
    while t < t_run:
        ens.step(50)
        for k, m in enumerate(ens.members):
            h = m.fields()[0][jb + 1:]
            hr = m.hazard().cpu().numpy()[jb + 1:]
            np.maximum(hmax[k], h, out=hmax[k])
            np.maximum(hrmax[k], hr, out=hrmax[k])
            t = m.diag()["t"]
            if arrival[k] is None and np.any(h[0, behind] > 0.01):
                arrival[k] = t
    out = []
    for k, L in enumerate(layers):
        out.append(dict(layers=L, barrier_m=L * LAYER_M, max_depth_downstream_m=float(hmax[k].max()),
                        max_hr_downstream=float(hrmax[k].max()),
                        wet_cells_downstream=int((hmax[k] > 0.01).sum()),
                        t_water_behind_line=arrival[k]))
    hr0 = out[0]["max_hr_downstream"]
    for o in out:
        o["max_hr_reduction_pct"] = 100.0 * (1.0 - o["max_hr_downstream"] / hr0) if hr0 > 0 else 0.0
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--quick", action="store_true", help="two group sizes x two layer counts, short runs")
    args = ap.parse_args(argv)
    t0 = time.perf_counter()
    if args.quick:
        res = dict(evacuation=[run_evacuation(evacuation_pair(population=300, q_peak=q), t_max=1200.0)
                               for q in (2.0, 10.0)],
                   deployment=run_deployment(deployment_sweep(population=300, groups=(0.2, 0.5), layers=(1, 2)),
                                             t_max=4 * 3600.0),
                   barrier_floods=barrier_floods(layers=(0, 1, 2), t_run=900.0))
    else:
        res = dict(evacuation=[run_evacuation(evacuation_pair(q_peak=q)) for q in BREACH_Q],
                   evacuation_stability=[run_evacuation(evacuation_pair(q_peak=q, bodies=True)) for q in BREACH_Q[2:]],
                   evacuation_wading=[run_evacuation(evacuation_pair(q_peak=q, bodies=True, wading=True))
                                      for q in BREACH_Q[2:]],
                   deployment=run_deployment(deployment_sweep()),
                   barrier_floods=barrier_floods())
    res["wall_s"] = time.perf_counter() - t0
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
