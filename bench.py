"""Benchmark of the coupled flood-pedestrian hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

Headline workload (the large sweep): 32 synthetic shopping centres of
2048 x 2048 cells of 0.25 m (random +3 m building blocks, a completed sandbag
line of U(0.2, 1.0) m, the triangular south inflow already under way, the
free area already wet), 50,000 evacuees each heading for the nearest of two
north exits: 134 M cells and 1.6 M people per step, stepped as one ensemble.
One step = one coupled time step of every scenario: flood update (Eq. 2),
pedestrian step (hazard, movement, roughness count), neighbour re-binning and
sandbag write-back, all on the GPU, from one set of graph-replayed launches.

Prints one JSON line: FV cell-updates/s over the K timed steps (inputs
resident in HBM), the roofline of the flood-update launch (HIP events around
back-to-back launches on the stream the kernels run on), the FP64 CPU oracle
(OpenMP on every host core) timed on a bounded sample of the same workload,
and secondary sections: the 512^2 shopping centre (a cache-resident,
latency-bound rate), an 8192^2 fully wet probe with the copy ceilings, the
64-scenario intervention sweep, and the learned update.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FV_BYTES_PER_CELL = 32   # read h, hu, hv, z (4 B each) + evacuee count (4 B); write h, hu, hv


def log(*a):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the first-order flood update's own source: fps_flood.hip from
    its cell record to the start of the second-order variant (its helpers and
    fv_step_kernel), and the parameter and state records it reads; edits to the
    other kernels leave it, and the counters taken on it, valid."""
    csrc = os.path.join(ROOT, "paper_1908_05232_amd", "csrc")
    text = open(os.path.join(csrc, "fps_flood.hip")).read()
    a = text.index("struct Cell {")
    b = text.index("// Second-order variant")
    h = hashlib.sha256(text[a:b].encode())
    inner = open(os.path.join(csrc, "fps_internal.h")).read()
    for rec in ("struct DevState {", "struct FvParams {"):
        i = inner.index(rec)
        h.update(inner[i:inner.index("};", i)].encode())
    return h.hexdigest()[:16]


def measured_traffic(workload, rows):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current flood kernel source at the same tile shape (rows
    per wave); else None."""
    path = os.path.join(ROOT, "profiles", f"fv_step_counters_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch_by_rows", {}).get(str(rows))


def host_info():
    """Host cores seen by this process and the CPU model (lscpu)."""
    import subprocess
    info = {"nproc": os.cpu_count(), "affinity_cores": len(os.sched_getaffinity(0))}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)"):
                info[k.strip()] = v.strip()
    except Exception as exc:      # lscpu missing: the counts above still stand
        info["lscpu"] = f"unavailable ({exc})"
    return info


def omp_threads():
    """Threads an OpenMP parallel region of the oracle's build uses."""
    import ctypes
    try:
        return int(ctypes.CDLL("libgomp.so.1").omp_get_max_threads())
    except OSError:
        return None


def cpu_baseline(sc, n_steps, what, omp=True):
    """The FP64 oracle (OpenMP build on every host core, or one thread) on the
    first n_steps of one scenario of the workload."""
    from oracle import oracle as O
    ref = O.OracleSim(sc, omp=omp)
    t0 = time.perf_counter()
    ref.run(n_steps)
    dt = time.perf_counter() - t0
    cells = sc.desc.nx * sc.desc.ny
    cores = omp_threads() if omp else 1
    return {"value": cells * n_steps / dt, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"first {n_steps} coupled steps of {what} ({cells * n_steps:.3g} cell-updates, "
                      f"{len(sc.agents['x']) if sc.agents else 0} agents, {dt:.1f} s wall, FP64 C, "
                      f"{'OpenMP, ' + str(cores) + ' threads' if omp else 'one thread'})",
            "wall_s": dt}


def ensemble_section(args, stream):
    """Batched ensemble: the pre-flood intervention sweep, all members stepped
    by one set of launches per coupled step."""
    import torch
    from paper_1908_05232_amd import fps, inputs as I
    scs = I.intervention_sweep(args.ens_scenarios, workers=8)
    log(f"ensemble: {len(scs)} scenarios built")
    cells = sum(sc.desc.nx * sc.desc.ny for sc in scs)
    agents = sum(len(sc.agents["x"]) for sc in scs)
    ens = fps.Ensemble(scs, stream=stream)
    ens.autotune()
    log("ensemble: autotuned")
    ens.step(args.ens_warmup)
    torch.cuda.synchronize()
    p0 = sum(m.diag()["ped_steps"] for m in ens.members)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ens.step(args.ens_steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    p1 = sum(m.diag()["ped_steps"] for m in ens.members)
    kms = ens.step_profiled(20)
    out = {"workload": f"intervention_sweep_{len(scs)} (grids 256/512/1024 at 0.25 m, barrier, responders, "
                       f"evacuees; seed 3303)",
           "scenarios": len(scs), "cells_per_step": cells, "agents": agents, "steps": args.ens_steps,
           "ms_per_step": ms / args.ens_steps,
           "cell_updates_per_s": cells * args.ens_steps / (ms * 1e-3),
           "scenario_steps_per_s": len(scs) * args.ens_steps / (ms * 1e-3),
           "ped_steps_per_s": (p1 - p0) / (ms * 1e-3),
           "flood_update_ms_per_launch": kms[0],
           "flood_update_GBs": FV_BYTES_PER_CELL * cells / (kms[0] * 1e-3) / 1e9,
           "kernel_ms_per_launch_in_step": {"flood_update": kms[0], "ped_step": kms[1], "end_of_step": kms[2],
                                            "bin_place": kms[3], "bin_sort": kms[4]}}
    ens.close()
    del ens
    torch.cuda.empty_cache()
    return out


def surrogate_section(args):
    """Learned flood update: train on finite-volume trajectories of 256^2
    random layouts, judge held-out pairs, then the surrogate-assisted
    ensemble against the plain finite-volume ensemble on large grids."""
    import numpy as np
    import torch
    from paper_1908_05232_amd import fps, surrogate as SG
    t_all = time.perf_counter()
    n, per = 256, 64
    pairs = args.sur_pairs
    n_traj = args.sur_traj // per * per
    ds = SG.Dataset(n_traj * pairs, n)
    t0 = time.perf_counter()
    fixed = []
    for b in range(n_traj // per):
        # half the layouts carry a completed sandbag line (raised bed) as in the sweeps
        cases = [SG.flood_case(100000 + b * per + k, n=n,
                               barrier_height=0.2 + 0.8 * ((b * per + k) % 7) / 6 if k % 2 else None)
                 for k in range(per)]
        fixed.append(SG.generate_pairs(cases, ds, warmup=50 + 25 * (b % 8), pairs=pairs, every=24))
        if b % 8 == 0:
            log(f"surrogate: trajectories {(b + 1) * per}/{n_traj}")
    t_gen = time.perf_counter() - t0
    sur = fps.Surrogate(args.sur_batch, n, n)
    sur.set_params(torch.tensor(SG.init_params(0)).cuda())
    (hist, t_train) = SG.timed(SG.train, sur, ds, args.sur_train_steps, args.sur_batch, lr=1e-3,
                               log_every=max(1, args.sur_train_steps // 10))
    log(f"surrogate: trained, loss {hist[0][1]:.4g} -> {hist[-1][1]:.4g}")
    flops_train = 3 * 230400 * n * n * args.sur_batch * args.sur_train_steps
    del ds
    torch.cuda.empty_cache()
    # held-out pairs
    held = [SG.flood_case(900000 + k, n=n, barrier_height=0.5 if k % 2 else None) for k in range(per)]
    kept = []
    hds = SG.Dataset(per * 2, n)
    SG.generate_pairs(held, hds, warmup=150, pairs=2, every=40, keep=kept)
    ev = SG.evaluate(sur, held, kept)
    log(f"surrogate: held-out {ev}")
    del hds, kept
    torch.cuda.empty_cache()
    # surrogate-assisted coupled ensemble against the plain finite-volume
    # coupled ensemble, same scenarios (members of the large sweep with the
    # step capped at 0.01 s), people walking in both arms
    big = SG.coupled_cases(args.sur_big_s, n=args.sur_big_n, n_evac=args.sur_big_people)
    log("surrogate: large cases built")
    params = sur.get_params()
    blocks = args.sur_blocks

    def run_plain():
        P = fps.Ensemble(big)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(blocks):
            P.step(SG.K_STEPS)
        torch.cuda.synchronize()
        return P, time.perf_counter() - t0

    def run_assisted(stride):
        A = SG.AssistedEnsemble(big, params, chunk=args.sur_chunk, stride=stride)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for b in range(blocks):
            A.block()
        torch.cuda.synchronize()
        return A, time.perf_counter() - t0

    P, t_plain = run_plain()
    P.close()
    del P
    torch.cuda.empty_cache()
    people = args.sur_big_s * args.sur_big_people
    runs = []
    for st in [int(v) for v in str(args.sur_strides).split(",") if v]:
        A, t_assist = run_assisted(st)
        stats = dict(A.stats)
        A.close()
        del A
        torch.cuda.empty_cache()
        # the bar at every person after every block: both arms again, in lockstep
        A, P = SG.AssistedEnsemble(big, params, chunk=args.sur_chunk, stride=st), fps.Ensemble(big)
        worst_bad, worst_dh = 0, 0.0
        for b in range(blocks):
            A.block()
            P.step(SG.K_STEPS)
            bad, dh = SG.bar_check(P, A)
            worst_bad, worst_dh = max(worst_bad, bad), max(worst_dh, dh)
            log(f"surrogate: stride {st}, block {b + 1}/{blocks}: {bad} people off, max |dh| {dh:.4f} m, "
                f"{A.stats}")
        A.close()
        P.close()
        del A, P
        torch.cuda.empty_cache()
        meets = worst_bad == 0
        runs.append({"judge_stride": st, "judge_hr_margin": 0.1, "judge_h_margin_m": 0.01,
                     "judged_people_per_block": stats["judged_people"] / blocks,
                     "judged_cell_fraction": stats["judged_cells"] / blocks,
                     "blocks_accepted": stats["accepted"], "blocks_fallback": stats["fallback"],
                     "cfl_fallback": stats["cfl_fallback"], "assisted_s": t_assist,
                     "ratio_assisted_over_fv": t_plain / t_assist,
                     "most_people_off_at_a_check": worst_bad, "max_dh_m": worst_dh, "meets_bar": meets,
                     "assisted_scenarios_per_s_at_bar": args.sur_big_s / t_assist if meets else None})
    # forward throughput alone (one chunk)
    sb = fps.Surrogate(args.sur_chunk, args.sur_big_n, args.sur_big_n)
    sb.set_params(params)
    x = torch.zeros((args.sur_chunk, args.sur_big_n, args.sur_big_n, 16), dtype=torch.bfloat16, device="cuda")
    yb = torch.empty((args.sur_chunk, args.sur_big_n, args.sur_big_n, 4), dtype=torch.float32, device="cuda")
    sb.forward(x, yb)
    _, t_fwd = SG.timed(sb.forward, x, yb)
    sb.close()
    px = args.sur_chunk * args.sur_big_n ** 2
    out = {
        "training": {"workload": f"{n_traj} finite-volume trajectories of {n}x{n} random layouts, {pairs} "
                                 f"pairs each (t -> t + {SG.K_STEPS} steps of 0.01 s)",
                     "pairs": n_traj * pairs, "generate_s": t_gen, "fixed_step_fraction": float(np.mean(fixed)),
                     "train_steps": args.sur_train_steps, "batch": args.sur_batch, "train_s": t_train,
                     "train_TFLOPs": flops_train / t_train / 1e12, "loss_history": hist},
        "held_out": ev,
        "assisted_vs_fv": {
            "workload": f"{args.sur_big_s} x {args.sur_big_n}^2 members of the large sweep, "
                        f"{args.sur_big_people} people walking in each, step capped at 0.01 s, {blocks} blocks of "
                        f"{SG.K_STEPS} steps",
            "people": people, "fv_s": t_plain, "fv_scenarios_per_s": args.sur_big_s / t_plain,
            "bar": "every person within 1 cm and the same hazard class after every block",
            "runs": runs,
            "forward_TFLOPs": 230400 * px / t_fwd / 1e12, "forward_ms_per_chunk": t_fwd * 1e3},
        "section_s": time.perf_counter() - t_all,
    }
    return out


def surrogate_probe(fwd_only=False):
    """Timing probe of the surrogate kernels alone (for the profiler): 23
    training steps and 20 forwards at 8 x 256^2, 6 forwards at 4 x 2048^2;
    with fwd_only, only 3 forwards at 4 x 2048^2."""
    import torch
    from paper_1908_05232_amd import fps, surrogate as SG
    params = torch.tensor(SG.init_params(0)).cuda()
    out = {}

    def timed(fn, reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    if not fwd_only:
        sur = fps.Surrogate(8, 256, 256)
        sur.set_params(params)
        g = torch.Generator(device="cuda").manual_seed(0)
        x = (torch.randn(8, 256, 256, 16, device="cuda", generator=g) * 0.5).bfloat16()
        x[..., 6:] = 0
        t = torch.randn(8, 256, 256, 4, device="cuda", generator=g) * 0.1
        t[..., 3] = 0
        for _ in range(3):
            sur.train_step(x, t, 1e-4)
        dt = timed(lambda: sur.train_step(x, t, 1e-4), 20)
        out["train_step_ms_8x256"] = dt * 1e3
        out["train_TFLOPs"] = 3 * 230400 * 8 * 65536 / dt / 1e12
        y = torch.empty(8, 256, 256, 4, device="cuda")
        dt = timed(lambda: sur.forward(x, y), 20)
        out["forward_ms_8x256"] = dt * 1e3
        out["forward_TFLOPs_8x256"] = 230400 * 8 * 65536 / dt / 1e12
    big = fps.Surrogate(4, 2048, 2048)
    big.set_params(params)
    xb = torch.zeros(4, 2048, 2048, 16, device="cuda", dtype=torch.bfloat16)
    yb = torch.empty(4, 2048, 2048, 4, device="cuda")
    big.forward(xb, yb)
    dt = timed(lambda: big.forward(xb, yb), 3 if fwd_only else 5)
    out["forward_ms_4x2048"] = dt * 1e3
    out["forward_TFLOPs_4x2048"] = 230400 * 4 * 2048 * 2048 / dt / 1e12
    print(json.dumps({"surrogate_probe": out}), flush=True)


def headline_section(args, stream):
    """The large sweep as one ensemble: K timed coupled steps (graph replay),
    then the flood launch timed alone and the per-kernel breakdown."""
    import torch
    from paper_1908_05232_amd import fps, inputs as I
    t0 = time.perf_counter()
    scs = I.large_sweep(args.large_s, n=args.large_n, n_evac=args.large_people, workers=8)
    log(f"headline: {len(scs)} scenarios of {args.large_n}^2 built in {time.perf_counter() - t0:.1f} s")
    cells = sum(sc.desc.nx * sc.desc.ny for sc in scs)
    agents = sum(len(sc.agents["x"]) for sc in scs)
    sample = scs[0]
    ens = fps.Ensemble(scs, stream=stream)
    del scs
    # the warm-up steps, untimed, in two parts: the tile shape is tuned on the
    # state after the first part, and the second part (one graph chunk)
    # captures the graph of the tuned shape
    chunk = 16
    ens.set_graph(0 if args.no_graph else chunk)
    ens.step(max(args.warmup - chunk, 0))
    if args.rows:
        for m in ens.members:
            m.set_rows_per_wave(args.rows)
    else:
        ens.autotune()
    rows = sorted({m.rows_per_wave() for m in ens.members})
    log(f"headline: rows per wave {rows}")
    ens.step(min(args.warmup, chunk))
    torch.cuda.synchronize()
    d0 = [m.diag() for m in ens.members]
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    ens.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    d1 = [m.diag() for m in ens.members]
    log(f"headline: {args.steps} steps in {ms:.2f} ms")
    kms = ens.step_profiled(args.profile_steps)
    fv_ms = ens.time_flood(args.flood_reps)
    ens.set_flux(fps.FPS_FLUX_HLL)
    fv_ms_hll = ens.time_flood(args.flood_reps)
    ens.set_flux(fps.FPS_FLUX_HLLC)
    ens.set_order(2)
    fv_ms_o2 = ens.time_flood(args.flood_reps)
    ens.set_order(1)
    wet = sum(float((m.h > 1e-5).float().mean()) for m in ens.members) / len(ens.members)
    out = {
        "cells": cells, "agents": agents, "rows": rows, "ms": ms, "fv_ms": fv_ms,
        "config": {"workload": f"large_sweep_{len(ens.members)}x{args.large_n}",
                   "scenarios": len(ens.members), "grid": [args.large_n, args.large_n], "dx_m": 0.25,
                   "cells_per_step": cells, "evacuees": agents, "rows_per_wave": rows,
                   "steps_timed": args.steps,
                   "sim_time_s": [min(d["t"] for d in d0), max(d["t"] for d in d1)],
                   "wet_cell_fraction_after": wet,
                   "recipe": "inputs.large_sweep(32, n=2048, n_evac=50000, seed=5)"},
        "secondary": {
            "ped-steps/s": (sum(d["ped_steps"] for d in d1) - sum(d["ped_steps"] for d in d0)) / (ms * 1e-3),
            "scenario_steps_per_s": len(ens.members) * args.steps / (ms * 1e-3),
            "flood_update_ms_per_launch": fv_ms,
            "flood_update_ms_per_launch_hll_flux": fv_ms_hll,
            "flood_update_ms_per_step_second_order": fv_ms_o2,
            "kernel_ms_per_launch_in_step": {"flood_update": kms[0], "ped_step": kms[1], "end_of_step": kms[2],
                                             "bin_place": kms[3], "bin_sort": kms[4]}},
    }
    ens.close()
    del ens
    torch.cuda.empty_cache()
    return out, sample


def stability_section(args, stream):
    """The pedestrian step without the body rules, with the stability rule
    (varied bodies standing in the flow) and with the stability and wading
    rules: 8 scenarios of 1024^2 cells, wet everywhere, with 50,000 evacuees
    each."""
    import copy
    import dataclasses
    import torch
    from paper_1908_05232_amd import fps, inputs as I
    scs = I.large_sweep(8, n=1024, n_evac=50000, seed=7)
    out = {"workload": "large_sweep_8x1024 with 50,000 evacuees each", "agents": 8 * 50000}
    bodies = [I.add_bodies(copy.deepcopy(sc), seed=k) for k, sc in enumerate(scs)]
    wading = [copy.deepcopy(sc) for sc in bodies]
    for sc in wading:
        sc.ped = dataclasses.replace(sc.ped, wading=1)
    for tag, members in (("off", scs), ("on", bodies), ("on_wading", wading)):
        ens = fps.Ensemble(members, stream=stream)
        ens.step(50)
        kms = ens.step_profiled(args.profile_steps)
        out[f"ped_step_ms_rule_{tag}"] = kms[1]
        out[f"unstable_people_rule_{tag}"] = sum(m.diag()["class_count"][5] for m in ens.members)
        ens.close()
        del ens
        torch.cuda.empty_cache()
    return out


def cache_resident_section(args, stream):
    """The 512^2 shopping centre with 2,000 evacuees: a 12.6 MB working set that
    stays in the caches, so its rate is set by launch and dependency latency."""
    import torch
    from paper_1908_05232_amd import fps, inputs as I
    sc = I.shopping_centre(n=512)
    cells = sc.desc.nx * sc.desc.ny
    sim = fps.Sim(sc, stream=stream)
    rows, _ = sim.autotune()
    sim.set_graph(0 if args.no_graph else 64)
    sim.step(args.small_warmup)
    torch.cuda.synchronize()
    d0 = sim.diag()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    sim.step(args.small_steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    d1 = sim.diag()
    kms = sim.step_profiled(500)
    fv_ms = sim.time_flood(500)
    sim.close()
    return {"workload": "shopping_centre_512 (cache-resident rate)", "bound": "latency",
            "cells": cells, "evacuees": len(sc.agents["x"]), "rows_per_wave": rows,
            "steps": args.small_steps, "ms_per_step": ms / args.small_steps,
            "cell_updates_per_s": cells * args.small_steps / (ms * 1e-3),
            "ped_steps_per_s": (d1["ped_steps"] - d0["ped_steps"]) / (ms * 1e-3),
            "sim_time_s": [d0["t"], d1["t"]],
            "flood_update_ms_per_launch": fv_ms,
            "flood_update_GBs_algorithmic": FV_BYTES_PER_CELL * cells / (fv_ms * 1e-3) / 1e9,
            "kernel_ms_per_launch_in_step": {"flood_update": kms[0], "ped_step": kms[1], "end_of_step": kms[2],
                                             "bin_place": kms[3], "bin_sort": kms[4]}}


def probe_section(args, stream):
    """The flood kernel on one fully wet 8192^2 grid, beside the copy ceilings
    of the part (torch's device copy and the library's own streaming copy)."""
    import torch
    from paper_1908_05232_amd import fps, inputs as I
    big = I.wet_probe(args.probe_n)
    bsim = fps.Sim(big, stream=stream)
    del big
    brows, _ = bsim.autotune()
    if args.no_graph:
        bsim.set_graph(0)
    bsim.step(4)
    bms = bsim.time_flood(args.probe_steps)
    bsim.set_flux(fps.FPS_FLUX_HLL)
    bms_hll = bsim.time_flood(args.probe_steps)
    bsim.set_flux(fps.FPS_FLUX_HLLC)
    bsim.set_order(2)
    bms_o2 = bsim.time_flood(args.probe_steps)
    bcells = args.probe_n * args.probe_n
    bach = FV_BYTES_PER_CELL * bcells / (bms * 1e-3) / 1e9
    probe = {"workload": f"wet_probe_{args.probe_n} (fully wet dam break, {bcells} cells)",
             "rows_per_wave": brows,
             "ms_per_launch": bms, "cell_updates_per_s": bcells / (bms * 1e-3),
             "achieved_GBs": bach, "frac": bach / HBM_PEAK_GBS,
             "hll_flux_ms_per_launch": bms_hll,
             "second_order_ms_per_step": bms_o2,
             "working_set_MB": (FV_BYTES_PER_CELL + 12) * bcells / 1e6}
    bsim.close()
    del bsim
    torch.cuda.empty_cache()
    # the practical streaming rate of the part: a plain 1 GiB device copy
    # (bytes read + bytes written per second)
    ca = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    cb = torch.empty_like(ca)
    for _ in range(3):
        cb.copy_(ca)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        cb.copy_(ca)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * ca.numel() * 4 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    probe["copy_1GiB_GBs"] = copy_gbs
    probe["frac_of_copy"] = bach / copy_gbs
    del ca, cb
    torch.cuda.empty_cache()
    return probe


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--large-s", type=int, default=32, help="scenarios of the headline sweep")
    ap.add_argument("--large-n", type=int, default=2048, help="grid side of the headline sweep")
    ap.add_argument("--large-people", type=int, default=50000, help="evacuees per scenario")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--flood-reps", type=int, default=50)
    ap.add_argument("--cpu-steps", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--oracle-full", action="store_true",
                    help="also time the oracle over the whole 20,000-step 512^2 run (one thread and OpenMP)")
    ap.add_argument("--rows", type=int, default=0,
                    help="rows per wave of the flood update on the headline workload (0: autotune)")
    ap.add_argument("--small-steps", type=int, default=20000)
    ap.add_argument("--small-warmup", type=int, default=200)
    ap.add_argument("--no-small", action="store_true")
    ap.add_argument("--probe-n", type=int, default=8192,
                    help="side of the fully wet grid used for the HBM probe (0 = skip)")
    ap.add_argument("--probe-steps", type=int, default=50)
    ap.add_argument("--no-graph", action="store_true",
                    help="launch every kernel eagerly (profilers trace graph-replayed kernels poorly)")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--ens-scenarios", type=int, default=64)
    ap.add_argument("--ens-steps", type=int, default=500)
    ap.add_argument("--ens-warmup", type=int, default=50)
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--sur-traj", type=int, default=2000)
    ap.add_argument("--sur-pairs", type=int, default=16)
    ap.add_argument("--sur-batch", type=int, default=8)
    ap.add_argument("--sur-train-steps", type=int, default=2000)
    ap.add_argument("--sur-big-s", type=int, default=32)
    ap.add_argument("--sur-big-n", type=int, default=2048)
    ap.add_argument("--sur-big-people", type=int, default=50000)
    ap.add_argument("--sur-blocks", type=int, default=10)
    ap.add_argument("--sur-chunk", type=int, default=4)
    ap.add_argument("--sur-strides", default="1,250",
                    help="judge every k-th person (plus those near a class boundary); one run each")
    ap.add_argument("--sur-probe", choices=["all", "forward"], default=None,
                    help="only time the surrogate kernels (profiler runs) and exit")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of 1 GiB (counter calibration) and exit")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline workload (profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1908_05232_amd import fps  # noqa: F401  (fails loudly without the HIP library)

    if args.sur_probe:
        surrogate_probe(fwd_only=args.sur_probe == "forward")
        return

    if args.copy_probe:
        n = 1 << 28                                   # 2^28 floats = 1 GiB each way
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": 4 * n}), flush=True)
        return

    stream = torch.cuda.current_stream()
    head, sample = headline_section(args, stream)
    cells, ms, fv_ms = head["cells"], head["ms"], head["fv_ms"]
    workload = head["config"]["workload"]
    value = cells * args.steps / (ms * 1e-3)
    achieved = FV_BYTES_PER_CELL * cells / (fv_ms * 1e-3) / 1e9
    traffic = measured_traffic(workload, head["rows"][0]) if len(head["rows"]) == 1 else None
    out = {
        "metric": "FV cell-updates/s",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": head["config"],
        "secondary": head["secondary"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "fv_step_kernel", "bytes_per_cell": FV_BYTES_PER_CELL,
                     "launch": f"one launch over the {cells} cells of every scenario",
                     "ms_per_launch": fv_ms},
    }
    if not args.headline_only:
        if not args.no_small:
            out["secondary"]["cache_resident_512"] = cache_resident_section(args, stream)
            log("cache-resident 512^2 done")
        if args.probe_n > 0:
            out["secondary"]["hbm_probe"] = probe_section(args, stream)
            log("probe done")
        if not args.no_ensemble:
            out["secondary"]["ensemble"] = ensemble_section(args, stream)
            out["secondary"]["stability_rule"] = stability_section(args, stream)
            log("stability rule done")
        if not args.no_surrogate:
            out["secondary"]["surrogate"] = surrogate_section(args)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(sample, args.cpu_steps, "one 2048^2 scenario of the same sweep")
        one = cpu_baseline(sample, max(2, args.cpu_steps // 4), "one 2048^2 scenario of the same sweep", omp=False)
        out["secondary"]["oracle_timing"] = {"host": host_info(), "one_thread": one}
        if args.oracle_full:
            from paper_1908_05232_amd import inputs as I
            sc2 = I.shopping_centre(n=512)
            out["secondary"]["oracle_timing"]["shopping_centre_512_full"] = {
                "openmp": cpu_baseline(sc2, 20000, "the 512^2 shopping centre (whole run)"),
                "one_thread": cpu_baseline(sc2, 20000, "the 512^2 shopping centre (whole run)", omp=False)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
