"""Benchmark of the coupled flood-pedestrian hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

Workload (synthetic shopping centre): 512 x 512 cells of 0.25 m with random
+3 m building blocks, a triangular inflow of 2 m^2/s peak over 600 s through
the central 30% of the south side, a transmissive north side, and 2,000
evacuees heading for two north exits.  One step = one coupled time step:
flood update (Eq. 2), pedestrian step (hazard, movement, roughness count),
neighbour re-binning and sandbag write-back, all on the GPU.

Prints one JSON line: FV cell-updates/s over the K timed steps (inputs
resident in HBM), the roofline of the flood-update kernel (HIP events around
each launch, on the stream the kernels run on), and the FP64 CPU oracle timed
on a bounded sample of the same workload on this host.
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


def kernel_source_hash():
    src = os.path.join(ROOT, "paper_1908_05232_amd", "csrc", "fps_flood.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def measured_traffic(workload, launches_cells):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current flood kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"fv_step_counters_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(sc, n_steps):
    """The FP64 oracle (single thread) on the first n_steps of the same workload."""
    from oracle import oracle as O
    ref = O.OracleSim(sc)
    t0 = time.perf_counter()
    ref.run(n_steps)
    dt = time.perf_counter() - t0
    cells = sc.desc.nx * sc.desc.ny
    return {"value": cells * n_steps / dt, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_steps} coupled steps of the same 512x512 workload "
                      f"({cells * n_steps:.3g} cell-updates, {dt:.1f} s, FP64 C, one thread)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--profile-steps", type=int, default=500)
    ap.add_argument("--cpu-steps", type=int, default=1000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--probe-n", type=int, default=8192,
                    help="side of the fully wet grid used for the HBM probe (0 = skip)")
    ap.add_argument("--probe-steps", type=int, default=50)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of 1 GiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1908_05232_amd import fps, inputs as I

    if args.copy_probe:
        n = 1 << 28                                   # 2^28 floats = 1 GiB each way
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": 4 * n}), flush=True)
        return

    workload = "shopping_centre_512"
    sc = I.shopping_centre(n=512)
    cells = sc.desc.nx * sc.desc.ny
    stream = torch.cuda.current_stream()
    sim = fps.Sim(sc, stream=stream)
    rows, _ = sim.autotune()          # flood-update tile shape for this grid

    sim.step(args.warmup)
    torch.cuda.synchronize()
    d0 = sim.diag()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    sim.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    d1 = sim.diag()
    value = cells * args.steps / (ms * 1e-3)
    ped_rate = (d1["ped_steps"] - d0["ped_steps"]) / (ms * 1e-3)

    # per-launch duration of each kernel, HIP events around every launch
    kms = sim.step_profiled(args.profile_steps)
    fv_ms = kms[0]
    achieved = FV_BYTES_PER_CELL * cells / (fv_ms * 1e-3) / 1e9
    traffic = measured_traffic(workload, cells)

    probe = None
    if args.probe_n > 0:
        # the same flood kernel on a working set well beyond the 256 MB cache
        big = I.wet_probe(args.probe_n)
        bsim = fps.Sim(big, stream=stream)
        del big
        brows, _ = bsim.autotune()
        bsim.step(4)
        bk = bsim.step_profiled(args.probe_steps)
        bcells = args.probe_n * args.probe_n
        bach = FV_BYTES_PER_CELL * bcells / (bk[0] * 1e-3) / 1e9
        probe = {"workload": f"wet_probe_{args.probe_n} (fully wet dam break, {bcells} cells)",
                 "rows_per_wave": brows,
                 "ms_per_launch": bk[0], "cell_updates_per_s": bcells / (bk[0] * 1e-3),
                 "achieved_GBs": bach, "frac": bach / HBM_PEAK_GBS,
                 "working_set_MB": (FV_BYTES_PER_CELL + 12) * bcells / 1e6}
        bsim.close()
        del bsim
        torch.cuda.empty_cache()

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
        "config": {"workload": workload, "cells": cells, "dx_m": sc.desc.dx, "rows_per_wave": rows,
                   "evacuees": len(sc.agents["x"]), "steps_timed": args.steps,
                   "sim_time_s": [d0["t"], d1["t"]]},
        "secondary": {"ped-steps/s": ped_rate,
                      "kernel_ms_per_launch": {"flood_update": kms[0], "ped_step": kms[1],
                                               "end_of_step": kms[2], "bin_place": kms[3],
                                               "bin_sort": kms[4]},
                      "hbm_probe": probe},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "fv_step_kernel", "bytes_per_cell": FV_BYTES_PER_CELL},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
