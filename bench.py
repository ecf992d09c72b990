"""Benchmark: cell-updates/s of the SSP-RK3 step at 2048 x 512 on one MI355X.

A cell-update is one cell advanced by one full step (CFL reduction, three fused
stages with the phase-change source).  The workload is the production jet mesh
(2048 x 512, axially stretched 1.002, radially clustered about the core lip,
ambient 218 K / 23.8 kPa / ice RH 1.1, synthetic inputs).  Timed: K steps of the
captured step graph with inputs resident in HBM, bracketed by synchronisation.

Prints ONE JSON line.  Headline ``value``: the mixed-precision path (FP32 storage,
fluxes and RK update, FP64 source); the plain FP64 path is reported beside it.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s at 2048x512 (mixed+surrogate vs plain FP64), % HBM roofline"
HBM_PEAK_GBS = 8000.0


def stage_bytes_per_cell(esz):
    # fused stage: read U^(s-1) and U^n, write U^(s) (15 variables); stage 1 does
    # not read U^n.  Average over the three launches of a step.
    return (2 * 15 * esz + 3 * 15 * esz + 3 * 15 * esz) / 3.0


def step_bytes_per_cell(esz):
    # 3 stages (8 array passes of 15 variables) + CFL pass over 5 gas variables
    return 8 * 15 * esz + 5 * esz


def run_path(binding, inputs, precision, steps, warmup, stage_reps):
    import torch
    m, c = inputs.config2(0)
    s = binding.Solver(m, c, precision)
    U = s.init()
    s.step_n(U, max(warmup, 1))            # includes autotuning + graph capture
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    sim_t = s.step_n(U, steps)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    cells = m["nx"] * m["nr"]
    d = s.diag(U)
    stage_ms = s.time_stage(U, stage_reps)
    esz = 8 if precision == binding.CP_FP64 else 4
    out = dict(cell_updates_per_s=cells * steps / (ms / 1e3), ms_per_step=ms / steps, wall_s=wall,
               sim_time_s=sim_t, tile=list(s.get_tile()), stage_ms=stage_ms,
               stage_bytes=stage_bytes_per_cell(esz) * cells, max_lnS_l=d["max_lnS_l"],
               active_cells=d["active_cells"], esz=esz, cells=cells)
    s.close()
    del U
    torch.cuda.empty_cache()
    return out


def run_batch(binding, inputs, steps):
    """64 plumes on meshes drawn from {256x64, 512x128, 1024x256}, mixed precision,
    one graph replay per step covering every plume."""
    import torch
    cases = inputs.config4(seed=0)
    bt = binding.Batch([m for m, _ in cases], [c for _, c in cases], binding.CP_MIXED)
    Us = bt.init()
    bt.step_n(Us, 3)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    bt.step_n(Us, steps)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    cells = sum(m["nx"] * m["nr"] for m, _ in cases)
    bt.close()
    del Us
    torch.cuda.empty_cache()
    return {"plumes": len(cases), "cells": cells, "steps": steps, "ms_per_step": ms / steps,
            "cell_updates_per_s": cells * steps / (ms / 1e3)}


def cpu_baseline(inputs, seconds_target=15.0):
    """The FP64 oracle on this host's cores, a bounded number of steps of the same
    2048 x 512 workload."""
    import oracle
    oracle.build(force=False)
    m, c = inputs.config2(0)
    o = oracle.Oracle(m, c)
    U = o.init()
    t0 = time.perf_counter()
    n = 0
    while True:
        o.run(U, 1)
        n += 1
        el = time.perf_counter() - t0
        if el > seconds_target or n >= 50:
            break
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": m["nx"] * m["nr"] * n / el, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": "%d SSP-RK3 steps of the 2048x512 workload (FP64 C oracle, OpenMP over rows, %.1f s)" % (n, el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--stage-reps", type=int, default=30)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--paths", default="fp64,mixed")
    ap.add_argument("--batch-steps", type=int, default=50, help="steps of the 64-plume batch (0: skip)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 512 MiB device copy (calibrates HBM byte counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the solver runs on a single MI355X "
              "(multi-GPU sharding is described in DESIGN.md but not built)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2504_20742_amd import binding, inputs
    binding.load()
    torch.cuda.set_device(0)
    if a.copy_calib:
        src = torch.empty(512 * 2 ** 20 // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("bench: copy calibration done (3 x 512 MiB)", file=sys.stderr, flush=True)
        del src, dst
    res = {}
    for p in a.paths.split(","):
        prec = binding.CP_FP64 if p == "fp64" else binding.CP_MIXED
        print("bench: path %s, %d warmup + %d timed steps" % (p, a.warmup, a.steps), file=sys.stderr, flush=True)
        res[p] = run_path(binding, inputs, prec, a.steps, a.warmup, a.stage_reps)
    head = res.get("mixed") or res.get("fp64")
    head_name = "mixed" if "mixed" in res else "fp64"
    dom = head
    achieved = dom["stage_bytes"] / (dom["stage_ms"] / 1e3) / 1e9
    line = {
        "metric": METRIC,
        "value": head["cell_updates_per_s"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head_name == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "production jet 2048x512 (x-stretch 1.002, r-clustered), SSP-RK3 CFL 0.5, "
                               "path=%s" % head_name,
                   "nx": 2048, "nr": 512, "cells": head["cells"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_stage (%s, tile %dx%d)" % (head_name, *head["tile"]),
                     "bytes_per_launch": dom["stage_bytes"], "ms_per_launch": dom["stage_ms"]},
        "paths": {k: {kk: v[kk] for kk in ("cell_updates_per_s", "ms_per_step", "stage_ms", "tile",
                                            "max_lnS_l", "active_cells")} for k, v in res.items()},
    }
    if "fp64" in res and "mixed" in res:
        line["mixed_over_fp64"] = res["mixed"]["cell_updates_per_s"] / res["fp64"]["cell_updates_per_s"]
    if a.batch_steps > 0:
        print("bench: 64-plume batch, %d steps" % a.batch_steps, file=sys.stderr, flush=True)
        line["batch_64_plumes"] = run_batch(binding, inputs, a.batch_steps)
    if not a.no_cpu:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(inputs)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
