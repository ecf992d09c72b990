"""Benchmark: cell-updates/s of the SSP-RK3 step at 2048 x 512 on one MI355X.

A cell-update is one cell advanced by one full step (CFL reduction, three fused
stages with the phase-change source).  Workloads, all synthetic and seeded:

* production jet 2048 x 512 (axial stretch 1.002, radial clustering about the core
  lip, ambient 218 K / 23.8 kPa / ice RH 1.1, lognormal soot), run three ways:
  plain FP64, mixed precision (FP32 storage, fluxes and RK update; FP64 source),
  and mixed precision with the learned source attached (the headline);
* its source-active twin (hydrogen-like core water, cold bypass) on the same
  mesh, where the phase-change source is live: the same three paths, the gain of
  the surrogate (mixed exact step time / mixed surrogate step time), the share of
  active cells it takes, and the error of each path against the FP64 path;
* 64 plumes of uneven size advanced in one captured graph (mixed precision, 2000 steps);
* one GPU's share of the production jet split into 2, 4 and 8 x-slabs (mixed and FP64),
  and the stage kernel on the 2048 x 2048 jet, whose states exceed the Infinity Cache.

Timed regions: K steps of the captured step graph with inputs resident in HBM,
bracketed by synchronisation.  The roofline entry is the fused stage kernel of the
headline path, timed with HIP events on the stream it is launched on; `traffic` and
`valu_issue` come from the committed rocprofv3 summaries in profiles/ while they were
taken on the kernel sources as they are.

Prints ONE JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s at 2048x512 (mixed+surrogate vs plain FP64), % HBM roofline"
HBM_PEAK_GBS = 8000.0
COUNTER_FILE = os.path.join(ROOT, "profiles", "k_stage_mixed_2048x512_counters.txt")
VALU_FILE = os.path.join(ROOT, "profiles", "k_stage_mixed_2048x512_valu.txt")
# vector-instruction issue limit: 256 CUs x 4 SIMDs, one wave64 FP32 instruction per
# SIMD every 4 cycles (16 lanes) at 2.4 GHz
VALU_PEAK_WAVE_INSTS = 256 * 4 * 2.4e9 / 4
KERNEL_SOURCES = ["paper_2504_20742_amd/csrc/cp_kernels.hip", "paper_2504_20742_amd/csrc/cp_physics.hpp",
                  "paper_2504_20742_amd/csrc/cp_internal.hpp"]


def stage_bytes_per_cell(esz):
    # fused stage: read U^(s-1) and U^n, write U^(s) (15 variables); stage 1 does
    # not read U^n.  Average over the three launches of a step.
    return (2 * 15 * esz + 3 * 15 * esz + 3 * 15 * esz) / 3.0


def kernel_source_hash(root=ROOT):
    """Hash of the stage-kernel sources with comments and white space removed (a
    comment edit does not change the kernel the counters were taken on)."""
    import re
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(root, p)) as f:
            txt = f.read()
        txt = re.sub(r"/\*.*?\*/", " ", txt, flags=re.S)
        txt = re.sub(r"//[^\n]*", " ", txt)
        h.update(" ".join(txt.split()).encode())
    return h.hexdigest()[:16]


def _counter_value(path, key, tile):
    """A per-launch figure from a committed rocprofv3 counter summary, if it was
    taken on the kernel sources as they are now and on this tile shape (else None)."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    if vals.get("tile") != "%dx%d" % tuple(tile):
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def measured_traffic(tile):
    """HBM bytes per stage launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)."""
    return _counter_value(COUNTER_FILE, "hbm_bytes_per_launch", tile)


def measured_valu(tile):
    """Vector-ALU wave-instructions per stage launch (SQ_INSTS_VALU)."""
    return _counter_value(VALU_FILE, "valu_wave_insts_per_launch", tile)


def condensed_water(s, U):
    """Condensed water (liquid of both populations + ice) per radian of the
    axisymmetric domain [kg]."""
    import math
    import torch
    xf, rf = s.faces()
    dx = torch.as_tensor(xf[1:] - xf[:-1], device=U.device, dtype=torch.float64)
    rdr = torch.as_tensor((rf[1:] - rf[:-1]) * 0.5 * (rf[1:] + rf[:-1]), device=U.device, dtype=torch.float64)
    liq = U[8].double() + (U[18].double() if U.shape[0] > 15 else 0.0)
    cond = 4.0 / 3.0 * math.pi * (1000.0 * liq + 917.0 * U[12].double())
    return float((cond * rdr[:, None] * dx[None, :]).sum())


def run_path(binding, m, c, precision, steps, warmup, stage_reps=0, sur=None, keep=False, tile=None, qmode=None,
             table_h=0.0, drift=False, bimodal=False):
    import torch
    s = binding.Solver(m, c, precision)
    if bimodal:
        s.set_bimodal(True)
    U = s.init()
    if drift:
        s.set_drift(True)
    if tile:
        s.set_tile(*tile)
    if qmode is not None:
        s.set_qmode(qmode)
    if table_h > 0.0:
        s.set_property_table(table_h)
    if sur is not None:
        s.sur_set(sur[0], sur[1])
        s.set_qmode(binding.CP_Q_SURROGATE)
    s.step_n(U, max(warmup, 1))            # includes autotuning + graph capture
    d0 = s.diag(U)
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
    out = dict(cell_updates_per_s=cells * steps / (ms / 1e3), ms_per_step=ms / steps, wall_s=wall,
               sim_time_s=sim_t, tile=list(s.get_tile()), max_lnS_l=d["max_lnS_l"],
               active_cells=d["active_cells"], esz=8 if precision == binding.CP_FP64 else 4, cells=cells)
    if d["active_cells"] > 0:
        out["condensed_water_per_rad"] = condensed_water(s, U)
        if bimodal:   # share of the droplet number in the homogeneously nucleated population
            n_het, n_hom = float(U[5].double().sum()), float(U[15].double().sum())
            out["homogeneous_droplet_number_share"] = n_hom / max(n_het + n_hom, 1e-300)
        # exact-source sub-steps over the timed steps, per cell-stage of the active set
        subs = d["nsub_total"] - d0["nsub_total"]
        out["source_substeps_per_step"] = subs / steps
        out["mean_nsub_per_active_cell_stage"] = subs / (3.0 * steps * d["active_cells"])
    if sur is not None:
        n_net = d["surrogate_cells"] - d0["surrogate_cells"]
        n_fb = d["fallback_cells"] - d0["fallback_cells"]
        out["network_cell_stages"] = n_net
        out["fallback_cell_stages"] = n_fb
        out["network_share"] = n_net / max(n_net + n_fb, 1.0)
    if stage_reps:
        out["stage_ms"] = s.time_stage(U, stage_reps)
        out["stage_bytes"] = stage_bytes_per_cell(out["esz"]) * cells
    s.close()
    if keep:
        out["U"] = U
    else:
        del U
        torch.cuda.empty_cache()
    return out


def rel_errors(U, Uref):
    """Relative L2 errors of U against Uref: gas state (rho, rho E, rho Y_v each, and
    the momentum vector), ice number (v = 9), total condensate+vapour water."""
    import torch
    a, b = U.double(), Uref.double()

    def rel(x, y):
        n = torch.linalg.vector_norm(y)
        return float(torch.linalg.vector_norm(x - y) / n) if float(n) > 0 else float(x.abs().max())

    mom = float(torch.sqrt(((a[1:3] - b[1:3]) ** 2).sum() / (b[1:3] ** 2).sum()))
    return {"gas": max(rel(a[0], b[0]), rel(a[3], b[3]), rel(a[4], b[4]), mom), "ice_mu0": rel(a[9], b[9])}


def train_surrogate(binding, inputs, log):
    """The network of the learned source, trained on the source-active jet on the
    production mesh (exact FP64 source of the library as the teacher)."""
    from paper_2504_20742_amd import surrogate
    m, c = inputs.sa2(0)
    t0 = time.perf_counter()
    net, norm, rep = surrogate.build(binding, [(m, c)], snapshots=8, every=25, epochs=8, max_rows=1000000)
    rep["seconds"] = time.perf_counter() - t0
    log("bench: surrogate trained on %d rows in %.1f s (val loss %.3f)" % (rep["rows"], rep["seconds"],
                                                                           rep["final_val_loss"]))
    return net, norm, rep


ACTIVE_PATHS = ("fp64", "mixed", "mixed_surrogate", "mixed_tables", "mixed_drift", "mixed_equilibrium",
                "fp64_bimodal", "mixed_bimodal")


def run_source_active(binding, inputs, steps, warmup, trained, which=ACTIVE_PATHS):
    """Source-active jet on the production mesh: FP64, mixed exact, mixed + surrogate,
    mixed with tabulated water properties, mixed with particle drift, the mixed path
    with the equilibrium comparison model, and two liquid populations in FP64 and
    mixed (`which` selects a subset; errors are reported against the FP64 path of the
    same model when it ran)."""
    import torch
    m, c = inputs.sa2(0)
    res = {}
    runs = {
        "fp64": lambda: run_path(binding, m, c, binding.CP_FP64, steps, warmup, keep=True),
        "mixed": lambda: run_path(binding, m, c, binding.CP_MIXED, steps, warmup, keep=True),
        "mixed_surrogate": lambda: run_path(binding, m, c, binding.CP_MIXED, steps, warmup,
                                            sur=(trained[0], trained[1].pack()), keep=True),
        # water properties from 0.25 K tables read by second-order Taylor expansion
        "mixed_tables": lambda: run_path(binding, m, c, binding.CP_MIXED, steps, warmup, keep=True, table_h=0.25),
        # droplets and crystals drifting against the gas (a model extension: its change
        # against the FP64 path without drift is the drift's own effect)
        "mixed_drift": lambda: run_path(binding, m, c, binding.CP_MIXED, steps, warmup, keep=True, drift=True),
        # the paper's comparison model (a different model: no error against the kinetics)
        "mixed_equilibrium": lambda: run_path(binding, m, c, binding.CP_MIXED, steps, warmup,
                                              qmode=binding.CP_Q_EQUILIBRIUM),
        # two liquid populations (19 variables): the mixed path against the FP64 path of
        # the same model
        "fp64_bimodal": lambda: run_path(binding, m, c, binding.CP_FP64, steps, warmup, keep=True, bimodal=True),
        "mixed_bimodal": lambda: run_path(binding, m, c, binding.CP_MIXED, steps, warmup, keep=True, bimodal=True),
    }
    for k in ACTIVE_PATHS:
        if k in which:
            res[k] = runs[k]()
    if "mixed_bimodal" in res and "fp64_bimodal" in res:
        res["mixed_bimodal"]["error_vs_fp64_bimodal"] = rel_errors(res["mixed_bimodal"]["U"],
                                                                  res["fp64_bimodal"]["U"])
    if "fp64" in res:
        for k in ("mixed", "mixed_surrogate", "mixed_tables", "mixed_drift"):
            if k in res:
                res[k]["error_vs_fp64"] = rel_errors(res[k]["U"], res["fp64"]["U"])
    for d in res.values():
        d.pop("U", None)
    torch.cuda.empty_cache()
    out = {k: {kk: v for kk, v in d.items() if kk not in ("esz", "cells", "wall_s")} for k, d in res.items()}
    if "mixed" in res and "mixed_surrogate" in res:
        out["gain"] = res["mixed"]["ms_per_step"] / res["mixed_surrogate"]["ms_per_step"]
    if "mixed" in which:
        out["exact_source_cost"] = exact_source_cost(binding, m, c, warmup)
    if "mixed" in res and "mixed_equilibrium" in res and res["mixed"].get("condensed_water_per_rad"):
        out["equilibrium_over_kinetic_condensed_water"] = (res["mixed_equilibrium"].get("condensed_water_per_rad", 0.0)
                                                           / res["mixed"]["condensed_water_per_rad"])
    if trained is not None:
        rep = trained[2]
        out["surrogate_training"] = {"rows": rep["rows"], "epochs": rep["epochs"], "seconds": rep["seconds"],
                                     "val_loss": rep["final_val_loss"]}
    out["steps"] = steps
    out["warmup"] = warmup
    return out


def exact_source_cost(binding, m, c, warmup, reps=10):
    """Cost of the exact sub-cycled source on the source-active state (mixed path):
    one cp_source call over the mesh, timed with HIP events; per active cell and per
    sub-step of those cells.  The call is latency-bound (its time is set by the
    stiffest cells' sequential sub-steps), so the per-cell figure is an average."""
    import torch
    s = binding.Solver(m, c, binding.CP_MIXED)
    U = s.init()
    s.step_n(U, max(warmup, 1))
    dt = s.cfl_dt(U)
    Q = s.source(U, dt)
    d = s.diag(U)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        s.source(U, dt, Q)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    subs = s.diag(U)["nsub_total"]     # counted from the last cp_source call on
    s.close()
    del U, Q
    torch.cuda.empty_cache()
    active = max(d["active_cells"], 1.0)
    out = {"ms_per_call": ms, "active_cells": d["active_cells"], "ns_per_active_cell": ms * 1e6 / active}
    if subs:
        out["substeps_per_call"] = subs
        out["ns_per_cell_substep"] = ms * 1e6 / subs
    return out


def run_mlp_inference(binding, net, rows, reps=5):
    """The learned source's network on `rows` synthetic feature rows: the fused MFMA
    inference kernel (all three layers in one launch), timed with HIP events."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(0)
    X = torch.randn((rows, 17), generator=g).cuda()
    for _ in range(3):
        net.forward(X)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        net.forward(X)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    flop = rows * 2.0 * (17 * 256 + 256 * 256 + 256 * 15)
    del X
    torch.cuda.empty_cache()
    return {"rows": rows, "ms": ms, "ns_per_row": ms * 1e6 / rows, "tflops": flop / ms / 1e9,
            "frac_of_bf16_dense_peak": flop / ms / 1e9 / 2500.0}


def copy_bandwidth(gib=1.0, reps=10):
    """Achievable HBM bandwidth: a plain device-to-device copy of `gib` GiB (bytes read
    + written per second), beside the 8 TB/s peak."""
    import torch
    n = int(gib * 2 ** 30) // 4
    src = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes": 2 * n * 4, "ms": ms, "GBps": 2 * n * 4 / ms / 1e6, "frac_of_peak": 2 * n * 4 / ms / 1e6 / HBM_PEAK_GBS}


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
    out = {"value": m["nx"] * m["nr"] * n / el, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
           "sample": "%d SSP-RK3 steps of the 2048x512 workload (FP64 C oracle, OpenMP over rows, %.1f s)" % (n, el)}
    # the same oracle on one thread (one step), and the host CPU
    try:
        import ctypes
        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(1)
        t0 = time.perf_counter()
        o.run(U, 1)
        out["value_1_thread"] = m["nx"] * m["nr"] / (time.perf_counter() - t0)
        gomp.omp_set_num_threads(cores)
    except OSError:
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                out["cpu_model"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--stage-reps", type=int, default=30)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--paths", default="fp64,mixed,mixed_surrogate")
    ap.add_argument("--active-steps", type=int, default=100, help="timed steps of the source-active jet (0: skip)")
    ap.add_argument("--active-warmup", type=int, default=200)
    ap.add_argument("--active-paths", default=",".join(ACTIVE_PATHS),
                    help="source-active paths to run (comma-separated subset of %s)" % ",".join(ACTIVE_PATHS))
    ap.add_argument("--batch-steps", type=int, default=2000, help="steps of the 64-plume batch (0: skip)")
    ap.add_argument("--mlp-rows", type=int, default=1 << 20, help="rows of the timed network inference (0: skip)")
    ap.add_argument("--tile", default="", help="stage tile of the production-jet paths, e.g. 32x8 (default: autotuned)")
    ap.add_argument("--hbm-copy-gib", type=float, default=1.0, help="size of the achievable-bandwidth copy (0: skip)")
    ap.add_argument("--slab-steps", type=int, default=100,
                    help="timed steps of the mixed and FP64 paths on one GPU's share of the production "
                         "jet split into 2, 4 and 8 x-slabs (1024, 512, 256 x 512 cells; 0: skip)")
    ap.add_argument("--big-mesh-steps", type=int, default=20,
                    help="timed steps of the mixed path on the 2048x2048 jet, whose states exceed the "
                         "256 MB Infinity Cache (0: skip)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 512 MiB device copy (calibrates HBM byte counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the solver runs on a single MI355X "
              "(multi-GPU sharding is designed but not built)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2504_20742_amd import binding, inputs
    binding.load()
    torch.cuda.set_device(0)
    log = lambda msg: print(msg, file=sys.stderr, flush=True)
    if a.copy_calib:
        src = torch.empty(512 * 2 ** 20 // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: copy calibration done (3 x 512 MiB)")
        del src, dst
    paths = [p for p in a.paths.split(",") if p]
    active = None
    trained = None
    active_paths = [p for p in a.active_paths.split(",") if p]
    for p in active_paths:
        if p not in ACTIVE_PATHS:
            ap.error("unknown source-active path %r" % p)
    if (a.active_steps > 0 and "mixed_surrogate" in active_paths) or "mixed_surrogate" in paths:
        trained = train_surrogate(binding, inputs, log)
    if a.active_steps > 0 and active_paths:
        log("bench: source-active jet 2048x512, paths %s, %d warmup + %d timed steps each"
            % (",".join(active_paths), a.active_warmup, a.active_steps))
        active = run_source_active(binding, inputs, a.active_steps, a.active_warmup, trained, active_paths)
    m, c = inputs.config2(0)
    res = {}
    for p in paths:
        prec = binding.CP_FP64 if p == "fp64" else binding.CP_MIXED
        log("bench: production jet, path %s, %d warmup + %d timed steps" % (p, a.warmup, a.steps))
        attach = (trained[0], trained[1].pack()) if p == "mixed_surrogate" else None
        tile = tuple(int(x) for x in a.tile.split("x")) if a.tile else None
        res[p] = run_path(binding, m, c, prec, a.steps, a.warmup, a.stage_reps, sur=attach, tile=tile, keep=True)
    if a.mlp_rows > 0:
        from paper_2504_20742_amd import surrogate
        if trained is None:
            net = binding.MLP(17, 256, 15)
            net.set_params(surrogate.init_params(0))
        else:
            net = trained[0]
        log("bench: network inference on %d rows" % a.mlp_rows)
        mlp = run_mlp_inference(binding, net, a.mlp_rows)
    else:
        mlp = None
    if not res:   # no production-jet path: the parts that ran, without a headline
        part = {"surrogate_inference": mlp, "source_active_2048x512": active}
        if a.batch_steps > 0:
            log("bench: 64-plume batch, %d steps" % a.batch_steps)
            part["batch_64_plumes"] = run_batch(binding, inputs, a.batch_steps)
        print(json.dumps(part), flush=True)
        return
    # accuracy of each path against the FP64 path after the same steps (same dt sequence
    # up to the FP32 CFL limit of the mixed paths), then the states are released
    if "fp64" in res:
        for k in res:
            if k != "fp64":
                res[k]["error_vs_fp64"] = rel_errors(res[k]["U"], res["fp64"]["U"])
    for d in res.values():
        d.pop("U", None)
    torch.cuda.empty_cache()
    head_name = "mixed_surrogate" if "mixed_surrogate" in res else ("mixed" if "mixed" in res else "fp64")
    head = res[head_name]
    achieved = head["stage_bytes"] / (head["stage_ms"] / 1e3) / 1e9
    traffic = measured_traffic(head["tile"])
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
        "dtype": "f64" if head_name == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "production jet 2048x512 (x-stretch 1.002, r-clustered), SSP-RK3 CFL 0.5, "
                               "path=%s, phase-change source %s" % (
                                   head_name, "active in %d cells" % head["active_cells"] if head["active_cells"]
                                   else "inactive (subsaturated everywhere)"),
                   "nx": 2048, "nr": 512, "cells": head["cells"],
                   # the source-active twin on the same mesh is reported beside it
                   "source_activity": {"active_cells": head["active_cells"], "max_lnS_l": head["max_lnS_l"],
                                       "network_cell_stages": head.get("network_cell_stages", 0)}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_stage (%s, tile %dx%d)" % ("f32" if head["esz"] == 4 else "f64", *head["tile"]),
                     "bytes_per_launch": head["stage_bytes"], "ms_per_launch": head["stage_ms"]},
        "paths": {k: dict({kk: v[kk] for kk in ("cell_updates_per_s", "ms_per_step", "stage_ms", "tile",
                                                 "max_lnS_l", "active_cells", "error_vs_fp64") if kk in v},
                          # end to end: algorithmic bytes of a cell-update (8 array passes of the
                          # three stages: 960 B in FP64, 480 B with FP32 storage) at the step rate
                          end_to_end_frac=v["cell_updates_per_s"] * (960.0 if v["esz"] == 8 else 480.0)
                          / (HBM_PEAK_GBS * 1e9))
                  for k, v in res.items()},
    }
    valu = measured_valu(head["tile"]) if head["esz"] == 4 else None
    if valu is not None:
        rate = valu / (head["stage_ms"] / 1e3)
        line["valu_issue"] = {"bound": "alu", "achieved": rate, "peak": VALU_PEAK_WAVE_INSTS,
                              "unit": "wave-instructions/s", "frac": rate / VALU_PEAK_WAVE_INSTS,
                              "insts_per_launch": valu}
    if "fp64" in res:
        line["over_fp64"] = {k: v["cell_updates_per_s"] / res["fp64"]["cell_updates_per_s"]
                             for k, v in res.items() if k != "fp64"}
    if active is not None:
        line["source_active_2048x512"] = active
    if mlp is not None:
        line["surrogate_inference"] = mlp
    if active is not None and mlp is not None and "exact_source_cost" in active:
        # the exact source per active cell (one call over the source-active jet) against
        # one network row: what the learned source would save per cell it takes over
        ex = active["exact_source_cost"]["ns_per_active_cell"]
        line["source_cost_per_cell"] = {"exact_ns_per_active_cell": ex, "network_ns_per_row": mlp["ns_per_row"],
                                        "exact_over_network": ex / mlp["ns_per_row"]}
    if a.hbm_copy_gib > 0:
        log("bench: %.1f GiB device copy (achievable HBM bandwidth)" % a.hbm_copy_gib)
        line["hbm_copy"] = copy_bandwidth(a.hbm_copy_gib)
    if a.slab_steps > 0:
        # a shard of the production jet at its real shape: n_x / k columns, all 512 rows
        # (the same 2 m x 0.5 m jet on a mesh of that size: same cell count and shape)
        line["slabs"] = {}
        for nxs in (1024, 512, 256):
            log("bench: %dx512 slab, %d steps" % (nxs, a.slab_steps))
            ms_, cs_ = inputs.config2(0, nxs, 512)
            line["slabs"]["%dx512" % nxs] = {
                p: {kk: v for kk, v in run_path(binding, ms_, cs_, prec, a.slab_steps, 10).items()
                    if kk in ("ms_per_step", "cell_updates_per_s", "tile")}
                for p, prec in (("mixed", binding.CP_MIXED), ("fp64", binding.CP_FP64))}
    if a.big_mesh_steps > 0:
        # the three FP32 states of 2048 x 512 (189 MB) fit in the 256 MB Infinity Cache;
        # at 2048 x 2048 (755 MB) they do not, so its stage time is a true-HBM figure
        log("bench: mixed path on the 2048x2048 jet, %d steps" % a.big_mesh_steps)
        mb, cb = inputs.config2(0, 2048, 2048)
        big = run_path(binding, mb, cb, binding.CP_MIXED, a.big_mesh_steps, 5, a.stage_reps)
        gbs = big["stage_bytes"] / (big["stage_ms"] / 1e3) / 1e9
        line["stage_2048x2048"] = {"cells": big["cells"], "ms_per_step": big["ms_per_step"],
                                   "cell_updates_per_s": big["cell_updates_per_s"], "stage_ms": big["stage_ms"],
                                   "tile": big["tile"], "achieved_GBps": gbs, "frac": gbs / HBM_PEAK_GBS}
    if a.batch_steps > 0:
        log("bench: 64-plume batch, %d steps" % a.batch_steps)
        line["batch_64_plumes"] = run_batch(binding, inputs, a.batch_steps)
    if not a.no_cpu:
        log("bench: CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(inputs)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
