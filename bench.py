"""Benchmark of the phase-field lattice Boltzmann step on one MI355X.

One step = one time step of both D2Q9 lattices (phase field f and flow g) over the whole
workload.  The default workload is the spinodal-decomposition case: 1024 x 1024 periodic,
phi0 = 0.5 + U[-0.01, 0.01] (seed 0), rho_l / rho_g = 3, sigma = 1e-3, W = 4, M = 0.1,
nu_l = 0.1, nu_g = 1.0.  The headline value is MLUPS (million lattice-node updates of both
lattices per second) with FP32 storage; FP64 and FP16-deviation storage are measured on
the same device and reported next to it with their max-norm error against the FP64 CPU
oracle over the same short horizon.

Prints ONE JSON line.  Inputs are resident in device memory before the timed region;
timing uses HIP events on the stream the library launches on.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (both lattices) and % HBM roofline, FP32/FP16 vs FP64 at stated error"
PEAK_HBM_GBS = 8000.0
# algorithmic bytes per lattice update of the fused step: 9 f + 9 g populations read and
# written once, plus the per-node state beside them read and written once: FP64 phi u of
# the previous step (2 doubles); reduced formats the FP32 planes phi_w, p_w, ux_w, uy_w
ALG_BYTES = {"f64": 36 * 8 + 4 * 8, "f32": 36 * 4 + 8 * 4, "f16": 36 * 2 + 8 * 4}
KERNEL_SRC = os.path.join(ROOT, "paper_1710_09541_amd", "csrc", "lbm_kernels.hip")


def kernel_source_hash():
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def workload(name):
    from paper_1710_09541_amd import cases
    if name == "spinodal1024":
        c = cases.spinodal(1024, seed=0)
        desc = ("spinodal decomposition 1024x1024 periodic, phi0=0.5+U[-0.01,0.01] seed 0, "
                "rho_l/rho_g=3, sigma=1e-3, W=4, M=0.1, nu_l=0.1, nu_g=1.0")
        return [c], desc
    if name == "spinodal4096":
        c = cases.spinodal(4096, seed=0)
        return [c], "spinodal decomposition 4096x4096 periodic (HBM-resident working set)"
    if name == "impact2048":
        c = cases.droplet_impact(2048, 512, D=256, Re=100)
        return [c], "droplet impact on a film 2048x512, D=256, Re=100, We=8000, ratio 1000"
    if name == "batch256":
        cs = cases.batch_ensemble(256, seed=1)
        return cs, "256 static-drop / layered-Poiseuille instances, grids 32..512 (seed 1)"
    raise SystemExit("unknown workload " + name)


def traffic_from_profile(wl, storage, nodes):
    """HBM bytes per launch from the committed rocprofv3 counter summary, scaled by the
    copy-kernel calibration; None if absent or taken on another version of the kernels."""
    path = os.path.join(ROOT, "profiles", "pmc_%s_%s.json" % (wl, storage))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def time_gpu(cs, storage, steps, warmup, kernel, tile_rows):
    import torch
    from paper_1710_09541_amd import lbm
    stream = torch.cuda.Stream()
    sim = lbm.Simulation(cs, storage=storage, kernel=kernel, tile_rows=tile_rows,
                         stream=stream.cuda_stream)
    info = sim.info()
    sim.step(warmup)
    stream.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    sim.close()
    return ms, info


def gpu_error(cs, storage, nsteps, ref):
    from paper_1710_09541_amd import lbm
    from tests.parity import errors
    with lbm.Simulation(cs, storage=storage) as sim:
        sim.step(nsteps)
        got = sim.moments(0)
    return errors(cs[0], got, ref)


def cpu_baseline(cs, steps):
    from oracle.oracle import OracleSim
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    c = cs[0]
    s = OracleSim(c, c["phi0"], c["ux0"], c["uy0"])
    s.step(1)
    t0 = time.perf_counter()
    s.step(steps)
    dt = time.perf_counter() - t0
    nodes = c["nx"] * c["ny"]
    ref = s.moments()
    return {"value": nodes * steps / dt / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": "%dx%d, %d steps after 1 warm-up step, FP64, OpenMP over rows, %.1f s"
                      % (c["nx"], c["ny"], steps, dt)}, ref


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="spinodal1024")
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--kernel", default="auto")
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--variants", default="f64,f16", help="other storages to time ('' for none)")
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        # a plain copy of known size: what the byte counters read for it calibrates them
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4,
                          "launches": 5}), flush=True)
        return

    from paper_1710_09541_amd import lbm
    lbm.load()

    cs, desc = workload(args.workload)
    nodes = sum(c["nx"] * c["ny"] for c in cs)
    print("[bench] workload %s, %d nodes, storage %s" % (args.workload, nodes, args.storage),
          file=sys.stderr, flush=True)

    base = None
    ref = None
    if not args.no_cpu_baseline and len(cs) == 1:
        base, ref = cpu_baseline(cs, args.cpu_steps)
        print("[bench] cpu baseline %.2f MLUPS (%s)" % (base["value"], base["sample"]),
              file=sys.stderr, flush=True)

    results = {}
    for st in [args.storage] + [v for v in args.variants.split(",") if v and v != args.storage]:
        ms, info = time_gpu(cs, st, args.steps, args.warmup, args.kernel, args.tile_rows)
        mlups = nodes * args.steps / (ms / 1e3) / 1e6
        per_launch_s = ms / 1e3 / args.steps
        ach = ALG_BYTES[st] * nodes / per_launch_s / 1e9
        r = {"mlups": mlups, "ms_per_step": ms / args.steps, "kernel": info["kernel"],
             "tile_rows": info["tile_rows"], "alg_bytes_per_lu": ALG_BYTES[st],
             "achieved_gbs": ach, "frac_hbm_peak": ach / PEAK_HBM_GBS}
        if ref is not None:
            e = gpu_error(cs, st, args.cpu_steps + 1, ref)
            r["max_norm_error_vs_oracle"] = {"steps": args.cpu_steps + 1, **e}
        results[st] = r
        print("[bench] %s: %.1f MLUPS, %.4f ms/step, %.0f GB/s algorithmic (%s)"
              % (st, mlups, ms / args.steps, ach, info), file=sys.stderr, flush=True)

    main_r = results[args.storage]
    kname = {1: "k_step (fused)", 2: "k_phi_plane + k_step (split)"}[main_r["kernel"]]
    traffic = traffic_from_profile(args.workload, args.storage, nodes)
    out = {
        "metric": METRIC,
        "value": round(main_r["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "f16": "f32"}[args.storage],
        "data": "synthetic",
        "config": {"workload": desc, "storage": args.storage, "nodes": nodes,
                   "kernel": kname, "tile_rows": main_r["tile_rows"]},
        "roofline": {"bound": "hbm", "achieved": round(main_r["achieved_gbs"], 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(main_r["frac_hbm_peak"], 4), "traffic": traffic,
                     "kernel": kname,
                     "alg_bytes_per_launch": ALG_BYTES[args.storage] * nodes},
        "cpu_baseline": base,
        "variants": {k: v for k, v in results.items()},
        "kernel_source_sha256": kernel_source_hash(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
