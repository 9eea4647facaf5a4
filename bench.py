"""Benchmark of the phase-field lattice Boltzmann step on one MI355X.

One step = one time step of both D2Q9 lattices (phase field f and flow g) over the whole
workload.  The default workload is the largest single-GPU configuration: a batch of 256
independent static-drop / layered-Poiseuille instances of uneven size (grids uniform in
32..512 per axis, density ratio 10/100/1000, seed 1; 19,195,714 nodes), advanced together
in one launch per step.  The headline value is MLUPS (million lattice-node updates of both
lattices per second) with FP32 storage; the FP64 and 16-bit formats are timed on the same
device and reported next to it.  Each format states its error against the FP64 CPU oracle:

* per instance, on a sample of the batch (every 16th instance) after the oracle's timed
  steps, max-norm errors of phi, u and p against the oracle run of each instance alone;
* field by field on the layered Poiseuille channel 16 x 512 after 1000 steps (walls,
  step viscosity, density ratio 1000), where the stated tolerances apply.

The roofline fraction counts the algorithmic bytes of the method: every population read
and written once, phi written and read once and phi u of the previous step read and
written once (168 B per lattice update in FP32, 336 in FP64, 96 with 16-bit
populations).  The kernel's own design moves a per-node state each way instead of the phi
plane and phi u: 12 bytes in FP32 (phi_w, u_w), 16 in FP64 (phi u) and with 16-bit
populations (phi_w, p_w, u_w), so 168 / 320 / 104 B; that figure is reported beside it.
HBM rates differ from one device to the next, so the line also carries what a plain
streaming pass over 1 GiB (an elementwise kernel: one read and one write per element) reaches
on the same device and the fraction of it achieved.

Also timed (unless --no-extra):
* the spinodal decomposition 1024 x 1024 (the earlier headline; phi0 = 0.5 + U[-0.01, 0.01],
  ratio 3) in all three formats, with the oracle's coarsening length beside it;
* the same spinodal at 4096 x 4096 and a static drop of radius 1024 at 4096 x 4096 (working sets
  far above the 256 MB last-level cache, so the bandwidth is HBM's);
* the spinodal with the D2Q5 phase-field lattice (5 instead of 9 f populations), with the normal
  of Eq. 29, and with the inverse-linear viscosity of Eq. 25;
* the static drop 64 x 64 and the Poiseuille channel 16 x 512 (both so small that launch
  latency dominates), and the droplet impact at 2048 x 512.

Prints ONE JSON line.  Inputs are resident in device memory before the timed region;
timing uses HIP events recorded on the stream the library launches on.
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
ESIZE = {"f64": 8, "f32": 4, "f16": 2}


def alg_bytes(storage, qf=9):
    """Bytes per lattice update that the fused step kernel moves by design, with a
    phase-field lattice of qf velocities: qf f and 9 g populations read and written once,
    plus the per-node state beside them read and written once (FP64: phi u of the previous
    step, 2 doubles; FP32: phi_w, ux_w, uy_w, 3 floats; 16-bit: phi_w, p_w, ux_w, uy_w,
    4 floats).  D2Q9: FP64 320, FP32 168, FP16 104."""
    state = {"f64": 16, "f32": 12, "f16": 16}[storage]
    return 2 * (qf + 9) * ESIZE[storage] + 2 * state


def method_bytes(storage, qf=9):
    """Algorithmic bytes per lattice update that the method itself must move: qf f and 9 g
    populations read and written once, phi written and read once and phi u of the previous
    step (two values) read and written once, all in the storage's word for the populations
    and its compute word for phi and phi u (FP64: 8 bytes; otherwise 4).  D2Q9: FP64 336,
    FP32 168, FP16 96 (phi and phi u in FP32)."""
    aux = 8 if storage == "f64" else 4
    return 2 * (qf + 9) * ESIZE[storage] + 6 * aux


TOL = {"f64": 1e-12, "f32": 1e-5, "f16": 1e-3}
KERNEL_SRC = os.path.join(ROOT, "paper_1710_09541_amd", "csrc", "lbm_kernels.hip")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def code_hash(text):
    """sha256 (first 16 hex digits) of C++ source with comments and blank space removed, so
    that only a change of the code itself marks measurements taken on it as stale."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    text = "\n".join(" ".join(l.split()) for l in text.splitlines() if l.strip())
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def kernel_source_hash():
    with open(KERNEL_SRC) as fh:
        return code_hash(fh.read())


def workload(name):
    from paper_1710_09541_amd import cases
    if name == "spinodal1024":
        c = cases.spinodal(1024, seed=0)
        desc = ("spinodal decomposition 1024x1024 periodic, phi0=0.5+U[-0.01,0.01] seed 0, "
                "rho_l/rho_g=3, sigma=1e-3, W=4, M=0.1, nu_l=0.1, nu_g=1.0")
        return [c], desc
    if name in ("spinodal1024_d2q5", "spinodal1024_eq29", "spinodal1024_nu_inverse"):
        c = cases.spinodal(1024, seed=0)
        if name.endswith("d2q5"):        # the D2Q5 phase-field lattice
            c["f_lattice"] = 5
            what = "D2Q5 phase-field lattice"
        elif name.endswith("eq29"):      # the normal of Eq. 29 (local non-equilibrium scheme)
            c["grad_scheme"] = cases.GRAD_LOCAL_NEQ
            what = "normal from Eq. 29"
        else:                            # the inverse-linear viscosity law of Eq. 25
            c["visc_law"] = cases.NU_INVERSE
            what = "viscosity law of Eq. 25"
        return [c], "spinodal decomposition 1024x1024 as spinodal1024, %s" % what
    if name == "spinodal4096":
        c = cases.spinodal(4096, seed=0)
        return [c], "spinodal decomposition 4096x4096 periodic, as spinodal1024 otherwise"
    if name == "impact2048":
        c = cases.droplet_impact(2048, 512, D=256, Re=100)
        return [c], "droplet impact on a film 2048x512, D=256, Re=100, We=8000, ratio 1000"
    if name == "batch256":
        cs = cases.batch_ensemble(256, seed=1)
        return cs, ("256 static-drop / layered-Poiseuille instances, grids uniform in 32..512 "
                    "per axis, density ratio 10/100/1000 (seed 1)")
    raise SystemExit("unknown workload " + name)


def traffic_from_profile(wl, storage):
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


def time_gpu(cs, storage, steps, warmup, kernel, tile_rows, final_stats=False, stores="auto",
             grid="auto", deal="auto"):
    """Milliseconds of `steps` steps after `warmup` untimed ones.  With final_stats, also
    the first instance's L and sum(phi) drift at the end (read after the timed region)."""
    import torch
    from paper_1710_09541_amd import lbm
    stream = torch.cuda.Stream()
    sim = lbm.Simulation(cs, storage=storage, kernel=kernel, tile_rows=tile_rows,
                         stream=stream.cuda_stream, stores=stores, grid=grid, deal=deal)
    info = sim.info()
    s0 = sim.reduce()["sum_phi"] if final_stats else None
    sim.step(warmup)
    stream.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    stats = None
    if final_stats:
        phi = sim.moments(0)["phi"]
        stats = {"steps": warmup + steps, "L": crossings_length(phi),
                 "sum_phi_drift": abs(float(sim.reduce()["sum_phi"]) - s0) / s0}
    sim.close()
    return ms, info, stats


def measure(cs, storage, steps, warmup, kernel="auto", tile_rows=0, final_stats=False,
            stores="auto", grid="auto", deal="auto"):
    nodes = sum(c["nx"] * c["ny"] for c in cs)
    qf = cs[0].get("f_lattice", 9)
    ms, info, stats = time_gpu(cs, storage, steps, warmup, kernel, tile_rows, final_stats, stores,
                               grid, deal)
    per_launch_s = ms / 1e3 / steps
    ach = alg_bytes(storage, qf) * nodes / per_launch_s / 1e9
    return {"mlups": nodes * steps / (ms / 1e3) / 1e6, "ms_per_step": ms / steps,
            "kernel": info["kernel"], "tile_rows": info["tile_rows"], "stores": info["stores"],
            "grid": info["grid"], "tile_order": ("rows" if info["strip"] == "rows"
                                                 else "strips of %d tiles" % info["strip"]),
            "narrow_tiles": info["narrow"], "deal": info["deal"],
            "f_lattice": qf,
            "alg_bytes_per_lu": alg_bytes(storage, qf), "achieved_gbs": ach,
            "frac_hbm_peak": ach / PEAK_HBM_GBS, "nodes": nodes, "steps": steps,
            **({"end_of_run": stats} if stats else {})}


def host_round_trip(cs, storage, steps, r):
    """The whole job as a host caller sees it: lbm_init from host fields (device buffers,
    the FP64 upload of phi0, ux0, uy0, the initial equilibria), `steps` steps, and
    lbm_moments back to host memory (five FP64 planes), timed on the host clock.  The launch
    configuration is the one the timed run used, given explicitly, so no autotuning runs."""
    import torch
    from paper_1710_09541_amd import lbm
    nodes = sum(c["nx"] * c["ny"] for c in cs)
    strip = "rows" if r["tile_order"] == "rows" else int(r["tile_order"].split()[2])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim = lbm.Simulation(cs, storage=storage, kernel=r["kernel"], tile_rows=r["tile_rows"],
                         stores=r["stores"], grid=r["grid"], strip=strip,
                         narrow=r["narrow_tiles"], deal=r["deal"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for k in range(len(cs)):
        sim.moments(k)
    t3 = time.perf_counter()
    sim.close()
    return {"steps": steps, "init_ms": (t1 - t0) * 1e3, "steps_ms": (t2 - t1) * 1e3,
            "moments_ms": (t3 - t2) * 1e3, "upload_bytes": 3 * 8 * nodes,
            "download_bytes": 5 * 8 * nodes,
            "mlups": nodes * steps / (t3 - t0) / 1e6}


def crossings_length(phi):
    n = phi.size
    s = phi >= 0.5
    cr = np.count_nonzero(s != np.roll(s, 1, axis=1)) + np.count_nonzero(s != np.roll(s, 1, axis=0))
    return 2.0 * n / max(cr, 1)


def spinodal_accuracy(c, storage, nsteps, ref):
    """L and sum(phi) drift of the GPU run against the oracle's, plus the field error."""
    from paper_1710_09541_amd import lbm
    from tests.parity import errors
    with lbm.Simulation([c], storage=storage) as sim:
        s0 = float(sim.moments(0)["phi"].sum())
        sim.step(nsteps)
        got = sim.moments(0)
    L_gpu, L_ref = crossings_length(got["phi"]), crossings_length(ref["phi"])
    e = errors(c, got, ref)
    return {"steps": nsteps, "L": L_gpu, "L_oracle": L_ref, "L_rel_err": abs(L_gpu / L_ref - 1),
            "sum_phi_drift": abs(float(got["phi"].sum()) - s0) / s0,
            "field_max_err": {k: e[k] for k in ("phi", "u", "p")}}


def poiseuille_parity(storage, ref_cache):
    from paper_1710_09541_amd import cases, lbm
    from tests.parity import errors, run_oracle
    c = cases.layered_poiseuille()
    if "pois" not in ref_cache:
        ref_cache["pois"] = run_oracle(c, 1000)
    with lbm.Simulation([c], storage=storage) as sim:
        sim.step(1000)
        got = sim.moments(0)
    e = errors(c, got, ref_cache["pois"])
    return {"case": "layered Poiseuille 16x512, ratio 1000, step mu, 1000 steps",
            "phi": e["phi"], "u": e["u"], "p": e["p"], "tol": TOL[storage],
            "within_tol": bool(e["u"] <= TOL[storage] and
                               (storage == "f16" or e["phi"] <= TOL[storage]))}


def host_cpu():
    """Model name of this host's CPU, as /proc/cpuinfo gives it."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    """Threads the oracle's OpenMP loops use by default on this host."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    return min(cores, int(os.environ.get("OMP_NUM_THREADS", cores)))


def set_oracle_threads(n):
    """Sets the OpenMP thread count of the calling thread's later parallel regions (the
    oracle's loops) through the OpenMP runtime the oracle is linked with."""
    import ctypes
    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))


def batch_cpu_baseline(cs, steps, every=16):
    """The FP64 oracle timed on this host's cores over a bounded sample of the batch: with
    all threads on every instance, and with one thread on every `every`-th instance.  Each
    instance is created, stepped once untimed and then `steps` timed steps; only the timed
    steps count.  Returns the baseline record and the oracle's moments of the sampled
    instances after 1 + steps steps, keyed by instance index."""
    from oracle.oracle import OracleSim
    threads = host_threads()
    runs = {}

    def run(idx, nthreads, keep):
        set_oracle_threads(nthreads)
        lu, secs = 0, 0.0
        for k in idx:
            c = cs[k]
            s = OracleSim(c, c["phi0"], c["ux0"], c["uy0"])
            s.step(1)
            t0 = time.perf_counter()
            s.step(steps)
            secs += time.perf_counter() - t0
            lu += c["nx"] * c["ny"] * steps
            if keep:
                runs[k] = s.moments()
            del s
        return lu / secs / 1e6, secs, lu

    sample = list(range(0, len(cs), every))
    all_mlups, all_s, all_lu = run(range(len(cs)), threads, False)
    one_mlups, one_s, one_lu = run(sample, 1, True)
    set_oracle_threads(threads)
    return {"value": all_mlups, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "host": host_cpu(),
            "value_1_thread": one_mlups, "cores_1_thread": 1,
            "sample": ("batch of %d instances, FP64, %d steps each after 1 untimed step: all "
                       "instances on %d threads (%.2e lattice updates, %.1f s); every %dth "
                       "instance (%d) on 1 thread (%.2e lattice updates, %.1f s)"
                       % (len(cs), steps, threads, all_lu, all_s, every, len(sample), one_lu,
                          one_s))}, runs


def batch_accuracy(cs, storage, steps, refs, r, masks):
    """Per-instance max-norm errors (phi, u, p) of the batched GPU run after `steps` steps
    against the oracle run of each sampled instance alone, in the launch configuration `r`
    of the timed run (no autotuning).  phi and p are also given outside each drop's interior
    plateau (masks, tests/parity.drop_interior_mask: a disc fixed from the case alone, where
    the oracle itself cannot be followed to the FP32 tolerance); the tolerance is judged
    there, and on u everywhere."""
    from paper_1710_09541_amd import lbm
    from tests.parity import errors, errors_outside
    strip = "rows" if r["tile_order"] == "rows" else int(r["tile_order"].split()[2])
    worst = {"phi": 0.0, "u": 0.0, "p": 0.0}
    judged = {"phi": 0.0, "u": 0.0, "p": 0.0}
    with lbm.Simulation(cs, storage=storage, kernel=r["kernel"], tile_rows=r["tile_rows"],
                        stores=r["stores"], grid=r["grid"], strip=strip,
                        narrow=r["narrow_tiles"], deal=r["deal"]) as sim:
        sim.step(steps)
        for k, ref in refs.items():
            got = sim.moments(k)
            e = errors(cs[k], got, ref)
            o = e if masks[k] is None else errors_outside(cs[k], got, ref, masks[k])
            for q in worst:
                worst[q] = max(worst[q], float(e[q]))
                judged[q] = max(judged[q], float(e[q] if q == "u" else o[q]))
    tol = TOL[storage]
    ok = judged["u"] <= tol and (storage == "f16" or judged["phi"] <= tol)
    return {"steps": steps, "instances": sorted(refs), "max_err": worst,
            "max_err_outside_drop_interiors": judged,
            "nodes_in_drop_interiors": int(sum(int(m.sum()) for m in masks.values()
                                               if m is not None)),
            "tol": tol, "within_tol": bool(ok)}


def copy_bandwidth(reps=10):
    """GB/s (bytes read + written) of a plain streaming pass over 1 GiB on this GPU: an
    elementwise kernel (y = -x, one read and one write per element), timed with HIP events
    over reps passes after three untimed ones.  The runtime's own device-to-device copy
    (torch copy_) reaches only about 80 % of this rate on MI355X; the elementwise kernel
    reaches what a hand-written one-vector-per-thread copy does."""
    import torch
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.neg(x, out=y)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        torch.neg(x, out=y)
    t1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * x.numel() * 4 * reps / (t0.elapsed_time(t1) / 1e3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return gbs


def cpu_baseline(c, steps):
    """The FP64 oracle timed on this host's cores over a bounded sample of the workload."""
    from oracle.oracle import OracleSim
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    s = OracleSim(c, c["phi0"], c["ux0"], c["uy0"])
    s.step(1)
    t0 = time.perf_counter()
    s.step(steps)
    dt = time.perf_counter() - t0
    nodes = c["nx"] * c["ny"]
    ref = s.moments()
    return {"value": nodes * steps / dt / 1e6, "unit": "MLUPS", "cores": min(cores, threads),
            "kind": "oracle", "host": host_cpu(),
            "sample": "%dx%d spinodal, %d steps after 1 untimed step, FP64, OpenMP over rows "
                      "(%d threads), %.1f s" % (c["nx"], c["ny"], steps, min(cores, threads), dt)
            }, ref


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="batch256")
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--kernel", default="auto")
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--stores", default="auto", choices=["auto", "cached", "streaming"])
    ap.add_argument("--grid", default="auto", choices=["auto", "tiles", "persistent"])
    def deal_arg(v):
        if v in ("auto", "bands"):
            return v
        if v.isdigit() and 1 <= int(v) <= 4096:
            return int(v)
        raise argparse.ArgumentTypeError("auto, bands or a chunk of 1 to 4096 tiles")
    ap.add_argument("--deal", default="auto", type=deal_arg,
                    help="tiles to the XCDs: auto, bands, or a chunk of 1 to 4096 tiles")
    ap.add_argument("--variants", default=None,
                    help="other storages to time, comma-separated ('none' for none; default "
                         "f64 for the batch, f64,f16 otherwise)")
    ap.add_argument("--cpu-steps", type=int, default=None,
                    help="oracle steps of the CPU baseline, also the accuracy horizon (default "
                         "40 for the batch, 1500 for a single spinodal)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads (spinodal 1024^2 and 4096^2, static drop "
                         "4096^2, rows f1-f3, small grids, impact)")
    ap.add_argument("--no-round-trip", action="store_true",
                    help="skip the host-to-host job timing (profiled runs: the step kernel's last "
                         "dispatches are then the timed ones)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates HBM byte counters) "
                         "and an elementwise streaming pass over the same bytes")
    args = ap.parse_args()
    deal = args.deal

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this implementation has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        # a plain copy of known size: what the byte counters read for it calibrates them;
        # then the elementwise streaming pass of copy_bandwidth over the same bytes, whose
        # traced duration is the device's streaming rate
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        for _ in range(5):
            torch.neg(x, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4,
                          "launches": 5, "streaming_passes": 5}), flush=True)
        return

    from paper_1710_09541_amd import lbm
    lbm.load()

    cs, desc = workload(args.workload)
    nodes = sum(c["nx"] * c["ny"] for c in cs)
    batch = len(cs) > 1
    single = len(cs) == 1 and cs[0].get("name") == "spinodal"
    log("workload %s, %d instance(s), %d nodes, storage %s" % (args.workload, len(cs), nodes,
                                                              args.storage))
    cpu_steps = args.cpu_steps if args.cpu_steps is not None else (40 if batch else 1500)
    variants = args.variants if args.variants is not None else "f64,f16"

    base = None
    ref = None
    batch_refs = None
    batch_masks = None
    if not args.no_cpu_baseline and single:
        base, ref = cpu_baseline(cs[0], cpu_steps)
        log("cpu baseline %.2f MLUPS (%s)" % (base["value"], base["sample"]))
    elif not args.no_cpu_baseline and batch:
        base, batch_refs = batch_cpu_baseline(cs, cpu_steps)
        log("cpu baseline %.2f MLUPS on %d threads, %.2f MLUPS on 1 thread (%s)"
            % (base["value"], base["cores"], base["value_1_thread"], base["sample"]))

    results = {}
    pois_ref = {}
    others = [] if variants in ("", "none") else variants.split(",")
    for st in [args.storage] + [v for v in others if v and v != args.storage]:
        r = measure(cs, st, args.steps, args.warmup, args.kernel, args.tile_rows,
                    final_stats=single, stores=args.stores, grid=args.grid, deal=deal)
        log("%s: %.1f MLUPS, %.4f ms/step, %.0f GB/s algorithmic (%d rows, %s stores, %s grid, "
            "tile order: %s, deal: %s)" % (st, r["mlups"], r["ms_per_step"], r["achieved_gbs"],
                                          r["tile_rows"], r["stores"], r["grid"], r["tile_order"],
                                          r["deal"]))
        if ref is not None:
            r["accuracy_vs_oracle"] = spinodal_accuracy(cs[0], st, cpu_steps + 1, ref)
            log("%s: accuracy %s" % (st, json.dumps(r["accuracy_vs_oracle"])))
        if batch_refs is not None:
            if batch_masks is None:
                from tests.parity import drop_interior_mask
                batch_masks = {k: drop_interior_mask(cs[k], cpu_steps + 1) for k in batch_refs}
            r["accuracy_vs_oracle"] = batch_accuracy(cs, st, cpu_steps + 1, batch_refs, r,
                                                     batch_masks)
            log("%s: per-instance accuracy %s" % (st, json.dumps(r["accuracy_vs_oracle"])))
        if not args.no_cpu_baseline:
            r["parity_vs_oracle"] = poiseuille_parity(st, pois_ref)
            log("%s: parity %s" % (st, json.dumps(r["parity_vs_oracle"])))
        results[st] = r

    # end of the timed runs: L of each format against the FP64 format's (which repeats the
    # oracle's arithmetic), over the whole timed horizon
    if "f64" in results and "end_of_run" in results["f64"]:
        L64 = results["f64"]["end_of_run"]["L"]
        for st, r in results.items():
            if "end_of_run" in r:
                r["end_of_run"]["L_rel_to_f64"] = abs(r["end_of_run"]["L"] / L64 - 1)
                log("%s: after %d steps L %.4f (rel. to FP64 %.2e), sum phi drift %.2e"
                    % (st, r["end_of_run"]["steps"], r["end_of_run"]["L"],
                       r["end_of_run"]["L_rel_to_f64"], r["end_of_run"]["sum_phi_drift"]))

    extra = {} if args.no_extra else extra_workloads(args, skip=args.workload)

    main_r = results[args.storage]
    # host to host: not the measured value (inputs are resident in HBM there), reported beside it
    trip = ([] if args.no_round_trip else
            [host_round_trip(cs, args.storage, n, main_r) for n in (1, args.steps)])
    for t in trip:
        log("host round trip, %d steps: init %.1f ms, steps %.1f ms, moments %.1f ms: %.1f MLUPS"
            % (t["steps"], t["init_ms"], t["steps_ms"], t["moments_ms"], t["mlups"]))
    kname = {1: "k_step (fused)", 2: "k_phi_plane + k_step (split)"}[main_r["kernel"]]
    qf = cs[0].get("f_lattice", 9)
    per_launch_s = main_r["ms_per_step"] / 1e3
    m_bytes = method_bytes(args.storage, qf) * nodes
    achieved = m_bytes / per_launch_s / 1e9
    copy_gbs = copy_bandwidth()
    log("device copy: %.0f GB/s; the step reaches %.1f %% of it" % (copy_gbs, 100 * achieved / copy_gbs))
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
        "config": {"workload": desc, "storage": args.storage, "instances": len(cs),
                   "nodes": nodes, "kernel": kname, "tile_rows": main_r["tile_rows"],
                   "stores": main_r["stores"], "grid": main_r["grid"],
                   "tile_order": main_r["tile_order"],
                   "narrow_tiles": main_r["narrow_tiles"], "deal": main_r["deal"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic_from_profile(args.workload, args.storage),
                     "kernel": kname,
                     "alg_bytes_per_lu": method_bytes(args.storage, qf),
                     "alg_bytes_per_launch": m_bytes,
                     "design_bytes_per_lu": main_r["alg_bytes_per_lu"],
                     "design_frac": round(main_r["frac_hbm_peak"], 4),
                     "launch_us": round(per_launch_s * 1e6, 3),
                     "copy_gbs": round(copy_gbs, 1),
                     "frac_of_copy": round(achieved / copy_gbs, 4)},
        "cpu_baseline": base,
        "host_round_trip": trip,
        "variants": results,
        "extra": extra,
        "kernel_source_sha256": kernel_source_hash(),
        "library_build_id": lbm.build_id(),
    }
    print(json.dumps(out), flush=True)


def extra_workloads(args, skip):
    """Every other workload, timed in its formats (see the module docstring)."""
    from paper_1710_09541_amd import cases
    extra = {}
    if skip != "spinodal1024":
        sp, _ = workload("spinodal1024")
        res = {}
        for st in ("f32", "f64", "f16"):
            r = measure(sp, st, max(args.steps, 2000), args.warmup, final_stats=True)
            res[st] = r
            extra["spinodal1024_" + st] = r
            log("spinodal 1024^2 %s: %.1f MLUPS, %.0f GB/s design bytes" % (st, r["mlups"],
                                                                           r["achieved_gbs"]))
        L64 = res["f64"]["end_of_run"]["L"]
        for r in res.values():
            r["end_of_run"]["L_rel_to_f64"] = abs(r["end_of_run"]["L"] / L64 - 1)
        del sp
    big, bdesc = workload("spinodal4096")
    for st in ("f32", "f64", "f16"):
        r = measure(big, st, 1000, 20)
        extra["spinodal4096_" + st] = r
        log("4096^2 %s: %.1f MLUPS, %.0f GB/s design bytes (%s stores, tile order: %s)"
            % (st, r["mlups"], r["achieved_gbs"], r["stores"], r["tile_order"]))
    del big
    # the static drop at 4096^2 (R = 1024): a single grid far above the last-level cache
    drop = [cases.static_drop(4096, 4096, R=1024.0)]
    for st in ("f32", "f64", "f16"):
        r = measure(drop, st, 300, 20)
        extra["static_drop4096_" + st] = r
        log("static drop 4096^2 %s: %.1f MLUPS, %.0f GB/s design bytes (%s stores, tile order: "
            "%s)" % (st, r["mlups"], r["achieved_gbs"], r["stores"], r["tile_order"]))
    del drop
    n_short = max(args.steps, 2000) // 4
    q5, _ = workload("spinodal1024_d2q5")
    for st in ("f32", "f64", "f16"):
        r = measure(q5, st, n_short, args.warmup)
        extra["spinodal1024_d2q5_" + st] = r
        log("1024^2 D2Q5 %s: %.1f MLUPS, %.0f GB/s design bytes" % (st, r["mlups"],
                                                                    r["achieved_gbs"]))
    # the normal of Eq. 29 (local non-equilibrium scheme) instead of the isotropic stencil's
    q29, _ = workload("spinodal1024_eq29")
    for st in ("f32", "f64", "f16"):
        r = measure(q29, st, n_short, args.warmup)
        extra["spinodal1024_eq29_" + st] = r
        log("1024^2 Eq. 29 %s: %.1f MLUPS, %.0f GB/s design bytes" % (st, r["mlups"],
                                                                      r["achieved_gbs"]))
    # the inverse-linear viscosity law of Eq. 25
    qnu, _ = workload("spinodal1024_nu_inverse")
    r = measure(qnu, "f32", n_short, args.warmup)
    extra["spinodal1024_nu_inverse_f32"] = r
    log("1024^2 Eq. 25 f32: %.1f MLUPS, %.0f GB/s design bytes" % (r["mlups"], r["achieved_gbs"]))
    small = [("static_drop64_f64", [cases.static_drop()], "f64", 2000),
             ("poiseuille16x512_f32", [cases.layered_poiseuille()], "f32", 5000),
             ("impact2048_f32", workload("impact2048")[0], "f32", 2000),
             ("impact2048_f16", workload("impact2048")[0], "f16", 2000)]
    for name, wcs, st, n in small:
        r = measure(wcs, st, n, 50)
        extra[name] = r
        log("%s: %.1f MLUPS, %.4f ms/step" % (name, r["mlups"], r["ms_per_step"]))
    if skip != "batch256":
        bcs, bdesc = workload("batch256")
        for st in ("f32", "f64"):
            r = measure(bcs, st, 200, 10)
            r["workload"] = bdesc
            extra["batch256_" + st] = r
            log("batch256 %s: %.1f MLUPS over %d nodes, %.0f GB/s design bytes"
                % (st, r["mlups"], r["nodes"], r["achieved_gbs"]))
    return extra


if __name__ == "__main__":
    main()
