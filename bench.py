"""Throughput of the plain leap-frog stepper on the 4M-triangle periodic FP32 workload.

Workload: periodic unit square, Delaunay triangulation of a 1415 x 1415 lattice jittered by
+-0.25 h (4,004,450 triangles, 6,006,675 edges), Gaussian-enveloped plane wave of 20 cells
per wavelength at a seeded random angle, dt = 0.5 * 2/omega_max (power iteration), FP32 fields
with FP64-derived coefficients.  One step = one edge half-step and one triangle half-step
over the whole mesh (10,011,125 cell-updates).

Prints one JSON line: cell-updates/s, ms per step, the roofline of the dominant kernel
(algorithmic bytes per launch / average launch time from HIP events in the timed region),
and the CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import re
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N_LATTICE = 1415


def parse(argv=None):
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10000)
    p.add_argument("--warmup", type=int, default=500)
    p.add_argument("--n", type=int, default=N_LATTICE, help="lattice size (default 1415)")
    p.add_argument("--order", default="morton", choices=["none", "random", "morton", "rcm"])
    p.add_argument("--fusion", type=int, default=0, help="steps per launch (0 = library default)")
    p.add_argument("--tile", type=int, default=0, help="fused tile size in triangles (0 = default)")
    p.add_argument("--prec", default="f32", choices=["f32", "f64"])
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--cpu-steps", type=int, default=0, help="oracle sample steps (0 = auto)")
    p.add_argument("--workload", default="torus1415",
                   choices=["torus1415", "plasma2830", "batch256", "learned", "modes70x101", "spectrum70x101",
                            "relax", "open1415", "tet100"],
                   help="torus1415 (the reported line), plasma2830 (16M triangles with a plasma "
                        "particle and a line source), batch256 (256 uneven meshes), learned "
                        "(train and evaluate the learned edge scale) or modes70x101 (the 128 "
                        "lowest modes of the 70 x 101 resonator of Fig. 4; --steps timed "
                        "solves, at most 20), spectrum70x101 (every mode of that resonator, one "
                        "solve), open1415 (the 1415 x 1415 box tied to a 16-layer PML frame), tet100 (12M "
                        "tetrahedra of a 100^3 BCC box, E on edges and B on faces) or relax "
                        "(jello relaxation of the 45 x 45 cavity and "
                        "the 1415 x 1415 torus: omega_max and so dt before and after)")
    p.add_argument("--relax-rounds", type=int, default=8)
    p.add_argument("--relax-iters", type=int, default=100)
    p.add_argument("--relax-step", type=float, default=0.05)
    p.add_argument("--train-meshes", type=int, default=64)
    p.add_argument("--train-n", type=int, default=316,
                   help="learned: training lattice size (316: 199,712 triangles per mesh)")
    p.add_argument("--eval-meshes", type=int, default=16)
    p.add_argument("--eval-n", type=int, default=707)
    p.add_argument("--iters", type=int, default=200)
    p.add_argument("--lr", type=float, default=3e-3)
    p.add_argument("--batch-meshes", type=int, default=4,
                   help="learned: meshes per Adam step (0: every (mesh, wave) pair each step)")
    p.add_argument("--batch-waves", type=int, default=4, help="learned: waves per mesh per Adam step")
    p.add_argument("--val-pairs", type=int, default=48,
                   help="learned: fixed (mesh, wave) pairs for the reported loss and the "
                        "constant-scale ablation (0: every pair)")
    p.add_argument("--graph", type=int, default=8, help="fused launches per HIP graph (0 = eager)")
    p.add_argument("--tune", action="store_true", help="batch256: run the autotuner first")
    p.add_argument("--modes-no-scale", action="store_true",
                   help="modes70x101: leave out the 1.6M-triangle apply measurement")
    p.add_argument("--modes-degree", type=int, default=0,
                   help="modes70x101: largest filter degree per iteration (0 = library default)")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain 512 MiB device copy (for counter calibration)")
    p.add_argument("--fusion-sweep", default="",
                   help="torus1415 or plasma2830: comma-separated KxT (steps per launch x tile triangles) "
                        "configurations of the fused kernel, each timed on the same mesh (graphs "
                        "of 8 launches, median of 5 regions of about --steps steps); one JSON "
                        "line per configuration, then exit")
    p.add_argument("--copy-sweep", action="store_true",
                   help="only print device copy rates against buffer size (torch copy and the "
                        "library's non-temporal probe), from 16 MiB to 4 GiB per buffer")
    p.add_argument("--traffic-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR",
                                                          "COPY_WRITE_DIR"),
                   help="turn rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE csv outputs of this bench "
                        "and of --copy-calibration into the stored traffic figure of k_fused "
                        "for --workload, then exit (no GPU use)")
    return p.parse_args(argv)


def traffic_file(workload, K):
    return os.path.join(ROOT, "profiles", f"traffic_k_fused_{workload}_k{K}_f32.json")


COPY_BYTES = 128 * 1024 * 1024 * 4     # --copy-calibration: bytes read and written per copy
# the fused kernel and its device-side contract (tile records, XCD mapping)
KERNEL_SOURCES = ["paper_1812_01448_amd/csrc/fused.hip", "paper_1812_01448_amd/csrc/tile.hpp"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, config, workload="torus1415"):
    """HBM bytes per launch from the committed counter summary of this depth, if it still
    applies (same kernel sources and launch configuration)."""
    try:
        with open(traffic_file(workload, config["steps_per_launch"])) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel") != kernel or t.get("source_hash") != kernel_source_hash():
        return None
    if any(t.get("config", {}).get(k) != v for k, v in config.items()):
        return None
    return t.get("bytes_per_launch")


def copy_calibration():
    import torch
    x = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": x.numel() * 4,
                      "launches": 5}), flush=True)


def copy_sweep():
    """Copy rate (bytes read + written per second) against buffer size. torch's copy uses
    ordinary loads and stores, whose lines the 256 MB Infinity Cache can keep between copies
    while source and destination fit in it; the library's probe uses non-temporal loads and
    stores. One JSON line per size."""
    import torch
    import paper_1812_01448_amd as ty
    for mib in (16, 32, 64, 96, 128, 192, 256, 512, 1024, 4096):
        nbytes = mib << 20
        x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        reps = max(20, int(2e9 // nbytes))
        for _ in range(5):
            y.copy_(x)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            y.copy_(x)
        b.record()
        b.synchronize()
        us = a.elapsed_time(b) * 1e3 / reps
        del x, y
        torch.cuda.empty_cache()
        nt = ty.copy_bandwidth(nbytes, min(reps, 1000))
        print(json.dumps({"mib_per_buffer": mib, "torch_copy_GBs": round(2 * nbytes / us / 1e3, 1),
                          "torch_copy_us": round(us, 2), "nt_probe_GBs": round(nt, 1),
                          "reps": reps}), flush=True)


def _pmc_values(folder, counter):
    """{kernel name: [counter value per dispatch]} from a rocprofv3 --pmc csv folder."""
    import csv
    import glob
    out = {}
    for path in glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            for row in csv.DictReader(f):
                if row["Counter_Name"] == counter:
                    out.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
    return out


def traffic_summary(args):
    """Scaled HBM bytes per fused launch from FETCH_SIZE / WRITE_SIZE (KiB per dispatch).

    Each counter is scaled by what it reads for the calibration copy (COPY_BYTES read and
    written per dispatch). A fused launch is one dispatch of k_fused per tile class, so its
    traffic is the sum over the k_fused kernels of their median per-dispatch values."""
    fetch_dir, write_dir, cfetch_dir, cwrite_dir = args.traffic_summary

    def copy_kib(folder, counter):
        vals = sorted(v for k, vs in _pmc_values(folder, counter).items() if "copyBuffer" in k
                      for v in vs)
        big = vals[-5:]                       # the five 512 MiB copies
        return float(np.median(big))

    cf, cw = copy_kib(cfetch_dir, "FETCH_SIZE"), copy_kib(cwrite_dir, "WRITE_SIZE")
    fetch_scale, write_scale = COPY_BYTES / 1024 / cf, COPY_BYTES / 1024 / cw
    per = {}
    for counter, folder in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        for name, vals in _pmc_values(folder, counter).items():
            if "k_fused" in name:
                per.setdefault(name, {})[counter] = (float(np.median(vals)), len(vals),
                                                     float(min(vals)), float(max(vals)))
    fetch = sum(v["FETCH_SIZE"][0] for v in per.values())
    write = sum(v["WRITE_SIZE"][0] for v in per.values())
    total = fetch * 1024 * fetch_scale + write * 1024 * write_scale
    if args.fusion < 2 or args.tile <= 0:
        raise SystemExit("--traffic-summary needs the --fusion and --tile the counters were taken with")
    cfg = {"triangles": {"torus1415": 4004450, "plasma2830": 16017830}[args.workload],
           "steps_per_launch": args.fusion, "tile_tris": args.tile, "prec": "f32", "order": "morton"}
    out = {"kernel": "k_fused", "workload": args.workload, "source_hash": kernel_source_hash(),
           "config": cfg, "copy_fetch_kib": cf, "copy_write_kib": cw,
           "fetch_scale": round(fetch_scale, 6), "write_scale": round(write_scale, 6),
           "per_kernel": {re.search(r"k_fused<[^>]*>", k).group(0): v for k, v in per.items()},
           "fetch_kib_per_launch_raw": fetch, "write_kib_per_launch_raw": write,
           "bytes_per_launch": int(round(total))}
    with open(traffic_file(args.workload, args.fusion), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)


def measure_copy_bandwidth():
    """Achievable device bandwidth (bytes read + written per second): the library's 16-byte
    non-temporal copy probe over 1 GiB, the reference beside the published HBM peak."""
    import paper_1812_01448_amd as ty
    return round(ty.copy_bandwidth(1 << 30, 10), 1)


def measure_torch_copy_bandwidth():
    """Device-to-device copy rate of torch's copy_ on a 512 MiB buffer (the kernel the
    counter calibration uses)."""
    import torch
    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(10):
        y.copy_(x)
    b.record()
    b.synchronize()
    gbs = 2 * COPY_BYTES * 10 / (a.elapsed_time(b) * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return round(gbs, 1)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def launch_stats(prof, graph_launches):
    """Average launch duration of the stepping kernel from the HIP-event totals of a timed
    region: whole graph replays (each holding `graph_launches` launches) plus the launches
    made outside a graph (a remainder shorter than one graph span).  Returns (kind, launches,
    avg_ms) with kind "fused" or "edge+tri" (one launch each per half-step), or None."""
    if not prof:
        return None
    g = prof.get("graph", {"count": 0, "total_ms": 0.0})
    if "fused" in prof or ("graph" in prof and "edge" not in prof):
        f = prof.get("fused", {"count": 0, "total_ms": 0.0})
        n = g["count"] * graph_launches + f["count"]
        return ("fused", n, (g["total_ms"] + f["total_ms"]) / n) if n else None
    e = prof.get("edge", {"count": 0, "total_ms": 0.0})
    t = prof.get("tri", {"count": 0, "total_ms": 0.0})
    steps = g["count"] * graph_launches + e["count"]
    return ("edge+tri", steps, (g["total_ms"] + e["total_ms"] + t["total_ms"]) / steps) \
        if steps else None


def region_depth(steps, default_k, short=100):
    """Fusion depth for a timed region of `steps` steps: the library default, except in a
    region shorter than `short` launches where the default would leave single steps over;
    there the deepest depth up to the default that splits the region into an even number of
    whole launches (so the region runs from graphs alone), if there is one."""
    if steps >= short * default_k or steps % (2 * default_k) == 0:
        return default_k
    for k in range(default_k, 1, -1):
        if steps % (2 * k) == 0:
            return k
    return default_k


def graph_size(steps, K, wanted):
    """Launches per graph: at most `wanted`, even, and no longer than the timed region, so
    that a short region still runs from graphs (0 when not even two launches fit)."""
    fit = steps // max(K, 1)
    g = min(wanted, fit - fit % 2)
    return g if g >= 2 else 0


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.copy_sweep:
        copy_sweep()
        return
    if args.fusion_sweep:
        fusion_sweep(args)
        return
    if args.traffic_summary:
        traffic_summary(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1 (the method "
                                   "shards by contiguous Morton ranges with halo exchange, "
                                   "which is not built)",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    run = {"batch256": bench_batch, "learned": bench_learned, "plasma2830": bench_plasma,
           "modes70x101": bench_modes, "spectrum70x101": bench_spectrum, "torus1415": bench_torus,
           "relax": bench_relax, "open1415": bench_open, "tet100": bench_tet}[args.workload]
    out = run(args)
    print(json.dumps(out), flush=True)


def single_step_rate(sim, bytes_step, steps=2000):
    """One launch per half-step (k_edge then k_tri), replayed from graphs of 8 steps: HIP-event
    time per step against the per-step algorithmic bytes."""
    sim.set_fusion(1, 0)
    sim.set_graph(8)
    sim.step(400)
    sim.sync()
    sim.set_profiling(True, kinds=["graph"])
    sim.step(steps)
    sim.sync()
    prof = sim.kernel_times()
    sim.set_profiling(False)
    st = launch_stats(prof, 8)
    ms = st[2]
    ach = bytes_step / (ms * 1e-3) / 1e9
    return {"kernels": "k_edge + k_tri, one launch per half-step, graphs of 8 steps",
            "ms_per_step": round(ms, 6), "achieved": round(ach, 1),
            "frac": round(ach / HBM_PEAK_GBS, 4), "steps_timed": st[1]}


def fusion_sweep(args):
    """Steps per launch and tile size of the fused kernel on the torus1415 (or plasma2830) mesh
    and start: for
    each configuration, graphs of 8 launches, a warm-up of 4 graph spans, then the median (and
    minimum) wall time per step over 5 regions of whole graph spans (about --steps steps)."""
    import paper_1812_01448_amd as ty
    from meshgen import lattice_mesh, periodic_wavevector, plane_wave_packet, random_angle, plasma_workload
    plasma = args.workload == "plasma2830"
    if plasma:
        w = plasma_workload()
        xy, tri, n = w["xy"], w["tri"], w["n"]
    else:
        n = args.n
        xy, tri = lattice_mesh(n, 0.25, 1, periodic=True)
    mesh = ty.Mesh(xy, tri, periodic=True)
    mesh.reorder(args.order, 0)
    lam, _, _ = mesh.cfl(max_iter=20000, rtol=1e-12, seed=0)
    dt = 0.5 * 2.0 / np.sqrt(lam)
    view = mesh.view()
    k, _, _ = periodic_wavevector(random_angle(2), 20.0, 1.0 / n)
    B0, E0 = plane_wave_packet(view["O"], view["C"], view["evec"] / view["elen"][:, None], k, dt,
                               sigma=0.1, center=(0.5, 0.5))
    sim = ty.Sim(mesh, dt, args.prec)
    sim.set_state("E", E0)
    sim.set_state("B", B0)
    if plasma:                  # the plasma particle and the line source: eager fused launches
        sim.set_media(w["wp2_tri"], w["nu"])
        sim.set_source(w["src_pairs"], w["src_weights"], w["src_omega"], w["src_cycles"])
    log(f"fusion sweep on {mesh.nt} triangles")
    for item in args.fusion_sweep.split(","):
        K, tile = (int(v) for v in item.lower().split("x"))
        sim.set_fusion(K, tile)
        sim.set_graph(8)
        span = 8 * K
        steps = span * max(1, round(args.steps / span))
        sim.step(4 * span)
        sim.sync()
        per = []
        for _ in range(5):
            t0 = time.perf_counter()
            sim.step(steps)
            sim.sync()
            per.append((time.perf_counter() - t0) / steps * 1e6)
        fi = sim.fusion_info()
        print(json.dumps({"workload": args.workload, "steps_per_launch": fi["steps_per_launch"], "tile": fi["tile"],
                          "us_per_step": round(float(np.median(per)), 3), "min_us_per_step": round(min(per), 3),
                          "cell_updates_per_s": round((mesh.ne + mesh.nt) / (np.median(per) * 1e-6), -8),
                          "tiles": fi["tiles"], "halo_ratio_tris": round(fi["local_tris"] / mesh.nt, 3),
                          "halo_ratio_edges": round(fi["local_edges"] / mesh.ne, 3), "steps_timed": steps}),
              flush=True)
    d = sim.diagnostics()
    if d["nonfinite"]:
        raise SystemExit("non-finite fields after the sweep")


def bench_torus(args, with_extras=True):
    """The reported line: the plain FP32 step on the 4M-triangle periodic mesh."""
    import torch
    import paper_1812_01448_amd as ty
    from meshgen import lattice_mesh, periodic_wavevector, plane_wave_packet, random_angle

    n = args.n
    t0 = time.time()
    xy, tri = lattice_mesh(n, 0.25, 1, periodic=True)
    log(f"mesh {n}x{n}: {len(tri)} triangles ({time.time() - t0:.1f} s)")
    mesh = ty.Mesh(xy, tri, periodic=True)
    mesh.reorder(args.order, 0)
    lam, iters, ok = mesh.cfl(max_iter=20000, rtol=1e-12, seed=0)
    dt = 0.5 * 2.0 / np.sqrt(lam)
    log(f"omega_max {np.sqrt(lam):.6e} ({iters} iterations, converged={ok}), dt {dt:.6e}")
    view = mesh.view()
    theta = random_angle(2)
    k, _, _ = periodic_wavevector(theta, 20.0, 1.0 / n)
    B0, E0 = plane_wave_packet(view["O"], view["C"], view["evec"] / view["elen"][:, None], k, dt,
                               sigma=0.1, center=(0.5, 0.5))

    torch.cuda.init()
    stream = torch.cuda.current_stream()
    sim = ty.Sim(mesh, dt, args.prec, stream=stream.cuda_stream)
    sim.set_state("E", E0)
    sim.set_state("B", B0)
    sim.set_fusion(args.fusion, args.tile)
    if args.fusion == 0:
        k_def = sim.fusion_info()["steps_per_launch"]
        k_run = region_depth(args.steps, k_def)
        if k_run != k_def:
            log(f"{args.steps} timed steps: {k_run} steps per launch (default {k_def}) so that "
                f"the region runs from whole graph spans")
            sim.set_fusion(k_run, args.tile)
    ne, nt = mesh.ne, mesh.nt
    cells = ne + nt

    sim.step(max(args.warmup, 1))
    sim.sync()
    fuse = sim.fusion_info()
    K = fuse["steps_per_launch"]
    glaunch = graph_size(args.steps, K, args.graph) if args.graph > 0 else 0
    sim.set_graph(glaunch)
    if glaunch:                                   # capture outside the timed region
        sim.step(K * glaunch)
    torch.cuda.synchronize()
    # HIP events bracket every graph replay and every launch made outside a graph inside the
    # timed region, on the simulation's stream
    sim.set_profiling(True, kinds=["graph", "fused"] if K > 1 else ["graph", "edge", "tri"])
    t_start = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof = sim.kernel_times()
    sim.set_profiling(False)
    diag = sim.diagnostics()
    log(f"timed {args.steps} steps in {elapsed:.4f} s; energy {diag['energy']:.6e} "
        f"nonfinite={diag['nonfinite']}; launches {prof}")

    ms_per_step = elapsed * 1e3 / args.steps
    value = cells * args.steps / elapsed
    esz = 4 if args.prec == "f32" else 8
    # algorithmic bytes: every cell read and written once, its coefficient and indices read
    # once, compulsory gathers counted once (64 B per triangle in FP32, 25.6 B per cell)
    bytes_edge = 3 * esz * ne + 8 * ne + esz * nt          # Et r/w + cE, R/L, B gather
    bytes_tri = 3 * esz * nt + 12 * nt + esz * ne           # B r/w + nB, A, Et gather
    step_bytes = bytes_edge + bytes_tri
    st = launch_stats(prof, glaunch)
    roofline = {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    if st is not None:
        kind, launches, avg_ms = st
        # a K-step fused launch must still move every cell once: its compulsory bytes are one
        # step's; the K - 1 further steps run from the tile held on chip
        per_launch = step_bytes
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        roofline.update({
            "kernel": "k_fused" if kind == "fused" else "k_edge+k_tri",
            "achieved": round(achieved, 1), "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None, "avg_launch_ms": round(avg_ms, 6), "launches_timed": launches,
            "steps_per_launch": K if kind == "fused" else 1,
            "timed_with": f"HIP events on the simulation stream: {prof.get('graph', {}).get('count', 0)} "
                          f"graph replays of {glaunch} launches, "
                          f"{prof.get('fused', prof.get('edge', {})).get('count', 0)} launches outside graphs",
            "algorithmic_bytes_per_launch": per_launch,
            "algorithmic_bytes_note": "64 B per triangle (25.6 B per cell): each cell's field read "
                                      "and written once, coefficient and indices read once, "
                                      "gathers counted once",
            "effective_GBs": round((K if kind == "fused" else 1) * step_bytes / (avg_ms * 1e-3) / 1e9, 1)})
        if kind == "fused":
            tr = measured_traffic("k_fused", {
                "triangles": nt, "steps_per_launch": K, "tile_tris": fuse["tile"],
                "prec": args.prec, "order": args.order})
            roofline["traffic"] = tr
            if tr:
                roofline["traffic_GBs"] = round(tr / (avg_ms * 1e-3) / 1e9, 1)
                roofline["traffic_frac"] = round(tr / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
            roofline["halo_ratio_tris"] = round(fuse["local_tris"] / nt, 3)
            roofline["halo_ratio_edges"] = round(fuse["local_edges"] / ne, 3)
    out = {
        "metric": "cell-updates/s (edges+tris) & HBM GB/s, plain vs learned at fixed phase error",
        "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.prec, "data": "synthetic",
        "config": {"workload": f"plain FP32 periodic jittered-lattice Delaunay {n}x{n} "
                               f"(+-0.25h), plane-wave packet 20 cells/lambda, CFL 0.5",
                   "triangles": nt, "edges": ne, "cell_updates_per_step": cells,
                   "order": args.order, "steps_per_launch": K, "tile_tris": fuse["tile"],
                   "graph_launches": glaunch, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": None,
    }
    if not with_extras:
        return out
    # further runs of 1,000 steps (median beside the timed region above)
    sim.set_graph(args.graph)
    reps = []
    for _ in range(5):
        torch.cuda.synchronize()
        t_r = time.perf_counter()
        sim.step(1000)
        torch.cuda.synchronize()
        reps.append((time.perf_counter() - t_r) * 1e3 / 1000)
    out["repeats_ms_per_step"] = [round(r, 5) for r in reps]
    out["median_ms_per_step"] = round(float(np.median(reps)), 5)
    # the boundary takes and returns host buffers in canonical order: state transfer cost
    torch.cuda.synchronize()
    t_io = time.perf_counter()
    E1, B1 = sim.get_state("E"), sim.get_state("B")
    t_get = time.perf_counter() - t_io
    t_io = time.perf_counter()
    sim.set_state("E", E1)
    sim.set_state("B", B1)
    torch.cuda.synchronize()
    out["host_io_ms"] = {"get_E_B": round((t_get) * 1e3, 1),
                         "set_E_B": round((time.perf_counter() - t_io) * 1e3, 1)}
    roofline["single_step"] = single_step_rate(sim, step_bytes)
    roofline["copy_GBs"] = measure_copy_bandwidth()
    roofline["torch_copy_GBs"] = measure_torch_copy_bandwidth()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(xy, tri, dt, args.cpu_steps)
    return out


def bench_plasma(args):
    """16M-triangle periodic mesh with a conforming plasma particle and a soft line source.

    One step = Drude current + source on the special edges, nodal charge by continuity,
    edge half-step, triangle half-step.  The FP32 working set (about 0.9 GB) exceeds the
    256 MB Infinity Cache, so this is the HBM-bound point of the path."""
    import torch
    import paper_1812_01448_amd as ty
    from meshgen import plasma_workload, periodic_wavevector, plane_wave_packet

    n = 2830 if args.n == N_LATTICE else args.n
    t0 = time.time()
    w = plasma_workload(n)
    xy, tri = w["xy"], w["tri"]
    log(f"plasma mesh {n}x{n}: {len(tri)} triangles, {int(w['inside'].sum())} inside the "
        f"particle, {len(w['src_pairs'])} source lines ({time.time() - t0:.1f} s)")
    mesh = ty.Mesh(xy, tri, periodic=True)
    mesh.reorder(args.order, 0)
    lam, iters, ok = mesh.cfl(max_iter=20000, rtol=1e-12, seed=0)
    dt = 0.5 * 2.0 / np.sqrt(lam)
    log(f"omega_max {np.sqrt(lam):.6e} ({iters} iterations, converged={ok}), dt {dt:.6e}")
    view = mesh.view()
    k, _, _ = periodic_wavevector(0.7, 20.0, 1.0 / n)
    B0, E0 = plane_wave_packet(view["O"], view["C"], view["evec"] / view["elen"][:, None], k, dt,
                               sigma=0.1, center=(0.5, 0.5))
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    sim = ty.Sim(mesh, dt, args.prec, stream=stream.cuda_stream)
    sim.set_media(w["wp2_tri"], w["nu"])
    sim.set_source(w["src_pairs"], w["src_weights"], w["src_omega"], w["src_cycles"])
    sim.set_state("E", E0)
    sim.set_state("B", B0)
    sim.set_fusion(args.fusion, args.tile)
    sim.set_graph(args.graph)
    sim.step(args.warmup)
    sim.sync()
    fuse = sim.fusion_info()
    K = fuse["steps_per_launch"]
    torch.cuda.synchronize()
    # an untimed profiled pass names the dominant kernel; the timed region then brackets
    # only that kernel's launches with HIP events
    kinds = ["fused"] if K > 1 else ["edge", "tri", "special", "charge"]
    sim.set_profiling(True, kinds=kinds)
    sim.step(max(20, min(200, args.steps // 10)))
    sim.sync()
    prof_all = sim.kernel_times()
    sim.set_profiling(False)
    dom = max(prof_all, key=lambda kk: prof_all[kk]["total_ms"])
    torch.cuda.synchronize()
    sim.set_profiling(True, kinds=[dom])
    t1 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    prof = sim.kernel_times()
    sim.set_profiling(False)
    diag = sim.diagnostics()
    log(f"timed {args.steps} steps in {elapsed:.4f} s; nonfinite={diag['nonfinite']}")
    ne, nt, nv = mesh.ne, mesh.nt, len(xy)
    esz = 4 if args.prec == "f32" else 8
    # special edges: plasma (either side inside the particle) and source lines
    R, L = view["R"], view["L"]
    special = (w["inside"][R] > 0) | (w["inside"][L] > 0)
    en = view["edge_nodes"].astype(np.int64)
    key = en[:, 0] * nv + en[:, 1]
    sp = np.sort(w["src_pairs"].astype(np.int64), axis=1)
    special[np.searchsorted(key, sp[:, 0] * nv + sp[:, 1])] = True
    n_special = int(special.sum())
    nodes = np.unique(en[special].ravel())
    n_inc = 2 * n_special
    bytes_edge = 3 * esz * ne + 8 * ne + esz * nt
    bytes_tri = 3 * esz * nt + 12 * nt + esz * ne
    # special: slot + j r/w + two Drude coefficients + source weight; charge: node, offset,
    # Q r/w, and per incidence its edge and coefficient
    bytes_special = n_special * (4 + 5 * esz)
    bytes_charge = len(nodes) * (8 + 2 * esz) + n_inc * (4 + esz)    # plus esz per decrement read
    # compulsory bytes of one launch: a single-step kernel moves its own cells once; a fused
    # launch (plain-class tiles, special-class tiles and the charge update of its K steps)
    # must still move every cell, special edge and charge node once, its K - 1 further steps
    # running from tiles held on chip
    step_bytes = bytes_edge + bytes_tri + bytes_special + bytes_charge
    algo = {"edge": bytes_edge, "tri": bytes_tri, "special": bytes_special, "charge": bytes_charge,
            "fused": step_bytes}
    avg_ms = prof[dom]["total_ms"] / prof[dom]["count"]
    achieved = algo[dom] / (avg_ms * 1e-3) / 1e9
    cells = ne + nt
    out = {
        "metric": "cell-updates/s (edges+tris), plasma particle and line source",
        "value": cells * args.steps / elapsed, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": f"periodic jittered-lattice Delaunay {n}x{n} (+-0.25h) with a "
                               f"conforming equilateral plasma particle (omega_p 0.8, nu 0.05 "
                               f"per mesh-unit time) and a soft line source, CFL 0.5",
                   "triangles": nt, "edges": ne, "special_edges": n_special,
                   "charge_nodes": int(len(nodes)), "order": args.order,
                   "steps_per_launch": K, "tile_tris": fuse["tile"],
                   "special_tiles": fuse["special_tiles"], "tiles": fuse["tiles"],
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": prof[dom]["name"], "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("k_fused", {
                         "triangles": nt, "steps_per_launch": K, "tile_tris": fuse["tile"],
                         "prec": args.prec, "order": args.order}, "plasma2830")
                     if dom == "fused" else None,
                     "avg_launch_ms": round(avg_ms, 5), "algorithmic_bytes_per_launch": algo[dom],
                     "effective_GBs": round(step_bytes * (K if dom == "fused" else 1)
                                            / (avg_ms * 1e-3) / 1e9, 1),
                     "step_effective_GBs": round(step_bytes * args.steps / elapsed / 1e9, 1)},
        "copy_GBs": measure_copy_bandwidth(),
        "cpu_baseline": None if args.no_cpu else cpu_baseline_plasma(708),
        "kernels": {kk: {"name": v["name"], "count": v["count"],
                         "avg_ms": round(v["total_ms"] / max(1, v["count"]), 5),
                         "algorithmic_GBs": round(algo[kk] / (v["total_ms"] / max(1, v["count"])
                                                               * 1e-3) / 1e9, 1)}
                    for kk, v in prof_all.items()},
    }
    tr = out["roofline"]["traffic"]
    if tr:
        out["roofline"]["traffic_GBs"] = round(tr / (avg_ms * 1e-3) / 1e9, 1)
        out["roofline"]["traffic_frac"] = round(out["roofline"]["traffic_GBs"] / HBM_PEAK_GBS, 4)
        out["roofline"]["traffic_frac_of_copy"] = round(out["roofline"]["traffic_GBs"] / out["copy_GBs"], 4)
    return out


def bench_batch(args):
    """256 independent periodic meshes, triangle counts log-uniform in [5k, 500k]."""
    import torch
    import paper_1812_01448_amd as ty
    from meshgen import lattice_mesh, periodic_wavevector, plane_wave_packet
    from meshgen.workloads import batch_lattice_sizes

    sizes = batch_lattice_sizes(256, seed=4)
    rng = np.random.default_rng(5)
    meshes, dts, init, init_xy = [], [], [], []
    t0 = time.time()
    for k, n in enumerate(sizes):
        xy, tri = lattice_mesh(int(n), 0.25, 1000 + k, periodic=True)
        init_xy.append((xy, tri))
        m = ty.Mesh(xy, tri, True)
        m.reorder(args.order)
        lam, _, _ = m.cfl()
        dt = 0.5 * 2 / np.sqrt(lam)
        v = m.view()
        kv, _, _ = periodic_wavevector(rng.uniform(0, 2 * np.pi), rng.uniform(8, 32), 1.0 / n)
        B0, E0 = plane_wave_packet(v["O"], v["C"], v["evec"] / v["elen"][:, None], kv, dt,
                                   sigma=0.1)
        meshes.append(m)
        dts.append(dt)
        init.append((E0, B0))
    log(f"batch of {len(sizes)} meshes built in {time.time() - t0:.1f} s")
    torch.cuda.init()
    batch = ty.Batch(meshes, dts, args.prec, stream=torch.cuda.current_stream().cuda_stream)
    for k, (E0, B0) in enumerate(init):
        batch.set_state(k, "E", E0)
        batch.set_state(k, "B", B0)
    info = batch.info()
    tuned = None
    if args.tune:
        batch.set_graph(args.graph)
        tuned = batch.tune(32, progress=lambda r: log(
            f"trial {r['order']} K={r['steps_per_launch']} tile={r['tile_tris']}: "
            f"{r['ms_per_step'] * 1e3:.1f} us per step"))
        best = min(tuned, key=lambda r: r["ms_per_step"])
        log(f"tuned: {best}")
    else:
        batch.set_fusion(args.fusion, args.tile)
    sim = batch.sim()
    batch.step(max(args.warmup, 1))
    batch.sync()
    fuse = sim.fusion_info()
    K = fuse["steps_per_launch"]
    glaunch = graph_size(args.steps, K, args.graph) if args.graph > 0 else 0
    batch.set_graph(glaunch)
    if glaunch:                                   # capture outside the timed region
        batch.step(K * glaunch)
    torch.cuda.synchronize()
    sim.set_profiling(True, kinds=["graph", "fused"] if K > 1 else ["graph", "edge", "tri"])
    t1 = time.perf_counter()
    batch.step(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    prof = sim.kernel_times()
    sim.set_profiling(False)
    cells = info["triangles"] + info["edges"]
    esz = 4 if args.prec == "f32" else 8
    step_bytes = (3 * esz + 8) * info["edges"] + esz * info["triangles"] + \
                 (3 * esz + 12) * info["triangles"] + esz * info["edges"]
    kind, launches, avg_ms = launch_stats(prof, glaunch)
    # compulsory bytes per launch: every cell of the union moved once (see the torus line)
    per_launch = step_bytes
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    kf = K if kind == "fused" else 1
    out = {
        "metric": "cell-updates/s (edges+tris), batched plain method",
        "value": cells * args.steps / elapsed, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps, "higher_is_better": True, "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": "256 periodic jittered-lattice Delaunay meshes, triangle counts "
                               "log-uniform in [5k, 500k], per-mesh dt and plane wave",
                   "members": info["members"], "triangles": info["triangles"],
                   "edges": info["edges"], "steps_per_launch": K, "tile_tris": fuse["tile"],
                   "graph_launches": glaunch, "order": args.order if not tuned else "tuned"},
        "roofline": {"bound": "hbm", "kernel": "k_fused" if kind == "fused" else "k_edge+k_tri",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "avg_launch_ms": round(avg_ms, 5),
                     "launches_timed": launches, "steps_per_launch": kf,
                     "algorithmic_bytes_per_launch": per_launch, "traffic": None,
                     "effective_GBs": round(kf * step_bytes / (avg_ms * 1e-3) / 1e9, 1)},
        "tune": tuned,
        "cpu_baseline": None if args.no_cpu else cpu_baseline_batch(sizes, dts, init_xy),
    }
    return out


MODES_WANTED, MODES_BLOCK, MODES_TOL = 128, 160, 1e-11


def fig4_mesh():
    """The 70 x 101 closed resonator of Fig. 4 at h = 1: jittered (+-0.1 h) triangular lattice."""
    from meshgen import box_tri_mesh
    return box_tri_mesh(70.0, 101.0, 1.0, 0.1, 0)


def fig4_reference_curves(count, Lx=70.0, Ly=101.0, h=1.0):
    """omega^2 of the closed resonator, lowest `count`: the continuum pi^2 ((m/Lx)^2 +
    (n/Ly)^2) and the structured square Yee grid of spacing h (B at the Lx/h x Ly/h cell
    centres), (4/h^2)(sin^2(m pi h/(2 Lx)) + sin^2(n pi h/(2 Ly))), m, n >= 0."""
    nx, ny = int(round(Lx / h)), int(round(Ly / h))
    mm, nn = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    exact = np.sort((np.pi ** 2 * ((mm / Lx) ** 2 + (nn / Ly) ** 2)).ravel())[:count]
    quad = np.sort((4 / h ** 2 * (np.sin(mm * np.pi * h / (2 * Lx)) ** 2 +
                                  np.sin(nn * np.pi * h / (2 * Ly)) ** 2)).ravel())[:count]
    return exact, quad


def bench_modes(args):
    """Lowest 128 modes of the Fig. 4 resonator (FP64), solved on the device end to end."""
    import torch
    import paper_1812_01448_amd as ty

    xy, tri, Lx, Ly = fig4_mesh()
    mesh = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    mesh.reorder("morton")
    torch.cuda.init()
    stream = torch.cuda.current_stream().cuda_stream
    solves = max(1, min(args.steps, 20))
    kw = dict(block=MODES_BLOCK, degree=args.modes_degree, tol=MODES_TOL, max_iter=400,
              stream=stream)
    for _ in range(min(args.warmup, 1)):
        mesh.modes(MODES_WANTED, want_vectors=False, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [mesh.modes(MODES_WANTED, want_vectors=False, **kw) for _ in range(solves)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    r = runs[-1]
    assert all(x["converged"] for x in runs)
    nt, nb = len(tri), MODES_BLOCK
    filter_applies = r["applies"] - (r["iters"] + 1)
    avg_ms = r["filter_ms"] / filter_applies
    # per apply: read the block row and the older row, write one row (24 nb B) + tables (44 B)
    per_launch = nt * (24 * nb + 44)
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    exact, quad = fig4_reference_curves(MODES_WANTED, Lx, Ly)
    om2 = r["omega2"]
    rel = lambda a, b: float(np.max(np.abs(np.sqrt(a[1:]) / np.sqrt(b[1:]) - 1)))
    log(f"{solves} solves: {r['iters']} iterations, {r['applies']} applies, filter "
        f"{r['filter_ms']:.1f} ms of {r['total_ms']:.1f} ms")
    out = {
        "metric": "resonator modes/s (lowest 128, residual <= 1e-11 of the lambda bound)",
        "value": MODES_WANTED * solves / elapsed, "unit": "modes/s", "n_gpus": 1,
        "steps": solves, "warmup": min(args.warmup, 1), "ms_per_step": elapsed * 1e3 / solves,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "Fig. 4 closed resonator 70 x 101, h = 1, jittered (+-0.1h) "
                               "triangular-lattice Delaunay mesh", "triangles": nt,
                   "modes": MODES_WANTED, "block": nb, "max_degree": args.modes_degree,
                   "iterations": r["iters"],
                   "applies": r["applies"], "lambda_bound": r["lambda_bound"]},
        "roofline": {"bound": "hbm", "kernel": "k_modes_apply2 (two columns per work-item, even block)",
                     "timed_with": "HIP events around the filter launches",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "avg_launch_ms": round(avg_ms, 5),
                     "algorithmic_bytes_per_launch": per_launch, "traffic": None,
                     "filter_share_of_solve": round(r["filter_ms"] / r["total_ms"], 4)},
        "fig4": {"max_rel_omega_dev_unstructured_vs_analytic": rel(om2, exact),
                 "max_rel_omega_dev_structured_quad_vs_analytic": rel(quad, exact),
                 "omega_mode_1_8": [float(v) for v in np.sqrt(np.abs(om2[1:9]))],
                 "omega_analytic_1_8": [float(v) for v in np.sqrt(exact[1:9])],
                 # Fig. 4's three curves at every 8th mode index: (index, unstructured mesh,
                 # structured square Yee grid, analytic)
                 "curves_every_8th": [[k, float(np.sqrt(abs(om2[k]))), float(np.sqrt(quad[k])),
                                       float(np.sqrt(exact[k]))]
                                      for k in list(range(0, MODES_WANTED, 8)) + [MODES_WANTED - 1]]},
        "apply_at_hbm_scale": None if args.modes_no_scale else modes_apply_at_scale(ty, stream),
        "cpu_baseline": None if args.no_cpu else cpu_baseline_modes(xy, tri, Lx, Ly),
    }
    return out


def bench_open(args):
    """The 1415 x 1415 box (4.6M triangles, a jittered triangular lattice) tied to a 16-layer PML
    frame (the paper's Conclusion), FP32, two launches per step (E, then B); a centred pulse
    leaves through the frame."""
    import torch
    import paper_1812_01448_amd as ty
    from meshgen import box_tri_mesh

    t0 = time.perf_counter()
    xy, tri, Lx, Ly = box_tri_mesh(1415.0, 1415.0, 1.0, 0.1, 11)
    mesh = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    prm = ty.pml(16, 1.0, 1.0, 3.0)
    torch.cuda.init()
    stream = torch.cuda.Stream()          # a stream of our own: graphs are captured on it
    probe = ty.Open(mesh, prm, 1.0, "f32", stream.cuda_stream)
    lam, iters, ok = probe.cfl(rtol=1e-6)
    del probe
    dt = 0.5 * 2 / np.sqrt(lam)
    sim = ty.Open(mesh, prm, dt, "f32", stream.cuda_stream)
    # fused stepping of the box (K steps per launch, the frame's band in single steps) unless
    # --fusion 1; the library's FP32 default depth for it is 7
    K = 1 if args.fusion == 1 else (args.fusion or 7)
    if K > 1:
        sim.set_fusion(mesh, K, args.tile)
    log(f"open1415: mesh, frame and omega_max (lambda {lam:.4g}, {iters} iterations) in "
        f"{time.perf_counter() - t0:.1f} s; {sim.nt} triangles, {sim.nf} frame cells, {sim.ne} edges")
    g = ty.open_frame(mesh, prm)
    r2 = np.sum((g["O"] - [Lx / 2, Ly / 2]) ** 2, axis=1)
    B0 = np.where(np.arange(sim.ncell) < sim.nt, np.exp(-r2 / (2 * 40.0 ** 2)), 0.0)
    sim.set_state("BX", B0)
    steps, warmup = args.steps, args.warmup
    sim.step(warmup)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    cells = sim.ne + sim.ncell
    B = sim.get_state("BX") + sim.get_state("BY")
    left = float(np.sum(g["S"][:sim.nt] * B[:sim.nt] ** 2) / np.sum(g["S"][:sim.nt] * B0[:sim.nt] ** 2))
    step_ms = open_step_ms(sim, steps, stream, segment=K * max(1, round(256 / K)))
    ne, nc, nf, nt = sim.ne, sim.ncell, sim.nf, sim.nt
    wall = ne - sim.n_inner                     # the frame's outer edges (one cell)
    frame_inner = ne - mesh.ne - wall           # the frame's own edges between two cells
    # algorithmic bytes (FP32), each array read or written once: E update: per inner edge the
    # line integral r/w, two cell ids and one coefficient, a decay factor per inner frame edge,
    # the ids of a wall edge; B of every cell and By of every frame cell read once.  B update:
    # per triangle three signed edge ids, dt/S and B r/w; per frame cell four ids, four
    # coefficients and Bx, By r/w; every edge's line integral read once
    edge_bytes = 20 * sim.n_inner + 8 * wall + 4 * frame_inner + 4 * nc + 4 * nf
    cell_bytes = 24 * nt + 48 * nf + 4 * ne
    step_bytes = edge_bytes + cell_bytes
    # a fused group of K steps must still move every cell once: its compulsory bytes are one
    # step's (as for the torus's fused launch); effective_GBs is K times that
    achieved = step_bytes / (K * step_ms * 1e-3) / 1e9
    out = {
        "metric": "cell-updates/s (edges + cells of the mixed mesh per step)",
        "value": cells * steps / elapsed, "unit": "cell-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": elapsed * 1e3 / steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "open boundary: 1415 x 1415 box, jittered (+-0.1h) triangular-lattice Delaunay "
                               "mesh, tied to a 16-layer PML frame of width 1 (sigma_max 1, cubic grading)",
                   "triangles": sim.nt, "frame_cells": nf, "edges": ne, "dt": dt, "omega_max": float(np.sqrt(lam)),
                   "pulse_energy_left_in_box": left},
        "roofline": {"bound": "hbm",
                     "kernel": ("k_fused over the box + k_open_edge / k_open_cell over the frame's band, groups of "
                                f"{K} steps" if K > 1 else "k_open_edge + k_open_cell (one step: the E and the B update)"),
                     "timed_with": ("HIP events on the launch stream around segments of about 256 steps "
                                    + ("(whole fused groups, replayed from graphs of 8 groups)" if K > 1
                                       else "(graphs of 8 steps)")),
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "steps_per_launch": K,
                     "effective_GBs": round(step_bytes / (step_ms * 1e-3) / 1e9, 1), "avg_step_ms": round(step_ms, 5),
                     "algorithmic_bytes_per_step": step_bytes, "traffic": None,
                     "per_kernel_bytes": {"k_open_edge": edge_bytes, "k_open_cell": cell_bytes}},
        "cpu_baseline": None if args.no_cpu else cpu_baseline_open(),
    }
    return out


def bench_tet(args):
    """The three-dimensional scheme (the Conclusion: tetrahedra, E on edges, B on faces): the
    Delaunay tetrahedralisation of a jittered (+-0.05 h) BCC lattice of 100^3 cubes (12M
    tetrahedra) with conducting walls, FP32, two launches per step (E, then B); a Gaussian B
    pulse at the centre."""
    import torch
    import paper_1812_01448_amd as ty
    from meshgen.tet import bcc_box

    t0 = time.perf_counter()
    xyz, tets, L = bcc_box(100, 100, 100, 1.0, 0.05, 0)
    t1 = time.perf_counter()
    T = ty.Tet(xyz, tets)
    t2 = time.perf_counter()
    lam, iters, ok = T.cfl(max_iter=5000, rtol=1e-6)
    dt = 0.5 * 2 / np.sqrt(lam)
    log(f"tet100: {T.nt} tetrahedra, {T.ne} edges, {T.nf} faces; input {t1 - t0:.1f} s, mesh {t2 - t1:.1f} s, "
        f"omega_max {np.sqrt(lam):.4g} ({iters} iterations) {time.perf_counter() - t2:.1f} s")
    v = T.view()
    face = v["face"]
    fa = xyz[face[:, 0]]
    nrm = np.cross(xyz[face[:, 1]] - fa, xyz[face[:, 2]] - fa)
    nz = nrm[:, 2] / np.linalg.norm(nrm, axis=1)
    r2 = np.sum((xyz[face].mean(axis=1) - 50.0) ** 2, axis=1)
    B0 = np.where(v["d"] > 0, np.exp(-r2 / (2 * 8.0 ** 2)) * nz, 0.0)
    del v, face, fa, nrm, nz, r2
    torch.cuda.init()
    stream = torch.cuda.Stream()
    sim = ty.TetSim(T, dt, "f32", stream.cuda_stream)
    sim.set_state("B", B0)
    steps, warmup = args.steps, args.warmup
    sim.step(warmup)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t3
    step_ms = open_step_ms(sim, steps, stream)
    ne, nf, ninc = T.ne, T.nf, T.n_incidences
    # algorithmic bytes (FP32), each array read or written once: E update: per edge its line
    # integral r/w and coefficient, per incidence one signed face id (the slices' padding is not
    # counted), every face's h once, a width and a start per slice of 64 edges; B update: per
    # face h r/w, three edge ids and one coefficient, every edge's line integral once
    edge_bytes = 12 * ne + 4 * ninc + 4 * nf + 8 * ((ne + 63) // 64)
    face_bytes = 24 * nf + 4 * ne
    step_bytes = edge_bytes + face_bytes
    achieved = step_bytes / (step_ms * 1e-3) / 1e9
    return {
        "metric": "cell-updates/s (edges + faces of the tetrahedral mesh per step)",
        "value": (ne + nf) * steps / elapsed, "unit": "cell-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": elapsed * 1e3 / steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "tetrahedra: 100 x 100 x 100 BCC box (h = 1, jitter 0.05 h, seed 0), Delaunay, "
                               "conducting walls",
                   "tetrahedra": T.nt, "edges": ne, "faces": nf, "incidences": ninc, "dt": dt,
                   "omega_max": float(np.sqrt(lam))},
        "roofline": {"bound": "hbm", "kernel": "k_tet_edge + k_tet_face (one step: the E and the B update)",
                     "timed_with": "HIP events on the launch stream around segments of 256 steps (graphs of 8 steps)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "launches_per_step": 2,
                     "avg_step_ms": round(step_ms, 5), "algorithmic_bytes_per_step": step_bytes, "traffic": None,
                     "per_kernel_bytes": {"k_tet_edge": edge_bytes, "k_tet_face": face_bytes}},
        "cpu_baseline": None if args.no_cpu else cpu_baseline_tet(),
    }


def cpu_baseline_tet():
    """The tetrahedral oracle (numpy, FP64) stepping a 20^3 BCC box of the same recipe: a
    per-cell rate."""
    from meshgen.tet import bcc_box
    from oracle.tet import TetMesh
    xyz, tets, L = bcc_box(20, 20, 20, 1.0, 0.05, 0)
    m = TetMesh(xyz, tets, L)
    E, B = np.zeros(m.ne), np.where(m.inner_face, 1.0, 0.0)
    m.step(E, B, 0.05, 2)
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < 10.0:
        E, B = m.step(E, B, 0.05, 10)
        n += 10
    el = time.perf_counter() - t0
    # the oracle's steps are numpy element-wise operations and scatter-adds: one thread
    return {"value": (m.ne + m.nf) * n / el, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} steps of the 20^3 BCC box ({m.nt} tetrahedra), numpy element-wise on one thread",
            **host_cpu()}


def open_step_ms(sim, steps, stream, segment=256):
    """Steady-state GPU time of one open-boundary (or tetrahedral) step from HIP events on the
    launch stream: one event pair per segment of about 256 steps (whole graphs or whole fused
    groups), the stream drained between segments. A pair around thousands of queued launches
    reads short on this runtime (its first timestamp is taken late), so the region is cut into
    segments; their event times agree with the wall clock of the same segments."""
    import torch
    total, done = 0.0, 0
    while done < steps:
        n = min(segment, steps - done)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sim.step(n)
        e1.record(stream)
        e1.synchronize()
        total += e0.elapsed_time(e1)
        done += n
    return total / steps


def cpu_baseline_open():
    """The open-boundary oracle (numpy, FP64) stepping a 192 x 192 box with the same frame
    recipe: a per-cell rate."""
    import oracle
    from oracle.open import OpenMesh
    from meshgen import box_tri_mesh
    xy, tri, Lx, Ly = box_tri_mesh(192.0, 192.0, 1.0, 0.1, 11)
    om = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    m = OpenMesh(om, 16, 1.0, 1.0)
    E, Bx, By = np.zeros(m.ne), np.ones(m.ncell), np.zeros(m.ncell)
    m.step(E, Bx, By, 0.1, 2)
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < 10.0:
        E, Bx, By = m.step(E, Bx, By, 0.1, 10)
        n += 10
    el = time.perf_counter() - t0
    # the oracle's steps are numpy element-wise operations and scatter-adds: one thread
    return {"value": (m.ne + m.ncell) * n / el, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} steps of the 192 x 192 box with the frame ({m.nt} triangles, {m.nf} frame cells), "
                      f"numpy element-wise on one thread", **host_cpu()}


SPECTRUM_TOL = 1e-10


def bench_spectrum(args):
    """Every mode of the Fig. 4 resonator (16,497 eigenpairs, FP64) on the device, vectors
    included (copied to the host in canonical order)."""
    import torch
    import paper_1812_01448_amd as ty

    xy, tri, Lx, Ly = fig4_mesh()
    mesh = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    mesh.reorder("morton")
    torch.cuda.init()
    stream = torch.cuda.current_stream().cuda_stream
    nt = len(tri)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = mesh.spectrum(tol=SPECTRUM_TOL, stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert r["converged"] and r["found"] == nt
    nb = 192
    avg_ms = r["sq_ms"] / r["sq_launches"]
    # per fused (K - sigma)^2 launch: the block read once, the older block read, one block
    # written (24 nb B per row) and the row's tables (44 B); the two-ring gathers of the block
    # come from the caches and are not counted again
    per_launch = nt * (24 * nb + 44)
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    om2 = r["omega2"]
    # Fig. 4's three curves against the mode index: the unstructured mesh (all n_t modes), the
    # structured square Yee grid (70 x 101 cells, 7,070 modes) and the continuum
    nq = 70 * 101
    exact, quad = fig4_reference_curves(nq, Lx, Ly)
    idx = list(range(0, nq, 256)) + [nq - 1]
    log(f"whole spectrum: {r['windows']} windows, {r['iters']} Rayleigh-Ritz steps, {r['applies']} "
        f"applies, filter {r['filter_ms']:.0f} ms of {r['total_ms']:.0f} ms")
    out = {
        "metric": "resonator modes/s (every eigenpair with its vector, residual <= 1e-10 of the "
                  "lambda bound)",
        "value": nt / elapsed, "unit": "modes/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": elapsed * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "whole spectrum of the Fig. 4 closed resonator 70 x 101, h = 1, "
                               "jittered (+-0.1h) triangular-lattice Delaunay mesh",
                   "triangles": nt, "modes": nt, "block": nb, "windows": r["windows"],
                   "rayleigh_ritz_steps": r["iters"], "applies": r["applies"],
                   "set_aside": r["below"], "retries": r["retries"],
                   "lambda_bound": r["lambda_bound"], "lambda_max": float(om2[-1]),
                   "max_residual": r["max_residual"], "min_boundary_gap": r["min_gap"]},
        "roofline": {"bound": "hbm", "kernel": "k_modes_apply_sq (fused (K - sigma)^2 block apply)",
                     "timed_with": "HIP events around the interior windows' filter passes",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "avg_launch_ms": round(avg_ms, 5),
                     "launches": r["sq_launches"], "algorithmic_bytes_per_launch": per_launch,
                     "traffic": None,
                     "filter_share_of_solve": round(r["filter_ms"] / r["total_ms"], 4)},
        "fig4_curves": {"index_every_256": idx,
                        "omega_unstructured": [float(np.sqrt(max(om2[k], 0.0))) for k in idx],
                        "omega_structured_quad": [float(np.sqrt(quad[k])) for k in idx],
                        "omega_analytic": [float(np.sqrt(exact[k])) for k in idx],
                        "omega_unstructured_top": float(np.sqrt(om2[-1]))},
        "cpu_baseline": None if args.no_cpu else cpu_baseline_spectrum(nt),
    }
    return out


def cpu_baseline_spectrum(nt_full):
    """The oracle's whole spectrum (dense library eigensolver, eigenvalues only, every host
    core) on the 40 x 58 box (5,427 triangles): the full-size solve takes minutes, so the
    sample is timed and scaled by the solver's n^3 work to the Fig. 4 size."""
    import oracle
    from meshgen import box_tri_mesh
    xy, tri, Lx, Ly = box_tri_mesh(40.0, 58.0, 1.0, 0.1, 3)
    om = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    t0 = time.perf_counter()
    om.spectrum(vectors=False)
    el = time.perf_counter() - t0
    scaled = el * (nt_full / om.nt) ** 3
    from threadpoolctl import threadpool_info
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return {"value": nt_full / scaled, "unit": "modes/s", "cores": threads, "kind": "oracle",
            "sample": f"eigenvalues (no vectors) of the 40 x 58 box, {om.nt} triangles, in {el:.1f} s, "
                      f"scaled by (n/{om.nt})^3 to {nt_full} triangles ({scaled:.0f} s)"}


def modes_apply_at_scale(ty, stream, nb=MODES_BLOCK):
    """The block apply where the block cannot stay in the caches: one filtering iteration (degree
    capped by the solver) on a 700 x 1000 resonator (1.6M triangles, block of 160, 1.64 GB per
    block); HIP-event time per application against its algorithmic bytes."""
    from meshgen import box_tri_mesh
    xy, tri, Lx, Ly = box_tri_mesh(700.0, 1000.0, 1.0, 0.1, 3)
    mesh = ty.Mesh(xy, tri, False, L=Lx, Ly=Ly)
    mesh.reorder("morton")
    r = mesh.modes(nb // 2, block=nb, degree=200, tol=1e-14, max_iter=1, want_vectors=False,
                   stream=stream)
    applies = r["applies"] - (r["iters"] + 1)
    ms = r["filter_ms"] / applies
    per = len(tri) * (24 * nb + 44)
    log(f"apply at scale: {len(tri)} triangles x {nb}: {ms * 1e3:.0f} us per application")
    return {"triangles": len(tri), "block": nb, "applications": applies,
            "avg_launch_ms": round(ms, 5), "algorithmic_bytes_per_launch": per,
            "achieved_GBs": round(per / (ms * 1e-3) / 1e9, 1),
            "frac_of_8TBs": round(per / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def cpu_baseline_modes(xy, tri, Lx, Ly):
    """The oracle's lowest 128 modes of the same mesh (library sparse shift-invert solver),
    one host thread."""
    import oracle
    from threadpoolctl import threadpool_limits
    om = oracle.OracleMesh(xy, tri, False, Lx, Ly)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        om.modes(MODES_WANTED)
        el = time.perf_counter() - t0
    return {"value": MODES_WANTED / el, "unit": "modes/s", "cores": 1, "kind": "oracle",
            "sample": f"one full solve of the same 128 modes ({el:.1f} s)"}


def cpu_baseline_batch(sizes, dts, meshes_xy, samples=8):
    """The FP64 oracle stepping 8 members of the batch (evenly spread over the sizes),
    single-threaded; rate = their cell-updates over their summed time."""
    import oracle
    order = np.argsort(sizes)
    pick = order[np.linspace(0, len(order) - 1, samples).astype(int)]
    cells, secs, desc = 0, 0.0, []
    for k in pick:
        xy, tri = meshes_xy[k]
        om = oracle.OracleMesh(xy, tri, True)
        E0 = np.zeros(om.ne)
        B0 = np.cos(2 * np.pi * om.O[:, 0])
        t1 = time.perf_counter()
        om.step(E0, B0, dts[k], 2)
        per = (time.perf_counter() - t1) / 2
        steps = int(max(2, min(2000, 1.5 / max(per, 1e-9))))
        t1 = time.perf_counter()
        om.step(E0, B0, dts[k], steps)
        secs += time.perf_counter() - t1
        cells += (om.ne + om.nt) * steps
        desc.append(f"{om.nt}x{steps}")
    log(f"oracle batch sample: {cells / secs:.3e} cell-updates/s")
    return {"value": cells / secs, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": "FP64 steps of 8 members (triangles x steps: " + ", ".join(desc) +
                      "), single-threaded plain C oracle"}


def _waves(n, cells, angles):
    from meshgen import periodic_wavevector
    return np.array([periodic_wavevector(a, r, 1.0 / n)[0] for r in cells for a in angles])


def _resolution_to_reach(r_grid, err, target):
    """Coarsest resolution r* with err(r) <= target for every r in [r*, 10] (linear
    interpolation between grid points)."""
    r_grid, err = np.asarray(r_grid, float), np.asarray(err, float)
    i10 = int(np.argmin(np.abs(r_grid - 10.0)))
    if err[i10] > target:                       # worse than plain at 10: scan finer grids
        for i in range(i10 + 1, len(r_grid)):
            if err[i] <= target:
                a, b = r_grid[i - 1], r_grid[i]
                return a + (b - a) * (err[i - 1] - target) / (err[i - 1] - err[i])
        return float(r_grid[-1])
    for i in range(i10, 0, -1):
        if err[i - 1] > target:
            a, b = r_grid[i - 1], r_grid[i]
            return b - (b - a) * (target - err[i]) / (err[i - 1] - err[i])
    return float(r_grid[0])


def bench_learned(args):
    """Train the learned edge scale on the GPU and evaluate it on held-out meshes.

    Training: periodic meshes (jitter 0.3) small enough to run inside one work-group, the
    time-stepped phase error of 12 angles x (8, 10, 16, 32) cells per wavelength.
    Evaluation: full E/B leap-frog runs on the GPU (FP32) of plane waves on held-out meshes,
    plain vs learned vs the best constant scale; the cost to reach the plain method's error
    at 10 cells per wavelength scales as (cells per wavelength)^3 / dt."""
    import torch
    import paper_1812_01448_amd as ty
    from meshgen import lattice_mesh

    angles_train = np.arange(12) * np.pi / 12
    angles_eval = np.arange(4) * np.pi / 8
    r_grid = [4.0, 5.0, 6.5, 8.0, 10.0]
    torch.cuda.init()
    t0 = time.time()
    train = []
    for k in range(args.train_meshes):
        xy, tri = lattice_mesh(args.train_n, 0.3, 100 + k, periodic=True)
        m = ty.Mesh(xy, tri, True)
        lam, _, _ = m.cfl()
        train.append((m, 0.5 * 2 / np.sqrt(lam)))
    W = _waves(args.train_n, (8, 10, 16, 32), angles_train)
    log(f"{len(train)} training meshes ({train[0][0].nt} triangles) in {time.time() - t0:.1f} s")
    learner = ty.Learner([m for m, _ in train], [d for _, d in train],
                         np.stack([W] * len(train)), phase=2.0)
    learner.init(seed=0)
    nM, nW = len(train), len(W)
    rng = np.random.default_rng(12345)
    # fixed validation pairs (spread over meshes and waves) for the reported loss and the
    # constant-scale ablation; every pair when --val-pairs is 0 or covers them all
    if 0 < args.val_pairs < nM * nW:
        val = [(int(b // nW), int(b % nW)) for b in
               np.sort(rng.choice(nM * nW, args.val_pairs, replace=False))]
    else:
        val = None
    minibatch = args.batch_meshes > 0 and args.batch_meshes * args.batch_waves < nM * nW

    def val_loss():
        learner.set_batch(val)
        lv, _, _ = learner.loss_grad(want_grad=False)
        return lv

    loss0 = val_loss()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if minibatch:
        # each Adam step: one wavelength (cycling through the four, so every pair of a batch
        # runs about as many recurrence steps and few launches carry only a straggler), then
        # batch_meshes meshes drawn without replacement and batch_waves of their 12 angles
        # each (seeded); waves are ordered angle-major, wavelength-minor
        n_cls = 4
        hist = []
        for it in range(args.iters):
            cls = it % n_cls
            ms = rng.choice(nM, min(args.batch_meshes, nM), replace=False)
            pairs = [(int(m), int(a) * n_cls + cls) for m in ms
                     for a in rng.choice(nW // n_cls, min(args.batch_waves, nW // n_cls), replace=False)]
            learner.set_batch(pairs)
            hist.append(float(learner.train(1, args.lr)[0]))
            if (it + 1) % 10 == 0:
                log(f"Adam step {it + 1}/{args.iters}: minibatch loss {hist[-1]:.4e} "
                    f"({time.perf_counter() - t1:.1f} s)")
        hist = np.array(hist)
    else:
        learner.set_batch(None)
        hist = learner.train(args.iters, args.lr)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    loss1 = val_loss()
    theta = learner.params()
    log(f"trained {args.iters} Adam steps in {train_s:.2f} s: validation loss {loss0:.4e} -> {loss1:.4e}")
    # constant-scale ablation: best single gamma for every edge on the validation pairs
    best_c, best_l = 1.0, loss0
    for c in np.arange(0.990, 1.0301, 0.002):
        th = np.zeros_like(theta)
        th[-1] = np.arctanh((c - 1.0) / 0.1)
        learner.set_params(th)
        lc, _, _ = learner.loss_grad(want_grad=False)
        if lc < best_l:
            best_c, best_l = float(c), lc
    learner.set_params(theta)
    log(f"best constant scale {best_c:.4f} (validation loss {best_l:.4e})")

    rows = []
    for k in range(args.eval_meshes):
        t_mesh = time.perf_counter()
        xy, tri = lattice_mesh(args.eval_n, 0.3, 200 + k, periodic=True)
        m = ty.Mesh(xy, tri, True)
        m.reorder("morton")
        gam = learner.gamma(m)
        w10 = _waves(args.eval_n, (10,), angles_eval)
        gate = m.gate(gam, w10, phase=2.0, prec="f32")
        const = np.full(m.ne, best_c)
        lam_c, _, _ = m.cfl(gamma=const)
        dt_c = 0.5 * 2 / np.sqrt(lam_c)
        row = {"triangles": m.nt, "accepted": bool(gate["accepted"]),
               "dt_ratio": gate["dt_learned"] / gate["dt_plain"],
               "dt_ratio_const": dt_c / gate["dt_plain"]}
        curves = {}
        use_l = gate["accepted"]
        for name, g, dt in (("plain", None, gate["dt_plain"]),
                            ("learned", gam if use_l else None,
                             gate["dt_learned"] if use_l else gate["dt_plain"]),
                            ("const", const, dt_c)):
            errs = m.phase_error_timestepped(dt, _waves(args.eval_n, r_grid, angles_eval), phase=2.0,
                                             samples=10, gamma=g, prec="f32")
            curves[name] = np.abs(np.array(errs)).reshape(len(r_grid), len(angles_eval)).mean(1)
        target = curves["plain"][r_grid.index(10.0)]
        for name in ("learned", "const"):
            rs = _resolution_to_reach(r_grid, curves[name], target)
            dtr = row["dt_ratio"] if (name == "learned" and use_l) else (
                1.0 if name == "learned" else row["dt_ratio_const"])
            row[f"r_star_{name}"] = rs
            row[f"cost_ratio_{name}"] = (10.0 / rs) ** 3 * dtr
            row[f"curve_{name}"] = [float(v) for v in curves[name]]
        row["curve_plain"] = [float(v) for v in curves["plain"]]
        row["err10_plain"] = float(target)
        row["err10_learned"] = float(curves["learned"][r_grid.index(10.0)])
        row["err10_const"] = float(curves["const"][r_grid.index(10.0)])
        rows.append(row)
        log(f"eval {k}: accepted {row['accepted']} err10 plain {row['err10_plain']:.4e} "
            f"learned {row['err10_learned']:.4e} const {row['err10_const']:.4e}; cost ratio "
            f"learned {row['cost_ratio_learned']:.3f} const {row['cost_ratio_const']:.3f} "
            f"({time.perf_counter() - t_mesh:.1f} s)")
    ratio = float(np.mean([r["cost_ratio_learned"] for r in rows]))
    step_s = train_s / max(1, args.iters)
    per_step_pairs = (min(args.batch_meshes, nM) * min(args.batch_waves, nW)) if minibatch else nM * nW
    if train[0][0].nt <= 4096:
        # LDS roofline of the training step's dominant kernel (k_ts_adjoint, one work-group per
        # mesh and wave): per leap-frog step of the B-only recurrence each triangle reads its 3
        # neighbours' x and v (complex: 12 floats) and writes its own 4, in both passes, and the
        # second pass reads 8 floats per edge for the gradient: (32 n_t + 8 n_e) x 4 B per step.
        lds_bytes = 0.0
        for m_, dt_ in train:
            for kv in W:
                nsteps = max(1, int(round(2.0 / (np.hypot(*kv) * dt_))))
                lds_bytes += nsteps * (32 * m_.nt + 8 * m_.ne) * 4.0
        lds_bytes *= per_step_pairs / (nM * nW)
        lds_peak = 256 * 128 * 2.4e9 / 1e12        # TB/s: 256 CUs x 128 B/clk x 2.4 GHz
        roofline = {"bound": "lds", "kernel": "k_ts_adjoint", "unit": "TB/s",
                    "achieved": round(lds_bytes / step_s / 1e12, 2), "peak": round(lds_peak, 1),
                    "frac": round(lds_bytes / step_s / 1e12 / lds_peak, 4),
                    "algorithmic_bytes_per_launch": lds_bytes, "avg_launch_ms": round(step_s * 1e3, 2),
                    "timed_with": "wall time of the training steps (the adjoint kernel is ~95 % of it)",
                    "peak_assumes": "128 B per clock per CU of LDS bandwidth", "traffic": None}
    else:
        # HBM roofline of the multi-work-group adjoint (k_gts_step, one launch per leap-frog
        # step of every active pair): per triangle and step it reads x, v (16 B), y, u (16 B),
        # its couplings and neighbour ids (24 B) and writes y, u, x, v (32 B); the second pass
        # adds its side words (12 B) and the accumulators of the edges it is R of (1.5 per
        # triangle, 16 B read and written): 88 B, then 124 B, per triangle and step.
        nt_, ne_ = train[0][0].nt, train[0][0].ne
        mean_steps = np.mean([[max(1, int(round(2.0 / (np.hypot(*kv) * dt_)))) for kv in W]
                              for _, dt_ in train])
        hbm_bytes = per_step_pairs * mean_steps * nt_ * (88.0 + 124.0)
        roofline = {"bound": "hbm", "kernel": "k_gts_step", "unit": "GB/s",
                    "achieved": round(hbm_bytes / step_s / 1e9, 1), "peak": HBM_PEAK_GBS,
                    "frac": round(hbm_bytes / step_s / 1e9 / HBM_PEAK_GBS, 4),
                    "algorithmic_bytes_per_launch": hbm_bytes, "avg_launch_ms": round(step_s * 1e3, 2),
                    "timed_with": "wall time of the Adam steps (both adjoint passes, the MLP kernels "
                                  "and the minibatch set-up)",
                    "per_step_pairs": per_step_pairs, "mean_recurrence_steps": float(mean_steps),
                    "traffic": None}
    cpu = None
    if not args.no_cpu:
        # the FP64 oracle's loss and gradient (time-stepped phase error with its adjoint) on a
        # sample of the training waves, scaled to one Adam step's pairs
        import oracle
        from oracle import learned as OL
        from meshgen import lattice_mesh as _lm
        xy, tri = _lm(args.train_n, 0.3, 100, periodic=True)
        om = oracle.OracleMesh(xy, tri, True)
        dt0 = train[0][1]
        # the shortest recurrence of the set: 8 cells per wavelength at 0 degrees
        sample = W[:1] if train[0][0].nt > 4096 else W[::12][:4]
        t1 = time.perf_counter()
        for kv in sample:
            OL.ts_phase_error_grad(om, np.ones(om.ne), dt0, kv, OL.ts_steps(kv, dt0))
        per_wave = (time.perf_counter() - t1) / len(sample)
        cpu = {"value": per_wave * per_step_pairs, "unit": "s per Adam step",
               "gpu_value": step_s, "cores": 1, "kind": "oracle",
               "sample": f"loss and exact gradient of {len(sample)} training wave(s) on one "
                         f"{om.nt}-triangle training mesh ({per_wave:.2f} s per wave), scaled to "
                         f"the {per_step_pairs} pairs of one Adam step; single-threaded numpy/scipy"}
        log(f"oracle training step (scaled): {cpu['value']:.1f} s vs GPU {cpu['gpu_value']:.3f} s")
    out = {
        "metric": "cell-updates to reach the plain method's phase error at 10 cells/lambda, "
                  "plain / learned",
        "value": ratio, "unit": "x", "higher_is_better": True, "n_gpus": 1, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "learned edge scale: %d training meshes of %d triangles, %d "
                               "held-out meshes of %d triangles, jitter 0.3"
                               % (len(train), train[0][0].nt, len(rows), rows[0]["triangles"]),
                   "minibatch": ("%d meshes x %d waves per Adam step, drawn at random (seeded), "
                                 "one wavelength per step in turn"
                                 % (min(args.batch_meshes, nM), min(args.batch_waves, nW)))
                   if minibatch else "every (mesh, wave) pair each Adam step",
                   "validation_pairs": len(val) if val else nM * nW,
                   "waves_train": "12 angles x (8, 10, 16, 32) cells/lambda, ~2 rad of travel",
                   "waves_eval": "4 angles x %s cells/lambda, full E/B stepping (FP32 fields, "
                                 "agrees with FP64 to 1e-8 in the error)" % r_grid,
                   "iters": args.iters, "lr": args.lr},
        "train": {"val_loss_initial": loss0, "val_loss_final": loss1, "seconds": train_s,
                  "ms_per_iter": 1e3 * train_s / max(1, args.iters),
                  "loss_history_every_50": [float(h) for h in hist[::50]]},
        "accepted": int(sum(r["accepted"] for r in rows)),
        "err10_plain": float(np.mean([r["err10_plain"] for r in rows])),
        "err10_learned": float(np.mean([r["err10_learned"] for r in rows])),
        "err10_const": float(np.mean([r["err10_const"] for r in rows])),
        "cost_ratio_const": float(np.mean([r["cost_ratio_const"] for r in rows])),
        "best_constant_scale": best_c,
        "dt_ratio": float(np.mean([r["dt_ratio"] for r in rows])),
        "r_grid": r_grid,
        "per_mesh": rows,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    return out


def cpu_baseline_plasma(n_sample):
    """The FP64 oracle on the plasma workload recipe at a smaller lattice (same particle,
    source, rates in mesh units): a per-cell rate of a smaller mesh of the same recipe, on
    one thread and on all OpenMP threads."""
    import oracle
    from meshgen import plasma_workload, periodic_wavevector, plane_wave_packet
    w = plasma_workload(n_sample)
    om = oracle.OracleMesh(w["xy"], w["tri"], True)
    dt = 0.5 * 2 / np.sqrt(om.power()[0])
    k, _, _ = periodic_wavevector(0.7, 20.0, 1.0 / n_sample)
    B0, E0 = plane_wave_packet(om.O, om.C, om.tangent, k, dt, sigma=0.1, center=(0.5, 0.5))
    wp2 = om.edge_wp2(w["wp2_tri"])
    src = (w["src_pairs"], w["src_weights"], w["src_omega"], w["src_cycles"])
    all_threads = oracle.get_threads()
    rates = {}
    for th in sorted({1, all_threads}):
        oracle.set_threads(th)
        ns, el = _timed_oracle_steps(
            om, lambda m: om.step(E0, B0, dt, m, wp2=wp2, nu=w["nu"], src=src), 6.0)
        rates[th] = ((om.ne + om.nt) * ns / el, ns)
    oracle.set_threads(all_threads)
    log(f"oracle plasma{n_sample}: {rates}")
    out = {"value": rates[all_threads][0], "unit": "cell-updates/s", "cores": all_threads,
           "kind": "oracle", "value_1_thread": rates[1][0],
           "sample": f"{rates[all_threads][1]} FP64 steps of the plasma recipe at "
                     f"{n_sample}x{n_sample} ({om.nt} triangles, particle and source; a smaller "
                     f"mesh than the benchmarked one, so a per-cell rate) on {all_threads} "
                     f"threads, {rates[1][1]} steps on one; plain C oracle"}
    out.update(host_cpu())
    return out


def bench_relax(args):
    """Jello relaxation (Section 3, Fig. 5b) of the workloads' meshes: the 45 x 45 closed cavity
    (jitter 0.2, five seeds) and the 1415 x 1415 torus (jitter 0.25).  omega_max sets the eq. 20
    step, so omega before / omega after is the factor by which the relaxed mesh needs fewer
    steps for the same simulated time."""
    import torch
    import paper_1812_01448_amd as ty
    from meshgen import lattice_mesh
    torch.cuda.init()
    stream = torch.cuda.current_stream().cuda_stream
    rows = []
    cases = [("cavity45", 45, 0.2, s, False) for s in range(5)] + [("torus1415", 1415, 0.25, 1, True)]
    for name, n, jit, seed, per in cases:
        xy, tri = lattice_mesh(n, jit, seed, periodic=per)
        m = ty.Mesh(xy, tri, per)
        t0 = time.perf_counter()
        x1, t1, om, st = m.relax(rounds=args.relax_rounds, iters=args.relax_iters, step=args.relax_step,
                                 stream=stream)
        el = time.perf_counter() - t0
        mr = ty.Mesh(x1, t1, per)
        info0, info1 = m.info(), mr.info()
        row = {"mesh": name, "seed": seed, "triangles": m.nt,
               "omega_initial": st["omega_initial"], "omega_relaxed": st["omega_best"],
               "dt_gain": st["omega_initial"] / st["omega_best"], "best_round": st["best_round"],
               "omega_rounds": [float(v) for v in om], "flips": st["flips"],
               "min_dual_ratio_initial": info0["min_dual_ratio"],
               "min_dual_ratio_relaxed": info1["min_dual_ratio"],
               "energy_initial": st["energy_initial"], "energy_final": st["energy_final"],
               "seconds": round(el, 2)}
        rows.append(row)
        log(f"{name} seed {seed}: omega_max {st['omega_initial']:.4e} -> {st['omega_best']:.4e} "
            f"(dt x{row['dt_gain']:.3f}, round {st['best_round']}), min d/|e| "
            f"{info0['min_dual_ratio']:.2e} -> {info1['min_dual_ratio']:.2e}, {st['flips']} flips, "
            f"{el:.1f} s; per round {np.array2string(om, precision=3)}")
    big = rows[-1]
    return {
        "metric": "eq. 20 time-step gain of the jello-relaxed mesh (omega_max before / after)",
        "value": big["dt_gain"], "unit": "x", "higher_is_better": True, "n_gpus": 1,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "jello relaxation: springs along edges and heights at equilateral "
                               "rest lengths, Euler steps, Lawson flips between rounds, best "
                               "iterate by omega_max; 45x45 cavity (jitter 0.2, seeds 0-4) and "
                               "1415x1415 torus (jitter 0.25)",
                   "rounds": args.relax_rounds, "iters_per_round": args.relax_iters,
                   "step": args.relax_step},
        "steps_for_1e4_plain_steps_of_time": 1e4 / big["dt_gain"],
        "cavity45_mean_dt_gain": float(np.mean([r["dt_gain"] for r in rows[:-1]])),
        "per_mesh": rows,
        "roofline": None, "cpu_baseline": None,
    }


def host_cpu():
    """CPU model, logical CPUs of the host and CPUs this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "cpus_allowed": len(os.sched_getaffinity(0))}


def _timed_oracle_steps(om, run, budget_s, steps=0):
    """(steps, seconds) of `run(steps)`: a one-step probe sizes a sample of about budget_s."""
    if steps <= 0:
        t1 = time.perf_counter()
        run(1)
        per = time.perf_counter() - t1
        steps = int(max(2, min(5000, budget_s / max(per, 1e-9))))
    t1 = time.perf_counter()
    run(steps)
    return steps, time.perf_counter() - t1


def cpu_baseline(xy, tri, dt, steps=0, budget_s=8.0):
    """The FP64 CPU oracle stepping the same mesh and start on a bounded sample of steps, on
    one thread and on all the threads OpenMP is given (the oracle's result does not depend on
    the count)."""
    import oracle
    t0 = time.time()
    om = oracle.OracleMesh(xy, tri, True)
    log(f"oracle mesh built in {time.time() - t0:.1f} s")
    from meshgen import periodic_wavevector, plane_wave_packet, random_angle
    n = int(round(np.sqrt(len(xy))))
    k, _, _ = periodic_wavevector(random_angle(2), 20.0, 1.0 / n)
    B0, E0 = plane_wave_packet(om.O, om.C, om.tangent, k, dt, sigma=0.1, center=(0.5, 0.5))
    cells = om.ne + om.nt
    all_threads = oracle.get_threads()
    rates = {}
    for th in sorted({1, all_threads}):
        oracle.set_threads(th)
        ns, el = _timed_oracle_steps(om, lambda m: om.step(E0, B0, dt, m), budget_s, steps)
        rates[th] = (cells * ns / el, ns, el)
        log(f"oracle {th} threads: {ns} steps in {el:.2f} s ({rates[th][0]:.3e} cell-updates/s)")
    oracle.set_threads(all_threads)
    rate, ns, el = rates[all_threads]
    out = {"value": rate, "unit": "cell-updates/s", "cores": all_threads, "kind": "oracle",
           "value_1_thread": rates[1][0],
           "sample": f"{ns} FP64 leap-frog steps of the same {om.nt}-triangle mesh and start on "
                     f"{all_threads} threads ({el:.1f} s), and {rates[1][1]} steps on one thread "
                     f"({rates[1][2]:.1f} s); plain C oracle, OpenMP over cells"}
    out.update(host_cpu())
    return out


if __name__ == "__main__":
    main()
