#!/usr/bin/env python3
"""Throughput of the random-network flow solve on one MI355X.

Default workload: the 512-network batch (2D sides 64-1024 and 3D sides
32-128, FBM conductances, diluted), solved together by rn_solve_batch with
the mixed-precision solver (FP32 inner CG, FP64 residual refresh, solution
and flux) to a relative true residual of 1e-8. One step = one batch. Inputs
are generated on the host, copied to HBM before the timed region and passed
by device pointer.

Prints one JSON line: value = network solves/s, the members' completion
latencies, the dominant pass kernel's roofline (floor bytes per swept node
over its device time, from HIP events the library records on the launch
stream around every launch), the plain FP64 CG comparisons (batched, one at a
time, and a Poisson-served stream against FIFO), and the CPU oracle's full
solves of a seeded sample of the members. The single-network workloads
(--workload fbm2d_2048, iid2d_128, strat3d_256) and the study workloads
(serve, aniso, fbmgen) remain available.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "network solves/s + p99 latency at 1e-8 resid vs plain FP64 CG; CG HBM GB/s"
SHAPES_CACHE = os.path.join(ROOT, "paper_1908_03301_amd", "shapes_gfx950.txt")
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "fbm2d_2048": dict(desc="2D 2048x2048, FBM ln g (H=0.7, sigma=1.5), i.i.d. occupancy 0.6, K_x and K_y",
                       make=lambda I: I.workload_fbm_2d_2048(), axes=(0, 1)),
    "iid2d_128": dict(desc="2D 128x128, ln g ~ N(0,1) i.i.d., K_x",
                      make=lambda I: I.workload_iid_2d_128(), axes=(0,)),
    "strat3d_256": dict(desc="3D 256^3 layered 1D-FBM ln g (H=0.8, sigma=2), occupancy 0.27, K_x and K_z",
                        make=lambda I: I.workload_strat_3d_256(), axes=(0, 2)),
}
MULTI = {
    "batch512": "512 independent networks in one batched launch sequence: 2D side U{64..1024} and 3D side "
                "U{32..128} (half each), FBM ln g (H~U(0.5,0.9), sigma=1), occupancy U(0.55,1) in 2D and "
                "U(0.3,1) in 3D, flow along x",
    "serve": "served request stream, Poisson arrivals at 0.7 x the measured batched saturation rate; nodes "
             "log-uniform in [1e4, 3e7], 2D/3D 50/50, FBM ln g (H=0.75, sigma=1.5), occupancy U(0.3,1), "
             "flow along x; requests cycle through a pre-generated seeded pool",
    "aniso": "permeability anisotropy study (Eq. 2, Fig. 10): 2D 512x512 FBM ln g (sigma from --sigma) with "
             "beta_x/beta_y in {1,2,4,8,16} and H in {0.75,0.35}, 16 networks each, K_x and K_y of every "
             "network in one batch",
    "fbmgen": "network generation (Eqs. 1-2, Table I's task): FBM node field by Fourier filtering, bonds and "
              "i.i.d. dilution for 2D 2048x2048 and 3D 256^3, on the GPU (random numbers resident in HBM) "
              "and with numpy on one core",
    "backbone": "backbone of the spanning cluster (rn_build_backbone, bonds resident in HBM) of the 2048^2 FBM "
                "network (occupancy 0.6), the 256^3 layered network (occupancy 0.27) and a 2048^2 RRN at "
                "p = 0.52 (Sec. VI, near p_c = 1/2), against the oracle's depth-first search on one core; "
                "then 2048^2 RRNs at p = 0.7, 0.6, 0.55, 0.52 solved (mixed, 1e-8) on the whole live set "
                "and with RN_OPT_BACKBONE",
}


def pass_bytes(dim: int, n: int, s: int, live: int) -> dict:
    """Algorithmic HBM bytes of one pass kernel launch.

    CG pass: a live node reads z, p, u and dim conductance arrays (s bytes
    each) and writes z, p, u: (dim + 6) s bytes; its Jacobi diagonal is the
    sum of the bonds it reads. One CG pass in kpend (4 for FP32, 2 for FP64)
    also reads the directions of the kpend - 1 passes before ((kpend - 1) s)
    and reads and writes the FP64 pressure (16): the figure is the average
    over kpend passes. Refresh pass: every node copies its FP64 pressure (16
    bytes) and reads its dim inner-precision bonds (s each); a live node also
    reads dim FP64 conductances and two directions and writes z, p, u:
    8 dim + 5 s bytes more.
    """
    kp = 4 if s == 4 else 2
    return {"cg": ((dim + 6) * s * kp + 16 + (kp - 1) * s) * live // kp,
            "refresh": (16 + dim * s) * n + (8 * dim + 5 * s) * live}


def cpu_info() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in ("rn_kernels.hip", "rn_device.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1908_03301_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload: str, key: str):
    """Counted HBM bytes per launch of one kernel on one workload, from the
    committed rocprofv3 counter summaries, if they were taken on the current
    kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "pass_kernel_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        e = d.get(workload, {}).get(key)
        if not e or e.get("kernel_hash") != kernel_hash():
            return None
        return {"bytes_per_launch": float(e["bytes_per_launch"])}
    except Exception:
        return None


def copy_ceiling_gbps(mib: int = 1024) -> float:
    """Device-to-device copy rate (read + write bytes / time) of a plain copy of
    MIB MiB between two fresh buffers, timed with events on the current stream:
    the practical HBM ceiling the pass kernel is compared with."""
    import torch
    nbytes = mib << 20
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(5):
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / best / 1e9


def run_solves(ctx, B, prob_by_axis, precision, tol, steps, warmup, max_iter=2_000_000, backbone=False,
               compact=False):
    lat, results = [], []
    o = B.opts(precision, tol, max_iter=max_iter, backbone=backbone, compact=compact)
    import torch
    for it in range(warmup + steps):
        for axis, pr in prob_by_axis:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = ctx.solve(pr, o)
            t1 = time.perf_counter()
            print(f"[bench] {'mixed' if precision == B.RN_MIXED else 'fp64'} axis={axis} "
                  f"{'warmup' if it < warmup else 'step'} {it}: {1e3 * (t1 - t0):.1f} ms iters={r.iters} "
                  f"refreshes={r.refreshes} launches={r.passes} status={r.status}", file=sys.stderr, flush=True)
            if it >= warmup:
                lat.append(t1 - t0)
                results.append((axis, r.as_dict()))
    return lat, results


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batch512", choices=sorted(WORKLOADS) + sorted(MULTI))
    ap.add_argument("--requests", type=int, default=160,
                    help="served stream: requests after the saturation run (batch512: 0 skips the leg)")
    ap.add_argument("--sat-requests", type=int, default=48,
                    help="served stream: requests submitted at once to measure the saturation rate")
    ap.add_argument("--pool", type=int, default=32, help="served stream: distinct networks generated for it")
    ap.add_argument("--cpu-sample", type=int, default=16, help="batch512: members the CPU oracle solves")
    ap.add_argument("--shapes", choices=("cache", "search", "builtin"), default="cache",
                    help="batch512: launch shapes from the shape cache the library wrote on an MI355X "
                         "(paper_1908_03301_amd/shapes_gfx950.txt), from rn_autotune run now (untimed), or the "
                         "built-in rules")
    ap.add_argument("--shapes-file", default=SHAPES_CACHE, help="the cache --shapes cache loads")
    ap.add_argument("--batch-size", type=int, default=512, help="batch512: networks in the batch")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--sigma", type=float, default=1.5, help="aniso: spread sigma of ln g")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 CG comparison leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-iters", type=int, default=60, help="oracle PCG iterations in the CPU sample")
    ap.add_argument("--single-axis", action="store_true", help="solve only the first flow axis (profiling)")
    ap.add_argument("--options", action="store_true",
                    help="single-network workloads: also time the mixed solve with RN_OPT_BACKBONE, RN_OPT_COMPACT "
                         "and both (extra keys; the headline stays the plain solve)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (counter calibration) and exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this solver has no multi-GPU path "
              "(independent networks would be routed to GPUs whole).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1908_03301_amd import binding as B
    from paper_1908_03301_amd import inputs as I

    if args.calibrate_copy:
        # reference dispatch for the HBM byte counters: reads and writes exactly
        # MIB MiB each (a copy between two fresh buffers, repeated 3 times)
        nbytes = args.calibrate_copy << 20
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes}), flush=True)
        return

    if args.workload in MULTI:
        run = {"batch512": batch_bench, "serve": serve_bench, "aniso": aniso_bench,
               "fbmgen": fbmgen_bench, "backbone": backbone_bench}[args.workload]
        out = run(args, B, I, np)
        print(json.dumps(out), flush=True)
        return

    wl = dict(WORKLOADS[args.workload])
    if args.single_axis:
        wl["axes"] = wl["axes"][:1]
    net = wl["make"](I)
    torch.cuda.set_device(0)
    gd = [torch.from_numpy(a).to("cuda") for a in net.g]
    torch.cuda.synchronize()
    probs = [(ax, B.problem(dim=net.dim, nx=net.nx, ny=net.ny, nz=net.nz, axis=ax, g=gd)) for ax in wl["axes"]]

    ctx = B.Context(0)
    ctx.set_stream(None)

    def leg(precision):
        lat, res = run_solves(ctx, B, probs, precision, args.tol, args.steps, args.warmup)
        for _, r in res:
            if r["status"] != 0 or not r["converged"]:
                raise SystemExit(f"solve failed: {r}")
        return lat, res

    lat_m, res_m = leg(B.RN_MIXED)
    total_m = sum(lat_m)
    solves = len(lat_m)
    value = solves / total_m

    # roofline of the pass kernel (mixed leg: FP32 inner passes and FP64 refreshes)
    # (each axis has its own live set)
    n = net.n
    n_live = res_m[0][1]["n_live"]
    pb = pass_bytes(net.dim, n, 4, n_live)
    loop_t = sum(r["t_loop_s"] for _, r in res_m)
    launches = sum(r["passes"] for _, r in res_m)
    iters = sum(r["iters"] for _, r in res_m)
    refr = sum(r["refreshes"] for _, r in res_m)
    alg_bytes = sum(r["iters"] * pass_bytes(net.dim, n, 4, r["n_live"])["cg"] +
                    r["refreshes"] * pass_bytes(net.dim, n, 4, r["n_live"])["refresh"] for _, r in res_m)
    live_iters = sum(r["n_live"] * r["iters"] for _, r in res_m)
    avg_launch_s = loop_t / max(launches, 1)
    achieved = alg_bytes / loop_t / 1e9
    tr = traffic_from_profiles(args.workload, "mixed")
    traffic = tr["bytes_per_launch"] if tr else None
    copy_gbps = copy_ceiling_gbps()
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "copy_ceiling": round(copy_gbps, 1), "frac_of_copy": round(achieved / copy_gbps, 4),
                "traffic_GBps": round(traffic / avg_launch_s / 1e9, 1) if traffic else None,
                "traffic_frac": round(traffic / avg_launch_s / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
                "kernel": f"pass{net.dim}d_kernel<float>", "avg_launch_us": round(avg_launch_s * 1e6, 2),
                "launches": launches, "cg_passes": iters, "refresh_passes": refr,
                "bytes_per_cg_pass": pb["cg"], "bytes_per_refresh_pass": pb["refresh"]}

    out = {"metric": METRIC, "value": round(value, 4), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(1e3 * total_m / args.steps, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "fp32+fp64", "data": "synthetic",
           "config": {"workload": wl["desc"], "nodes": n, "solves_per_step": len(wl["axes"]), "tol": args.tol,
                      "precision": "fp32 inner CG + fp64 refresh/solution/flux", "inputs": "resident in HBM"},
           "latency_ms": {"p50": round(1e3 * float(np.percentile(lat_m, 50)), 3),
                          "p99": round(1e3 * float(np.percentile(lat_m, 99)), 3)},
           "roofline": roofline,
           "live_node_iters_per_s": round(live_iters / loop_t, 1)}
    out["results"] = {f"K_axis{ax}": r["K"] for ax, r in res_m[: len(wl["axes"])]}
    out["iters_mixed"] = {f"axis{ax}": r["iters"] for ax, r in res_m[: len(wl["axes"])]}

    if len(probs) > 1:
        # context: every axis of the network in one rn_solve_batch, so that
        # the passes of the solves share launches (not the headline value)
        walls = []
        for it in range(args.warmup + 1):
            torch.cuda.synchronize()
            t = time.perf_counter()
            rb = ctx.solve_batch([pr for _, pr in probs], B.opts(B.RN_MIXED, args.tol))
            w = time.perf_counter() - t
            if any(r.status != 0 or not r.converged for r in rb):
                raise SystemExit("batched axes failed")
            if it >= args.warmup:
                walls.append(w)
        out["axes_batched"] = {"solves_per_s": round(len(probs) / min(walls), 4),
                               "wall_ms": round(1e3 * min(walls), 3),
                               "K": {f"axis{ax}": r.K for (ax, _), r in zip(probs, rb)}}

    if args.options:
        # the same mixed solves with the backbone and compact options (their setup included)
        variants = {}
        for name, bb, cp in (("backbone", True, False), ("compact", False, True), ("backbone_compact", True, True)):
            lat_v, res_v = run_solves(ctx, B, probs, B.RN_MIXED, args.tol, args.steps, args.warmup, backbone=bb,
                                      compact=cp)
            for _, r in res_v:
                if r["status"] != 0 or not r["converged"]:
                    raise SystemExit(f"solve failed ({name}): {r}")
            k = len(wl["axes"])
            variants[name] = {
                "solves_per_s": round(len(lat_v) / sum(lat_v), 4),
                "speedup_vs_plain": round((len(lat_v) / sum(lat_v)) / value, 3),
                "iters": {f"axis{ax}": r["iters"] for ax, r in res_v[:k]},
                "n_backbone": {f"axis{ax}": r["n_backbone"] for ax, r in res_v[:k]},
                "loop_ms": {f"axis{ax}": round(1e3 * r["t_loop_s"], 2) for ax, r in res_v[:k]},
                "K_rel_diff_vs_plain": max(abs(a[1]["K"] / b[1]["K"] - 1.0) for a, b in zip(res_v[:k], res_m[:k]))}
        out["options"] = variants

    if not args.no_fp64:
        lat_d, res_d = leg(B.RN_FP64)
        loop_d = sum(r["t_loop_s"] for _, r in res_d)
        bytes_d = sum(r["iters"] * pass_bytes(net.dim, n, 8, r["n_live"])["cg"] +
                      r["refreshes"] * pass_bytes(net.dim, n, 8, r["n_live"])["refresh"] for _, r in res_d)
        out["fp64_cg"] = {"solves_per_s": round(len(lat_d) / sum(lat_d), 4),
                          "p50_ms": round(1e3 * float(np.percentile(lat_d, 50)), 3),
                          "p99_ms": round(1e3 * float(np.percentile(lat_d, 99)), 3),
                          "iters": {f"axis{ax}": r["iters"] for ax, r in res_d[: len(wl["axes"])]},
                          "loop_GBps": round(bytes_d / loop_d / 1e9, 1),
                          "K": {f"axis{ax}": r["K"] for ax, r in res_d[: len(wl["axes"])]}}
        out["mixed_vs_fp64_speedup"] = round(value / out["fp64_cg"]["solves_per_s"], 3)
        out["mixed_K_rel_diff_vs_fp64"] = max(
            abs(a[1]["K"] / b[1]["K"] - 1.0) for a, b in zip(res_m[: len(wl["axes"])], res_d[: len(wl["axes"])]))
    ctx.close()

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(net, wl, args, res_d if not args.no_fp64 else None)
    print(json.dumps(out), flush=True)


def _gen_batch(spec):
    from paper_1908_03301_amd import inputs as I
    return I.batch_network(spec)


def _gen_aniso(job):
    from paper_1908_03301_amd import inputs as I
    spec, sigma = job
    return I.aniso_network(spec, sigma=sigma)


def _gen_stream(req):
    from paper_1908_03301_amd import inputs as I
    return I.stream_network(req)


def generate(fn, items, label):
    """Seeded networks generated in a process pool (same bytes as serial generation)."""
    from concurrent.futures import ProcessPoolExecutor
    out = [None] * len(items)
    t0 = time.time()
    workers = max(1, min(8, len(os.sched_getaffinity(0)) - 1))
    with ProcessPoolExecutor(max_workers=workers) as ex:
        for k, net in enumerate(ex.map(fn, items, chunksize=4)):
            out[k] = net
            if (k + 1) % 32 == 0 or k + 1 == len(items):
                print(f"[bench] {label}: generated {k + 1}/{len(items)} networks in {time.time() - t0:.1f}s",
                      file=sys.stderr, flush=True)
    return out


def _contract(args, value, unit, total_s, steps, config, dtype="fp32+fp64"):
    return {"metric": METRIC, "value": round(value, 4), "unit": unit, "n_gpus": 1, "steps": steps,
            "warmup": args.warmup, "ms_per_step": round(1e3 * total_s / max(steps, 1), 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config}


def _net_bytes(r, dim, n, s):
    pb = pass_bytes(dim, n, s, r.n_live)
    return r.iters * pb["cg"] + r.refreshes * pb["refresh"]


# Algorithmic bytes per swept node (every lattice node of the network): the
# compulsory floor of one CG iteration, s (d + 7) (bonds read once; x, r, p
# read and written once; the Jacobi diagonal read once), and of one FP64
# outer step of the mixed solve, 8 d + 32 (FP64 bonds and residual, the
# solution read and written). The two-pass fused design figure s (d + 12) is
# reported beside it.
def floor_cg(dim: int, s: int) -> int:
    return s * (dim + 7)


def floor_refresh(dim: int) -> int:
    return 8 * dim + 32


def two_pass_cg(dim: int, s: int) -> int:
    return s * (dim + 12)


PATHS = ("2d_full", "2d_small", "3d")
KERNEL_NAME = {(0, "fp32"): "pass2d_kernel<float, 0>", (1, "fp32"): "pass2d_kernel<float, 1>",
               (2, "fp32"): "pass3d_kernel<float>", (0, "fp64"): "pass2d_kernel<double, 0>",
               (1, "fp64"): "pass2d_kernel<double, 1>", (2, "fp64"): "pass3d_kernel<double>"}


def kernel_accounting(B, nets, probs, results_per_step, precision, stats):
    """Per pass kernel (path x precision): device time and launches from the
    library's event timing, algorithmic bytes from every member's iteration and
    refresh counts (floor figures per swept node), and the live-node bytes of
    the pass as built (pass_bytes) beside them."""
    s = 4 if precision == B.RN_MIXED else 8
    pname = "fp32" if precision == B.RN_MIXED else "fp64"
    plan_path = [B.rn_plan(pr, B.opts(precision))["path"] for pr in probs]
    rows = {}
    for path in range(3):
        secs = stats["pass_device_s"][path][precision]
        launches = stats["pass_timed_launches"][path][precision]
        if launches == 0:
            continue
        floor_b = live_b = two_b = 0
        cg = refr = swept_iters = 0
        for res in results_per_step:
            for k, (net, r) in enumerate(zip(nets, res)):
                if plan_path[k] != path:
                    continue
                floor_b += r.iters * floor_cg(net.dim, s) * net.n + r.refreshes * floor_refresh(net.dim) * net.n
                two_b += r.iters * two_pass_cg(net.dim, s) * net.n + r.refreshes * floor_refresh(net.dim) * net.n
                pb = pass_bytes(net.dim, net.n, s, r.n_live)
                live_b += r.iters * pb["cg"] + r.refreshes * pb["refresh"]
                cg += r.iters
                refr += r.refreshes
                swept_iters += r.iters * net.n
        rows[f"{PATHS[path]}_{pname}"] = {
            "kernel": KERNEL_NAME[(path, pname)], "device_s": secs, "launches": launches,
            "avg_launch_us": 1e6 * secs / launches, "cg_passes": cg, "refresh_passes": refr,
            "floor_bytes": floor_b, "two_pass_bytes": two_b, "live_node_bytes": live_b,
            "floor_GBps": floor_b / secs / 1e9, "swept_node_iters_per_s": swept_iters / secs}
    return rows


def batch_bench(args, B, I, np):
    """512 uneven networks solved together (rn_solve_batch), mixed precision to tol.

    value = networks solved per second over the timed batches. Latency is the
    completion time of each member from the call. The roofline is the pass
    kernel with the most device time (HIP events around every launch, on the
    launch stream, over the timed batches): the floor bytes of every CG
    iteration and FP64 outer step of its members over its device time.
    Compared with the same batch in FP64, with plain FP64 CG run one network
    at a time, and with a Poisson-served stream against plain FP64 CG served
    first in first out (--requests 0 skips it). The CPU oracle solves a seeded
    sample of the members in worker processes while the GPU comparison legs
    run.
    """
    import tempfile
    import torch
    shapes = {"source": "built-in rules"}
    if args.shapes == "cache" and os.path.exists(args.shapes_file):
        B.rn_tune_load(args.shapes_file)
        rows = [l.split() for l in open(args.shapes_file) if l.strip() and not l.startswith("#")]
        shapes = {"source": f"rn_tune_load of {os.path.relpath(args.shapes_file, ROOT)} (written by rn_autotune "
                            f"on an MI355X)", "table": [" ".join(r) for r in rows]}
    elif args.shapes == "search":
        # the launch-shape search of every size class (untimed, like a warmup)
        c = B.Context(0)
        path = os.path.join(tempfile.mkdtemp(prefix="rn_shapes_"), "shapes.txt")
        t = time.perf_counter()
        c.autotune(path)
        c.close()
        rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
        shapes = {"source": "rn_autotune on this device before the timed batches",
                  "search_s": round(time.perf_counter() - t, 2),
                  "table": [" ".join(r) for r in rows]}
        print(f"[bench] launch-shape search: {len(rows)} classes in {shapes['search_s']} s", file=sys.stderr,
              flush=True)
    specs = I.batch_specs(args.batch_size)
    nets = generate(_gen_batch, specs, "batch")
    gd = [[torch.from_numpy(a).to("cuda") for a in n.g] for n in nets]
    torch.cuda.synchronize()
    probs = [B.problem(dim=n.dim, nx=n.nx, ny=n.ny, nz=n.nz, axis=0, g=g) for n, g in zip(nets, gd)]
    ctx = B.Context(0)

    def run(prec, steps, timed_stats=False):
        walls, per_step, lat = [], [], []
        for it in range(args.warmup + steps):
            if timed_stats and it == args.warmup:
                ctx.set_timing(True)           # clears the accumulated launch times
            torch.cuda.synchronize()
            t = time.perf_counter()
            res = ctx.solve_batch(probs, B.opts(prec, args.tol))
            w = time.perf_counter() - t
            bad = [r.status for r in res if r.status != 0]
            print(f"[bench] batch prec={'mixed' if prec == B.RN_MIXED else 'fp64'} "
                  f"{'warmup' if it < args.warmup else 'step'} {it}: {w:.3f}s failed={len(bad)}",
                  file=sys.stderr, flush=True)
            if bad:
                raise SystemExit(f"batch members failed: {bad[:5]}")
            if it >= args.warmup:
                walls.append(w)
                per_step.append(res)
                lat.extend(r.t_total_s for r in res)
        st = ctx.stats() if timed_stats else None
        if timed_stats:
            ctx.set_timing(False)
        return walls, per_step, lat, st

    walls_m, steps_m, lat_m, st_m = run(B.RN_MIXED, args.steps, timed_stats=True)
    tot_m = sum(walls_m)
    value = len(probs) * len(walls_m) / tot_m
    res_m = steps_m[-1]
    config = {"workload": MULTI["batch512"], "networks": len(probs), "nodes": int(sum(n.n for n in nets)),
              "nodes_2d": int(sum(n.n for n in nets if n.dim == 2)),
              "nodes_3d": int(sum(n.n for n in nets if n.dim == 3)), "tol": args.tol,
              "precision": "fp32 inner CG + fp64 refresh/solution/flux", "x0": "linear profile",
              "preconditioner": "Jacobi", "inputs": "resident in HBM",
              "launch_shapes": shapes["source"]}
    out = _contract(args, value, "solves/s", tot_m, len(walls_m), config)
    out["latency_ms"] = {"p50": round(1e3 * float(np.percentile(lat_m, 50)), 2),
                         "p99": round(1e3 * float(np.percentile(lat_m, 99)), 2),
                         "of": "completion time of each batch member from the rn_solve_batch call"}
    out["batch_wall_s"] = [round(w, 3) for w in walls_m]
    out["launch_shapes"] = shapes
    kern = kernel_accounting(B, nets, probs, steps_m, B.RN_MIXED, st_m)
    if not kern:
        # no per-launch times: pass rounds replayed from a hipGraph (RN_GRAPHS=1) record no events
        out["roofline"] = None
        out["roofline_note"] = "no per-launch device times: pass rounds were replayed from a hipGraph"
        out["iters_mixed"] = {"median": int(np.median([r.iters for r in res_m])),
                              "max": int(max(r.iters for r in res_m))}
        ctx.close()
        return out
    dom_key = max(kern, key=lambda k: kern[k]["device_s"])
    dom = kern[dom_key]
    traffic = traffic_from_profiles("batch512", dom_key)
    achieved = dom["floor_GBps"]
    out["roofline"] = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": round(traffic["bytes_per_launch"]) if traffic else None,
        "kernel": dom["kernel"], "avg_launch_us": round(dom["avg_launch_us"], 2), "launches": dom["launches"],
        "bytes_per_launch": round(dom["floor_bytes"] / dom["launches"]),
        "bytes_model": "floor per swept node: s(d+7) per CG iteration, 8d+32 per FP64 outer step",
        "two_pass_GBps": round(dom["two_pass_bytes"] / dom["device_s"] / 1e9, 1),
        "live_node_GBps": round(dom["live_node_bytes"] / dom["device_s"] / 1e9, 1),
        "traffic_GBps": round(traffic["bytes_per_launch"] / (dom["device_s"] / dom["launches"]) / 1e9, 1)
        if traffic else None,
        "timing": "HIP events recorded by the library on the launch stream between consecutive pass launches"}
    out["kernels"] = {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                      for k, v in kern.items()}
    all_secs = sum(v["device_s"] for v in kern.values())
    all_floor = sum(v["floor_bytes"] for v in kern.values())
    out["all_pass_kernels_floor_GBps"] = round(all_floor / all_secs / 1e9, 1)
    out["pass_device_s_per_batch"] = round(all_secs / len(walls_m), 4)
    out["live_node_iters_per_s"] = round(sum(r.n_live * r.iters for res in steps_m for r in res) / tot_m, 1)
    out["iters_mixed"] = {"median": int(np.median([r.iters for r in res_m])),
                          "max": int(max(r.iters for r in res_m))}

    cpu_job = None
    if not args.no_cpu:
        cpu_job = start_cpu_baseline(specs, args)

    if not args.no_fp64:
        walls_d, steps_d, _, _ = run(B.RN_FP64, 1)
        res_d = steps_d[-1]
        out["fp64_batched_solves_per_s"] = round(len(probs) / min(walls_d), 4)
        # plain FP64 CG, one network at a time
        t = time.perf_counter()
        lat_d = []
        for pr in probs:
            r = ctx.solve(pr, B.opts(B.RN_FP64, args.tol))
            if r.status != 0:
                raise SystemExit(f"fp64 solve failed: {r.as_dict()}")
            lat_d.append(time.perf_counter() - t)
        w = time.perf_counter() - t
        out["fp64_cg_one_at_a_time"] = {"solves_per_s": round(len(probs) / w, 4),
                                        "p50_ms": round(1e3 * float(np.percentile(lat_d, 50)), 2),
                                        "p99_ms": round(1e3 * float(np.percentile(lat_d, 99)), 2)}
        out["mixed_batched_vs_fp64_one_at_a_time"] = round(value / out["fp64_cg_one_at_a_time"]["solves_per_s"], 3)
        out["mixed_batched_vs_fp64_batched"] = round(value / out["fp64_batched_solves_per_s"], 3)
        out["max_K_rel_diff_mixed_vs_fp64"] = float(max(abs(a.K / b.K - 1.0) for a, b in zip(res_m, res_d)
                                                        if b.K > 0))
    ctx.close()
    del gd, probs
    torch.cuda.empty_cache()

    if args.requests > 0:
        out["serve"] = serve_leg(args, B, I, np)

    if cpu_job is not None:
        out["cpu_baseline"] = finish_cpu_baseline(cpu_job, args)
        out["vs_cpu_oracle"] = round(value / out["cpu_baseline"]["value"], 1)
    return out


def _oracle_member(job):
    """One full oracle solve (mask, assembly, Jacobi-PCG from the linear
    profile, flux) of batch member k in this worker process; seconds and
    iterations."""
    k, spec, tol = job
    import oracle
    from paper_1908_03301_amd import inputs as I
    net = I.batch_network(spec)
    t = time.perf_counter()
    r = oracle.solve(net, tol=tol, want_pressure=False, x0=oracle.X0_LINEAR, precond=oracle.JACOBI)
    return k, time.perf_counter() - t, r.iters, r.converged, net.n


def start_cpu_baseline(specs, args):
    """Start the oracle on a seeded uniform sample of the batch members, one
    member per worker process (single-threaded C), on the host's cores while
    the GPU comparison legs run."""
    from concurrent.futures import ProcessPoolExecutor
    import numpy as np
    rng = np.random.default_rng(190803301 + 77)
    sample = sorted(int(k) for k in rng.choice(len(specs), size=min(args.cpu_sample, len(specs)), replace=False))
    # the machine's CPU share is 16 cores; two stay free for the threads driving the GPU
    cores = max(1, min(16, len(os.sched_getaffinity(0))) - 2)
    ex = ProcessPoolExecutor(max_workers=cores)
    futs = [ex.submit(_oracle_member, (k, specs[k], args.tol)) for k in sample]
    print(f"[bench] cpu oracle: {len(sample)} sampled members on {cores} worker processes", file=sys.stderr,
          flush=True)
    return {"ex": ex, "futs": futs, "cores": cores, "sample": sample, "t0": time.perf_counter(),
            "members": len(specs)}


def finish_cpu_baseline(job, args):
    rows = [f.result() for f in job["futs"]]
    wall = time.perf_counter() - job["t0"]
    job["ex"].shutdown()
    secs = sum(r[1] for r in rows)
    cores = job["cores"]
    one = len(rows) / secs
    return {"value": round(one * cores, 4), "unit": "solves/s", "cores": cores, "kind": "oracle",
            "value_1_core": round(one, 5),
            "sample": (f"{len(rows)} of the {job['members']} batch members (seeded uniform draw: "
                       f"{job['sample']}), each solved in full by the oracle (mask, assembly, Jacobi-PCG from "
                       f"the linear profile to tol {args.tol}, flux) in its own single-threaded worker process; "
                       f"value = cores x sampled solves / their summed solve seconds ({secs:.1f} s; wall "
                       f"{wall:.1f} s on {cores} processes), i.e. the batch's solves/s on that many cores "
                       f"under a uniform sample"),
            "members": [{"member": r[0], "nodes": r[4], "seconds": round(r[1], 2), "iters": r[2],
                         "converged": bool(r[3])} for r in rows],
            "cpu": cpu_info(), "threads_per_solve": 1}


def aniso_bench(args, B, I, np):
    """K_x / K_y of anisotropic FBM networks (Eq. 2): both axes of every network
    in one rn_solve_batch, mixed precision to tol; the ratio's range per
    (H, beta_x / beta_y) is the quantity of Fig. 10."""
    import torch
    specs = I.aniso_specs()
    nets = generate(_gen_aniso, [(sp, args.sigma) for sp in specs], "aniso")
    gd = [[torch.from_numpy(a).to("cuda") for a in n.g] for n in nets]
    torch.cuda.synchronize()
    probs = [B.problem(dim=2, nx=n.nx, ny=n.ny, nz=1, axis=ax, g=g) for n, g in zip(nets, gd) for ax in (0, 1)]
    ctx = B.Context(0)
    walls, res = [], None
    for it in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = ctx.solve_batch(probs, B.opts(B.RN_MIXED, args.tol))
        w = time.perf_counter() - t
        print(f"[bench] aniso {'warmup' if it < args.warmup else 'step'} {it}: {w:.3f}s", file=sys.stderr, flush=True)
        if any(r.status != 0 or not r.converged for r in res):
            raise SystemExit("aniso batch member failed")
        if it >= args.warmup:
            walls.append(w)
    ctx.close()
    value = len(probs) * len(walls) / sum(walls)
    table = {}
    for k, sp in enumerate(specs):
        kx, ky = res[2 * k].K, res[2 * k + 1].K
        table.setdefault(f"H={sp.H:g} beta_x/beta_y={sp.ratio:g}", []).append(kx / ky if ky > 0 else float("inf"))
    summary = {key: {"min": round(min(v), 3), "median": round(float(np.median(v)), 3), "max": round(max(v), 3),
                     "networks": len(v)} for key, v in table.items()}
    out = _contract(args, value, "solves/s", sum(walls), len(walls),
                    {"workload": MULTI["aniso"], "sigma": args.sigma, "networks": len(nets), "solves": len(probs),
                     "nodes": sum(n.n for n in nets), "tol": args.tol,
                     "precision": "fp32 inner CG + fp64 refresh/solution/flux", "inputs": "resident in HBM"})
    out["Kx_over_Ky"] = summary
    return out


def fbmgen_bench(args, B, I, np):
    """Nodes generated per second: field + bonds + dilution, GPU (rn_fbm_field,
    rn_fbm_bonds) against the numpy generator, on the same random numbers."""
    import torch
    ctx = B.Context(0)
    rows = {}
    for dim, shape, H in ((2, (2048, 2048), 0.7), (3, (256, 256, 256), 0.8)):
        rng = I.rng_for(123)
        noise = rng.standard_normal(shape)
        u = [rng.random(shape) for _ in range(dim)]
        n = int(np.prod(shape))
        nx, ny, nz = shape[-1], shape[-2], (shape[0] if dim == 3 else 1)
        nd = torch.from_numpy(noise).cuda()
        ud = [torch.from_numpy(a).cuda() for a in u]
        phi = torch.empty_like(nd)
        g = [torch.empty_like(nd) for _ in range(dim)]
        walls = []
        for it in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            ctx.fbm_field(dim, nx, ny, nz, H, nd, phi)
            ctx.fbm_bonds(dim, nx, ny, nz, phi, 1.5, False, g, u=ud, occupancy=0.6)
            torch.cuda.synchronize()
            if it >= args.warmup:
                walls.append(time.perf_counter() - t)
        t = time.perf_counter()
        ref = I.bonds_from_node_field(I.fbm_filter(noise, H), 1.5)
        ref = [np.where(uk < 0.6, a, 0.0) for uk, a in zip(u, ref)]
        t_np = time.perf_counter() - t
        err = max(float(np.max(np.abs(a.cpu().numpy() - r) / np.maximum(r, 1e-300))) for a, r in zip(g, ref))
        rows[f"{dim}D {'x'.join(map(str, shape[::-1]))}"] = {
            "gpu_ms": round(1e3 * min(walls), 3), "numpy_s": round(t_np, 3),
            "gpu_nodes_per_s": round(n / min(walls)), "numpy_nodes_per_s": round(n / t_np),
            "speedup": round(t_np / min(walls), 1), "max_rel_diff_bonds": err}
        print(f"[bench] fbmgen {dim}D: gpu {1e3 * min(walls):.2f} ms, numpy {t_np:.2f} s", file=sys.stderr,
              flush=True)
    ctx.close()
    total_n = sum(v["gpu_nodes_per_s"] * v["gpu_ms"] / 1e3 for v in rows.values())
    total_t = sum(v["gpu_ms"] / 1e3 for v in rows.values())
    out = _contract(args, total_n / total_t, "nodes/s", total_t, args.steps,
                    {"workload": MULTI["fbmgen"], "inputs": "random numbers resident in HBM"}, dtype="f64")
    out["metric"] = "network generation nodes/s (FBM field + bonds + dilution)"
    out["cases"] = rows
    return out


def backbone_bench(args, B, I, np):
    """Lattice nodes per second of rn_build_backbone (mask + backbone), the
    oracle's Hopcroft-Tarjan search timed beside it on one core."""
    import torch

    import oracle
    ctx = B.Context(0)
    nets = {"2D 2048^2 FBM occ 0.6": I.workload_fbm_2d_2048(),
            "3D 256^3 layered occ 0.27": I.workload_strat_3d_256(),
            "2D 2048^2 RRN p 0.52": I.iid_network(2, 2048, 2048, 1, sigma=0.0, occupancy=0.52, index=7)}
    rows, total_n, total_t = {}, 0, 0.0
    for label, net in nets.items():
        gd = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in net.g]
        m = torch.zeros(net.shape, dtype=torch.uint8, device="cuda")
        pr = B.problem(dim=net.dim, nx=net.nx, ny=net.ny, nz=net.nz, axis=net.axis, g=gd, mask_out=m)
        walls = []
        for it in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            nl, nb = ctx.build_backbone(pr)
            torch.cuda.synchronize()
            if it >= args.warmup:
                walls.append(time.perf_counter() - t)
        t = time.perf_counter()
        ref, nlr, nbr = oracle.backbone(net)
        t_cpu = time.perf_counter() - t
        same = bool(np.array_equal(m.cpu().numpy(), ref))
        row = {"nodes": net.n, "n_live": nl, "n_backbone": nb, "backbone_fraction_of_live": round(nb / max(nl, 1), 4),
               "gpu_ms": round(1e3 * min(walls), 3), "oracle_s": round(t_cpu, 3),
               "gpu_nodes_per_s": round(net.n / min(walls)), "speedup_vs_oracle": round(t_cpu / min(walls), 1),
               "mask_equals_oracle": same}
        rows[label] = row
        total_n += net.n
        total_t += min(walls)
        print(f"[bench] backbone {label}: gpu {1e3 * min(walls):.1f} ms, oracle {t_cpu:.2f} s, "
              f"live {nl} backbone {nb}, equal {same}", file=sys.stderr, flush=True)
        del gd, m
        torch.cuda.empty_cache()
    # the RRN toward p_c (Sec. VI, Fig. 7's networks): mixed solves of the whole live set against
    # RN_OPT_BACKBONE (its backbone pass included), wall time from the call to the result
    study = {}
    for p in (0.7, 0.6, 0.55, 0.52):
        net = I.iid_network(2, 2048, 2048, 1, sigma=0.0, occupancy=p, index=700 + int(100 * p))
        gd = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in net.g]
        pr = B.problem(dim=2, nx=net.nx, ny=net.ny, g=gd)
        row = {}
        for name, bb in (("live_set", False), ("backbone", True)):
            best = None
            for it in range(2):
                torch.cuda.synchronize()
                t = time.perf_counter()
                r = ctx.solve(pr, B.opts(B.RN_MIXED, args.tol, backbone=bb))
                torch.cuda.synchronize()
                dt = time.perf_counter() - t
                best = dt if best is None else min(best, dt)
            row[name] = {"s": round(best, 4), "iters": int(r.iters), "K": r.K, "converged": bool(r.converged),
                         "n_live": int(r.n_live), "n_backbone": int(r.n_backbone)}
        row["speedup"] = round(row["live_set"]["s"] / row["backbone"]["s"], 3)
        row["K_rel_diff"] = abs(row["backbone"]["K"] / row["live_set"]["K"] - 1.0) if row["live_set"]["K"] else 0.0
        study[f"p={p}"] = row
        print(f"[bench] RRN 2048^2 p={p}: live set {row['live_set']['iters']} iters {row['live_set']['s']:.3f} s, "
              f"backbone {row['backbone']['iters']} iters {row['backbone']['s']:.3f} s", file=sys.stderr, flush=True)
        del gd
        torch.cuda.empty_cache()
    ctx.close()
    out = _contract(args, total_n / total_t, "nodes/s", total_t, args.steps,
                    {"workload": MULTI["backbone"], "inputs": "bonds resident in HBM"}, dtype="int32")
    out["metric"] = "backbone nodes/s (connectivity mask + biconnected block of the inlet-outlet edge)"
    out["cases"] = rows
    out["rrn_toward_pc"] = study
    return out


def serve_leg(args, B, I, np):
    """Served stream (rn_submit / rn_poll) against plain FP64 CG served first in first out.

    Requests cycle through a pool of pre-generated networks (device
    resident). The mixed server's saturation rate is measured first with
    --sat-requests requests submitted at once; the stream then arrives as a
    Poisson process at 0.7 times that rate. The same arrival times are
    replayed against plain FP64 CG solving one request at a time in arrival
    order. Latency = completion time - arrival time.
    """
    import torch
    reqs = I.stream_requests(args.pool, rate_per_s=1.0)
    pool = generate(_gen_stream, reqs, "stream pool")
    gd = [[torch.from_numpy(a).to("cuda") for a in n.g] for n in pool]
    torch.cuda.synchronize()
    probs = [B.problem(dim=n.dim, nx=n.nx, ny=n.ny, nz=n.nz, axis=0, g=g) for n, g in zip(pool, gd)]
    om, od = B.opts(B.RN_MIXED, args.tol), B.opts(B.RN_FP64, args.tol)

    def serve(arrivals, order, c):
        nreq = len(arrivals)
        lat, submitted, done = [None] * nreq, {}, 0
        tstart = time.perf_counter()
        i = 0
        while done < nreq:
            now = time.perf_counter() - tstart
            while i < nreq and arrivals[i] <= now:
                submitted[c.submit(probs[order[i]], om)] = (i, tstart + arrivals[i])
                i += 1
            for t in list(submitted):
                st, r = c.poll(t)
                if st == B.RN_EAGAIN:
                    continue
                k, ta = submitted.pop(t)
                if st != 0:
                    raise SystemExit(f"served request failed: {st}")
                lat[k] = time.perf_counter() - ta
                done += 1
            time.sleep(0.0002)
        return lat, time.perf_counter() - tstart

    # saturation: everything submitted at t = 0
    nsat = args.sat_requests
    c = B.Context(0)
    _, make = serve([0.0] * nsat, [i % len(pool) for i in range(nsat)], c)
    sat = nsat / make
    c.close()
    rate = 0.7 * sat
    nreq = args.requests
    rng = I.rng_for(50_000_000)
    arrivals = list(np.cumsum(rng.exponential(1.0 / rate, nreq)))
    order = [int(k) for k in rng.integers(0, len(pool), nreq)]
    print(f"[bench] serve: saturation {sat:.2f} solves/s, stream of {nreq} at {rate:.2f}/s", file=sys.stderr,
          flush=True)
    c = B.Context(0)
    lat, make = serve(arrivals, order, c)
    c.close()
    # plain FP64 CG, first in first out, same arrivals
    ctx = B.Context(0)
    lat_d = []
    tstart = time.perf_counter()
    for k in range(nreq):
        now = time.perf_counter() - tstart
        if arrivals[k] > now:
            time.sleep(arrivals[k] - now)
        r = ctx.solve(probs[order[k]], od)
        if r.status != 0:
            raise SystemExit(f"fp64 request failed: {r.as_dict()}")
        lat_d.append(time.perf_counter() - tstart - arrivals[k])
    make_d = time.perf_counter() - tstart
    ctx.close()
    del gd, probs
    torch.cuda.empty_cache()
    out = {"workload": MULTI["serve"], "requests": nreq, "pool": len(pool),
           "pool_nodes": int(sum(n.n for n in pool)), "rate_per_s": round(rate, 3),
           "saturation_solves_per_s": round(sat, 3), "saturation_requests": nsat,
           "solves_per_s": round(nreq / make, 3),
           "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 2),
           "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 2),
           "fp64_cg_fifo": {"solves_per_s": round(nreq / make_d, 3),
                            "p50_ms": round(1e3 * float(np.percentile(lat_d, 50)), 2),
                            "p99_ms": round(1e3 * float(np.percentile(lat_d, 99)), 2)}}
    out["p99_vs_fp64_fifo"] = round(out["fp64_cg_fifo"]["p99_ms"] / out["p99_ms"], 3)
    return out


def serve_bench(args, B, I, np):
    """The served stream alone (value = its solves/s at 0.7 x saturation)."""
    leg = serve_leg(args, B, I, np)
    out = _contract(args, leg["solves_per_s"], "solves/s", leg["requests"] / leg["solves_per_s"], leg["requests"],
                    {"workload": MULTI["serve"], "requests": leg["requests"], "pool": leg["pool"],
                     "rate_per_s": leg["rate_per_s"], "tol": args.tol,
                     "precision": "fp32 inner CG + fp64 refresh/solution/flux", "inputs": "resident in HBM"})
    out["latency_ms"] = {"p50": leg["p50_ms"], "p99": leg["p99_ms"]}
    out["serve"] = leg
    return out


def cpu_baseline(net, wl, args, res_fp64):
    """The CPU oracle (plain C, FP64, one thread) on a bounded sample of a single-network workload.

    Sample: mask + assembly + final flux on the full network (max_iter 0), and
    the same plus `cpu_iters` PCG iterations; the per-solve time is
    extrapolated to the iteration count the GPU FP64 solve of the same network
    needed (the same Jacobi-PCG from the same linear-profile initial guess and
    the same tolerance). The batch workload times full oracle solves instead.
    """
    import oracle
    n0 = net.with_axis(wl["axes"][0])
    t0 = time.perf_counter()
    oracle.solve(n0, tol=args.tol, max_iter=0, want_pressure=False, x0=oracle.X0_LINEAR)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.solve(n0, tol=args.tol, max_iter=args.cpu_iters, want_pressure=False, x0=oracle.X0_LINEAR)
    t_m = time.perf_counter() - t0
    t_iter = max(t_m - t_setup, 1e-9) / args.cpu_iters
    if res_fp64:
        it = res_fp64[0][1]["iters"]
        basis = "GPU FP64 iteration count of the same solve"
    else:
        it = args.cpu_iters
        basis = "sample iterations only"
    t_solve = t_setup + it * t_iter
    return {"value": round(1.0 / t_solve, 6), "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"{wl['desc']}, axis {wl['axes'][0]}: mask+assembly+flux {t_setup:.2f}s, "
                       f"{t_iter * 1e3:.1f} ms per PCG iteration over {args.cpu_iters} iterations, "
                       f"extrapolated to {it} iterations ({basis}); tol {args.tol}"),
            "cpu": cpu_info(), "sec_per_solve": round(t_solve, 2)}


if __name__ == "__main__":
    main()
