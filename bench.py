#!/usr/bin/env python3
"""Throughput of the random-network flow solve on one MI355X.

One step solves one synthetic network for K_x and K_y (two solves) with the
mixed-precision solver (FP32 inner CG, FP64 residual refresh, solution and
flux) to a relative true residual of 1e-8; plain FP64 CG is timed on the same
inputs and tolerance for comparison. Inputs are generated on the host, copied
to HBM before the timed region and passed by device pointer.

Prints one JSON line: value = network solves/s (mixed), latency percentiles,
the pass kernel's roofline (algorithmic bytes / device time of the iteration
loop, measured with HIP events on the launch stream) and the CPU oracle timed
on a bounded sample of the same workload.
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
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "fbm2d_2048": dict(desc="2D 2048x2048, FBM ln g (H=0.7, sigma=1.5), i.i.d. occupancy 0.6, K_x and K_y",
                       make=lambda I: I.workload_fbm_2d_2048(), axes=(0, 1)),
    "iid2d_128": dict(desc="2D 128x128, ln g ~ N(0,1) i.i.d., K_x",
                      make=lambda I: I.workload_iid_2d_128(), axes=(0,)),
    "strat3d_256": dict(desc="3D 256^3 layered 1D-FBM ln g (H=0.8, sigma=2), occupancy 0.27, K_x and K_z",
                        make=lambda I: I.workload_strat_3d_256(), axes=(0, 2)),
}


def pass_bytes(dim: int, n: int, s: int, live: int) -> dict:
    """Algorithmic HBM bytes of one pass kernel launch.

    CG pass: every node reads 1/d (s bytes); a live node also reads r, p, q
    and dim conductance arrays (s bytes each) and its FP64 pressure, and
    writes r, p, q and the pressure: (dim + 6) s + 16 bytes. Refresh pass:
    every node reads 1/d and copies its FP64 pressure (16 bytes); a live node
    also reads dim FP64 conductances and p and writes r, p, q:
    8 dim + 4 s bytes more.
    """
    return {"cg": s * n + ((dim + 6) * s + 16) * live,
            "refresh": (s + 16) * n + (8 * dim + 4 * s) * live}


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


def traffic_from_profiles(workload: str, precision: str):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if current."""
    path = os.path.join(ROOT, "profiles", "pass_kernel_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        e = d.get(workload, {}).get(precision)
        if not e or e.get("kernel_hash") != kernel_hash():
            return None
        return float(e["bytes_per_launch"])
    except Exception:
        return None


def run_solves(ctx, B, prob_by_axis, precision, tol, steps, warmup, max_iter=2_000_000):
    lat, results = [], []
    o = B.opts(precision, tol, max_iter=max_iter)
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
    ap.add_argument("--workload", default="fbm2d_2048", choices=sorted(WORKLOADS))
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 CG comparison leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-iters", type=int, default=60, help="oracle PCG iterations in the CPU sample")
    ap.add_argument("--single-axis", action="store_true", help="solve only the first flow axis (profiling)")
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
    n = net.n
    n_live = res_m[0][1]["n_live"]
    pb = pass_bytes(net.dim, n, 4, n_live)
    loop_t = sum(r["t_loop_s"] for _, r in res_m)
    launches = sum(r["passes"] for _, r in res_m)
    iters = sum(r["iters"] for _, r in res_m)
    refr = sum(r["refreshes"] for _, r in res_m)
    alg_bytes = iters * pb["cg"] + refr * pb["refresh"]
    avg_launch_s = loop_t / max(launches, 1)
    achieved = alg_bytes / loop_t / 1e9
    traffic = traffic_from_profiles(args.workload, "mixed")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
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
           "roofline": roofline}
    out["results"] = {f"K_axis{ax}": r["K"] for ax, r in res_m[: len(wl["axes"])]}
    out["iters_mixed"] = {f"axis{ax}": r["iters"] for ax, r in res_m[: len(wl["axes"])]}

    if not args.no_fp64:
        lat_d, res_d = leg(B.RN_FP64)
        pbd = pass_bytes(net.dim, n, 8, res_d[0][1]["n_live"])
        loop_d = sum(r["t_loop_s"] for _, r in res_d)
        bytes_d = sum(r["iters"] for _, r in res_d) * pbd["cg"] + sum(r["refreshes"] for _, r in res_d) * pbd["refresh"]
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


def cpu_baseline(net, wl, args, res_fp64):
    """The CPU oracle (plain C, FP64, one thread) on a bounded sample of the workload.

    Sample: mask + assembly + final flux on the full network (max_iter 0), and
    the same plus `cpu_iters` PCG iterations; the per-solve time is extrapolated
    to the iteration count the GPU FP64 solve of the same network needed (same
    Jacobi-PCG from x = 0 and the same tolerance).
    """
    import oracle
    n0 = net.with_axis(wl["axes"][0])
    t0 = time.perf_counter()
    oracle.solve(n0, tol=args.tol, max_iter=0, want_pressure=False)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.solve(n0, tol=args.tol, max_iter=args.cpu_iters, want_pressure=False)
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
