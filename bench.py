"""Benchmark: ms per 500-waypoint batch and G point-link queries/s.

One step = forward kinematics of every waypoint (lsdf_fk_batch) plus the
clearance query (lsdf_query_min_distance) over 500 waypoints x 20,000
obstacle points x 7 links with 64^3 FP32 link grids, inputs resident in HBM.
Prints one JSON line.  One GPU only.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ms per 500-waypoint batch; G point-link queries/s; grid vs MLP-SDF at ≤1 mm"
PEAK_FP32_VECTOR_TFLOPS = 157.3       # MI355X published FP32 vector peak
FLOP_PER_PAIR = 24                    # map to grid coordinates (9 FMA) + 6 box compares
FLOP_PER_INBOX_PAIR = 28              # cell + fraction (6), 7 lerps (21), min (1)
BYTES_PER_INBOX_PAIR = 32             # 8 gathered FP32 corners


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def profiled_traffic(kernel_source: str, summary: str):
    """HBM bytes per launch measured by the rocprofv3 FETCH_SIZE/WRITE_SIZE
    runs recorded in the profile summary, or None when the kernel source has
    changed since (the summary stores a hash of the source it measured)."""
    import hashlib
    try:
        lines = dict(l.split(": ", 1) for l in open(summary).read().splitlines() if ": " in l)
        src = hashlib.sha256(open(kernel_source, "rb").read()).hexdigest()[:16]
        if lines.get("query_kernel_source_sha256_16", "").strip() != src:
            return None
        return int(float(lines["query_kernel_traffic_bytes_per_launch"]))
    except (OSError, KeyError, ValueError):
        return None


def count_inbox_pairs(T: np.ndarray, lo, hi, points: np.ndarray) -> int:
    """Pairs (c, i, j) whose point lies in link i's box at waypoint c (double
    precision; used only to price the in-box work for the roofline)."""
    total = 0
    P = points.astype(np.float64)
    C, L = T.shape[:2]
    for i in range(L):
        R = T[:, i, :, :3].astype(np.float64)     # [C][3][3]
        t = T[:, i, :, 3].astype(np.float64)      # [C][3]
        for c0 in range(0, C, 50):
            l = np.einsum("cba,cjb->cja", R[c0:c0 + 50], P[None] - t[c0:c0 + 50, None, :])
            inside = np.all((l >= lo[i]) & (l <= hi[i]), axis=-1)
            total += int(inside.sum())
    return total


def cpu_baseline(w, budget_s: float = 12.0):
    """The CPU oracle (double-precision kinematics + query) on the same
    workload, repeated for about budget_s seconds."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    log(f"cpu baseline: building oracle grids ({threads} threads)")
    grids = oracle.workload_grids(w)
    reps, t_total = 0, 0.0
    while t_total < budget_s and reps < 200:
        t0 = time.perf_counter()
        T = oracle.fk(w.robot.dh, w.q, w.robot.base_T)
        cl = oracle.query_f64(T, w.grid_lo, w.grid_hi, w.grid_n, grids, w.points)
        oracle.reduce(cl)
        t_total += time.perf_counter() - t0
        reps += 1
    sec = t_total / reps
    return {"value": round(w.C * w.M * w.L / sec / 1e9, 4), "unit": "G point-link queries/s",
            "ms_per_batch": round(sec * 1e3, 3), "cores": threads, "kind": "oracle",
            "sample": f"full {w.name} batch (C={w.C}, M={w.M}, L={w.L}) repeated {reps}x; "
                      "double-precision kinematics + query, OpenMP over waypoints"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="paper")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB mebibytes (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the clearance query is measured on a single MI355X "
              "(see the sharding notes in DESIGN.md); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2309_12543_amd import lsdf

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: 5 copies of {args.copy_probe} MiB")
        return
    lsdf.load_library()
    w = synth.make_workload(args.workload)
    log(f"workload {w.name}: C={w.C} M={w.M} L={w.L} n={int(w.grid_n[0, 0])}")
    gs = lsdf.build_robot_grids(w.robot.links, w.grid_lo, w.grid_hi, w.grid_n, device=dev)
    q = torch.as_tensor(w.q, dtype=torch.float32, device=dev)
    pts = torch.as_tensor(w.points, dtype=torch.float32, device=dev)
    T = torch.empty((w.C, w.L, 3, 4), dtype=torch.float32, device=dev)
    dist = torch.empty(w.C, dtype=torch.float32, device=dev)
    link = torch.empty(w.C, dtype=torch.int32, device=dev)
    ws = torch.zeros(lsdf.query_workspace_size(w.C, w.L, w.M), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    def step(ev=None):
        lsdf.fk_batch(w.robot.dh, q, base_T=w.robot.base_T, out=T)
        if ev is not None:
            ev[0].record()
        lsdf.query_min_distance(T, gs, pts, workspace=ws, out=(dist, link, None))
        if ev is not None:
            ev[1].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    pairs = w.C * w.M * w.L
    value = pairs / (ms_per_step / 1e3) / 1e9

    Tn = T.cpu().numpy()
    inbox = count_inbox_pairs(Tn, w.grid_lo.astype(np.float64), w.grid_hi.astype(np.float64), w.points)
    flop = FLOP_PER_PAIR * pairs + FLOP_PER_INBOX_PAIR * inbox
    achieved = flop / (kernel_ms / 1e3) / 1e12
    rec = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "G point-link queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.C} waypoints x {w.M} points x {w.L} links, "
                               f"{int(w.grid_n[0, 0])}^3 FP32 link grids",
                   "waypoints": w.C, "points": w.M, "links": w.L, "grid_nodes": int(w.grid_n[0, 0]),
                   "parallelism": "single GPU"},
        "query_kernel_ms": round(kernel_ms, 5),
        "inbox_pair_fraction": round(inbox / pairs, 5),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4),
                     "traffic": profiled_traffic(os.path.join(ROOT, "paper_2309_12543_amd", "csrc", "query.hip"),
                                                 os.path.join(ROOT, "profiles", "query_kernel_paper.txt")),
                     "kernel": "query_kernel (timed with its finalize kernel: one lsdf_query_min_distance call)",
                     "algorithmic_flop": flop},
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
