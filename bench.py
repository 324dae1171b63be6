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


def time_calls(fn, steps, warmup):
    """Mean duration (ms) of fn() measured with HIP events on the current stream."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in ev]))


def learned_variant(dev, epochs: int, steps: int, judge_waypoints: int = 8):
    """The learned form on the 500 x 100,000 x 7 workload (64^3 grids): per-link
    networks trained on the GPU (untimed), then the grid-only query and the
    network-plus-fallback query timed on the same inputs, and the learned
    clearances judged against the oracle's exact minimum on sampled waypoints."""
    import torch

    import oracle
    import synth
    from paper_2309_12543_amd import learned, lsdf

    w = synth.make_workload("learned")
    log(f"learned variant: C={w.C} M={w.M} L={w.L}, training {epochs} epochs")
    gs = lsdf.build_robot_grids(w.robot.links, w.grid_lo, w.grid_hi, w.grid_n, device=dev)
    cen, half = synth.mlp_domain(w.grid_lo.astype(np.float64), w.grid_hi.astype(np.float64))
    n = 1 << 20
    S = torch.as_tensor(np.stack([synth.mlp_samples(m, w.grid_lo[i], w.grid_hi[i], n, synth.BASE_SEED + 4 + i)
                                  for i, m in enumerate(w.robot.links)]).astype(np.float32), device=dev)
    t0 = time.perf_counter()
    labels = learned.labels_for_samples(w.robot.links, gs, S)
    params = torch.as_tensor(synth.mlp_init(w.L, synth.BASE_SEED + 5).astype(np.float32), device=dev)
    hist = learned.train(params, (cen, half), S, labels, epochs=epochs, batch=4096, lr=3e-3, lr_final=3e-5,
                         log_every=max(1, epochs // 4), log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    doms = lsdf.make_domains(cen, half)
    q = torch.as_tensor(w.q, dtype=torch.float32, device=dev)
    pts = torch.as_tensor(w.points, dtype=torch.float32, device=dev)
    T = lsdf.fk_batch(w.robot.dh, q, base_T=w.robot.base_T)
    ws = torch.zeros(lsdf.query_workspace_size(w.C, w.L, w.M), dtype=torch.uint8, device=dev)
    outg = (torch.empty(w.C, device=dev), torch.empty(w.C, dtype=torch.int32, device=dev), None)
    outm = (torch.empty(w.C, device=dev), torch.empty(w.C, dtype=torch.int32, device=dev), None)
    grid_ms = time_calls(lambda: lsdf.query_min_distance(T, gs, pts, workspace=ws, out=outg), steps * 10, 5)
    mlp_ms = time_calls(lambda: lsdf.query_min_distance_mlp(T, gs, params, doms, pts, margin=0.05, workspace=ws,
                                                            out=outm), steps, 1)
    d_grid = outg[0].cpu().numpy().astype(np.float64)
    d_mlp = outm[0].cpu().numpy().astype(np.float64)
    # judge: exact minimum of grid-in-box / mesh-outside over each link's domain
    sel = np.linspace(0, w.C - 1, judge_waypoints).round().astype(int)
    log(f"learned variant: judging {len(sel)} waypoints with the oracle")
    grids = oracle.workload_grids(w)
    T64 = oracle.fk(w.robot.dh, w.q[sel], w.robot.base_T)
    jcl = oracle.judge_min(T64, w.grid_lo, w.grid_hi, w.grid_n, grids, w.robot.links, cen, half, w.points)
    judge, _ = oracle.reduce(jcl)
    both = np.isfinite(judge) & np.isfinite(d_mlp[sel])
    err = np.abs(d_mlp[sel][both] - judge[both]) * 1e3
    pairs = w.C * w.M * w.L
    return {
        "workload": f"{w.name}: {w.C} waypoints x {w.M} points x {w.L} links, 64^3 FP32 grids, "
                    f"3-128-128-128-1 SiLU network per link (bf16 MFMA, FP32 accumulate), fallback below 5 cm",
        "grid_ms_per_batch": round(grid_ms, 4),
        "mlp_ms_per_batch": round(mlp_ms, 3),
        "grid_gq_s": round(pairs / (grid_ms / 1e3) / 1e9, 2),
        "mlp_gq_s": round(pairs / (mlp_ms / 1e3) / 1e9, 2),
        "judged_waypoints": int(len(sel)),
        "max_err_mm": round(float(err.max()), 3) if err.size else None,
        "mean_err_mm": round(float(err.mean()), 3) if err.size else None,
        "grid_inf_waypoints": int(np.sum(~np.isfinite(d_grid))),
        "mlp_inf_waypoints": int(np.sum(~np.isfinite(d_mlp))),
        "train_s": round(train_s, 1),
        "train_epochs": epochs,
        "train_samples_per_link": n,
        "final_train_l1_mm": [round(1e3 * float(x), 2) for x in hist[-1]],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="paper")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--learned-epochs", type=int, default=400,
                    help="training epochs of the learned variant (0 skips the learned variant)")
    ap.add_argument("--learned-steps", type=int, default=5)
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
    if args.learned_epochs > 0:
        rec["learned"] = learned_variant(dev, args.learned_epochs, args.learned_steps)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
