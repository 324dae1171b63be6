"""Benchmark: ms per 500-waypoint batch and G point-link queries/s.

One step = forward kinematics of every waypoint plus the clearance query
over 500 waypoints x 20,000 obstacle points x 7 links with 64^3 FP32 link
grids, inputs resident in HBM, as one lsdf_query_from_joints call (the
kinematics run in the query's first kernel); the same step as two calls
(lsdf_fk_batch, lsdf_query_min_distance) and as a graph replay is reported
beside it.  Prints one JSON line.  One GPU only.
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
# the same ALUs without packed FP32 (the library is built with it off): 256 CUs x 4 SIMDs x 16 lanes
# x one FMA (2 FLOP) per clock x 2.4 GHz
PEAK_FP32_UNPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
FLOP_PER_TEST = 24                    # map a point or a sphere centre to grid coordinates (9 FMA) + 6 compares
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


def culled_work(T: np.ndarray, lo, hi, points: np.ndarray, block: int = 8):
    """Work of the culled method at waypoint-link granularity, in double
    precision: (sphere tests, pairs in blocks whose sphere reaches the link's
    box, pairs inside the box).  Every (waypoint, link, 8-point block) needs
    one sphere test; a surviving block needs the point test of its points;
    an in-box pair needs the interpolation.  Used only to price the kernel's
    compulsory work for the roofline."""
    P = points.astype(np.float64)
    M = P.shape[0]
    nb = (M + block - 1) // block
    pad = np.concatenate([P, np.repeat(P[-1:], nb * block - M, axis=0)]).reshape(nb, block, 3)
    cnt = np.full(nb, block)
    cnt[-1] = M - (nb - 1) * block
    bmin, bmax = pad.min(axis=1), pad.max(axis=1)
    cen = 0.5 * (bmin + bmax)
    rad = np.sqrt(((pad - cen[:, None, :]) ** 2).sum(-1)).max(axis=1)
    C, L = T.shape[:2]
    tests = C * L * nb
    surv_pairs, inbox = 0, 0
    for i in range(L):
        mid = 0.5 * (lo[i] + hi[i])
        hw = 0.5 * (hi[i] - lo[i])
        R = T[:, i, :, :3].astype(np.float64)
        t = T[:, i, :, 3].astype(np.float64)
        for c0 in range(0, C, 25):
            Rc, tc = R[c0:c0 + 25], t[c0:c0 + 25]
            lc = np.einsum("cba,cjb->cja", Rc, cen[None] - tc[:, None, :])              # [c][block][3]
            surv = np.all(np.abs(lc - mid) <= hw + rad[None, :, None], axis=-1)          # [c][block]
            surv_pairs += int((surv * cnt[None, :]).sum())
            lp = np.einsum("cba,cjb->cja", Rc, P[None] - tc[:, None, :])
            inbox += int(np.all((lp >= lo[i]) & (lp <= hi[i]), axis=-1).sum())
    return tests, surv_pairs, inbox


_ORACLE_GRIDS = {}


def oracle_grids(w):
    """The oracle's double-precision grids of a workload's robot (cached by
    node count: every workload uses the same robot and boxes)."""
    import oracle
    key = int(w.grid_n[0, 0])
    if key not in _ORACLE_GRIDS:
        log(f"oracle grids {key}^3 (double, brute force)")
        _ORACLE_GRIDS[key] = oracle.workload_grids(w)
    return _ORACLE_GRIDS[key]


def cpu_model() -> str:
    """The host CPU's model name (the `model name` line of /proc/cpuinfo,
    which is what lscpu prints)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, budget_s: float = 12.0):
    """The CPU oracle (double-precision kinematics + query) on the same
    workload, repeated for about budget_s seconds on all the host's threads,
    then three batches on one thread (median)."""
    import oracle
    grids = oracle_grids(w)

    def batch():
        t0 = time.perf_counter()
        T = oracle.fk(w.robot.dh, w.q, w.robot.base_T)
        cl = oracle.query_f64(T, w.grid_lo, w.grid_hi, w.grid_n, grids, w.points)
        oracle.reduce(cl)
        return time.perf_counter() - t0

    threads = oracle.max_threads()
    log(f"cpu baseline ({threads} threads)")
    reps, t_total = 0, 0.0
    while t_total < budget_s and reps < 200:
        t_total += batch()
        reps += 1
    sec = t_total / reps
    oracle.set_threads(1)
    one = float(np.median([batch() for _ in range(3)]))
    oracle.set_threads(threads)
    return {"value": round(w.C * w.M * w.L / sec / 1e9, 4), "unit": "G point-link queries/s",
            "ms_per_batch": round(sec * 1e3, 3), "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
            "host_cpus": os.cpu_count(),
            "sample": f"full {w.name} batch (C={w.C}, M={w.M}, L={w.L}) repeated {reps}x; "
                      "double-precision kinematics + query, OpenMP over waypoints",
            "single_thread": {"ms_per_batch": round(one * 1e3, 3),
                              "value": round(w.C * w.M * w.L / one / 1e9, 4), "sample": "median of 3 full batches"}}


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


def dense_cloud(w, M: int, seed: int = 71) -> np.ndarray:
    """M points packed inside the links' boxes along the path: each is a
    uniform point of link i's grid box placed with link i's pose at a random
    waypoint, so nearly every 8-point block reaches some waypoint's box (the
    case of an obstacle right against the arm)."""
    import oracle
    rng = np.random.default_rng(seed)
    T = oracle.fk(w.robot.dh, w.q, w.robot.base_T)
    c = rng.integers(0, w.C, M)
    i = rng.integers(0, w.L, M)
    lo, hi = w.grid_lo.astype(np.float64)[i], w.grid_hi.astype(np.float64)[i]
    loc = rng.uniform(lo, hi)
    R, t = T[c, i, :, :3], T[c, i, :, 3]
    return (np.einsum("mab,mb->ma", R, loc) + t).astype(np.float32).astype(np.float64)


def scene_line(dev, w, label: str, steps: int, warmup: int):
    """A non-headline workload timed like the headline one: the prepared
    fused step (wall time over K steps), its device time, the query kernel
    alone (events), and the kernel's roofline fraction from the culled
    method's algorithmic work."""
    import torch

    from paper_2309_12543_amd import lsdf

    gs = lsdf.build_robot_grids(w.robot.links, w.grid_lo, w.grid_hi, w.grid_n, device=dev)
    q = torch.as_tensor(w.q, dtype=torch.float32, device=dev)
    pts = torch.as_tensor(w.points, dtype=torch.float32, device=dev)
    T = torch.empty((w.C, w.L, 3, 4), dtype=torch.float32, device=dev)
    call = lsdf.PreparedQueryFromJoints(w.robot.dh, q, gs, pts, base_T=w.robot.base_T, link_T=T)
    ms = time_calls(call, steps, warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda._sleep(int(2.4e9 * 0.02))
    e0.record()
    for _ in range(steps):
        call()
    e1.record()
    torch.cuda.synchronize()
    gpu_ms = e0.elapsed_time(e1) / steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record()
        b.record()
    for a, b in ev:
        lsdf.set_kernel_events(a, b)
        call()
    torch.cuda.synchronize()
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    tests, surv, inbox = culled_work(T.cpu().numpy(), w.grid_lo.astype(np.float64), w.grid_hi.astype(np.float64),
                                     w.points)
    flop = FLOP_PER_TEST * (tests + surv) + FLOP_PER_INBOX_PAIR * inbox
    achieved = flop / (kernel_ms / 1e3) / 1e12
    pairs = w.C * w.M * w.L
    return {"workload": label, "ms_per_step": round(ms, 5), "gpu_ms_per_step": round(gpu_ms, 5),
            "value": round(pairs / (ms / 1e3) / 1e9, 2), "unit": "G point-link queries/s",
            "query_kernel_ms": round(kernel_ms, 5), "inbox_pair_fraction": round(inbox / pairs, 5),
            "sphere_survivor_pair_fraction": round(surv / pairs, 5),
            "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_VECTOR_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4),
                         "algorithmic_flop": flop,
                         "inbox_pair_corner_tb_per_s": round(BYTES_PER_INBOX_PAIR * inbox / (kernel_ms / 1e3) / 1e12,
                                                             4)}}


def extra_scenes(dev, steps: int, warmup: int):
    """The tiny workload (50 waypoints x 2,000 points uniform in a 2 m cube,
    32^3 grids) and a dense cloud at the paper size (500 x 20,000, every
    point packed inside some link's box along the path)."""
    import synth
    out = {}
    t = synth.make_workload("tiny")
    log("extra scene: tiny")
    out["tiny"] = scene_line(dev, t, f"tiny: {t.C} waypoints x {t.M} points uniform in a 2 m cube x {t.L} links, "
                                     f"32^3 FP32 grids", steps, warmup)
    w = synth.make_workload("paper")
    w.points = dense_cloud(w, w.M)
    log("extra scene: dense cloud")
    out["dense"] = scene_line(dev, w, f"dense: {w.C} waypoints x {w.M} points packed in the links' boxes along "
                                      f"the path x {w.L} links, 64^3 FP32 grids", steps, warmup)
    return out


def learned_variant(dev, steps: int, epochs=None, judge_waypoints: int = 50):
    """The learned form on the 500 x 100,000 x 7 workload (64^3 grids): per-link
    networks trained on the GPU (untimed; the library's recipe, or with
    ``epochs`` only that many epochs of its first phase, for profiling runs),
    then the grid-only query and the
    network-plus-fallback query timed on the same inputs, and the learned
    clearances judged against the oracle's exact minimum on sampled waypoints."""
    import torch

    import oracle
    import synth
    from paper_2309_12543_amd import learned, lsdf

    w = synth.make_workload("learned")
    log(f"learned variant: C={w.C} M={w.M} L={w.L}, training "
        + ("with the library's recipe" if epochs is None else f"{epochs} epochs (profiling run)"))
    gs = lsdf.build_robot_grids(w.robot.links, w.grid_lo, w.grid_hi, w.grid_n, device=dev)
    cen, half = synth.mlp_domain(w.grid_lo.astype(np.float64), w.grid_hi.astype(np.float64))
    core = synth.mlp_core(w.grid_lo, w.grid_hi)
    n = 1 << 20
    S = torch.as_tensor(np.stack([synth.mlp_samples(m, w.grid_lo[i], w.grid_hi[i], n, synth.BASE_SEED + 4 + i)
                                  for i, m in enumerate(w.robot.links)]).astype(np.float32), device=dev)
    t0 = time.perf_counter()
    labels = learned.labels_for_samples(w.robot.links, gs, S)
    bound = learned.remainder_bounds((cen, half, core), S, labels)
    params = torch.as_tensor(synth.mlp_init(w.L, synth.BASE_SEED + 5).astype(np.float32), device=dev)
    if epochs is None:
        hist = learned.fit(params, (cen, half, core, bound), S, labels, log_every=400, log=log)
    else:
        hist = learned.train(params, (cen, half, core, bound), S, labels, epochs=epochs, batch=learned.BATCH,
                             lr=learned.LR, lr_final=learned.LR_FINAL)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    doms = lsdf.make_domains(cen, half, core, bound)
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
    # per-link minima too (same calls, with link_dist), for the far-field judge
    lg = lsdf.query_min_distance(T, gs, pts, workspace=ws, link_dist=True)[2].cpu().numpy().astype(np.float64)
    lm = lsdf.query_min_distance_mlp(T, gs, params, doms, pts, margin=0.05, workspace=ws,
                                     link_dist=True)[2].cpu().numpy().astype(np.float64)
    # judge: exact minimum of grid-in-box / mesh-outside over each link's domain
    sel = np.linspace(0, w.C - 1, judge_waypoints).round().astype(int)
    log(f"learned variant: judging {len(sel)} waypoints with the oracle")
    grids = oracle_grids(w)
    T64 = oracle.fk(w.robot.dh, w.q[sel], w.robot.base_T)
    jcl = oracle.judge_min(T64, w.grid_lo, w.grid_hi, w.grid_n, grids, w.robot.links, cen, half, w.points)
    judge, _ = oracle.reduce(jcl)
    both = np.isfinite(judge) & np.isfinite(d_mlp[sel])
    err = np.abs(d_mlp[sel][both] - judge[both]) * 1e3
    # the moving links 1-6 (link 0 stands 4 cm from the table at every
    # waypoint, so the grid fallback decides every whole-robot clearance)
    g6, m6, j6 = lg[sel][:, 1:], lm[sel][:, 1:], jcl[:, 1:]
    far = ~np.isfinite(g6) & np.isfinite(j6)
    near = np.isfinite(g6) & np.isfinite(j6)
    ef = np.abs(m6[far] - j6[far]) * 1e3
    en = np.abs(m6[near] - j6[near]) * 1e3
    eg = np.abs(g6[near] - j6[near]) * 1e3
    gw, mw, jw = g6.min(1), m6.min(1), j6.min(1)
    farw = ~np.isfinite(gw) & np.isfinite(jw)
    ew = np.abs(mw[farw] - jw[farw]) * 1e3
    pairs = w.C * w.M * w.L

    def stats(e):
        return {"max_mm": round(float(e.max()), 3), "mean_mm": round(float(e.mean()), 3),
                "p99_mm": round(float(np.percentile(e, 99)), 3)} if e.size else None
    return {
        "workload": f"{w.name}: {w.C} waypoints x {w.M} points x {w.L} links, 64^3 FP32 grids, "
                    f"3-128-128-128-1 SiLU network per link (bf16 MFMA, FP32 accumulate), its share bounded, plus the "
                    f"distance to the link's core box; tiles that cannot hold a minimum skipped; fallback below 5 cm",
        "grid_ms_per_batch": round(grid_ms, 4),
        "mlp_ms_per_batch": round(mlp_ms, 3),
        "grid_gq_s": round(pairs / (grid_ms / 1e3) / 1e9, 2),
        "mlp_gq_s": round(pairs / (mlp_ms / 1e3) / 1e9, 2),
        "judged_waypoints": int(len(sel)),
        "max_err_mm": round(float(err.max()), 3) if err.size else None,
        "mean_err_mm": round(float(err.mean()), 3) if err.size else None,
        "whole_robot_note": "every whole-robot clearance here is the base link's 4 cm to the table, which the "
                            "grid fallback gives exactly",
        "far_field_links_1_6": {
            "link_minima_judged": int(g6.size),
            "grid_inf_exact_finite": int(far.sum()),
            "network_finite_there": int(np.isfinite(m6[far]).sum()),
            "exact_range_m": [round(float(j6[far].min()), 4), round(float(j6[far].max()), 4)] if far.any() else None,
            "network_error": stats(ef),
            "meets_1mm": bool(ef.size and ef.max() <= 1.0),
            "waypoints_without_grid_answer": int(farw.sum()),
            "waypoint_network_error": stats(ew)},
        "inside_capture_range_links_1_6": {"link_minima": int(near.sum()), "learned_error": stats(en),
                                           "grid_error": stats(eg)},
        "grid_inf_waypoints": int(np.sum(~np.isfinite(d_grid))),
        "mlp_inf_waypoints": int(np.sum(~np.isfinite(d_mlp))),
        "train_s": round(train_s, 1),
        "train_recipe": ({"batch": learned.BATCH, "epochs": learned.EPOCHS, "lr": [learned.LR, learned.LR_FINAL],
                          "mining_rounds": [{"lr": lr, "epochs": e} for lr, e in learned.MINE_ROUNDS],
                          "mined_fraction": learned.MINE_FRACTION, "mined_repeat": learned.MINE_REPEAT,
                          "epochs_total": int(len(hist))} if epochs is None else
                         f"profiling run: {epochs} epochs of the first phase only (accuracy figures not the recipe's)"),
        "train_samples_per_link": n,
        "remainder_bounds_m": [round(float(b), 3) for b in bound],
        "final_train_l1_mm": [round(1e3 * float(x), 2) for x in hist[-1]],
        **learned_pair_stats(w, T, pts, params, cen, half, core, bound, margin=0.05),
    }


def learned_pair_stats(w, T, pts, params, cen, half, core, bound, margin: float, sample: int = 1 << 20,
                       seed: int = 7):
    """On a seeded sample of (waypoint, point) pairs per link: the fraction
    inside the network's domain, and among those the fraction whose estimate
    falls below the margin (the pairs that take the exact grid value when
    their point is in the grid box)."""
    import torch

    from paper_2309_12543_amd import lsdf

    gen = torch.Generator().manual_seed(seed)
    ci = torch.randint(0, w.C, (sample,), generator=gen).to(pts.device)
    ji = torch.randint(0, w.M, (sample,), generator=gen).to(pts.device)
    x = pts[ji]
    n_dom = n_fb = 0
    for i in range(w.L):
        R = T[ci, i, :, :3]
        d = x - T[ci, i, :, 3]
        lp = (R * d[:, :, None]).sum(dim=1)          # R^T (x - t)
        c = torch.as_tensor(cen[i], dtype=torch.float32, device=pts.device)
        h = torch.as_tensor(half[i], dtype=torch.float32, device=pts.device)
        inside = ((lp - c).abs() <= h).all(dim=1)
        lpi = lp[inside].contiguous()
        n_dom += int(lpi.shape[0])
        if lpi.shape[0]:
            m = lsdf.mlp_eval(params[i].contiguous(), (cen[i:i + 1], half[i:i + 1], core[i:i + 1], bound[i]), lpi)
            n_fb += int((m < margin).sum().item())
    return {"pair_sample_per_link": sample,
            "in_domain_pair_fraction": round(n_dom / (sample * w.L), 4),
            "fallback_fraction_of_in_domain": round(n_fb / max(1, n_dom), 5)}


def gather_roof(dev, iters: int = 64, reps: int = 5):
    """Sustained rate of trilinear-style gathers (8 corners of a random cell)
    from an FP32 grid that fits one XCD's L2 (64^3, 1 MB), one the size of
    the seven link grids (121^3, 7.1 MB) and one only HBM holds (645^3,
    1.07 GB): cells per second and the 32 B of corners per cell."""
    import torch

    from paper_2309_12543_amd import lsdf

    threads = 256 * 8 * 256
    res = {}
    for name, n in (("l2_1mb", 64), ("grids_7mb", 121), ("hbm_1gb", 645)):
        g = torch.rand(n ** 3, dtype=torch.float32, device=dev)
        out = torch.empty(threads, dtype=torch.float32, device=dev)
        ms = time_calls(lambda: lsdf.gather_roof(g, n, iters, threads, out=out), reps, 2)
        cells = threads * iters
        res[name] = {"n": n, "ms": round(ms, 4), "g_cells_per_s": round(cells / (ms / 1e3) / 1e9, 2),
                     "corner_tb_per_s": round(32 * cells / (ms / 1e3) / 1e12, 3)}
        del g, out
    return res


def precision_variant(dev, steps: int, judge_waypoints: int = 16):
    """128^3 grids stored as FP32, bfloat16 and binary16 on the 500 x 100,000
    x 7 workload: time per batch and the per-waypoint clearance error against
    the double-precision oracle (its own grids, kinematics and query) on
    sampled waypoints."""
    import torch

    import oracle
    import synth
    from paper_2309_12543_amd import lsdf

    w = synth.make_workload("precision")
    log(f"precision variant: C={w.C} M={w.M} L={w.L} n={int(w.grid_n[0, 0])}")
    q = torch.as_tensor(w.q, dtype=torch.float32, device=dev)
    pts = torch.as_tensor(w.points, dtype=torch.float32, device=dev)
    T = lsdf.fk_batch(w.robot.dh, q, base_T=w.robot.base_T)
    ws = torch.zeros(lsdf.query_workspace_size(w.C, w.L, w.M), dtype=torch.uint8, device=dev)
    sel = np.linspace(0, w.C - 1, judge_waypoints).round().astype(int)
    grids = oracle_grids(w)
    T64 = oracle.fk(w.robot.dh, w.q[sel], w.robot.base_T)
    ref, _ = oracle.reduce(oracle.query_f64(T64, w.grid_lo, w.grid_hi, w.grid_n, grids, w.points))
    out = {"workload": f"{w.name}: {w.C} waypoints x {w.M} points x {w.L} links, {int(w.grid_n[0, 0])}^3 grids",
           "judged_waypoints": int(len(sel))}
    for name, tdt in (("f32", torch.float32), ("bf16", torch.bfloat16), ("f16", torch.float16)):
        gs = lsdf.build_robot_grids(w.robot.links, w.grid_lo, w.grid_hi, w.grid_n, device=dev, dtype=tdt)
        res = (torch.empty(w.C, device=dev), torch.empty(w.C, dtype=torch.int32, device=dev), None)
        ms = time_calls(lambda: lsdf.query_min_distance(T, gs, pts, workspace=ws, out=res), steps, 5)
        d = res[0].cpu().numpy().astype(np.float64)[sel]
        both = np.isfinite(d) & np.isfinite(ref)
        err = np.abs(d[both] - ref[both]) * 1e3
        out[name] = {"query_ms": round(ms, 4), "grid_mb": round(gs.buf.numel() * gs.buf.element_size() / 1e6, 2),
                     "max_err_mm": round(float(err.max()), 4) if err.size else None,
                     "mean_err_mm": round(float(err.mean()), 4) if err.size else None,
                     "finite_pattern_equal": bool(np.array_equal(np.isfinite(d), np.isfinite(ref)))}
        del gs
    return out


def batched_variant(dev, steps: int, warmup: int):
    """64 re-planned trajectories, each against its own cloud (50-1,000
    waypoints and 5,000-200,000 points per trajectory, 64^3 FP32 grids), in
    one batched call: the tiling picked by the autotuner, then the step
    (kinematics of every waypoint + the batched query) timed eagerly and as a
    graph replay, and the query kernel alone."""
    import torch

    import synth
    from paper_2309_12543_amd import lsdf
    from paper_2309_12543_amd.step_graph import StepGraph

    t0 = time.perf_counter()
    w = synth.make_batched()
    log(f"batched variant: K={w.K} sum C={w.C} sum M={w.M} ({time.perf_counter() - t0:.1f} s to generate)")
    gs = lsdf.build_robot_grids(w.robot.links, w.grid_lo, w.grid_hi, w.grid_n, device=dev)
    q = torch.as_tensor(w.q, dtype=torch.float32, device=dev)
    pts = torch.as_tensor(w.points, dtype=torch.float32, device=dev)
    co = torch.as_tensor(w.c_off, dtype=torch.int32, device=dev)
    mo = torch.as_tensor(w.m_off, dtype=torch.int64, device=dev)
    T = lsdf.fk_batch(w.robot.dh, q, base_T=w.robot.base_T)
    ws = torch.zeros(lsdf.query_batched_workspace_size(w.K, w.C, w.L, w.M), dtype=torch.uint8, device=dev)
    best, best_ms, _ = lsdf.query_autotune(T, gs, pts, co, mo, reps=5, workspace=ws)
    log(f"batched variant: autotuner picked {best} ({best_ms:.3f} ms per call)")
    res = {}
    for name, tun in (("default", None), ("tuned", best)):
        out = (torch.empty(w.C, device=dev), torch.empty(w.C, dtype=torch.int32, device=dev), None)
        kev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for a, b in kev:
            a.record()
            b.record()
        it = iter(range(10 ** 9))

        def one(timed):
            if timed:
                lsdf.set_kernel_events(*kev[next(it)])
            lsdf.query_from_joints(w.robot.dh, q, gs, pts, base_T=w.robot.base_T, c_offsets=co, m_offsets=mo,
                                   link_T=T, tuning=tun, workspace=ws, out=out)

        for _ in range(warmup):
            one(False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            one(False)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t1) * 1e3 / steps
        for _ in range(steps):       # instrumented pass: events around the query kernel
            one(True)
        torch.cuda.synchronize()
        kms = float(np.mean([a.elapsed_time(b) for a, b in kev]))
        res[name] = {"ms_per_step": round(ms, 4), "query_kernel_ms": round(kms, 4), "out": out}
    sg = StepGraph(w.robot.dh, w.robot.base_T, gs, w.C, w.M, w.K, tuning=best)
    sg.load(q, pts, co, mo)
    graph_ms = time_calls(sg.replay, steps, warmup)
    d_t, l_t, _ = res["tuned"]["out"]
    d_d, l_d, _ = res["default"]["out"]
    same = bool(torch.equal(sg.dist.view(torch.int32), d_t.view(torch.int32)) and torch.equal(sg.link, l_t)
                and torch.equal(d_d.view(torch.int32), d_t.view(torch.int32)) and torch.equal(l_d, l_t))
    pairs = w.pairs()
    for r in res.values():
        r.pop("out")
    return {
        "workload": f"batched: {w.K} trajectories, waypoints U{{50..1000}} (sum {w.C}), points U{{5000..200000}} "
                    f"(sum {w.M}), {w.L} links, 64^3 FP32 grids, own scene per trajectory",
        "pairs": pairs,
        "autotuned": {"chunk_points": best.chunk_points, "blocks_per_cu": best.blocks_per_cu,
                      "autotune_ms_per_call": round(best_ms, 4)},
        "default": res["default"],
        "tuned": res["tuned"],
        "graph_replay_ms_per_step": round(graph_ms, 4),
        "gq_s_tuned_eager": round(pairs / (res["tuned"]["ms_per_step"] / 1e3) / 1e9, 1),
        "gq_s_graph": round(pairs / (graph_ms / 1e3) / 1e9, 1),
        "results_identical_across_tilings_and_graph": same,
    }


def robot_sdf_variant(dev, steps: int, judge_waypoints: int = 16):
    """The paper's own pipeline on the same 500 x 20,000 x 7 workload: Robot
    SDFs of every waypoint over a 4 m environment of 3.125 cm voxels (the
    preparation), then the gather-only runtime; against the per-point query
    on time, memory and error (both judged against the double-precision
    oracle at the points on sampled waypoints)."""
    import torch

    import oracle
    import synth
    from paper_2309_12543_amd import lsdf

    w = synth.make_workload("paper")
    lo, r, n = (-2.0, -2.0, -2.0), 1.0 / 32.0, (128, 128, 128)
    env = lsdf.make_env(lo, r, n)
    log(f"robot-sdf variant: C={w.C} env {n} voxels of {r * 100:.3f} cm")
    gs = lsdf.build_robot_grids(w.robot.links, w.grid_lo, w.grid_hi, w.grid_n, device=dev)
    q = torch.as_tensor(w.q, dtype=torch.float32, device=dev)
    pts = torch.as_tensor(w.points, dtype=torch.float32, device=dev)
    T = lsdf.fk_batch(w.robot.dh, q, base_T=w.robot.base_T)
    rs = torch.empty((w.C, n[2], n[1], n[0]), dtype=torch.float32, device=dev)
    build_ms = time_calls(lambda: lsdf.robot_sdf_build(T, gs, env, out=rs), max(3, steps // 10), 1)
    d_rs = torch.empty(w.C, dtype=torch.float32, device=dev)
    run_ms = time_calls(lambda: lsdf.robot_sdf_query(rs, env, pts, out=d_rs), steps, 5)
    d_q, _ = lsdf.query_min_distance(T, gs, pts)
    torch.cuda.synchronize()
    sel = np.linspace(0, w.C - 1, judge_waypoints).round().astype(int)
    grids = oracle_grids(w)
    T64 = oracle.fk(w.robot.dh, w.q[sel], w.robot.base_T)
    ref, _ = oracle.reduce(oracle.query_f64(T64, w.grid_lo, w.grid_hi, w.grid_n, grids, w.points))
    a = d_rs.cpu().numpy().astype(np.float64)[sel]
    b = d_q.cpu().numpy().astype(np.float64)[sel]
    ok = np.isfinite(ref) & np.isfinite(a) & np.isfinite(b)
    e_rs, e_q = np.abs(a[ok] - ref[ok]) * 1e3, np.abs(b[ok] - ref[ok]) * 1e3
    flat = np.floor((w.points - np.array(lo)) / r).astype(np.int64)
    occ = len(np.unique((flat[:, 2] * n[1] + flat[:, 1]) * n[0] + flat[:, 0]))
    out = {
        "workload": f"paper: {w.C} waypoints x {w.M} points x {w.L} links; environment {n[0]}^3 voxels of "
                    f"{r * 100:.3f} cm over a 4 m cube",
        "prep_ms_robot_sdf_build": round(build_ms, 3),
        "runtime_ms_gather": round(run_ms, 4),
        "robot_sdf_gb": round(rs.numel() * 4 / 1e9, 3),
        "occupied_voxels": occ,
        "judged_waypoints": int(ok.sum()),
        "max_err_mm_robot_sdf": round(float(e_rs.max()), 3) if e_rs.size else None,
        "mean_err_mm_robot_sdf": round(float(e_rs.mean()), 3) if e_rs.size else None,
        "max_err_mm_per_point_query": round(float(e_q.max()), 5) if e_q.size else None,
        "discretisation_bound_mm": round(0.5 * np.sqrt(3) * r * 1e3, 2),
    }
    del rs
    torch.cuda.empty_cache()
    return out


def random_rotations_dev(n: int, gen, dev):
    """Uniform random rotations [n][3][3] on the device (unit quaternions)."""
    import torch
    q = torch.randn((n, 4), generator=gen, device=dev, dtype=torch.float64)
    q = q / q.norm(dim=1, keepdim=True)
    w, x, y, z = q.unbind(1)
    R = torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        torch.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        torch.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1)], 1)
    return R.to(torch.float32).contiguous()


def frnn_variant(dev, train_steps: int, test_rotations: int):
    """The paper's tiny network for the grid transformation (Sec. III-B-1):
    trained on random rotations with the L1 loss and Adam, its maximum error
    over random rotations, and the Robot SDFs of the 500-waypoint workload
    built through it against the exact build (time and difference)."""
    import math

    import torch

    import synth
    from paper_2309_12543_amd import lsdf

    w = synth.make_workload("paper")
    lo, r, n = (-2.0, -2.0, -2.0), 1.0 / 32.0, (128, 128, 128)
    far = max(math.sqrt(max(sum((w.grid_hi[i, a] if (k >> a) & 1 else w.grid_lo[i, a]) ** 2 for a in range(3))
                            for k in range(8))) for i in range(w.L))
    m = int(math.ceil(far / r)) + 2
    npar = lsdf.frnn_nparam(m)
    log(f"frnn variant: block half-width m={m} ({(2 * m) ** 3} voxels, {npar} parameters), {train_steps} steps")
    gen = torch.Generator(device=dev)
    gen.manual_seed(synth.BASE_SEED + 7)
    # uniform +-1/sqrt(fan_in) initialisation of both layers
    fan = np.concatenate([np.full(32 * 9 + 32, 1 / 3.0), np.full(npar - 32 * 10, 1 / math.sqrt(32.0))])
    P = ((torch.rand(npar, generator=gen, device=dev, dtype=torch.float32) * 2 - 1) *
         torch.as_tensor(fan, dtype=torch.float32, device=dev)).contiguous()
    mm, vv = torch.zeros_like(P), torch.zeros_like(P)
    grad = torch.empty_like(P)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    lr0, lr1 = 1e-2, 1e-5
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Rall = random_rotations_dev(64 * train_steps, gen, dev)      # every step's batch, drawn at once
    for t in range(1, train_steps + 1):
        lr = lr1 + 0.5 * (lr0 - lr1) * (1 + math.cos(math.pi * t / train_steps))
        lsdf.frnn_train_step(P, m, Rall[64 * (t - 1):64 * t], adam=(mm, vv), t=t, lr=lr, grad=grad, loss=loss)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del Rall
    Rt = random_rotations_dev(test_rotations, gen, dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    err = float(lsdf.frnn_max_error(P, m, Rt).item())
    eval_s = time.perf_counter() - t0
    env = lsdf.make_env(lo, r, n)
    gs = lsdf.build_robot_grids(w.robot.links, w.grid_lo, w.grid_hi, w.grid_n, device=dev)
    q = torch.as_tensor(w.q, dtype=torch.float32, device=dev)
    T = lsdf.fk_batch(w.robot.dh, q, base_T=w.robot.base_T)
    Csub = 100
    rs_exact = lsdf.robot_sdf_build(T[:Csub].contiguous(), gs, env)
    rs_nn = torch.empty_like(rs_exact)
    nn_ms = time_calls(lambda: lsdf.robot_sdf_build_frnn(T[:Csub].contiguous(), gs, env, P, m, out=rs_nn), 3, 1)
    ex_ms = time_calls(lambda: lsdf.robot_sdf_build(T[:Csub].contiguous(), gs, env, out=rs_exact), 3, 1)
    both = torch.isfinite(rs_exact) & torch.isfinite(rs_nn)
    ad = (rs_exact[both] - rs_nn[both]).abs()
    diff = float(ad.max().item()) if ad.numel() else None
    # a voxel centre within the network's error of a link box's face can fall
    # inside the box in one build and outside in the other: the voxel then
    # takes another link's value (or +inf), a jump of centimetres that says
    # nothing about the transform's accuracy; so the share of voxels that
    # differ is reported beside the maximum
    n_both = int(ad.numel())
    over_01mm = int((ad > 1e-4).sum().item())
    over_1mm = int((ad > 1e-3).sum().item())
    del ad
    mismatch = int((torch.isfinite(rs_exact) != torch.isfinite(rs_nn)).sum().item())
    del rs_exact, rs_nn
    torch.cuda.empty_cache()
    return {
        "network": f"9-32-{3 * (2 * m) ** 3} ReLU, block half-width {m} voxels of {r * 100:.3f} cm (e_r = {m * r:.3f} m)",
        "train_steps": train_steps, "batch": 64, "lr": "Adam, cosine 1e-2 -> 1e-5", "train_s": round(train_s, 2),
        "final_l1": float(loss.item()),
        "test_rotations": test_rotations, "max_error_normalised": err, "max_error_mm": round(err * m * r * 1e3, 3),
        "max_error_eval_s": round(eval_s, 2),
        "robot_sdf_build_ms_100_waypoints": {"network": round(nn_ms, 3), "exact": round(ex_ms, 3)},
        "robot_sdf_max_abs_diff_mm": round(diff * 1e3, 3) if diff is not None else None,
        "robot_sdf_voxels_finite_in_both": n_both,
        "robot_sdf_voxels_differing_over_0.1mm": over_01mm,
        "robot_sdf_voxels_differing_over_1mm": over_1mm,
        "robot_sdf_finite_pattern_mismatches": mismatch,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="paper")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--learned-epochs", type=int, default=None,
                    help="train only this many epochs of the recipe's first phase (profiling runs); 0 skips the "
                         "learned variant; default: the library's recipe (about 90 s)")
    ap.add_argument("--learned-steps", type=int, default=5)
    ap.add_argument("--no-precision", action="store_true", help="skip the 128^3 bf16/fp16 storage variant")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-trajectory batched variant")
    ap.add_argument("--no-extra-scenes", action="store_true", help="skip the tiny and dense-cloud lines")
    ap.add_argument("--no-robot-sdf", action="store_true", help="skip the paper's Robot-SDF pipeline comparator")
    ap.add_argument("--frnn-steps", type=int, default=10000,
                    help="training steps of the grid-transformation network (0 skips that variant)")
    ap.add_argument("--frnn-rotations", type=int, default=100000,
                    help="random rotations of its max-error test (the paper uses 10^7)")
    ap.add_argument("--only", choices=["learned", "scenes", "precision", "batched", "robot-sdf", "frnn"], default=None,
                    help="run only this variant (for profiling) and print its record as one JSON line")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB mebibytes (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the clearance query is measured on a single MI355X "
              "(sharding waypoints over GPUs is designed, not built); use --gpus 1", file=sys.stderr)
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
    if args.only:
        only = {"learned": lambda: learned_variant(dev, args.learned_steps, args.learned_epochs),
                "scenes": lambda: extra_scenes(dev, 50, 5),
                "precision": lambda: precision_variant(dev, 50),
                "batched": lambda: batched_variant(dev, 20, 3),
                "robot-sdf": lambda: robot_sdf_variant(dev, 50),
                "frnn": lambda: frnn_variant(dev, args.frnn_steps, args.frnn_rotations)}
        print(json.dumps({"variant": args.only, **only[args.only]()}), flush=True)
        return
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

    # per step: events around the query call, and events the library records
    # around the query kernel alone (lsdf_set_kernel_events)
    call_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
    kern_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(2 * args.steps)]
    for a, b in call_ev + kern_ev:      # create the events before handing them to the library
        a.record()
        b.record()

    # The timed steps carry no events: an event recorded between two kernels
    # of the step adds a few µs to it.  Separate instrumented passes record
    # events around the query call and around the query kernel alone.
    def step_separate(k=None, instrument=False):
        # lsdf_fk_batch, then lsdf_query_min_distance
        lsdf.fk_batch(w.robot.dh, q, base_T=w.robot.base_T, out=T)
        if instrument and k is not None:
            call_ev[k][0].record()
            lsdf.set_kernel_events(*kern_ev[k])
        lsdf.query_min_distance(T, gs, pts, workspace=ws, out=(dist, link, None))
        if instrument and k is not None:
            call_ev[k][1].record()

    # lsdf_query_from_joints: the kinematics inside the query's first kernel,
    # its arguments marshalled once (a control loop refills q and the points
    # in place), so that a step costs the host one ctypes call
    fused_call = lsdf.PreparedQueryFromJoints(w.robot.dh, q, gs, pts, base_T=w.robot.base_T, link_T=T,
                                              workspace=ws, out=(dist, link, None))

    def step_fused(k=None, instrument=False):
        if instrument and k is not None:
            lsdf.set_kernel_events(*kern_ev[args.steps + k])
        fused_call()

    def step_wrapper(k=None):
        # the same call through the convenience wrapper, which checks and
        # marshals every argument on every call
        lsdf.query_from_joints(w.robot.dh, q, gs, pts, base_T=w.robot.base_T, link_T=T, workspace=ws,
                               out=(dist, link, None))

    def run(step):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            step(k)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps

    def gpu_only(step):
        # device time per step: the steps are queued behind a 20 ms sleep
        # kernel, so the GPU runs them back to back whatever the host's pace
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda._sleep(int(2.4e9 * 0.02))
        e0.record()
        for _ in range(args.steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    log(f"timing {args.steps} steps (separate calls, then the fused call)")
    sep_ms = run(step_separate)
    d_sep, l_sep = dist.clone(), link.clone()
    ms_per_step = run(step_fused)
    fused_same = bool(torch.equal(dist.view(torch.int32), d_sep.view(torch.int32)) and torch.equal(link, l_sep))
    wrapper_ms = run(step_wrapper)
    gpu_fused_ms = gpu_only(step_fused)
    gpu_sep_ms = gpu_only(step_separate)
    log("instrumented passes (events around the query call and kernel)")
    sep_ev_ms = run(lambda k=None: step_separate(k, instrument=True))
    fused_ev_ms = run(lambda k=None: step_fused(k, instrument=True))
    call_ms = float(np.mean([a.elapsed_time(b) for a, b in call_ev]))
    kernel_ms_sep = float(np.mean([a.elapsed_time(b) for a, b in kern_ev[:args.steps]]))
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in kern_ev[args.steps:]]))
    pairs = w.C * w.M * w.L
    value = pairs / (ms_per_step / 1e3) / 1e9

    # the same step captured once in a graph and replayed
    from paper_2309_12543_amd.step_graph import StepGraph
    sg = StepGraph(w.robot.dh, w.robot.base_T, gs, w.C, w.M, 1)
    sg.load(q, pts, torch.tensor([0, w.C], dtype=torch.int32, device=dev),
            torch.tensor([0, w.M], dtype=torch.int64, device=dev))
    graph_ms = run(lambda k=None: sg.replay())
    same = bool(torch.equal(sg.dist.view(torch.int32), d_sep.view(torch.int32)) and torch.equal(sg.link, l_sep))
    del sg

    # warm grids, cold points: every step reads its own copy of the cloud,
    # from a pool larger than the Infinity Cache (256 MB), so the points come
    # from HBM while the grids stay cached
    n_cold = max(args.steps + args.warmup, (300 << 20) // (w.M * 12) + 1)
    cold = torch.empty((n_cold, w.M, 3), dtype=torch.float32, device=dev)
    cold[:] = pts
    ck = [0]

    def step_cold():
        lsdf.query_from_joints(w.robot.dh, q, gs, cold[ck[0] % n_cold], base_T=w.robot.base_T, link_T=T,
                               workspace=ws, out=(dist, link, None))
        ck[0] += 1

    cold_ms = run(lambda k=None: step_cold())
    cold_same = bool(torch.equal(dist.view(torch.int32), d_sep.view(torch.int32)))
    del cold
    call_q = np.percentile([a.elapsed_time(b) for a, b in call_ev], [5, 50, 95])
    kern_q = np.percentile([a.elapsed_time(b) for a, b in kern_ev[args.steps:]], [5, 50, 95])

    Tn = T.cpu().numpy()
    tests, surv_pairs, inbox = culled_work(Tn, w.grid_lo.astype(np.float64), w.grid_hi.astype(np.float64), w.points)
    flop = FLOP_PER_TEST * (tests + surv_pairs) + FLOP_PER_INBOX_PAIR * inbox
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
        "step": "lsdf_query_from_joints (arguments marshalled once): kinematics in the query's first kernel, "
                "then the query and finalize kernels",
        "separate_calls_ms_per_step": round(sep_ms, 5),
        "wrapper_call_ms_per_step": round(wrapper_ms, 5),
        "gpu_ms_per_step": {"fused": round(gpu_fused_ms, 5), "separate_calls": round(gpu_sep_ms, 5),
                            "how": "steps queued behind a sleep kernel: device time with no host wait"},
        "instrumented_ms_per_step": {"separate_calls": round(sep_ev_ms, 5), "fused": round(fused_ev_ms, 5)},
        "separate_calls_equal_fused": fused_same,
        "query_call_ms": round(call_ms, 5),
        "query_call_ms_p5_p50_p95": [round(float(v), 5) for v in call_q],
        "query_kernel_ms_p5_p50_p95": [round(float(v), 5) for v in kern_q],
        "cold_points_ms_per_step": round(cold_ms, 5),
        "cold_points_cloud_copies": n_cold,
        "cold_points_equal": cold_same,
        "query_kernel_ms": round(kernel_ms, 5),
        "query_kernel_ms_separate_calls": round(kernel_ms_sep, 5),
        "graph_replay_ms_per_step": round(graph_ms, 5),
        "graph_equals_eager": same,
        "inbox_pair_fraction": round(inbox / pairs, 5),
        "sphere_survivor_pair_fraction": round(surv_pairs / pairs, 5),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4),
                     "traffic": profiled_traffic(os.path.join(ROOT, "paper_2309_12543_amd", "csrc", "query.hip"),
                                                 os.path.join(ROOT, "profiles", "query_kernel_paper.txt")),
                     "kernel": "query_kernel (its own launch, timed by events the library records around it)",
                     "peak_unpacked_fp32": round(PEAK_FP32_UNPACKED_TFLOPS, 1),
                     "frac_of_unpacked_fp32": round(achieved / PEAK_FP32_UNPACKED_TFLOPS, 4),
                     "algorithmic_flop": flop,
                     "work": {"sphere_tests": tests, "point_tests_in_surviving_blocks": surv_pairs,
                              "inbox_pairs": inbox, "flop_per_test": FLOP_PER_TEST,
                              "flop_per_inbox_pair": FLOP_PER_INBOX_PAIR}},
    }
    roof = gather_roof(dev)
    rec["gather_roof"] = roof
    rec["roofline"]["gather"] = {
        "inbox_pair_corner_tb_per_s": round(BYTES_PER_INBOX_PAIR * inbox / (kernel_ms / 1e3) / 1e12, 4),
        "roof_corner_tb_per_s_7mb": roof["grids_7mb"]["corner_tb_per_s"]}
    if not args.no_extra_scenes:
        rec["extra_scenes"] = extra_scenes(dev, 50, 5)
    if args.learned_epochs != 0:
        rec["learned"] = learned_variant(dev, args.learned_steps, args.learned_epochs)
    if not args.no_precision:
        rec["precision"] = precision_variant(dev, 50)
    if not args.no_batched:
        rec["batched"] = batched_variant(dev, 20, 3)
    if not args.no_robot_sdf:
        rec["robot_sdf_pipeline"] = robot_sdf_variant(dev, 50)
        if args.frnn_steps > 0:
            rec["robot_sdf_pipeline"]["grid_transformation_network"] = frnn_variant(dev, args.frnn_steps,
                                                                                    args.frnn_rotations)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
