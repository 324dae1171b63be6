"""GPU parity of the clearance path (fk_batch, build_link_sdf,
query_min_distance) against the CPU oracle, through the C ABI.

* query stage: bit-exact against the oracle's single-precision twin when both
  get the same FP32 poses and grids (out_dist, out_link and the per-link
  minima, +inf patterns included);
* fk_batch: within 5e-6 of the oracle's double-precision kinematics;
* build_link_sdf: within 2e-6 m of the oracle's double-precision grid;
* end to end (GPU kinematics, GPU grids, GPU query) against the all-double
  oracle: every per-link minimum within 1e-5 m of the double one, except
  where a pair proven to lie within the two sides' coordinate difference of
  a box face decides it (then between the double minima with and without
  such pairs); argmin equal outside near-ties.
"""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

TOL_E2E = 1e-5        # metres, FP32 end to end vs the double oracle


def say(*a):
    print("[gpu]", *a, flush=True)


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_12543_amd import lsdf
    lsdf.load_library()
    return lsdf


@pytest.fixture(scope="module")
def paper():
    return synth.make_workload("paper")


@pytest.fixture(scope="module")
def paper_grids(orc, paper):
    return orc.workload_grids(paper)


def upload_grids(B, w, grids64):
    gs = B.GridSet(w.grid_lo, w.grid_hi, w.grid_n, device="cuda")
    for i, g in enumerate(grids64):
        gs.set_grid(i, g.astype(np.float32))
    return gs


def to_dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def run_query(B, T32, gs, pts32, link_dist=True):
    say("query C=%d L=%d M=%d" % (T32.shape[0], T32.shape[1], pts32.shape[0]))
    d, l, ld = B.query_min_distance(to_dev(T32), gs, to_dev(pts32.reshape(-1, 3)), link_dist=True)
    torch.cuda.synchronize()
    return d.cpu().numpy(), l.cpu().numpy(), ld.cpu().numpy()


def twin(orc, w, T32, grids64, pts32):
    cl = orc.query_f32(T32, w.grid_lo, w.grid_hi, w.grid_n, [g.astype(np.float32) for g in grids64], pts32)
    d, l = orc.reduce(cl)
    return d, l, cl


def assert_bit_exact(gpu, ref):
    gd, gl, gld = gpu
    rd, rl, rcl = ref
    assert np.array_equal(gld.view(np.uint32), rcl.view(np.uint32)), \
        f"per-link minima differ at {np.argwhere(gld.view(np.uint32) != rcl.view(np.uint32))[:5]}"
    assert np.array_equal(gd.view(np.uint32), rd.view(np.uint32))
    assert np.array_equal(gl, rl)


# ---------------------------------------------------------------------------
# kinematics
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["tiny", "paper"])
def test_fk_batch_matches_oracle(B, orc, name):
    w = synth.make_workload(name)
    rng = np.random.default_rng(30)
    base = np.concatenate([np.linalg.qr(rng.normal(size=(3, 3)))[0] * [1, 1, 1], rng.normal(size=(3, 1)) * 0.2], 1)
    if np.linalg.det(base[:, :3]) < 0:
        base[:, 0] *= -1
    for b in (None, base):
        say("fk_batch", name, "C=%d" % w.C, "base" if b is not None else "identity")
        T = B.fk_batch(w.robot.dh, to_dev(w.q), base_T=b)
        torch.cuda.synchronize()
        ref = orc.fk(w.robot.dh, w.q, b)
        err = np.abs(T.cpu().numpy().astype(np.float64) - ref)
        assert err[..., 3].max() < 5e-6, err[..., 3].max()      # metres
        assert err[..., :3].max() < 5e-6, err[..., :3].max()    # rotation entries


def test_fk_batch_ragged_and_empty(B, orc, tiny):
    for C in (1, 63, 65, 257):
        q = tiny.q[np.arange(C) % tiny.C]
        T = B.fk_batch(tiny.robot.dh, to_dev(q))
        torch.cuda.synchronize()
        assert np.abs(T.cpu().numpy() - orc.fk(tiny.robot.dh, q)).max() < 5e-6
    T = B.fk_batch(tiny.robot.dh, torch.zeros((0, 6), dtype=torch.float32, device="cuda"))
    assert T.shape == (0, 7, 3, 4)


# ---------------------------------------------------------------------------
# query stage: bit-exact against the single-precision twin
# ---------------------------------------------------------------------------

def test_query_bit_exact_tiny(B, orc, tiny, tiny_grids):
    T32 = orc.fk(tiny.robot.dh, tiny.q, tiny.robot.base_T).astype(np.float32)
    gs = upload_grids(B, tiny, tiny_grids)
    pts = tiny.points.astype(np.float32)
    assert_bit_exact(run_query(B, T32, gs, pts), twin(orc, tiny, T32, tiny_grids, pts))


@pytest.mark.parametrize("C,M", [(37, 5000), (1, 1), (3, 2049), (129, 16385), (5, 0)])
def test_query_bit_exact_ragged(B, orc, tiny, tiny_grids, C, M):
    """Several point tiles with a ragged tail, ragged configuration tiles,
    a single point, and the empty cloud."""
    rng = np.random.default_rng(31 + C)
    q = synth.make_waypoints(tiny.robot.qmin, tiny.robot.qmax, C, 99 + C)
    T32 = orc.fk(tiny.robot.dh, q, tiny.robot.base_T).astype(np.float32)
    # points near the arm, so that most links see some of them
    origins = T32[:, :, :, 3].reshape(-1, 3).astype(np.float64)
    pts = (origins[rng.integers(0, origins.shape[0], M)] + rng.normal(0, 0.15, size=(M, 3))).astype(np.float32)
    gs = upload_grids(B, tiny, tiny_grids)
    gpu = run_query(B, T32, gs, pts)
    ref = twin(orc, tiny, T32, tiny_grids, pts)
    assert_bit_exact(gpu, ref)
    if M == 0:
        assert np.all(gpu[0] == np.inf) and np.all(gpu[1] == -1)
    elif M > 100:
        assert np.isfinite(gpu[2]).mean() > 0.3


def test_query_bit_exact_paper_scale(B, orc, paper, paper_grids):
    """500 waypoints x 20,000 points x 7 links, 64^3 grids: the full size, in
    the launch configuration the benchmark times."""
    T32 = orc.fk(paper.robot.dh, paper.q, paper.robot.base_T).astype(np.float32)
    gs = upload_grids(B, paper, paper_grids)
    pts = paper.points.astype(np.float32)
    gpu = run_query(B, T32, gs, pts)
    ref = twin(orc, paper, T32, paper_grids, pts)
    assert_bit_exact(gpu, ref)
    assert np.isfinite(gpu[0]).mean() > 0.5


def test_query_sixteen_links_and_one_link(B, orc, tiny, tiny_grids):
    T = orc.fk(tiny.robot.dh, tiny.q, tiny.robot.base_T).astype(np.float32)
    pts = tiny.points.astype(np.float32)
    # 16 links: the 7 real ones repeated; ties must resolve to the lowest index
    idx = np.arange(16) % 7
    w16 = synth.Workload("t16", tiny.robot, tiny.q, tiny.points, tiny.grid_lo[idx], tiny.grid_hi[idx],
                         tiny.grid_n[idx], {})
    g16 = [tiny_grids[i] for i in idx]
    gs = upload_grids(B, w16, g16)
    gpu = run_query(B, np.ascontiguousarray(T[:, idx]), gs, pts)
    ref = twin(orc, w16, np.ascontiguousarray(T[:, idx]), g16, pts)
    assert_bit_exact(gpu, ref)
    assert np.all(gpu[1] < 7)
    w1 = synth.Workload("t1", tiny.robot, tiny.q, tiny.points, tiny.grid_lo[3:4], tiny.grid_hi[3:4],
                        tiny.grid_n[3:4], {})
    gs1 = upload_grids(B, w1, tiny_grids[3:4])
    assert_bit_exact(run_query(B, np.ascontiguousarray(T[:, 3:4]), gs1, pts),
                     twin(orc, w1, np.ascontiguousarray(T[:, 3:4]), tiny_grids[3:4], pts))


def test_query_bit_exact_non_cubic_grids(B, orc, tiny):
    """Grids with different node counts per axis take the per-axis box test."""
    n = np.array([[24, 32, 40], [40, 24, 32], [32, 40, 24], [24, 24, 40], [40, 40, 24], [33, 17, 29], [16, 48, 20]],
                 dtype=np.int32)
    w = synth.Workload("nc", tiny.robot, tiny.q, tiny.points, tiny.grid_lo, tiny.grid_hi, n, {})
    grids = [orc.build_grid(m, w.grid_lo[i].astype(np.float64), w.grid_hi[i].astype(np.float64), n[i])
             for i, m in enumerate(w.robot.links)]
    T32 = orc.fk(w.robot.dh, w.q, w.robot.base_T).astype(np.float32)
    gs = upload_grids(B, w, grids)
    pts = w.points.astype(np.float32)
    assert_bit_exact(run_query(B, T32, gs, pts), twin(orc, w, T32, grids, pts))


def test_query_culling_is_exact_on_faces_and_nonrigid_poses(B, orc, tiny, tiny_grids):
    """The block culling must never drop a pair the box test keeps: points
    placed on box faces and corners (then jittered by a few ulps), and poses
    whose rotation part is scaled and sheared, still give the twin's bits."""
    rng = np.random.default_rng(33)
    C = 40
    T = orc.fk(tiny.robot.dh, tiny.q[:C], tiny.robot.base_T)
    A = np.array([[1.3, 0.2, 0.0], [0.0, 0.7, 0.1], [0.05, 0.0, 1.1]])   # not a rotation
    T[: C // 2, :, :, :3] = T[: C // 2, :, :, :3] @ A
    T32 = T.astype(np.float32)
    pts = []
    for c in range(0, C, 3):
        for i in range(tiny.L):
            lo, hi = tiny.grid_lo[i].astype(np.float64), tiny.grid_hi[i].astype(np.float64)
            for _ in range(6):
                l = rng.uniform(lo, hi)
                a = rng.integers(0, 3)
                l[a] = lo[a] if rng.uniform() < 0.5 else hi[a]           # on a face
                if rng.uniform() < 0.3:
                    l = np.where(rng.uniform(size=3) < 0.5, lo, hi)     # a corner
                R, t = T32[c, i, :, :3].astype(np.float64), T32[c, i, :, 3].astype(np.float64)
                x = R @ l + t
                pts.append(x * (1 + rng.integers(-4, 5, size=3) * 2.0 ** -23))
    pts = np.array(pts, dtype=np.float32)
    pts = np.concatenate([pts, tiny.points[:500].astype(np.float32)])
    gs = upload_grids(B, tiny, tiny_grids)
    gpu = run_query(B, T32, gs, pts)
    ref = twin(orc, tiny, T32, tiny_grids, pts)
    assert_bit_exact(gpu, ref)
    assert np.isfinite(gpu[2]).mean() > 0.5


@pytest.mark.parametrize("chunk_points,blocks_per_cu", [(8192, 1), (256, 0), (32, 2)])
def test_query_bit_exact_when_block_lists_fill(B, orc, tiny, tiny_grids, chunk_points, blocks_per_cu):
    """A cloud packed inside the links' boxes makes nearly every block reach
    some lane's box, so each workgroup's list of surviving blocks fills (it
    holds 128) and the waves test the rest of their blocks themselves: both
    paths must give the twin's bits, at every tiling."""
    rng = np.random.default_rng(71)
    C = min(64, len(tiny.q))
    T32 = orc.fk(tiny.robot.dh, tiny.q[:C], tiny.robot.base_T).astype(np.float32)
    pts = []
    for _ in range(8192):
        c, i = rng.integers(0, C), rng.integers(0, tiny.L)
        l = rng.uniform(tiny.grid_lo[i], tiny.grid_hi[i])
        pts.append(T32[c, i, :, :3].astype(np.float64) @ l + T32[c, i, :, 3])
    pts = np.array(pts, dtype=np.float32)
    gs = upload_grids(B, tiny, tiny_grids)
    say(f"full lists: chunk_points={chunk_points} blocks_per_cu={blocks_per_cu} C={C} M={len(pts)}")
    d, l, ld = B.query_min_distance_batched(
        to_dev(T32), gs, to_dev(pts), to_dev([0, C], torch.int32), to_dev([0, len(pts)], torch.int64),
        link_dist=True, tuning=B.make_tuning(chunk_points, blocks_per_cu, 2))
    torch.cuda.synchronize()
    gpu = d.cpu().numpy(), l.cpu().numpy(), ld.cpu().numpy()
    assert_bit_exact(gpu, twin(orc, tiny, T32, tiny_grids, pts))
    assert np.isfinite(gpu[2]).mean() > 0.9


@pytest.mark.parametrize("dt", ["bf16", "f16"])
def test_query_bit_exact_half_storage(B, orc, tiny, tiny_grids, paper, paper_grids, dt):
    """16-bit grids: the kernel widens each corner exactly to FP32, so the
    result equals the twin run on the rounded values, bit for bit."""
    tdt = torch.bfloat16 if dt == "bf16" else torch.float16
    for w, grids in ((tiny, tiny_grids), (paper, paper_grids)):
        T32 = orc.fk(w.robot.dh, w.q, w.robot.base_T).astype(np.float32)
        gs = B.GridSet(w.grid_lo, w.grid_hi, w.grid_n, device="cuda", dtype=tdt)
        for i, g in enumerate(grids):
            gs.set_grid(i, g.astype(np.float32))
        rounded = [gs.grid(i).float().cpu().numpy().astype(np.float64) for i in range(w.L)]
        pts = w.points.astype(np.float32)
        say(f"query {dt} grids, {w.name}")
        assert_bit_exact(run_query(B, T32, gs, pts), twin(orc, w, T32, rounded, pts))


@pytest.mark.parametrize("dt", ["bf16", "f16"])
def test_build_link_sdf_half_storage(B, orc, tiny, tiny_grids, dt):
    """build_link_sdf rounds its FP32 distance once into the storage type:
    within one ulp of the storage format of the oracle's rounded value."""
    tdt = torch.bfloat16 if dt == "bf16" else torch.float16
    u = 2.0 ** -8 if dt == "bf16" else 2.0 ** -11
    gs = B.build_robot_grids(tiny.robot.links, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, dtype=tdt)
    torch.cuda.synchronize()
    for i in range(tiny.L):
        got = gs.grid(i).float().cpu().numpy().astype(np.float64)
        want = torch.tensor(tiny_grids[i].astype(np.float32)).to(tdt).double().numpy()
        assert np.all(np.abs(got - want) <= 2 * u * np.abs(want) + 1e-7), i


def test_query_workspace_reuse_across_shapes(B, orc, tiny, tiny_grids):
    """One workspace serving calls of different sizes, holding random bytes
    before the first call: a call ignores what the workspace holds (the
    first kernel clears the keys), so a later call with more configurations
    reads no stale bytes as keys."""
    gs = upload_grids(B, tiny, tiny_grids)
    rng = np.random.default_rng(34)
    ws = torch.randint(0, 256, (B.query_workspace_size(200, 7, 20000),), dtype=torch.uint8, device="cuda")
    for C, M in ((3, 2049), (129, 16385), (7, 300), (200, 20000)):
        q = synth.make_waypoints(tiny.robot.qmin, tiny.robot.qmax, C, 199 + C)
        T32 = orc.fk(tiny.robot.dh, q, tiny.robot.base_T).astype(np.float32)
        origins = T32[:, :, :, 3].reshape(-1, 3).astype(np.float64)
        pts = (origins[rng.integers(0, origins.shape[0], M)] + rng.normal(0, 0.15, size=(M, 3))).astype(np.float32)
        say(f"shared workspace C={C} M={M}")
        d, l, ld = B.query_min_distance(to_dev(T32), gs, to_dev(pts), link_dist=True, workspace=ws)
        torch.cuda.synchronize()
        assert_bit_exact((d.cpu().numpy(), l.cpu().numpy(), ld.cpu().numpy()), twin(orc, tiny, T32, tiny_grids, pts))


def test_query_workspace_contents_ignored_and_repeatable(B, orc, tiny, tiny_grids):
    T32 = to_dev(orc.fk(tiny.robot.dh, tiny.q, tiny.robot.base_T).astype(np.float32))
    gs = upload_grids(B, tiny, tiny_grids)
    pts = to_dev(tiny.points.astype(np.float32))
    ws = torch.full((B.query_workspace_size(tiny.C, 7, tiny.M),), 0xFF, dtype=torch.uint8, device="cuda")
    say("query repeat x3 with a private workspace, refilled with 0xFF before each call")
    outs = []
    for _ in range(3):
        outs.append(B.query_min_distance(T32, gs, pts, link_dist=True, workspace=ws))
        ws.fill_(0xFF)
    torch.cuda.synchronize()
    for d, l, ld in outs[1:]:
        assert torch.equal(d, outs[0][0]) and torch.equal(l, outs[0][1]) and torch.equal(ld, outs[0][2])
    # permuting the cloud changes nothing, bit for bit
    perm = torch.as_tensor(np.random.default_rng(32).permutation(tiny.M), device="cuda")
    d2, l2, ld2 = B.query_min_distance(T32, gs, pts[perm].contiguous(), link_dist=True, workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(ld2, outs[0][2]) and torch.equal(l2, outs[0][1])


# ---------------------------------------------------------------------------
# grid construction and the whole path
# ---------------------------------------------------------------------------

def test_build_link_sdf_matches_oracle(B, orc, tiny, tiny_grids):
    say("build_link_sdf tiny, 7 links of 32^3")
    gs = B.build_robot_grids(tiny.robot.links, tiny.grid_lo, tiny.grid_hi, tiny.grid_n)
    torch.cuda.synchronize()
    for i in range(tiny.L):
        got = gs.grid(i).cpu().numpy().astype(np.float64)
        err = np.abs(got - tiny_grids[i])
        assert err.max() < 2e-6, (i, err.max())


def _double_intervals(orc, w, grids64, T32, T64, chunk=25):
    """Per (c, i), the interval the FP32 path's per-link minimum must lie in,
    from the double oracle's per-pair dump.  A pair can be in link i's grid
    box on one side and out of it on the other only when its double grid
    coordinates lie within the two sides' coordinate difference of a box
    face.  That difference is bounded per pair by the pose part (the FP32
    poses the GPU computed against the double ones, the link-frame points
    compared exactly in double) plus the rounding bound of the
    single-precision map (r10_bound).  Pairs clear of every face by more
    than that are surely in or surely out; the interval runs from the
    minimum over pairs possibly in the box to the minimum over pairs surely
    in it, each widened by TOL_E2E."""
    import r10_bound as rb
    lo64, hi64 = w.grid_lo.astype(np.float64), w.grid_hi.astype(np.float64)
    invh = (w.grid_n - 1.0) / (hi64 - lo64)
    P = w.points.astype(np.float64)
    C = T64.shape[0]
    lo = np.empty((C, w.L))
    hi = np.empty((C, w.L))
    for c0 in range(0, C, chunk):
        cs = slice(c0, min(C, c0 + chunk))
        u, v = orc.query_f64_each(T64[cs], lo64, hi64, w.grid_n, grids64, P)
        T3 = T32[cs].astype(np.float64)
        T6 = T64[cs]
        l32 = P @ T3[..., :3] - T3[..., 3][:, :, None, :] @ T3[..., :3]      # R^T (x - t), [c][L][M][3]
        l64 = P @ T6[..., :3] - T6[..., 3][:, :, None, :] @ T6[..., :3]
        du = np.abs(l32 - l64) * invh[None, :, None, :] + rb.coord_bound(T3, lo64, hi64, w.grid_n, P)
        slack = rb.face_slack(u, w.grid_n)
        surely = (slack > du).all(-1)
        maybe = (slack >= -du).all(-1)
        lo[cs] = np.where(maybe, v, np.inf).min(-1) - TOL_E2E
        hi[cs] = np.where(surely, v, np.inf).min(-1) + TOL_E2E
    return lo, hi


@pytest.mark.parametrize("name", ["tiny", "paper"])
def test_end_to_end_vs_double_oracle(B, orc, name, tiny_grids, paper_grids):
    """The whole path on the GPU (FP32 kinematics, GPU-built grids, FP32
    query) against the all-double oracle.  Every per-link minimum, at any
    distance, must lie in the interval the oracle's per-pair dump gives it
    (_double_intervals): the only slack beyond TOL_E2E is for pairs proven
    to lie within the two sides' coordinate difference of a box face, and
    the test reports how many minima such pairs widened.  Per waypoint the
    clearance lies between the links' interval ends and the argmin is a link
    whose interval can hold the minimum (the only one, outside near-ties)."""
    w = synth.make_workload(name)
    grids64 = tiny_grids if name == "tiny" else paper_grids
    say("end-to-end", name, "C=%d M=%d" % (w.C, w.M))
    gs = B.build_robot_grids(w.robot.links, w.grid_lo, w.grid_hi, w.grid_n)
    T = B.fk_batch(w.robot.dh, to_dev(w.q), base_T=w.robot.base_T)
    d, l, ld = B.query_min_distance(T, gs, to_dev(w.points), link_dist=True)
    torch.cuda.synchronize()
    d, l, ld = d.cpu().numpy().astype(np.float64), l.cpu().numpy(), ld.cpu().numpy().astype(np.float64)
    T32 = T.cpu().numpy()
    T64 = orc.fk(w.robot.dh, w.q, w.robot.base_T)
    lo, hi = _double_intervals(orc, w, grids64, T32, T64)
    cl = orc.query_f64(T64, w.grid_lo, w.grid_hi, w.grid_n, grids64, w.points)
    bad = ~((ld >= lo) & (ld <= hi))
    assert not bad.any(), [(c, i, ld[c, i], lo[c, i], hi[c, i]) for c, i in np.argwhere(bad)[:5]]
    fin = np.isfinite(cl) & np.isfinite(ld)
    widened = np.isfinite(hi) & (hi - np.where(np.isfinite(lo), lo, hi) > 2 * TOL_E2E + 1e-12) | (np.isinf(hi) & np.isfinite(lo))
    differ = (np.isfinite(cl) != np.isfinite(ld)) | (fin & (np.abs(np.where(fin, ld - cl, 0.0)) > TOL_E2E))
    err = np.abs(ld[fin] - cl[fin])
    say(f"end-to-end: {ld.size} link minima, {np.isfinite(ld).sum()} finite; max |gpu - double| = "
        f"{err.max() if err.size else 0.0:.3g} m; {widened.sum()} intervals widened by near-face pairs, "
        f"{differ.sum()} minima differ from the double one by more than {TOL_E2E} (all inside their intervals)")
    assert differ.sum() <= widened.sum()
    assert widened.sum() <= max(2, 0.01 * ld.size)
    # per waypoint
    assert np.array_equal(d, ld.min(axis=1))
    assert np.all((d >= lo.min(axis=1)) & (d <= hi.min(axis=1)))
    cand = lo <= hi.min(axis=1, keepdims=True)                   # links that can hold the minimum
    fin_c = np.isfinite(d)
    assert np.all(cand[fin_c, l[fin_c]])
    single = fin_c & (cand.sum(axis=1) == 1)
    assert np.array_equal(l[single], np.argmax(cand[single], axis=1))
    say(f"  argmin: {single.sum()} waypoints with one possible link (equal), {(fin_c & ~single).sum()} near-ties")
    assert np.all((l == -1) == ~np.isfinite(d))


def test_prepared_call_matches_the_wrapper(B, orc, tiny, tiny_grids):
    """The prepared fused call (arguments marshalled once) gives the
    convenience wrapper's bits, also after new joint angles and points are
    written into its buffers in place."""
    gs = upload_grids(B, tiny, tiny_grids)
    q = to_dev(tiny.q)
    pts = to_dev(tiny.points)
    T = torch.empty((tiny.C, tiny.L, 3, 4), dtype=torch.float32, device="cuda")
    call = B.PreparedQueryFromJoints(tiny.robot.dh, q, gs, pts, base_T=tiny.robot.base_T, link_T=T,
                                     link_dist=True)
    for k in range(3):
        if k:
            q.copy_(torch.roll(q, 7, 0))
            pts.copy_(torch.roll(pts, 333, 0) * 0.9)
        say(f"prepared call, round {k}")
        call()
        want = B.query_from_joints(tiny.robot.dh, q, gs, pts, base_T=tiny.robot.base_T, link_dist=True)
        torch.cuda.synchronize()
        for a, b in zip((call.dist, call.link, call.link_dist), want):
            assert torch.equal(a.view(torch.int32), b.view(torch.int32)), k
        assert torch.isfinite(call.dist).any()


@pytest.fixture(scope="module")
def precision_ws(orc):
    w = synth.make_workload("precision")
    say("oracle grids 128^3 (double, brute force)")
    return w, orc.workload_grids(w)


@pytest.mark.parametrize("dt", ["f32", "bf16", "f16"])
def test_query_precision_scale_sampled(B, orc, precision_ws, dt):
    """The precision workload at full size (500 waypoints x 100,000 points x
    7 links, 128^3 grids stored as FP32, bfloat16 or binary16) in the launch
    configuration the benchmark times: 16 sampled waypoints bit for bit
    against the single-precision twin on the same rounded grids, and the
    clearance within the storage bound of the double oracle (u times the
    link's largest |node| plus 1e-5 m, u = 2^-8, 2^-11, 0)."""
    w, grids64 = precision_ws
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[dt]
    u = {"f32": 0.0, "bf16": 2.0 ** -8, "f16": 2.0 ** -11}[dt]
    gs = B.GridSet(w.grid_lo, w.grid_hi, w.grid_n, device="cuda", dtype=tdt)
    for i, g in enumerate(grids64):
        gs.set_grid(i, g.astype(np.float32))
    # the twin's grids: the oracle's values rounded on the CPU (FP64 -> FP32 -> storage type, nearest even)
    rounded = [torch.tensor(g.astype(np.float32)).to(tdt).float().numpy().astype(np.float64) for g in grids64]
    T32 = orc.fk(w.robot.dh, w.q, w.robot.base_T).astype(np.float32)
    pts = w.points.astype(np.float32)
    say(f"precision scale {dt}: C={w.C} M={w.M} n=128")
    d, l, ld = B.query_min_distance(to_dev(T32), gs, to_dev(pts), link_dist=True)
    torch.cuda.synchronize()
    d, l, ld = d.cpu().numpy(), l.cpu().numpy(), ld.cpu().numpy()
    sel = np.linspace(0, w.C - 1, 16).round().astype(int)
    ref = twin(orc, w, T32[sel], rounded, pts)
    assert_bit_exact((d[sel], l[sel], ld[sel]), ref)
    assert np.isfinite(d).mean() > 0.5
    # against the double oracle (its own kinematics and grids)
    rd, _ = orc.reduce(orc.query_f64(orc.fk(w.robot.dh, w.q[sel], w.robot.base_T), w.grid_lo, w.grid_hi, w.grid_n,
                                     grids64, w.points))
    fin = np.isfinite(rd) & np.isfinite(d[sel])
    bound = u * max(np.abs(g).max() for g in grids64) + 1e-5
    err = np.abs(d[sel][fin].astype(np.float64) - rd[fin])
    say(f"  {dt}: max |gpu - double| {err.max():.3g} m over {fin.sum()} waypoints (bound {bound:.3g} m)")
    assert err.max() <= bound
