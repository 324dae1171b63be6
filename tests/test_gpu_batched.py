"""GPU parity of the batched clearance query (many trajectories, each a path
against its own cloud, in one call) through the C ABI.

* bit-exact against the oracle's single-precision twin run trajectory by
  trajectory, with ragged sizes, empty trajectories and point ranges that
  start and end inside 8-point blocks;
* bit-exact against the plain query called once per trajectory;
* every tiling (chunk size, workgroups per CU) gives the same bits;
* offset tables out of order or out of range are clamped as documented;
* a planning step captured in a graph gives the eager step's bits on every
  replay, with new inputs loaded between replays;
* the autotuner returns one of its candidates and the problem's results;
* at the full batched size (64 trajectories, 50-1000 configurations and
  5,000-200,000 points each, 64^3 grids), sampled configurations match the
  twin bit for bit.
"""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-batched]", *a, flush=True)


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_12543_amd import lsdf
    lsdf.load_library()
    return lsdf


def to_dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def upload_grids(B, w, grids64):
    gs = B.GridSet(w.grid_lo, w.grid_hi, w.grid_n, device="cuda")
    for i, g in enumerate(grids64):
        gs.set_grid(i, g.astype(np.float32))
    return gs


@pytest.fixture(scope="module")
def small():
    """7 trajectories of the tiny robot (32^3 grids): 0-150 configurations and
    0-2,500 points each, with trajectory 2 given no points and trajectory 4
    no configurations."""
    w = synth.make_batched(K=7, C_range=(1, 150), M_range=(1, 2500), n=32)
    Cs, Ms = np.diff(w.c_off), np.diff(w.m_off)
    Ms[2] = 0
    Cs[4] = 0
    keep_q = np.concatenate([np.arange(w.c_off[k], w.c_off[k] + Cs[k]) for k in range(w.K)])
    keep_p = np.concatenate([np.arange(w.m_off[k], w.m_off[k] + Ms[k]) for k in range(w.K)])
    w.q, w.points = w.q[keep_q], w.points[keep_p]
    w.c_off = np.concatenate([[0], np.cumsum(Cs)]).astype(np.int64)
    w.m_off = np.concatenate([[0], np.cumsum(Ms)]).astype(np.int64)
    assert any(w.m_off[1:] % 8 != 0)
    return w


def poses32(orc, w):
    return orc.fk(w.robot.dh, w.q, w.robot.base_T).astype(np.float32)


def gpu_batched(B, T32, gs, pts32, c_off, m_off, tuning=None):
    say(f"batched K={len(c_off) - 1} C={T32.shape[0]} M={pts32.shape[0]} tuning={tuning}")
    d, l, ld = B.query_min_distance_batched(to_dev(T32), gs, to_dev(pts32.reshape(-1, 3)),
                                            to_dev(c_off, torch.int32), to_dev(m_off, torch.int64),
                                            link_dist=True, tuning=tuning)
    torch.cuda.synchronize()
    return d.cpu().numpy(), l.cpu().numpy(), ld.cpu().numpy()


def twin_batched(orc, w, T32, grids64, pts32, c_off, m_off):
    g32 = [g.astype(np.float32) for g in grids64]
    cl = orc.query_batched(orc.query_f32, T32, w.grid_lo, w.grid_hi, w.grid_n, g32, pts32, c_off, m_off)
    cl = cl.astype(np.float32)
    d, l = orc.reduce(cl)
    return d, l, cl


def assert_bit_exact(gpu, ref):
    gd, gl, gld = gpu
    rd, rl, rcl = ref
    assert np.array_equal(gld.view(np.uint32), rcl.view(np.uint32)), \
        f"per-link minima differ at {np.argwhere(gld.view(np.uint32) != rcl.view(np.uint32))[:5]}"
    assert np.array_equal(gd.view(np.uint32), rd.astype(np.float32).view(np.uint32))
    assert np.array_equal(gl, rl)


def test_batched_bit_exact_vs_twin(B, orc, small, tiny_grids):
    T32 = poses32(orc, small)
    pts = small.points.astype(np.float32)
    gs = upload_grids(B, small, tiny_grids)
    got = gpu_batched(B, T32, gs, pts, small.c_off, small.m_off)
    ref = twin_batched(orc, small, T32, tiny_grids, pts, small.c_off, small.m_off)
    assert_bit_exact(got, ref)
    d = got[0]
    # trajectory 2 has no points: +inf and -1 for all of its configurations
    c0, c1 = small.c_off[2], small.c_off[3]
    assert c1 > c0 and np.all(np.isinf(d[c0:c1])) and np.all(got[1][c0:c1] == -1)
    assert np.isfinite(d).sum() > 50


def test_batched_equals_plain_per_trajectory(B, orc, small, tiny_grids):
    T32 = poses32(orc, small)
    pts = small.points.astype(np.float32)
    gs = upload_grids(B, small, tiny_grids)
    bd, bl, bld = gpu_batched(B, T32, gs, pts, small.c_off, small.m_off)
    for k in range(small.K):
        c0, c1, m0, m1 = small.c_off[k], small.c_off[k + 1], small.m_off[k], small.m_off[k + 1]
        if c1 == c0:
            continue
        say(f"plain trajectory {k}: C={c1 - c0} M={m1 - m0}")
        d, l, ld = B.query_min_distance(to_dev(T32[c0:c1]), gs, to_dev(pts[m0:m1].reshape(-1, 3)), link_dist=True)
        torch.cuda.synchronize()
        assert np.array_equal(ld.cpu().numpy().view(np.uint32), bld[c0:c1].view(np.uint32))
        assert np.array_equal(d.cpu().numpy().view(np.uint32), bd[c0:c1].view(np.uint32))
        assert np.array_equal(l.cpu().numpy(), bl[c0:c1])


@pytest.mark.parametrize("chunk,bpc,sched", [(8, 8, 1), (24, 3, 2), (64, 1, 1), (1024, 16, 2), (8192, 2, 1),
                                             (40, 8, 2), (520, 8, 2), (128, 5, 1)])
def test_tiling_does_not_change_bits(B, orc, small, tiny_grids, chunk, bpc, sched):
    """Chunk size, workgroups per CU and schedule change no result bit."""
    T32 = poses32(orc, small)
    pts = small.points.astype(np.float32)
    gs = upload_grids(B, small, tiny_grids)
    ref = gpu_batched(B, T32, gs, pts, small.c_off, small.m_off)
    got = gpu_batched(B, T32, gs, pts, small.c_off, small.m_off, tuning=B.make_tuning(chunk, bpc, sched))
    for a, b in zip(got, ref):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_bad_offsets_are_clamped(B, orc, small, tiny_grids):
    """Offsets out of order, negative or beyond C / M: the device clamps each
    trajectory's range (documented); the results follow the clamped ranges,
    configurations covered twice take the smaller minimum."""
    T32 = poses32(orc, small)
    pts = small.points.astype(np.float32)
    C, M = T32.shape[0], pts.shape[0]
    c_off = np.array([-5, 40, 20, 90, C + 1000, 60, C], dtype=np.int64)
    m_off = np.array([3, 1000, 500, -7, M + 10 ** 9, 2000, 4000], dtype=np.int64)
    gs = upload_grids(B, small, tiny_grids)
    got = gpu_batched(B, T32, gs, pts, c_off, m_off)
    ref = twin_batched(orc, small, T32, tiny_grids, pts, c_off, m_off)
    assert_bit_exact(got, ref)


@pytest.mark.parametrize("fused", [True, False])
def test_step_graph_replays_match_eager(B, orc, small, tiny_grids, fused):
    """FK + batched query captured once; each replay after loading a new
    batch (fewer trajectories, other sizes) gives the eager step's bits."""
    from paper_2309_12543_amd.step_graph import StepGraph
    gs = upload_grids(B, small, tiny_grids)
    dh, base = small.robot.dh, small.robot.base_T
    C_cap, M_cap, K_cap = small.C + 7, small.M + 5, small.K + 2
    say(f"capture StepGraph C_cap={C_cap} M_cap={M_cap} K_cap={K_cap}")
    g = StepGraph(dh, base, gs, C_cap, M_cap, K_cap, link_dist=True, fused=fused)
    batches = [(small.c_off, small.m_off, small.C, small.M)]
    # a second batch: the first 4 trajectories with the last one's points trimmed
    c2 = small.c_off[:5].copy()
    m2 = small.m_off[:5].copy()
    m2[-1] -= 3
    batches.append((c2, m2, int(c2[-1]), int(m2[-1])))
    # a third: a single trajectory of everything
    batches.append((np.array([0, small.C]), np.array([0, small.M]), small.C, small.M))
    q32 = small.q.astype(np.float32)
    pts = small.points.astype(np.float32)
    for rep, (c_off, m_off, C, M) in enumerate(batches * 2):
        q_d, p_d = to_dev(q32[:C]), to_dev(pts[:M])
        co, mo = to_dev(c_off, torch.int32), to_dev(m_off, torch.int64)
        g.load(q_d, p_d, co, mo)
        say(f"replay {rep}: K={len(c_off) - 1} C={C} M={M}")
        d, l, ld = g.replay()
        torch.cuda.synchronize()
        got = (d[:C].cpu().numpy(), l[:C].cpu().numpy(), ld[:C].cpu().numpy())
        # eager: the same calls outside the graph
        T = B.fk_batch(dh, q_d, base)
        ref = B.query_min_distance_batched(T, gs, p_d, co, mo, link_dist=True)
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert np.array_equal(a.view(np.uint32), b.cpu().numpy().view(np.uint32)), f"replay {rep}"
        # rows past the batch are empty
        assert torch.all(torch.isinf(d[C:])) and torch.all(l[C:] == -1)


@pytest.mark.parametrize("batched", [False, True])
def test_query_from_joints_equals_separate_calls(B, orc, small, tiny_grids, batched):
    """Kinematics inside the query's first kernel: the poses it stores and
    the clearances are the bits of lsdf_fk_batch followed by the query."""
    gs = upload_grids(B, small, tiny_grids)
    q = to_dev(small.q.astype(np.float32))
    pts = to_dev(small.points.astype(np.float32))
    dh, base = small.robot.dh, small.robot.base_T
    kw = {}
    if batched:
        kw = dict(c_offsets=to_dev(small.c_off, torch.int32), m_offsets=to_dev(small.m_off, torch.int64))
    say(f"query_from_joints batched={batched} C={small.C} M={small.M}")
    T_ref = B.fk_batch(dh, q, base)
    if batched:
        ref = B.query_min_distance_batched(T_ref, gs, pts, kw["c_offsets"], kw["m_offsets"], link_dist=True)
    else:
        ref = B.query_min_distance(T_ref, gs, pts, link_dist=True)
    T_out = torch.full_like(T_ref, float("nan"))
    got = B.query_from_joints(dh, q, gs, pts, base_T=base, link_T=T_out, link_dist=True, **kw)
    got2 = B.query_from_joints(dh, q, gs, pts, base_T=base, link_dist=True, **kw)     # no pose output
    torch.cuda.synchronize()
    assert torch.equal(T_out.view(torch.int32), T_ref.view(torch.int32))
    for a, b, c in zip(got, ref, got2):
        assert torch.equal(a.view(torch.int32), b.view(torch.int32))
        assert torch.equal(c.view(torch.int32), b.view(torch.int32))


def test_autotune_returns_a_candidate(B, orc, small, tiny_grids):
    T32 = poses32(orc, small)
    pts = small.points.astype(np.float32)
    gs = upload_grids(B, small, tiny_grids)
    cands = [(64, 8, 1), (128, 8, 2), (512, 4, 2)]
    say("autotune over 3 candidates")
    best, ms, (d, l) = B.query_autotune(to_dev(T32), gs, to_dev(pts), to_dev(small.c_off, torch.int32),
                                        to_dev(small.m_off, torch.int64), candidates=cands, reps=3)
    torch.cuda.synchronize()
    assert best.as_tuple() in cands and ms > 0
    ref = twin_batched(orc, small, T32, tiny_grids, pts, small.c_off, small.m_off)
    assert np.array_equal(d.cpu().numpy().view(np.uint32), ref[0].astype(np.float32).view(np.uint32))
    assert np.array_equal(l.cpu().numpy(), ref[1])
    say(f"autotune: best {best} at {ms:.4f} ms")


@pytest.fixture(scope="module")
def full_batch():
    say("generating the full batched workload (64 trajectories)")
    return synth.make_batched()


@pytest.fixture(scope="module")
def grids64(orc):
    say("oracle grids 64^3")
    return orc.workload_grids(synth.make_workload("paper"))


def test_full_batch_sampled_configurations(B, orc, full_batch, grids64):
    w = full_batch
    assert w.K == 64 and w.grid_n[0, 0] == 64
    T32 = poses32(orc, w)
    pts = w.points.astype(np.float32)
    gs = upload_grids(B, w, grids64)
    d, l, ld = gpu_batched(B, T32, gs, pts, w.c_off, w.m_off)
    rng = np.random.default_rng(71)
    g32 = [g.astype(np.float32) for g in grids64]
    checked = 0
    for k in rng.choice(w.K, size=8, replace=False):
        c0, c1, m0, m1 = w.c_off[k], w.c_off[k + 1], w.m_off[k], w.m_off[k + 1]
        cs = np.sort(rng.choice(np.arange(c0, c1), size=3, replace=False))
        cl = orc.query_f32(T32[cs], w.grid_lo, w.grid_hi, w.grid_n, g32, pts[m0:m1])
        rd, rl = orc.reduce(cl)
        assert np.array_equal(ld[cs].view(np.uint32), cl.view(np.uint32)), (k, cs)
        assert np.array_equal(d[cs].view(np.uint32), rd.astype(np.float32).view(np.uint32))
        assert np.array_equal(l[cs], rl)
        checked += 3
    say(f"full batch: {checked} sampled configurations bit-exact; finite {np.isfinite(d).mean():.3f}")
