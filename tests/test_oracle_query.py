"""Pins of the oracle's grid sampling and query (paper Sec. III-A).

* An affine field is reproduced exactly by trilinear interpolation, so a grid
  holding n.x - c must return n.l - c at every in-box point l; gradients that
  differ per axis and unequal node counts catch axis or index mix-ups.
* Grid nodes return their stored value.
* Trilinear interpolation agrees with scipy's regular-grid linear
  interpolator (an independent library routine for the same definition).
* The interpolated SDF stays within half a cell diagonal of the exact mesh
  distance (the |r_r|/2 discretisation bound of Sec. III-B).
* The whole query is invariant under a rigid motion of the scene, and the
  min-reductions are unchanged by permuting, duplicating, adding far points
  or splitting the cloud.
"""
import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator


def affine_grid(lo, hi, n, grad, c0):
    xs = [np.linspace(lo[a], hi[a], n[a]) for a in range(3)]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    return grad[0] * X + grad[1] * Y + grad[2] * Z - c0


IDENT = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)


def one_pose(R=np.eye(3), t=np.zeros(3)):
    return np.concatenate([R, t[:, None]], axis=1)[None, None]   # [1][1][3][4]


def rand_rot(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q @ np.diag(np.sign(np.diag(r)))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def test_affine_field_exact_f64(orc):
    lo, hi, n = np.array([-0.3, -0.2, -0.1]), np.array([0.2, 0.4, 0.3]), np.array([9, 13, 6])
    grad, c0 = np.array([0.3, -0.7, 0.5]), 0.05
    G = affine_grid(lo, hi, n, grad, c0)
    rng = np.random.default_rng(10)
    R, t = rand_rot(rng), rng.normal(size=3) * 0.3
    L = rng.uniform(lo, hi, size=(200, 3))           # link-frame points
    P = L @ R.T + t                                     # world points
    for j in range(0, 200, 7):
        cl = orc.query_f64(one_pose(R, t), lo[None], hi[None], n[None], [G], P[j:j + 1])
        assert cl[0, 0] == pytest.approx(L[j] @ grad - c0, abs=1e-12)


def test_affine_field_f32_within_rounding(orc):
    lo = np.array([-0.3, -0.2, -0.1], np.float32)
    hi = np.array([0.2, 0.4, 0.3], np.float32)
    n = np.array([9, 13, 6])
    grad, c0 = np.array([0.3, -0.7, 0.5]), 0.05
    G = affine_grid(lo.astype(np.float64), hi.astype(np.float64), n, grad, c0)
    rng = np.random.default_rng(11)
    L = rng.uniform(lo, hi, size=(300, 3)).astype(np.float32)
    vals = []
    for j in range(300):
        cl = orc.query_f32(one_pose().astype(np.float32), lo[None], hi[None], n[None],
                           [G.astype(np.float32)], L[j:j + 1])
        vals.append(cl[0, 0])
    want = L.astype(np.float64) @ grad - c0
    # node rounding (1/2 ulp), coordinate rounding (a few ulp of u times the
    # cell slope) and 7 lerps: well inside 2e-6 for |values| < 0.5
    assert np.max(np.abs(np.array(vals, np.float64) - want)) < 2e-6


def test_nodes_return_stored_values(orc):
    # power-of-two spacing: node coordinates are exact in both precisions
    lo, n = np.array([-0.5, -0.25, -1.0]), np.array([5, 9, 17])
    h = np.array([0.25, 0.0625, 0.125])
    hi = lo + h * (n - 1)
    rng = np.random.default_rng(12)
    G = rng.normal(size=(n[2], n[1], n[0]))
    ks = np.stack([rng.integers(0, n[a], size=60) for a in range(3)], axis=1)
    ks[:3] = n - 1                                          # the far corner is a node too
    for k in ks:
        p = lo + k * h
        cl = orc.query_f64(one_pose(), lo[None], hi[None], n[None], [G], p[None])
        assert cl[0, 0] == G[k[2], k[1], k[0]]
        cl32 = orc.query_f32(one_pose().astype(np.float32), lo[None].astype(np.float32),
                             hi[None].astype(np.float32), n[None], [G.astype(np.float32)],
                             p[None].astype(np.float32))
        assert cl32[0, 0] == np.float32(G[k[2], k[1], k[0]]) + np.float32(0.0)


def test_trilinear_matches_scipy(orc):
    rng = np.random.default_rng(13)
    n = np.array([7, 5, 11])
    G = rng.normal(size=(n[2], n[1], n[0]))
    interp = RegularGridInterpolator((np.arange(n[2]), np.arange(n[1]), np.arange(n[0])), G)
    for _ in range(200):
        u = rng.uniform(0, n - 1)
        assert orc.trilinear_f64(G, u) == pytest.approx(float(interp([u[2], u[1], u[0]])[0]), abs=1e-13)


def test_outside_box_is_infinite_and_faces_are_inside(orc):
    lo, hi, n = np.array([0.0, 0, 0]), np.array([1.0, 1, 1]), np.array([3, 3, 3])
    G = np.ones((3, 3, 3))
    pts = np.array([[1.0, 1.0, 1.0], [0.0, 0.5, 1.0]])
    cl = orc.query_f64(one_pose(), lo[None], hi[None], n[None], [G], pts)
    assert cl[0, 0] == 1.0
    for p in ([1.0 + 1e-9, 0.5, 0.5], [0.5, -1e-9, 0.5], [0.5, 0.5, 2.0]):
        cl = orc.query_f64(one_pose(), lo[None], hi[None], n[None], [G], np.array([p]))
        assert cl[0, 0] == np.inf
    cl = orc.query_f64(one_pose(), lo[None], hi[None], n[None], [G], np.zeros((0, 3)))
    assert cl[0, 0] == np.inf
    d, link = orc.reduce(cl)
    assert d[0] == np.inf and link[0] == -1


def test_grid_within_half_cell_diagonal(orc, tiny, tiny_grids):
    rng = np.random.default_rng(14)
    for i in (1, 3, 5):
        m = tiny.robot.links[i]
        lo, hi, n = tiny.grid_lo[i].astype(np.float64), tiny.grid_hi[i].astype(np.float64), tiny.grid_n[i]
        h = (hi - lo) / (n - 1)
        L = rng.uniform(lo, hi, size=(150, 3))
        exact = orc.mesh_sdf(L, m.verts, m.tris, m.comp_first)
        got = np.array([orc.query_f64(one_pose(), lo[None], hi[None], n[None], [tiny_grids[i]], L[j:j + 1])[0, 0]
                        for j in range(L.shape[0])])
        assert np.all(np.abs(got - exact) <= orc.grid_bound(h) + 1e-12)


def world_query(orc, w, grids, T, pts):
    return orc.query_f64(T, w.grid_lo, w.grid_hi, w.grid_n, grids, pts)


def test_rigid_motion_invariance(orc, tiny, tiny_grids):
    rng = np.random.default_rng(15)
    q = tiny.q[:6]
    pts = tiny.points[:500]
    T = orc.fk(tiny.robot.dh, q, tiny.robot.base_T)
    ref = world_query(orc, tiny, tiny_grids, T, pts)
    R, t = rand_rot(rng), rng.normal(size=3)
    base = np.concatenate([R, t[:, None]], axis=1)
    T2 = orc.fk(tiny.robot.dh, q, base)
    got = world_query(orc, tiny, tiny_grids, T2, pts @ R.T + t)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(got))
    assert np.max(np.abs(got[fin] - ref[fin])) < 1e-9
    assert fin.sum() > 10


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_reduction_properties_bit_identical(orc, tiny, tiny_grids, prec):
    rng = np.random.default_rng(16)
    q = tiny.q[::10]
    pts = tiny.points[:600]
    T = orc.fk(tiny.robot.dh, q, tiny.robot.base_T)
    if prec == "f64":
        run = lambda P: orc.query_f64(T, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, tiny_grids, P)
    else:
        g32 = [g.astype(np.float32) for g in tiny_grids]
        run = lambda P: orc.query_f32(T.astype(np.float32), tiny.grid_lo, tiny.grid_hi, tiny.grid_n,
                                      g32, P.astype(np.float32))
    ref = run(pts)
    assert np.array_equal(run(pts[rng.permutation(600)]), ref)                  # permutation
    assert np.array_equal(run(np.concatenate([pts, pts[:100]])), ref)         # duplicates
    far = rng.uniform(50, 60, size=(50, 3))
    assert np.array_equal(run(np.concatenate([far, pts])), ref)               # far points
    split = np.minimum(run(pts[:250]), run(pts[250:]))                          # split and min
    assert np.array_equal(split, ref)


def test_reduce_ties_lowest_link(orc):
    cl = np.array([[3.0, 1.0, 1.0, 2.0], [np.inf, np.inf, np.inf, np.inf], [0.5, 0.7, 0.5, 0.5]])
    d, link = orc.reduce(cl)
    assert list(link) == [1, -1, 0] and d[0] == 1.0 and d[1] == np.inf
    d32, link32 = orc.reduce(cl.astype(np.float32))
    assert list(link32) == [1, -1, 0]


def test_grid_vs_exact_mesh_distance_tiny(orc, tiny, tiny_grids):
    """Brute force on a tiny input: the per-waypoint clearance from the grids
    is within half a cell diagonal of the exact mesh distance, wherever the
    clearance is below the box padding (beyond it a point may lie outside
    every box and count as +inf by construction)."""
    q = tiny.q[:5]
    T = orc.fk(tiny.robot.dh, q, tiny.robot.base_T)
    # 50 points scattered around the link origins, so that most clearances are small
    rng = np.random.default_rng(17)
    origins = T[:, :, :, 3].reshape(-1, 3)
    pts = origins[rng.integers(0, origins.shape[0], 50)] + rng.normal(0, 0.08, size=(50, 3))
    grid_cl = world_query(orc, tiny, tiny_grids, T, pts)
    exact_cl = orc.exact_min(T, tiny.robot.links, pts)
    h = (tiny.grid_hi.astype(np.float64) - tiny.grid_lo) / (tiny.grid_n - 1)
    bound = max(orc.grid_bound(hh) for hh in h)
    dg, _ = orc.reduce(grid_cl)
    de, _ = orc.reduce(exact_cl)
    checked = 0
    for c in range(5):
        if de[c] < 0.05 - bound:
            assert abs(dg[c] - de[c]) <= bound + 1e-12
            checked += 1
    assert checked >= 3
    # per link as well: an in-box link minimum is within the bound of the exact one
    fin = np.isfinite(grid_cl) & (exact_cl < 0.05 - bound)
    assert np.all(np.abs(grid_cl[fin] - exact_cl[fin]) <= bound + 1e-12)


def test_f32_twin_close_to_f64(orc, tiny, tiny_grids):
    T = orc.fk(tiny.robot.dh, tiny.q, tiny.robot.base_T)
    T32 = T.astype(np.float32)
    cl64 = orc.query_f64(T32.astype(np.float64), tiny.grid_lo, tiny.grid_hi, tiny.grid_n, tiny_grids,
                         tiny.points)
    cl32 = orc.query_f32(T32, tiny.grid_lo, tiny.grid_hi, tiny.grid_n,
                         [g.astype(np.float32) for g in tiny_grids], tiny.points)
    both = np.isfinite(cl64) & np.isfinite(cl32)
    assert both.mean() > 0.99
    assert np.max(np.abs(cl64[both] - cl32[both])) < 1e-6


def test_judge_min_against_brute_force(orc, tiny, tiny_grids):
    """The pruned judge equals the unpruned definition: grid values for the
    points in each box, exact mesh distances for the others (inside the
    network domain)."""
    import synth
    q = tiny.q[:3]
    T = orc.fk(tiny.robot.dh, q, tiny.robot.base_T)
    rng = np.random.default_rng(18)
    origins = T[:, :, :, 3].reshape(-1, 3)
    pts = np.concatenate([origins[rng.integers(0, origins.shape[0], 60)] + rng.normal(0, 0.15, size=(60, 3)),
                          rng.uniform(-1.5, 1.5, size=(60, 3))])
    dc, dh = synth.mlp_domain(tiny.grid_lo.astype(np.float64), tiny.grid_hi.astype(np.float64), far=0.4)
    got = orc.judge_min(T, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, tiny_grids, tiny.robot.links, dc, dh, pts)
    grid_cl = orc.query_f64(T, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, tiny_grids, pts)
    want = np.full_like(got, np.inf)
    for c in range(T.shape[0]):
        for i in range(tiny.L):
            R, t = T[c, i, :, :3], T[c, i, :, 3]
            loc = (pts - t) @ R
            indom = np.all(np.abs((loc - dc[i]) / dh[i]) <= 1.0, axis=1)
            for j in np.flatnonzero(indom):
                v = orc.query_f64(T[c:c + 1, i:i + 1], tiny.grid_lo[i:i + 1], tiny.grid_hi[i:i + 1],
                                  tiny.grid_n[i:i + 1], [tiny_grids[i]], pts[j:j + 1])[0, 0]
                if not np.isfinite(v):
                    m = tiny.robot.links[i]
                    v = orc.mesh_sdf(loc[j:j + 1], m.verts, m.tris, m.comp_first)[0]
                want[c, i] = min(want[c, i], v)
    assert np.array_equal(np.isfinite(got), np.isfinite(want))
    fin = np.isfinite(got)
    assert np.max(np.abs(got[fin] - want[fin])) < 1e-12
    assert (got[fin] < grid_cl[fin]).any() or np.isinf(grid_cl).any()   # some minima come from outside a box


@pytest.mark.parametrize("dt,u", [("bf16", 2.0 ** -8), ("f16", 2.0 ** -11)])
def test_half_storage_error_bound(orc, tiny, tiny_grids, dt, u):
    """Rounding the stored node values to a 16-bit format moves each node by
    at most u |v| (u = 2^-8 for bfloat16, 2^-11 for binary16); trilinear
    interpolation is a convex combination of 8 nodes, so every per-link
    minimum moves by at most u times the largest |node| of its link (plus
    the FP32 rounding of the interpolation itself)."""
    import torch
    tdt = torch.bfloat16 if dt == "bf16" else torch.float16
    g32 = [g.astype(np.float32) for g in tiny_grids]
    gq = [torch.tensor(g).to(tdt).float().numpy() for g in g32]
    T32 = orc.fk(tiny.robot.dh, tiny.q, tiny.robot.base_T).astype(np.float32)
    a = orc.query_f32(T32, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, g32, tiny.points)
    b = orc.query_f32(T32, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, gq, tiny.points)
    assert np.array_equal(np.isfinite(a), np.isfinite(b))
    fin = np.isfinite(a)
    bound = np.array([u * np.abs(g).max() for g in g32])[None, :].repeat(a.shape[0], 0)
    assert np.all(np.abs(a - b)[fin] <= bound[fin] * (1 + 1e-3) + 4e-7)
    assert np.abs(a - b)[fin].max() > 0       # the rounding is visible


def test_batched_is_per_configuration_min_over_covering_trajectories(orc, tiny, tiny_grids):
    """The batched oracle against the definition taken configuration by
    configuration: each configuration's per-link minima are one plain query
    over the union of the points of every trajectory whose clamped range
    covers it (+inf when none does).  Offsets include an unsorted pair, a
    negative entry, entries past C and M, and overlapping ranges."""
    g32 = [g.astype(np.float32) for g in tiny_grids]
    T = orc.fk(tiny.robot.dh, tiny.q[:30], tiny.robot.base_T).astype(np.float32)
    pts = tiny.points[:900].astype(np.float32)
    C, M = T.shape[0], pts.shape[0]
    c_off = [-3, 8, 5, 14, 40, 22, 27]
    m_off = [0, 300, 1200, 100, 650, -1, 899]
    got = orc.query_batched(orc.query_f32, T, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, g32, pts, c_off, m_off)
    ranges = []
    for k in range(len(c_off) - 1):
        c0 = min(max(c_off[k], 0), C)
        c1 = min(max(c_off[k + 1], c0), C)
        m0 = min(max(m_off[k], 0), M)
        m1 = min(max(m_off[k + 1], m0), M)
        ranges.append((c0, c1, m0, m1))
    assert ranges[1] == (8, 8, 300, 900) and ranges[4] == (30, 30, 650, 650)
    covered = 0
    for c in range(C):
        idx = [np.arange(m0, m1) for (c0, c1, m0, m1) in ranges if c0 <= c < c1]
        idx = np.unique(np.concatenate(idx)) if idx else np.zeros(0, int)
        if idx.size == 0:
            assert np.all(np.isinf(got[c]))
            continue
        covered += 1
        want = orc.query_f32(T[c:c + 1], tiny.grid_lo, tiny.grid_hi, tiny.grid_n, g32, pts[idx])[0]
        assert np.array_equal(got[c].astype(np.float32).view(np.uint32), want.view(np.uint32)), c
    assert covered >= 20 and np.isfinite(got).any()


def test_twin_within_rounding_bound_of_double_per_pair(orc, paper, paper_grids):
    """The single-precision twin against the double definition of Sec. III-A,
    pair by pair on the paper workload (20 of its 500 configurations, every
    link and point), with the same FP32 poses and FP32 grids on both sides so
    that only the arithmetic differs.  Every pair the twin keeps lies within
    the rounding bound of its operation order (tests/r10_bound.py) of the
    double value; a pair kept by one side only lies within the coordinate
    bound of a box face.  A transposed rotation in the twin's input moves the
    values far outside that bound, so the bound has teeth."""
    import r10_bound as rb
    w = paper
    sel = np.arange(0, w.C, 25)
    T32 = orc.fk(w.robot.dh, w.q[sel], w.robot.base_T).astype(np.float32)
    T64 = T32.astype(np.float64)
    g32 = [g.astype(np.float32) for g in paper_grids]
    g64 = [g.astype(np.float64) for g in g32]
    lo, hi = w.grid_lo.astype(np.float64), w.grid_hi.astype(np.float64)
    pts = w.points.astype(np.float32)
    v32 = orc.query_f32_each(T32, w.grid_lo, w.grid_hi, w.grid_n, g32, pts).astype(np.float64)
    u64, v64 = orc.query_f64_each(T64, lo, hi, w.grid_n, g64, pts.astype(np.float64))
    du = rb.coord_bound(T64, lo, hi, w.grid_n, pts)
    slack = rb.face_slack(u64, w.grid_n)
    in64 = (slack >= 0).all(-1)
    in32 = np.isfinite(v32)
    assert in32.sum() > 10000, in32.sum()
    diff = in64 != in32
    near_face = (slack >= -du).all(-1) & (slack <= du).any(-1)
    assert np.all(near_face[diff]), np.argwhere(diff & ~near_face)[:5]
    vb = rb.value_bound(du, g64)
    err = np.abs(v32 - v64)
    assert np.all(err[in32] <= vb[in32]), np.max(err[in32] / vb[in32])
    print(f"[oracle] {in32.sum()} kept pairs, {diff.sum()} kept by one side only; max |twin - double| "
          f"{err[in32].max():.3g} m, bound up to {vb[in32].max():.3g} m, max ratio {np.max(err[in32] / vb[in32]):.3g}")
    # teeth: the twin fed R instead of R^T
    Tt = T32[:1].copy()
    Tt[..., :3] = np.swapaxes(Tt[..., :3], -1, -2)
    vt = orc.query_f32_each(Tt, w.grid_lo, w.grid_hi, w.grid_n, g32, pts).astype(np.float64)[0]
    both = np.isfinite(vt) & in64[0]
    moved = (np.abs(vt - v64[0]) > vb[0]) | (np.isfinite(vt) != in64[0])
    assert moved.sum() > 0.5 * max(1, (np.isfinite(vt) | in64[0]).sum()), (moved.sum(), both.sum())
