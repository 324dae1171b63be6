"""Pins of the oracle's Robot-SDF pipeline (the paper's own method,
Sec. III-A, Eq. 1-4): alignment, transformed Link SDFs, per-voxel minimum
over links, and the gather-only runtime.

* Alignment (Eq. 1-3) on hand-worked positions: block corner, residual
  shift in [-r/2, r/2], block centre on the grid line nearest the origin.
* The Robot SDF built through the alignment and the transformation of
  Eq. 4 (G = R^T (P_j - dt)) equals, voxel by voxel, the plain per-point
  query evaluated at the voxel centres (R^T (x_v - t) by definition): a
  wrong block corner, a wrong sign of the shift or a transposed rotation
  moves every value.
* The runtime's result is the minimum of the Robot SDF over the voxels the
  points fall in, with the voxelisation written independently here.
* Against the exact mesh distance at the points themselves, the pipeline's
  error stays within half a voxel diagonal plus the grid bound (the
  |r_e|/2 + |r_r|/2 of Sec. III-B-1).
"""
import math

import numpy as np
import pytest

R_ENV = 1.0 / 16.0          # voxel edge (a power of two: centres are exact)
ENV_LO = np.array([-1.5, -1.5, -1.5])
ENV_N = np.array([48, 48, 48], dtype=np.int32)


def block_halfwidths(w):
    """m_i: the block of link i reaches every voxel whose centre may fall in
    the link's grid box (farthest box corner from the link origin, plus the
    shift, plus two voxels)."""
    m = []
    for i in range(w.L):
        corners = np.array([[x, y, z] for x in (w.grid_lo[i, 0], w.grid_hi[i, 0]) for y in (w.grid_lo[i, 1], w.grid_hi[i, 1])
                            for z in (w.grid_lo[i, 2], w.grid_hi[i, 2])], dtype=np.float64)
        m.append(int(math.ceil(np.linalg.norm(corners, axis=1).max() / R_ENV)) + 2)
    return np.array(m, dtype=np.int32)


@pytest.mark.parametrize("t,k,dt", [
    ((0.0, 0.0, 0.0), (24 - 5, 24 - 5, 24 - 5), (0.0, 0.0, 0.0)),
    ((0.03, -0.03, 0.0313), (24 - 5, 24 - 5, 25 - 5), (0.03, -0.03, 0.0313 - 0.0625)),
    ((0.5, -1.0, 1.2), (32 - 5, 8 - 5, 43 - 5), (0.0, 0.0, 1.2 - (43 * 0.0625 - 1.5))),
])
def test_align_hand_cases(orc, t, k, dt):
    kk, dd = orc.align(np.array(t), ENV_LO, R_ENV, 5)
    assert tuple(kk) == k
    assert np.allclose(dd, dt, atol=1e-12)
    assert np.all(np.abs(dd) <= R_ENV / 2 + 1e-12)
    centre = ENV_LO + (kk + 5) * R_ENV
    assert np.allclose(np.array(t) - centre, dd, atol=1e-12)


def test_robot_sdf_equals_plain_query_at_voxel_centres(orc, tiny, tiny_grids):
    T = orc.fk(tiny.robot.dh, tiny.q[[3, 17, 41]], tiny.robot.base_T)
    m = block_halfwidths(tiny)
    rs = orc.robot_sdf_f64(T, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, tiny_grids, m, ENV_LO, R_ENV, ENV_N)
    V = int(np.prod(ENV_N))
    centres = orc.voxel_centres(ENV_LO, R_ENV, ENV_N, np.arange(V)).astype(np.float64)
    per_link = orc.query_f64(T, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, tiny_grids, centres[:1])   # shape check
    assert per_link.shape == (3, tiny.L)
    for c in range(3):
        want = np.full(V, np.inf)
        for i in range(tiny.L):
            # the plain query, one voxel centre at a time, per link (chunks of centres)
            Ti = T[c:c + 1, i:i + 1]
            vals = np.array([orc.query_f64(Ti, tiny.grid_lo[i:i + 1], tiny.grid_hi[i:i + 1], tiny.grid_n[i:i + 1],
                                           [tiny_grids[i]], centres[v:v + 1])[0, 0] for v in candidate_voxels(T[c, i], m[i])])
            idx = candidate_voxels(T[c, i], m[i])
            want[idx] = np.minimum(want[idx], vals)
        got = rs[c].reshape(-1)
        fin = np.isfinite(want)
        assert np.array_equal(fin, np.isfinite(got)), c
        assert fin.sum() > 300
        assert np.max(np.abs(got[fin] - want[fin])) < 1e-9


def candidate_voxels(Tci, m):
    """Flat indices of the voxels within m + 1 voxels of the link origin (a
    superset of the block; the plain query gives +inf beyond the box)."""
    t = Tci[:, 3]
    c = np.floor((t - ENV_LO) / R_ENV).astype(int)
    rng = [np.arange(max(0, c[a] - m - 1), min(ENV_N[a], c[a] + m + 2)) for a in range(3)]
    Z, Y, X = np.meshgrid(rng[2], rng[1], rng[0], indexing="ij")
    return ((Z * ENV_N[1] + Y) * ENV_N[0] + X).reshape(-1)


def test_runtime_is_min_over_occupied_voxels(orc, tiny, tiny_grids):
    T = orc.fk(tiny.robot.dh, tiny.q[[5, 25]], tiny.robot.base_T)
    m = block_halfwidths(tiny)
    rs = orc.robot_sdf_f64(T, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, tiny_grids, m, ENV_LO, R_ENV, ENV_N)
    rng = np.random.default_rng(80)
    pts = np.concatenate([tiny.points[:500], rng.uniform(-2.0, 2.0, size=(100, 3))])      # some outside
    got = orc.robot_sdf_query(rs, ENV_LO, R_ENV, ENV_N, pts)
    v = np.floor((pts - ENV_LO) / R_ENV).astype(np.int64)
    ok = np.all((v >= 0) & (v < ENV_N), axis=1)
    assert 0 < ok.sum() < len(pts)
    flat = (v[ok, 2] * ENV_N[1] + v[ok, 1]) * ENV_N[0] + v[ok, 0]
    want = rs.reshape(2, -1)[:, flat].min(axis=1)
    assert np.array_equal(got, want)
    assert orc.voxel_index(pts[~ok][0], ENV_LO, R_ENV, ENV_N) == -1


def test_pipeline_error_within_voxel_and_grid_bounds(orc, tiny, tiny_grids):
    """Against the exact mesh distance at the points: the Robot-SDF result
    reads the grid interpolant at voxel centres instead of the points, so
    it stays within half a voxel diagonal (the centre is that close to the
    point, and the exact distance is 1-Lipschitz) plus the grid bound."""
    sel = [7, 29]
    T = orc.fk(tiny.robot.dh, tiny.q[sel], tiny.robot.base_T)
    m = block_halfwidths(tiny)
    rs = orc.robot_sdf_f64(T, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, tiny_grids, m, ENV_LO, R_ENV, ENV_N)
    # points near the arm, all inside their voxels' link boxes' reach
    origins = T[:, :, :, 3].reshape(-1, 3)
    rng = np.random.default_rng(81)
    pts = origins[rng.integers(0, len(origins), 300)] + rng.normal(0, 0.06, size=(300, 3))
    got = orc.robot_sdf_query(rs, ENV_LO, R_ENV, ENV_N, pts)
    exact, _ = orc.reduce(orc.exact_min(T, tiny.robot.links, pts))
    h = (tiny.grid_hi[0].astype(np.float64) - tiny.grid_lo[0]) / (tiny.grid_n[0] - 1)
    hmax = max(orc.grid_bound((tiny.grid_hi[i].astype(np.float64) - tiny.grid_lo[i]) / (tiny.grid_n[i] - 1))
               for i in range(tiny.L))
    bound = 0.5 * math.sqrt(3) * R_ENV + hmax
    assert np.all(np.isfinite(got))
    assert np.all(np.abs(got - exact) <= bound + 1e-9), (np.abs(got - exact).max(), bound)
    assert h.shape == (3,)
