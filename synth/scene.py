"""Seeded obstacle clouds.

* ``uniform_cube``: points uniform in the 2 m cube [-1, 1]^3 around the base.
* ``human_table``: a human-like cluster of 10 ellipsoids (head, torso, two
  upper arms, two forearms, two thighs, two shins) plus a table slab, both
  voxelised; the points are the centres of the occupied voxels, the form in
  which the paper feeds obstacles to its runtime (Sec. III-A, Sec. IV-C uses
  4 cm voxels of a recorded Kinect cloud, which is not available here).

Exactly M points are returned.  With V occupied voxels: V > M keeps a seeded
subsample without replacement; V < M adds M - V extra points, each the centre
of a uniformly drawn occupied voxel jittered uniformly inside that voxel.  The
result is ordered by voxel raster index (x fastest), the order a voxel scan
produces.  Input generation only.
"""
from __future__ import annotations

import math

import numpy as np

FLOOR_Z = -0.75     # the human stands on a floor 0.75 m below the base / table top


def uniform_cube(M: int, seed: int, half: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(-half, half, size=(M, 3))


def _rot_xy(ax: float, ay: float) -> np.ndarray:
    cx, sx, cy, sy = math.cos(ax), math.sin(ax), math.cos(ay), math.sin(ay)
    rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    return rx @ ry


def _rot_z(a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def human_ellipsoids(rng: np.random.Generator):
    """Ten ellipsoids (centre, rotation, semi-axes) in the person's frame
    (feet at z = 0, facing +x).  Limbs hang from their proximal joint, each
    joint angle jittered by N(0, 15 deg)."""
    jit = lambda: rng.normal(0.0, 15.0 * math.pi / 180.0)
    ell = []
    ell.append((np.array([0.0, 0.0, 1.58]), np.eye(3), np.array([0.09, 0.10, 0.12])))   # head
    ell.append((np.array([0.0, 0.0, 1.18]), np.eye(3), np.array([0.11, 0.18, 0.28])))   # torso
    for side in (-1.0, 1.0):
        shoulder = np.array([0.0, side * 0.23, 1.40])
        r_up = _rot_xy(jit(), jit())
        up_axis = r_up @ np.array([0.0, 0.0, -1.0])
        ell.append((shoulder + 0.15 * up_axis, r_up, np.array([0.05, 0.05, 0.15])))    # upper arm
        elbow = shoulder + 0.30 * up_axis
        r_fo = r_up @ _rot_xy(jit() - 0.6, jit())
        fo_axis = r_fo @ np.array([0.0, 0.0, -1.0])
        ell.append((elbow + 0.13 * fo_axis, r_fo, np.array([0.04, 0.04, 0.13])))       # forearm
        hip = np.array([0.0, side * 0.09, 0.90])
        r_th = _rot_xy(jit(), jit())
        th_axis = r_th @ np.array([0.0, 0.0, -1.0])
        ell.append((hip + 0.22 * th_axis, r_th, np.array([0.08, 0.08, 0.22])))         # thigh
        knee = hip + 0.44 * th_axis
        r_sh = r_th @ _rot_xy(jit(), jit())
        sh_axis = r_sh @ np.array([0.0, 0.0, -1.0])
        ell.append((knee + 0.21 * sh_axis, r_sh, np.array([0.06, 0.06, 0.21])))        # shin
    return ell


def human_table(M: int, voxel: float, seed: int, return_info: bool = False):
    rng = np.random.default_rng(seed)
    # person: centre 0.3-1.5 m from the base at a random azimuth and yaw
    dist = rng.uniform(0.3, 1.5)
    az = rng.uniform(-math.pi, math.pi)
    yaw = rng.uniform(-math.pi, math.pi)
    R_p = _rot_z(yaw)
    t_p = np.array([dist * math.cos(az), dist * math.sin(az), FLOOR_Z])
    solids = []
    for c, R, s in human_ellipsoids(rng):
        solids.append((R_p @ c + t_p, R_p @ R, s))
    # table: 1.2 x 0.8 m slab, one voxel thick, top at z = 0, centred 0.6 m away
    taz = rng.uniform(-math.pi, math.pi)
    t_c = np.array([0.6 * math.cos(taz), 0.6 * math.sin(taz)])
    t_R = _rot_z(taz)[:2, :2]   # local x = radial (0.8 m side), local y = tangential (1.2 m)

    # bounding box of everything, in voxel indices (voxel i spans [i, i+1) * voxel)
    mins, maxs = [], []
    for c, R, s in solids:
        ext = np.abs(R) @ s
        mins.append(c - ext)
        maxs.append(c + ext)
    corners = np.array([[sx * 0.4, sy * 0.6] for sx in (-1, 1) for sy in (-1, 1)]) @ t_R.T + t_c
    mins.append(np.array([corners[:, 0].min(), corners[:, 1].min(), -voxel]))
    maxs.append(np.array([corners[:, 0].max(), corners[:, 1].max(), 0.0]))
    lo = np.floor(np.min(mins, axis=0) / voxel).astype(np.int64) - 1
    hi = np.ceil(np.max(maxs, axis=0) / voxel).astype(np.int64) + 1
    ix = np.arange(lo[0], hi[0])
    iy = np.arange(lo[1], hi[1])
    iz = np.arange(lo[2], hi[2])
    occ = np.zeros((iz.size, iy.size, ix.size), dtype=bool)
    Z, Y, X = np.meshgrid((iz + 0.5) * voxel, (iy + 0.5) * voxel, (ix + 0.5) * voxel, indexing="ij")
    P = np.stack([X, Y, Z], axis=-1)
    for c, R, s in solids:
        q = (P - c) @ R           # coordinates in the ellipsoid frame
        occ |= ((q / s) ** 2).sum(axis=-1) <= 1.0
    loc = (P[..., :2] - t_c) @ t_R
    occ |= (np.abs(loc[..., 0]) <= 0.4) & (np.abs(loc[..., 1]) <= 0.6) & (Z > -voxel) & (Z < 0.0)

    flat = np.flatnonzero(occ.ravel())            # raster order, x fastest
    centres = P.reshape(-1, 3)[flat]
    V = flat.size
    if V >= M:
        keep = np.sort(rng.choice(V, size=M, replace=False))
        pts, order_key = centres[keep], flat[keep].astype(np.float64)
    else:
        extra_src = rng.integers(0, V, size=M - V)
        jitter = rng.uniform(-0.5 * voxel, 0.5 * voxel, size=(M - V, 3))
        pts = np.concatenate([centres, centres[extra_src] + jitter])
        key = np.concatenate([flat, flat[extra_src]]).astype(np.float64)
        order_key = key + np.concatenate([np.zeros(V), 0.5 + np.arange(M - V) / (2.0 * (M - V))])
    pts = pts[np.argsort(order_key, kind="stable")]
    if return_info:
        return pts, {"occupied_voxels": int(V), "person_distance_m": float(dist)}
    return pts
