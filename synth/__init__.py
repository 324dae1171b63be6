"""Seeded synthetic inputs shared by the library's tests, the benchmark and
the oracle's tests.  This package holds input generation only (robot
parameters and meshes, waypoints, obstacle clouds, grid boxes); none of the
distance method's arithmetic is here.

Base seed 230912543; sub-streams: DH and meshes S+0, waypoints S+2+100*traj,
scene S+3+100*traj, network samples S+4+link, network initial weights S+5,
trajectory sizes of a batched workload S+6.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .robot import (GRID_PAD, MLP_FAR, Mesh, Robot, box_mesh, capsule_mesh, grid_box, make_robot, mlp_core, mlp_domain, mlp_init,
                    mlp_samples, sphere_mesh, surface_points, union_mesh)
from .scene import human_table, uniform_cube
from .traj import make_waypoints

BASE_SEED = 230912543


@dataclass
class Workload:
    name: str
    robot: Robot
    q: np.ndarray            # float64 [C][dof]
    points: np.ndarray       # float64 [M][3] (values exactly representable in float32)
    grid_lo: np.ndarray      # float32 [L][3]
    grid_hi: np.ndarray      # float32 [L][3]
    grid_n: np.ndarray       # int32 [L][3]
    info: dict

    @property
    def C(self) -> int:
        return int(self.q.shape[0])

    @property
    def M(self) -> int:
        return int(self.points.shape[0])

    @property
    def L(self) -> int:
        return self.robot.n_links


# name -> (C, M, cloud kind, voxel size, grid nodes per axis)
WORKLOADS = {
    # 50 waypoints x 2,000 points uniform in a 2 m cube, 32^3 grids
    "tiny": (50, 2000, "cube", None, 32),
    # 500 waypoints x 20,000 points (2 cm voxels of a person + table), 64^3 grids
    "paper": (500, 20000, "scene", 0.02, 64),
    # 500 waypoints x 100,000 points (1 cm voxels), 128^3 grids (precision study)
    "precision": (500, 100000, "scene", 0.01, 128),
    # 500 waypoints x 100,000 points (1 cm voxels), 64^3 grids (learned variant)
    "learned": (500, 100000, "scene", 0.01, 64),
}


def make_workload(name: str = "tiny", C: int | None = None, M: int | None = None,
                  n: int | None = None, traj: int = 0, seed: int = BASE_SEED) -> Workload:
    C0, M0, kind, voxel, n0 = WORKLOADS[name]
    C = C0 if C is None else C
    M = M0 if M is None else M
    n = n0 if n is None else n
    robot = make_robot(seed + 0)
    q = make_waypoints(robot.qmin, robot.qmax, C, seed + 2 + 100 * traj)
    info = {"workload": name, "C": C, "M": M, "n": n}
    if kind == "cube":
        pts = uniform_cube(M, seed + 3 + 100 * traj)
    else:
        pts, sinfo = human_table(M, voxel, seed + 3 + 100 * traj, return_info=True)
        info.update(sinfo)
        info["voxel_m"] = voxel
    pts = pts.astype(np.float32).astype(np.float64)
    los, his = [], []
    for mesh in robot.links:
        lo, hi = grid_box(mesh)
        los.append(lo)
        his.append(hi)
    grid_lo = np.array(los, dtype=np.float32)
    grid_hi = np.array(his, dtype=np.float32)
    grid_n = np.full((robot.n_links, 3), n, dtype=np.int32)
    return Workload(name, robot, q, pts, grid_lo, grid_hi, grid_n, info)


@dataclass
class BatchedWorkload:
    """K trajectories of one robot, each a path and its own obstacle cloud,
    concatenated: trajectory k owns q[c_off[k]:c_off[k+1]] and
    points[m_off[k]:m_off[k+1]]."""
    name: str
    robot: Robot
    q: np.ndarray            # float64 [sum C_k][dof]
    points: np.ndarray       # float64 [sum M_k][3] (values exactly representable in float32)
    c_off: np.ndarray        # int64 [K+1]
    m_off: np.ndarray        # int64 [K+1]
    grid_lo: np.ndarray
    grid_hi: np.ndarray
    grid_n: np.ndarray
    info: dict

    @property
    def K(self) -> int:
        return int(self.c_off.size - 1)

    @property
    def C(self) -> int:
        return int(self.q.shape[0])

    @property
    def M(self) -> int:
        return int(self.points.shape[0])

    @property
    def L(self) -> int:
        return self.robot.n_links

    def pairs(self) -> int:
        """Point-link queries of the whole batch: sum_k C_k M_k L."""
        return int((np.diff(self.c_off) * np.diff(self.m_off)).sum()) * self.L


def make_batched(K: int = 64, C_range=(50, 1000), M_range=(5000, 200000), n: int = 64, voxel: float = 0.02,
                 kind: str = "scene", seed: int = BASE_SEED) -> BatchedWorkload:
    """K re-planned trajectories with their own clouds: C_k and M_k drawn
    uniformly from the inclusive ranges (stream S+6), waypoints of trajectory
    k from stream S+2+100k and its scene from S+3+100k.  kind "cube" uses
    uniform points in the 2 m cube instead of the voxelised person and
    table.  Ranges may include 0 (empty trajectories)."""
    robot = make_robot(seed + 0)
    rng = np.random.default_rng(seed + 6)
    Cs = rng.integers(C_range[0], C_range[1] + 1, size=K)
    Ms = rng.integers(M_range[0], M_range[1] + 1, size=K)
    qs, ps = [], []
    occupied = []
    for k in range(K):
        C, M = int(Cs[k]), int(Ms[k])
        qs.append(make_waypoints(robot.qmin, robot.qmax, C, seed + 2 + 100 * k) if C > 0
                  else np.zeros((0, robot.dof)))
        if M == 0:
            ps.append(np.zeros((0, 3)))
        elif kind == "cube":
            ps.append(uniform_cube(M, seed + 3 + 100 * k))
        else:
            pts, sinfo = human_table(M, voxel, seed + 3 + 100 * k, return_info=True)
            occupied.append(sinfo["occupied_voxels"])
            ps.append(pts)
    q = np.concatenate(qs).reshape(-1, robot.dof)
    pts = np.concatenate(ps).reshape(-1, 3).astype(np.float32).astype(np.float64)
    c_off = np.concatenate([[0], np.cumsum(Cs)]).astype(np.int64)
    m_off = np.concatenate([[0], np.cumsum(Ms)]).astype(np.int64)
    los, his = zip(*(grid_box(mesh) for mesh in robot.links))
    grid_lo = np.array(los, dtype=np.float32)
    grid_hi = np.array(his, dtype=np.float32)
    grid_n = np.full((robot.n_links, 3), n, dtype=np.int32)
    info = {"workload": "batched", "K": K, "C_range": list(C_range), "M_range": list(M_range), "n": n,
            "voxel_m": voxel if kind == "scene" else None, "sum_C": int(Cs.sum()), "sum_M": int(Ms.sum())}
    if occupied:
        info["occupied_voxels_mean"] = float(np.mean(occupied))
    return BatchedWorkload("batched", robot, q, pts, c_off, m_off, grid_lo, grid_hi, grid_n, info)


__all__ = ["BatchedWorkload", "make_batched", "BASE_SEED", "GRID_PAD", "Mesh", "Robot", "Workload", "WORKLOADS", "box_mesh",
           "capsule_mesh", "grid_box", "human_table", "make_robot", "make_waypoints",
           "make_workload", "sphere_mesh", "uniform_cube", "union_mesh", "MLP_FAR", "mlp_core", "mlp_domain", "mlp_init",
           "mlp_samples", "surface_points"]
