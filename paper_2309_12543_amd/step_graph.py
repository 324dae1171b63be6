"""A whole planning step captured once in a HIP graph and replayed.

The paper re-plans trajectories continually against the latest obstacle
cloud (Sec. IV); one such step is forward kinematics of every trajectory's
configurations followed by the clearance query of each trajectory against
its own points.  The step is three to five short kernels, so at small sizes
launch overhead rivals the work: capturing the launches once
(torch.cuda.CUDAGraph over liblsdf.so's calls on the capture stream) and
replaying them removes it.  Nothing in the step reads back to the host (the
trajectory ranges live in device arrays), so one captured graph serves any
set of trajectories that fits its capacities.
"""
from __future__ import annotations

import torch

from . import lsdf


class StepGraph:
    """Static buffers of fixed capacity plus the captured step.

    Usage: ``g = StepGraph(dh, base_T, grids, C_cap, M_cap, K_cap)``, then per
    step ``g.load(q, points, c_offsets, m_offsets)`` (copies into the static
    buffers; unused trajectory slots become empty) and ``g.replay()``, which
    returns views of the static outputs (dist [C_cap], link [C_cap]).
    """

    def __init__(self, dh, base_T, grids: lsdf.GridSet, C_cap: int, M_cap: int, K_cap: int, *, tuning=None,
                 link_dist: bool = False, fused: bool = True, device="cuda"):
        """fused: kinematics inside the query's first kernel
        (lsdf_query_from_joints, one launch fewer) instead of lsdf_fk_batch
        followed by the batched query; both give the same bits."""
        dev = torch.device(device)
        self.dh, self.base_T, self.grids, self.tuning, self.fused = dh, base_T, grids, tuning, fused
        self.dof = len(dh)
        self.C_cap, self.M_cap, self.K_cap = int(C_cap), int(M_cap), int(K_cap)
        L = grids.L
        if L != self.dof + 1:
            raise ValueError(f"grids has {L} links, the arm has {self.dof + 1} frames")
        self.q = torch.zeros((self.C_cap, self.dof), dtype=torch.float32, device=dev)
        self.points = torch.zeros((self.M_cap, 3), dtype=torch.float32, device=dev)
        self.c_off = torch.zeros(self.K_cap + 1, dtype=torch.int32, device=dev)
        self.m_off = torch.zeros(self.K_cap + 1, dtype=torch.int64, device=dev)
        self.link_T = torch.zeros((self.C_cap, L, 3, 4), dtype=torch.float32, device=dev)
        self.dist = torch.zeros(self.C_cap, dtype=torch.float32, device=dev)
        self.link = torch.zeros(self.C_cap, dtype=torch.int32, device=dev)
        self.link_dist = torch.zeros((self.C_cap, L), dtype=torch.float32, device=dev) if link_dist else None
        need = lsdf.query_batched_workspace_size(self.K_cap, self.C_cap, L, self.M_cap)
        self.workspace = torch.zeros(need, dtype=torch.uint8, device=dev)
        # eager run on a side stream first (as torch requires before capture)
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            self._step()
        torch.cuda.current_stream(dev).wait_stream(side)
        torch.cuda.synchronize(dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._step()

    def _step(self):
        if self.fused:
            lsdf.query_from_joints(self.dh, self.q, self.grids, self.points, base_T=self.base_T,
                                   c_offsets=self.c_off, m_offsets=self.m_off, link_T=self.link_T,
                                   link_dist=self.link_dist is not None, tuning=self.tuning,
                                   workspace=self.workspace, out=(self.dist, self.link, self.link_dist))
            return
        lsdf.fk_batch(self.dh, self.q, self.base_T, out=self.link_T)
        lsdf.query_min_distance_batched(self.link_T, self.grids, self.points, self.c_off, self.m_off,
                                        link_dist=self.link_dist is not None, tuning=self.tuning,
                                        workspace=self.workspace, out=(self.dist, self.link, self.link_dist))

    def load(self, q: torch.Tensor, points: torch.Tensor, c_offsets: torch.Tensor, m_offsets: torch.Tensor):
        """Copies one step's inputs (device tensors) into the static buffers.
        K = len(c_offsets) - 1 <= K_cap trajectories; slots K..K_cap-1 are
        made empty by repeating the last offset."""
        C, M, K = int(q.shape[0]), int(points.shape[0]), int(c_offsets.numel()) - 1
        if C > self.C_cap or M > self.M_cap or K > self.K_cap or K < 1:
            raise ValueError(f"step (C={C}, M={M}, K={K}) exceeds the capacities "
                             f"({self.C_cap}, {self.M_cap}, {self.K_cap})")
        self.q[:C].copy_(q)
        self.points[:M].copy_(points)
        self.c_off[:K + 1].copy_(c_offsets)
        self.m_off[:K + 1].copy_(m_offsets)
        self.c_off[K + 1:].copy_(c_offsets[K:K + 1].expand(self.K_cap - K))
        self.m_off[K + 1:].copy_(m_offsets[K:K + 1].expand(self.K_cap - K))

    def replay(self):
        self.graph.replay()
        if self.link_dist is not None:
            return self.dist, self.link, self.link_dist
        return self.dist, self.link
