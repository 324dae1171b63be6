"""Synthetic 6-DoF arm: standard-DH parameters and closed triangle meshes per link.

Input generation only. Nothing here evaluates a distance, a kinematic chain
or a grid sample: those are the method's steps and live in the library (and,
independently, in the oracle). The robot stands in for the paper's DENSO
VS-060 (Sec. IV-C), whose model is not available.

Conventions
-----------
* Standard (distal) DH: joint k moves frame k relative to frame k-1 by
  Rz(theta_k) Tz(d_k) Tx(a_k) Rx(alpha_k).  Link 0 is the fixed base, so a
  6-joint arm has 7 links and link k's mesh is expressed in frame k.
* Meshes are closed, outward-oriented (counter-clockwise seen from outside)
  triangle soups; a link is a union of closed components listed by
  ``comp_first`` (first triangle of each component, plus the total).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

DEG = math.pi / 180.0
JOINT_LIMIT = 170.0 * DEG
GRID_PAD = 0.05  # metres of padding around each link's bounding box


@dataclass
class Mesh:
    verts: np.ndarray          # float64 [nv][3]
    tris: np.ndarray           # int32 [nt][3]
    comp_first: np.ndarray     # int32 [ncomp+1]

    @property
    def ncomp(self) -> int:
        return int(self.comp_first.shape[0] - 1)


@dataclass
class Robot:
    # DH table, one row per joint: a, alpha, d, theta_offset (metres / radians)
    dh: np.ndarray                              # float64 [dof][4]
    qmin: np.ndarray                            # float64 [dof]
    qmax: np.ndarray                            # float64 [dof]
    base_T: np.ndarray                          # float64 [3][4], link 0 -> world
    links: list = field(default_factory=list)   # list[Mesh], dof+1 entries

    @property
    def dof(self) -> int:
        return int(self.dh.shape[0])

    @property
    def n_links(self) -> int:
        return self.dof + 1


# ----------------------------------------------------------------------------
# Closed primitive meshes
# ----------------------------------------------------------------------------

def _frame_from_axis(w: np.ndarray):
    w = w / np.linalg.norm(w)
    helper = np.array([1.0, 0.0, 0.0]) if abs(w[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    u = np.cross(w, helper)
    u /= np.linalg.norm(u)
    v = np.cross(w, u)
    return u, v, w


def capsule_mesh(p0, p1, r, nseg=16, nring=4):
    """Capsule (segment p0-p1 swept by radius r) as a closed UV mesh whose
    vertices lie on the exact surface.  2*nseg fan triangles plus
    (2*nring-1)*2*nseg band triangles (256 for the defaults)."""
    p0 = np.asarray(p0, dtype=np.float64)
    p1 = np.asarray(p1, dtype=np.float64)
    u, v, w = _frame_from_axis(p1 - p0)
    rings = []
    # lower hemisphere around p0: latitudes -pi/2 + k*step, k = 1..nring (last is the equator)
    step = (math.pi / 2) / nring
    for k in range(1, nring + 1):
        rings.append((p0, -math.pi / 2 + k * step))
    # upper hemisphere around p1: latitudes k*step, k = 0..nring-1 (first is the equator)
    for k in range(0, nring):
        rings.append((p1, k * step))
    verts = [p0 - r * w]
    for centre, phi in rings:
        for s in range(nseg):
            th = 2 * math.pi * s / nseg
            d = math.cos(phi) * (math.cos(th) * u + math.sin(th) * v) + math.sin(phi) * w
            verts.append(centre + r * d)
    verts.append(p1 + r * w)
    verts = np.array(verts)
    tris = []
    nr = len(rings)
    ring_start = lambda j: 1 + j * nseg
    bottom, top = 0, len(verts) - 1
    for s in range(nseg):
        s1 = (s + 1) % nseg
        tris.append((bottom, ring_start(0) + s1, ring_start(0) + s))
    for j in range(nr - 1):
        a0, b0 = ring_start(j), ring_start(j + 1)
        for s in range(nseg):
            s1 = (s + 1) % nseg
            tris.append((a0 + s, a0 + s1, b0 + s1))
            tris.append((a0 + s, b0 + s1, b0 + s))
    last = ring_start(nr - 1)
    for s in range(nseg):
        s1 = (s + 1) % nseg
        tris.append((top, last + s, last + s1))
    tris = np.array(tris, dtype=np.int32)
    return _orient_outward(verts, tris)


def sphere_mesh(c, r, nseg=16, nring=8):
    """UV sphere with vertices on the exact surface (a capsule of zero length)."""
    c = np.asarray(c, dtype=np.float64)
    verts = [c - np.array([0, 0, r])]
    lats = [-math.pi / 2 + k * math.pi / nring for k in range(1, nring)]
    for phi in lats:
        for s in range(nseg):
            th = 2 * math.pi * s / nseg
            verts.append(c + r * np.array([math.cos(phi) * math.cos(th),
                                           math.cos(phi) * math.sin(th),
                                           math.sin(phi)]))
    verts.append(c + np.array([0, 0, r]))
    verts = np.array(verts)
    tris = []
    nr = len(lats)
    rs = lambda j: 1 + j * nseg
    top = len(verts) - 1
    for s in range(nseg):
        s1 = (s + 1) % nseg
        tris.append((0, rs(0) + s1, rs(0) + s))
    for j in range(nr - 1):
        for s in range(nseg):
            s1 = (s + 1) % nseg
            tris.append((rs(j) + s, rs(j) + s1, rs(j + 1) + s1))
            tris.append((rs(j) + s, rs(j + 1) + s1, rs(j + 1) + s))
    for s in range(nseg):
        s1 = (s + 1) % nseg
        tris.append((top, rs(nr - 1) + s, rs(nr - 1) + s1))
    return _orient_outward(verts, np.array(tris, dtype=np.int32))


def box_mesh(centre, half):
    """Axis-aligned box, 8 vertices and 12 triangles."""
    c = np.asarray(centre, dtype=np.float64)
    h = np.asarray(half, dtype=np.float64)
    verts = np.array([[c[0] + sx * h[0], c[1] + sy * h[1], c[2] + sz * h[2]]
                      for sz in (-1, 1) for sy in (-1, 1) for sx in (-1, 1)])
    # vertex index = x + 2y + 4z
    quads = [(0, 2, 3, 1),  # z-
             (4, 5, 7, 6),  # z+
             (0, 1, 5, 4),  # y-
             (2, 6, 7, 3),  # y+
             (0, 4, 6, 2),  # x-
             (1, 3, 7, 5)]  # x+
    tris = []
    for a, b, cc, d in quads:
        tris.append((a, b, cc))
        tris.append((a, cc, d))
    return _orient_outward(verts, np.array(tris, dtype=np.int32))


def _signed_volume(verts, tris):
    a, b, c = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)


def _orient_outward(verts, tris):
    # Every primitive here is convex and built with one consistent winding,
    # so the sign of the enclosed volume tells the orientation.
    if _signed_volume(verts, tris) < 0:
        tris = tris[:, [0, 2, 1]].copy()
    return verts, tris


def union_mesh(parts) -> Mesh:
    """Concatenate closed components into one link mesh."""
    verts, tris, first = [], [], [0]
    off = 0
    for v, t in parts:
        verts.append(v)
        tris.append(t + off)
        off += v.shape[0]
        first.append(first[-1] + t.shape[0])
    return Mesh(np.concatenate(verts).astype(np.float64),
                np.concatenate(tris).astype(np.int32),
                np.array(first, dtype=np.int32))


# ----------------------------------------------------------------------------
# The arm
# ----------------------------------------------------------------------------

def make_robot(seed: int) -> Robot:
    """6-joint arm with alpha = (pi/2, 0, pi/2, -pi/2, pi/2, 0),
    a = (0, U, U, 0, 0, 0), d = (U, 0, 0, U, 0, U), U ~ U[0.1, 0.5] m,
    limits +-170 deg.  Each moving link is a capsule from the previous joint
    frame's origin to its own origin plus one or two joint housings; the
    base is a 0.3 x 0.3 x 0.1 m box plus a vertical capsule."""
    rng = np.random.default_rng(seed)
    alpha = np.array([math.pi / 2, 0.0, math.pi / 2, -math.pi / 2, math.pi / 2, 0.0])
    U = lambda: float(rng.uniform(0.1, 0.5))
    a = np.array([0.0, U(), U(), 0.0, 0.0, 0.0])
    d = np.array([U(), 0.0, 0.0, U(), 0.0, U()])
    dh = np.stack([a, alpha, d, np.zeros(6)], axis=1)
    links = [union_mesh([box_mesh((0.0, 0.0, -0.05), (0.15, 0.15, 0.05)),
                         capsule_mesh((0.0, 0.0, 0.0), (0.0, 0.0, 0.12), 0.09)])]
    for k in range(6):
        r = float(rng.uniform(0.04, 0.08))
        ak, alk, dk = a[k], alpha[k], d[k]
        # origin of frame k-1 written in frame k: Rx(-alpha)(-a, 0, -d)
        prev = np.array([-ak, -dk * math.sin(alk), -dk * math.cos(alk)])
        if np.linalg.norm(prev) > 1e-6:
            parts = [capsule_mesh(prev, (0.0, 0.0, 0.0), r)]
        else:
            # coincident joint origins (a = d = 0): a wrist housing across x_k
            parts = [capsule_mesh((-1.2 * r, 0.0, 0.0), (1.2 * r, 0.0, 0.0), r)]
        # housing of the next joint (its axis is z_k)
        parts.append(capsule_mesh((0.0, 0.0, -1.2 * r), (0.0, 0.0, 1.2 * r), 1.15 * r))
        if rng.uniform() < 0.5:
            parts.append(box_mesh(prev, (0.9 * r, 0.9 * r, 0.9 * r)))
        links.append(union_mesh(parts))
    base_T = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)
    return Robot(dh=dh, qmin=np.full(6, -JOINT_LIMIT), qmax=np.full(6, JOINT_LIMIT),
                 base_T=base_T, links=links)


def grid_box(mesh: Mesh, pad: float = GRID_PAD):
    """Link grid box: tight bounding box of the mesh vertices grown by ``pad``."""
    lo = mesh.verts.min(axis=0) - pad
    hi = mesh.verts.max(axis=0) + pad
    return lo, hi


# ----------------------------------------------------------------------------
# Samples for the learned per-link SDF (input generation only: positions and
# initial weights; labels are computed by the library or the oracle)
# ----------------------------------------------------------------------------

MLP_FAR = 1.0      # metres the network's domain extends beyond the grid box


def mlp_domain(lo, hi, far: float = MLP_FAR):
    """Centre and half extent of a link's network domain: its grid box grown
    by `far` on every side."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return (lo + hi) / 2, (hi - lo) / 2 + far


def mlp_core(lo, hi, pad: float = GRID_PAD):
    """Half extents of a link's core box, centred on its grid box (and
    network domain): the mesh's bounding box, i.e. the grid box shrunk by the
    pad it was grown by.  The surrogate adds the distance to this box to its
    network's output."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return np.maximum((hi - lo) / 2 - pad, 0.0)


def surface_points(mesh: Mesh, n: int, rng: np.random.Generator) -> np.ndarray:
    """Uniform points on the mesh surface (area-weighted triangles, uniform
    barycentric coordinates)."""
    a, b, c = (mesh.verts[mesh.tris[:, k]] for k in range(3))
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    t = rng.choice(len(area), size=n, p=area / area.sum())
    r1, r2 = rng.uniform(size=n), rng.uniform(size=n)
    s = np.sqrt(r1)
    return ((1 - s)[:, None] * a[t] + (s * (1 - r2))[:, None] * b[t] + (s * r2)[:, None] * c[t])


def mlp_samples(mesh: Mesh, lo, hi, n: int, seed: int, far: float = MLP_FAR):
    """n link-frame training positions: 20 % near the surface (surface point
    + N(0, 2 cm)), 10 % in the band around it (surface point + N(0, 15 cm)),
    50 % in the shell where the network's answers are used (surface point +
    a uniform random direction times a distance uniform in [0, 60 cm]), 10 %
    uniform in the grid box and 10 % uniform in the network's domain."""
    rng = np.random.default_rng(seed)
    n_near, n_band, n_shell, n_box = int(0.2 * n), int(0.1 * n), int(0.5 * n), int(0.1 * n)
    n_dom = n - n_near - n_band - n_shell - n_box
    cen, half = mlp_domain(lo, hi, far)
    near = surface_points(mesh, n_near, rng) + rng.normal(0.0, 0.02, size=(n_near, 3))
    band = surface_points(mesh, n_band, rng) + rng.normal(0.0, 0.15, size=(n_band, 3))
    u = rng.normal(size=(n_shell, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    shell = surface_points(mesh, n_shell, rng) + u * rng.uniform(0.0, 0.6, size=(n_shell, 1))
    box = rng.uniform(lo, hi, size=(n_box, 3))
    dom = rng.uniform(cen - half, cen + half, size=(n_dom, 3))
    pts = np.concatenate([near, band, shell, box, dom])
    return pts[rng.permutation(n)]


def mlp_init(n_links: int, seed: int, hidden: int = 128) -> np.ndarray:
    """Initial parameters [n_links][33665]: every weight and bias uniform in
    +-1/sqrt(fan_in) (the common default for fully connected layers)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_links):
        parts = []
        for fan_in, fan_out in ((3, hidden), (hidden, hidden), (hidden, hidden), (hidden, 1)):
            bound = 1.0 / np.sqrt(fan_in)
            parts.append(rng.uniform(-bound, bound, size=fan_out * fan_in))
            parts.append(rng.uniform(-bound, bound, size=fan_out))
        out.append(np.concatenate(parts))
    return np.stack(out)
