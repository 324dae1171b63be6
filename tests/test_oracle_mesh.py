"""Pins of the oracle's mesh signed distance against closed forms.

The link SDF grids of the method (Sec. III-A, "Link SDFs") are samples of a
signed distance to the link geometry.  The oracle computes it by brute force
over triangles; these tests tie that to exact distances of boxes, spheres and
capsules, to a dense brute-force search over a triangle, and to the values
the winding number must take.
"""
import math

import numpy as np
import pytest

from synth import box_mesh, capsule_mesh, sphere_mesh, union_mesh


def box_sdf(p, centre, half):
    q = np.abs(np.asarray(p) - centre) - half
    return np.linalg.norm(np.maximum(q, 0.0), axis=-1) + np.minimum(q.max(axis=-1), 0.0)


def seg_dist(p, a, b):
    ab = b - a
    t = np.clip(((p - a) @ ab) / (ab @ ab), 0.0, 1.0)
    return np.linalg.norm(p - (a + t[:, None] * ab), axis=-1)


def test_box_exact_inside_and_outside(orc):
    centre = np.array([0.03, -0.02, 0.05])
    half = np.array([0.1, 0.2, 0.3])          # unequal, so any axis mix-up shows
    v, t = box_mesh(centre, half)
    rng = np.random.default_rng(1)
    P = centre + rng.uniform(-0.4, 0.4, size=(400, 3))
    got = orc.mesh_sdf(P, v, t)
    want = box_sdf(P, centre, half)
    assert np.max(np.abs(got - want)) < 1e-12
    assert (got < 0).sum() > 20 and (got > 0).sum() > 20


def test_disjoint_union_is_min(orc):
    a = box_mesh((-0.3, 0, 0), (0.1, 0.1, 0.1))
    b = box_mesh((0.3, 0.1, 0), (0.05, 0.15, 0.1))
    m = union_mesh([a, b])
    rng = np.random.default_rng(2)
    P = rng.uniform(-0.6, 0.6, size=(300, 3))
    P[:20] = np.array([-0.3, 0, 0]) + rng.uniform(-0.09, 0.09, size=(20, 3))
    got = orc.mesh_sdf(P, m.verts, m.tris, m.comp_first)
    want = np.minimum(box_sdf(P, np.array([-0.3, 0, 0]), np.array([0.1, 0.1, 0.1])),
                      box_sdf(P, np.array([0.3, 0.1, 0]), np.array([0.05, 0.15, 0.1])))
    assert np.max(np.abs(got - want)) < 1e-12


def facet_bound(r, nseg, nring_half):
    # every face of these UV meshes lies inside a spherical cap whose angular
    # radius is at most the larger of the two vertex spacings
    ang = max(2 * math.pi / nseg, (math.pi / 2) / nring_half)
    return r * (1 - math.cos(ang))


def test_sphere_within_facet_bound(orc):
    c, r = np.array([0.1, -0.2, 0.05]), 0.3
    v, t = sphere_mesh(c, r, nseg=32, nring=16)
    rng = np.random.default_rng(3)
    P = c + rng.uniform(-0.8, 0.8, size=(300, 3))
    got = orc.mesh_sdf(P, v, t)
    want = np.linalg.norm(P - c, axis=1) - r
    assert np.max(np.abs(got - want)) <= facet_bound(r, 32, 8) + 1e-12
    # the mesh is inscribed: it never sticks out of the sphere
    assert np.all(got >= want - 1e-12)


def test_capsule_within_facet_bound(orc):
    p0, p1, r = np.array([0.0, 0.1, -0.1]), np.array([0.25, -0.1, 0.2]), 0.07
    v, t = capsule_mesh(p0, p1, r)
    assert t.shape[0] == 256
    rng = np.random.default_rng(4)
    P = 0.5 * (p0 + p1) + rng.uniform(-0.4, 0.4, size=(400, 3))
    got = orc.mesh_sdf(P, v, t)
    want = seg_dist(P, p0, p1) - r
    assert np.max(np.abs(got - want)) <= facet_bound(r, 16, 4) + 1e-12
    assert np.all(got >= want - 1e-12)


def test_winding_number_values(orc):
    v, t = capsule_mesh((0, 0, 0), (0.2, 0.1, 0.0), 0.05)
    inside = [np.array([0.1, 0.05, 0.0]), np.array([0.0, 0.0, 0.02])]
    outside = [np.array([0.3, 0.3, 0.3]), np.array([0.1, 0.05, 0.2]), np.array([-1.0, 0, 0])]
    for p in inside:
        assert abs(orc.winding_number(p, v, t) - 1.0) < 1e-9
    for p in outside:
        assert abs(orc.winding_number(p, v, t)) < 1e-9
    # reversed orientation flips the sign
    assert abs(orc.winding_number(inside[0], v, t[:, [0, 2, 1]]) + 1.0) < 1e-9


def test_point_triangle_regions(orc):
    a, b, c = np.array([0.0, 0, 0]), np.array([1.0, 0, 0]), np.array([0.0, 2.0, 0])
    # above the interior: the height
    assert orc.point_triangle_distance([0.2, 0.3, 0.7], a, b, c) == pytest.approx(0.7, abs=1e-15)
    # vertex region of b
    p = np.array([1.5, -0.5, 0.2])
    assert orc.point_triangle_distance(p, a, b, c) == pytest.approx(np.linalg.norm(p - b), abs=1e-15)
    # edge region of bc: distance to the line through b and c
    p = np.array([1.0, 1.0, -0.3])
    e = (c - b) / np.linalg.norm(c - b)
    foot = b + ((p - b) @ e) * e
    assert orc.point_triangle_distance(p, a, b, c) == pytest.approx(np.linalg.norm(p - foot), abs=1e-14)


def test_point_triangle_vs_dense_search(orc):
    rng = np.random.default_rng(5)
    k = 200
    s, t = np.meshgrid(np.arange(k + 1), np.arange(k + 1), indexing="ij")
    keep = s + t <= k
    s, t = s[keep] / k, t[keep] / k
    for _ in range(20):
        tri = rng.normal(size=(3, 3))
        samples = tri[0] + s[:, None] * (tri[1] - tri[0]) + t[:, None] * (tri[2] - tri[0])
        # sample spacing bounds how far the dense minimum can sit above the true one
        spacing = max(np.linalg.norm(tri[1] - tri[0]), np.linalg.norm(tri[2] - tri[0]),
                      np.linalg.norm(tri[2] - tri[1])) / k
        p = rng.normal(size=3) * 1.5
        brute = np.min(np.linalg.norm(samples - p, axis=1))
        got = orc.point_triangle_distance(p, *tri)
        assert got <= brute + 1e-12
        assert got >= brute - spacing


def test_robot_links_are_closed(orc, tiny):
    # a point far away sees total solid angle 0; the base-link box centre sees 1
    for m in tiny.robot.links:
        for k in range(m.ncomp):
            t0, t1 = int(m.comp_first[k]), int(m.comp_first[k + 1])
            assert abs(orc.winding_number([5.0, 5.0, 5.0], m.verts, m.tris, t0, t1)) < 1e-9
            centroid = m.verts[np.unique(m.tris[t0:t1])].mean(axis=0)
            assert abs(orc.winding_number(centroid, m.verts, m.tris, t0, t1) - 1.0) < 1e-9
