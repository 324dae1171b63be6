"""Pins of the oracle's forward kinematics (the link poses T_{i,c} of
Sec. III-A) against geometry derived by hand for the standard DH step
Rz(theta) Tz(d) Tx(a) Rx(alpha)."""
import math

import numpy as np
import pytest


def test_single_joint_geometry(orc):
    rng = np.random.default_rng(20)
    for _ in range(20):
        a, alpha, d, off = rng.uniform(-1, 1), rng.uniform(-3, 3), rng.uniform(-1, 1), rng.uniform(-1, 1)
        q = rng.uniform(-3, 3)
        T = orc.fk(np.array([[a, alpha, d, off]]), np.array([[q]]))[0]
        th = q + off
        assert np.allclose(T[0], np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1), atol=0)
        R, o = T[1][:, :3], T[1][:, 3]
        # the origin moves d along z, then a along the rotated x
        assert np.allclose(o, [a * math.cos(th), a * math.sin(th), d], atol=1e-14)
        # x_1 is x_0 turned by theta about z_0; z_1 is z_0 tilted by alpha about x_1
        assert np.allclose(R[:, 0], [math.cos(th), math.sin(th), 0], atol=1e-14)
        assert np.allclose(R[:, 2], [math.sin(th) * math.sin(alpha), -math.cos(th) * math.sin(alpha),
                                     math.cos(alpha)], atol=1e-14)


def test_planar_chain_closed_form(orc):
    rng = np.random.default_rng(21)
    a = rng.uniform(0.1, 0.5, size=5)
    dh = np.stack([a, np.zeros(5), np.zeros(5), np.zeros(5)], axis=1)
    q = rng.uniform(-3, 3, size=(10, 5))
    T = orc.fk(dh, q)
    for c in range(10):
        ang = np.cumsum(q[c])
        pos = np.cumsum(a * np.cos(ang)), np.cumsum(a * np.sin(ang))
        assert np.allclose(T[c, 1:, 0, 3], pos[0], atol=1e-13)
        assert np.allclose(T[c, 1:, 1, 3], pos[1], atol=1e-13)
        assert np.allclose(T[c, 1:, 2, 3], 0.0, atol=1e-15)
        assert np.allclose(T[c, -1, 0, 0], math.cos(ang[-1]), atol=1e-13)


def axis_rotation(axis, ang):
    k = axis / np.linalg.norm(axis)
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


def test_joint_rotates_distal_frames_about_its_axis(orc, tiny):
    """Turning joint k by delta rotates every frame k, k+1, ... rigidly about
    the axis z_{k-1} through the origin of frame k-1, and leaves frames
    0..k-1 alone: a structural fact of any serial chain."""
    rng = np.random.default_rng(22)
    dh = tiny.robot.dh
    for _ in range(5):
        q = rng.uniform(-2, 2, size=6)
        T = orc.fk(dh, q[None])[0]
        for k in range(1, 7):
            delta = rng.uniform(-1, 1)
            q2 = q.copy()
            q2[k - 1] += delta
            T2 = orc.fk(dh, q2[None])[0]
            Rax = axis_rotation(T[k - 1][:, 2], delta)
            o = T[k - 1][:, 3]
            for f in range(7):
                if f < k:
                    assert np.allclose(T2[f], T[f], atol=1e-14)
                else:
                    assert np.allclose(T2[f][:, :3], Rax @ T[f][:, :3], atol=1e-12)
                    assert np.allclose(T2[f][:, 3], o + Rax @ (T[f][:, 3] - o), atol=1e-12)


def test_rotations_orthonormal_and_base(orc, tiny):
    rng = np.random.default_rng(23)
    T = orc.fk(tiny.robot.dh, tiny.q)
    R = T[..., :3]
    eye = np.einsum("cliq,cliz->clqz", R, R)
    assert np.allclose(eye, np.eye(3), atol=1e-13)
    assert np.allclose(np.linalg.det(R), 1.0, atol=1e-13)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    base = np.concatenate([q, rng.normal(size=(3, 1))], axis=1)
    Tb = orc.fk(tiny.robot.dh, tiny.q, base)
    assert np.allclose(Tb[..., :3], np.einsum("ab,clbz->claz", q, R), atol=1e-13)
    assert np.allclose(Tb[..., 3], np.einsum("ab,clb->cla", q, T[..., 3]) + base[:, 3], atol=1e-13)


def test_zero_configuration_of_the_synthetic_arm(orc, tiny):
    """At q = 0 consecutive frame origins differ by the DH offsets: |o_k -
    o_{k-1}| = sqrt(a_k^2 + d_k^2) (the link lengths)."""
    dh = tiny.robot.dh
    T = orc.fk(dh, np.zeros((1, 6)))[0]
    steps = np.linalg.norm(np.diff(T[:, :, 3], axis=0), axis=1)
    assert np.allclose(steps, np.hypot(dh[:, 0], dh[:, 2]), atol=1e-14)
