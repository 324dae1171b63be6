"""Pins of the oracle's tiny grid-transformation network (Sec. III-B-1,
Eq. 4-5): the target R^T P, the forward pass, the L1 loss and its gradient.

* The target equals R^T P written independently here with numpy (a
  transposed rotation or a wrong voxel order fails).
* A network built by hand to represent R^T P exactly (pairs of ReLU units
  carry each rotation entry as relu(x) - relu(-x)) reproduces the target:
  this pins the parameter layout and the output order.
* The analytic gradient matches central differences.
"""
import numpy as np
import pytest

H = 32


def random_rotations(n, seed):
    rng = np.random.default_rng(seed)
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1)], 1)


def centres(m):
    w = 2 * m
    jz, jy, jx = np.meshgrid(np.arange(w), np.arange(w), np.arange(w), indexing="ij")
    return np.stack([(jx + 0.5) / m - 1, (jy + 0.5) / m - 1, (jz + 0.5) / m - 1], -1).reshape(-1, 3)


def test_target_is_rotated_voxel_centres(orc):
    m = 3
    R = random_rotations(5, 100)
    got = orc.frnn_target(m, R).reshape(5, -1, 3)
    P = centres(m)
    want = np.einsum("sba,jb->sja", R, P)
    assert np.abs(got - want).max() < 1e-15
    assert np.abs(P).max() == pytest.approx(1 - 0.5 / m)


def exact_params(m):
    P = centres(m)
    V = P.shape[0]
    W1 = np.zeros((H, 9))
    for k in range(9):
        W1[2 * k, k] = 1.0
        W1[2 * k + 1, k] = -1.0
    b1 = np.zeros(H)
    W2 = np.zeros((3 * V, H))
    for j in range(V):
        for a in range(3):
            for b in range(3):
                k = 3 * b + a                      # x_k = R[b][a]
                W2[3 * j + a, 2 * k] = P[j, b]
                W2[3 * j + a, 2 * k + 1] = -P[j, b]
    return np.concatenate([W1.ravel(), b1, W2.ravel(), np.zeros(3 * V)])


def test_hand_built_network_is_exact(orc):
    m = 2
    p = exact_params(m)
    assert p.size == orc.frnn_nparam(m)
    R = random_rotations(7, 101)
    out = orc.frnn_forward(p, m, R)
    assert np.abs(out - orc.frnn_target(m, R)).max() < 1e-15
    loss, _ = orc.frnn_loss_grad(p, m, R)
    assert loss < 1e-15


def test_gradient_matches_central_differences(orc):
    m = 1
    rng = np.random.default_rng(102)
    n = orc.frnn_nparam(m)
    p = rng.normal(scale=0.3, size=n)
    R = random_rotations(6, 103)
    loss, g = orc.frnn_loss_grad(p, m, R)
    assert loss > 0
    h = 1e-6
    for k in rng.choice(n, size=60, replace=False):
        e = np.zeros(n)
        e[k] = h
        fd = (orc.frnn_loss_grad(p + e, m, R)[0] - orc.frnn_loss_grad(p - e, m, R)[0]) / (2 * h)
        assert fd == pytest.approx(g[k], rel=1e-5, abs=1e-9), k
