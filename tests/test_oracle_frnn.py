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

from frnn_util import centres, exact_params, random_rotations


def test_target_is_rotated_voxel_centres(orc):
    m = 3
    R = random_rotations(5, 100)
    got = orc.frnn_target(m, R).reshape(5, -1, 3)
    P = centres(m)
    want = np.einsum("sba,jb->sja", R, P)
    assert np.abs(got - want).max() < 1e-15
    assert np.abs(P).max() == pytest.approx(1 - 0.5 / m)


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
