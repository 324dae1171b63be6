"""Pins of the oracle's learned-SDF network (3 -> 128 -> 128 -> 128 -> 1,
SiLU), its L1 loss gradient and its Adam step.

* forward: equal to the same network assembled from PyTorch's CPU Linear
  and SiLU layers in float64 (an independent library implementation);
* gradient: equal to PyTorch autograd of the L1 loss in float64, and to
  central finite differences;
* bfloat16 rounding: equal to PyTorch's float32 -> bfloat16 conversion, in
  the forward pass and at the two backward rounding points (the deltas of
  layers 3 and 2), against PyTorch autograd in float64 with the same casts;
* Adam: the first two steps against their closed forms.
"""
import numpy as np
import pytest
import torch

H = 128


def rand_params(orc, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    P = np.empty(orc.mlp_nparam())
    W1, b1, W2, b2, W3, b3, w4, b4 = orc.mlp_unpack(P)
    for W, fan in ((W1, 3), (b1, 3), (W2, H), (b2, H), (W3, H), (b3, H), (w4, H), (b4, H)):
        W[...] = rng.uniform(-1, 1, size=W.shape) * scale / np.sqrt(fan)
    return P


def torch_net(orc, P):
    W1, b1, W2, b2, W3, b3, w4, b4 = [torch.tensor(a) for a in orc.mlp_unpack(P)]
    net = torch.nn.Sequential(torch.nn.Linear(3, H), torch.nn.SiLU(), torch.nn.Linear(H, H), torch.nn.SiLU(),
                              torch.nn.Linear(H, H), torch.nn.SiLU(), torch.nn.Linear(H, 1)).double()
    with torch.no_grad():
        net[0].weight.copy_(W1); net[0].bias.copy_(b1)
        net[2].weight.copy_(W2); net[2].bias.copy_(b2)
        net[4].weight.copy_(W3); net[4].bias.copy_(b3)
        net[6].weight.copy_(w4[None]); net[6].bias.copy_(b4)
    return net


def test_forward_matches_torch(orc):
    P = rand_params(orc, 1, scale=2.0)
    X = np.random.default_rng(2).uniform(-1, 1, size=(64, 3))
    got = orc.mlp_forward(P, X)
    want = torch_net(orc, P)(torch.tensor(X)).detach().numpy()[:, 0]
    assert np.max(np.abs(got - want)) < 1e-12


def test_loss_grad_matches_torch_autograd(orc):
    P = rand_params(orc, 3, scale=2.0)
    rng = np.random.default_rng(4)
    X = rng.uniform(-1, 1, size=(40, 3))
    Y = rng.uniform(-2, 2, size=40)
    loss, g = orc.mlp_loss_grad(P, X, Y)
    net = torch_net(orc, P)
    out = net(torch.tensor(X))[:, 0]
    tl = torch.nn.functional.l1_loss(out, torch.tensor(Y))
    tl.backward()
    tg = np.concatenate([net[0].weight.grad.numpy().ravel(), net[0].bias.grad.numpy(),
                         net[2].weight.grad.numpy().ravel(), net[2].bias.grad.numpy(),
                         net[4].weight.grad.numpy().ravel(), net[4].bias.grad.numpy(),
                         net[6].weight.grad.numpy().ravel(), net[6].bias.grad.numpy()])
    assert loss == pytest.approx(tl.item(), abs=1e-14)
    assert np.max(np.abs(g - tg)) < 1e-13 * max(1.0, np.abs(tg).max())


def test_loss_grad_central_differences(orc):
    P = rand_params(orc, 5, scale=2.0)
    rng = np.random.default_rng(6)
    X = rng.uniform(-1, 1, size=(16, 3))
    Y = orc.mlp_forward(P, X) + rng.choice([-1.0, 1.0], size=16) * 0.5   # far from the kinks of |r|
    _, g = orc.mlp_loss_grad(P, X, Y)
    idx = np.concatenate([rng.choice(384, 8, replace=False),                 # W1
                          384 + rng.choice(128, 4, replace=False),           # b1
                          512 + rng.choice(H * H, 8, replace=False),         # W2
                          16640 + rng.choice(H * H, 8, replace=False),       # W3
                          33280 + rng.choice(H, 4, replace=False), [33664]])  # w4, b4
    h = 1e-6
    for k in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[k] += h
        Pm[k] -= h
        fd = (orc.mlp_loss_grad(Pp, X, Y)[0] - orc.mlp_loss_grad(Pm, X, Y)[0]) / (2 * h)
        assert fd == pytest.approx(g[k], rel=1e-6, abs=1e-9), k


def test_bf16_rounding_matches_torch(orc):
    # a network whose only path is w4 * h3 with h3 = SiLU(b3): the bf16 twin
    # must round w4 and SiLU(b3) exactly as torch rounds float32 to bfloat16
    P = np.zeros(orc.mlp_nparam())
    W1, b1, W2, b2, W3, b3, w4, b4 = orc.mlp_unpack(P)
    rng = np.random.default_rng(7)
    b3[:] = rng.normal(size=H)
    w4[:] = rng.normal(size=H)
    got = orc.mlp_forward(P, np.zeros((1, 3)), bf16=True)[0]
    sil = torch.nn.functional.silu(torch.tensor(b3)).float().bfloat16().double()
    want = float((torch.tensor(w4).float().bfloat16().double() * sil).sum())
    assert got == pytest.approx(want, abs=1e-12)
    assert abs(got - orc.mlp_forward(P, np.zeros((1, 3)))[0]) > 1e-6     # rounding did happen


class _RoundValue(torch.autograd.Function):
    """Value rounded to bfloat16 (float64 -> float32 -> bfloat16, torch's own
    round-to-nearest-even), gradient passed through unchanged."""
    @staticmethod
    def forward(ctx, x):
        return x.float().bfloat16().double()

    @staticmethod
    def backward(ctx, g):
        return g


class _RoundGrad(torch.autograd.Function):
    """Value unchanged, gradient rounded to bfloat16 on its way back."""
    @staticmethod
    def forward(ctx, x):
        return x.clone()

    @staticmethod
    def backward(ctx, g):
        return g.float().bfloat16().double()


def _torch_bf16_grad(orc, P, X, Y, round_d3=True, round_d2=True, round_d1=False):
    """L1 loss gradient of the network by PyTorch autograd in float64, with
    the weights and the activations h1..h3 rounded to bfloat16 in the forward
    pass and the gradients at the pre-activations z3, z2 (optionally z1)
    rounded in the backward pass."""
    rv, rg = _RoundValue.apply, _RoundGrad.apply
    ts = [torch.tensor(a, requires_grad=True) for a in orc.mlp_unpack(P)]
    W1, b1, W2, b2, W3, b3, w4, b4 = ts
    x = torch.tensor(X)
    z1 = x @ rv(W1).T + b1
    if round_d1:
        z1 = rg(z1)
    h1 = rv(torch.nn.functional.silu(z1))
    z2 = h1 @ rv(W2).T + b2
    if round_d2:
        z2 = rg(z2)
    h2 = rv(torch.nn.functional.silu(z2))
    z3 = h2 @ rv(W3).T + b3
    if round_d3:
        z3 = rg(z3)
    h3 = rv(torch.nn.functional.silu(z3))
    m = h3 @ rv(w4) + b4
    loss = torch.nn.functional.l1_loss(m, torch.tensor(Y))
    loss.backward()
    return loss.item(), np.concatenate([t.grad.numpy().ravel() for t in ts])


def test_bf16_backward_rounding_matches_torch(orc):
    """The bfloat16 twin's gradient (the GPU kernels' rounding points: weights
    and activations in the forward pass, the deltas of layers 3 and 2 before
    they are multiplied) against PyTorch autograd in float64 with the same
    casts placed independently.  Moving, dropping or adding one backward
    rounding point changes the gradient far beyond the agreement found."""
    P = rand_params(orc, 9, scale=2.0)
    rng = np.random.default_rng(10)
    X = rng.uniform(-1, 1, size=(48, 3))
    Y = orc.mlp_forward(P, X, bf16=True) + rng.choice([-0.5, 0.5], size=48)
    loss, g = orc.mlp_loss_grad(P, X, Y, bf16=True)
    tl, tg = _torch_bf16_grad(orc, P, X, Y)
    scale = np.abs(tg).max()
    assert loss == pytest.approx(tl, abs=1e-13)
    assert np.max(np.abs(g - tg)) <= 1e-12 * scale
    for variant in ({"round_d3": False}, {"round_d2": False}, {"round_d1": True}):
        _, vg = _torch_bf16_grad(orc, P, X, Y, **variant)
        assert np.max(np.abs(g - vg)) > 1e-6 * scale, variant


def test_adam_first_two_steps_closed_form(orc):
    rng = np.random.default_rng(8)
    n = 50
    P0 = rng.normal(size=n)
    g1, g2 = rng.normal(size=n), rng.normal(size=n)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    P, m, v = P0.copy(), np.zeros(n), np.zeros(n)
    orc.adam_step(P, m, v, g1, 1, lr, b1, b2, eps)
    # step 1: bias-corrected moments are g and g^2, so the step is lr * g / (|g| + eps)
    assert np.allclose(P, P0 - lr * g1 / (np.abs(g1) + eps), rtol=0, atol=1e-15)
    P1 = P.copy()
    orc.adam_step(P, m, v, g2, 2, lr, b1, b2, eps)
    mh = (b1 * (1 - b1) * g1 + (1 - b1) * g2) / (1 - b1 ** 2)
    vh = (b2 * (1 - b2) * g1 ** 2 + (1 - b2) * g2 ** 2) / (1 - b2 ** 2)
    assert np.allclose(P, P1 - lr * mh / (np.sqrt(vh) + eps), rtol=0, atol=1e-15)


# ---------------------------------------------------------------------------
# learned clearance with the margin fallback (orc_query_mlp)
# ---------------------------------------------------------------------------

def _mlp_setup(orc, tiny, C=4):
    import synth
    T32 = orc.fk(tiny.robot.dh, tiny.q[:C], tiny.robot.base_T).astype(np.float32)
    dc, dh = synth.mlp_domain(tiny.grid_lo.astype(np.float64), tiny.grid_hi.astype(np.float64))
    pts = tiny.points[:600].astype(np.float32)
    return T32, dc, dh, pts


def _in_domain(T32, dc, dh, pts):
    """[C][L][M] domain membership and normalised inputs, numpy double."""
    T = T32.astype(np.float64)
    loc = np.einsum("jb,clba->clja", pts.astype(np.float64), T[..., :3]) \
        - np.einsum("clb,clba->cla", T[..., 3], T[..., :3])[:, :, None, :]
    X = (loc - dc[None, :, None, :]) / dh[None, :, None, :]
    return np.all(np.abs(X) <= 1.0, axis=-1), X


def test_query_mlp_without_fallback_is_network_min(orc, tiny):
    """margin = -inf: every in-domain pair takes the network's value, so the
    per-link minimum is the bfloat16 twin network's minimum over the points
    in that link's domain (domain test and inputs formed here in numpy)."""
    T32, dc, dh, pts = _mlp_setup(orc, tiny)
    P = np.stack([rand_params(orc, 20 + i) for i in range(tiny.L)])
    g32 = [g.astype(np.float32) for g in orc.workload_grids(tiny)]
    got = orc.query_mlp(T32, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, g32, pts, P, dc, dh, -np.inf)
    ind, X = _in_domain(T32, dc, dh, pts)
    for c in range(T32.shape[0]):
        for i in range(tiny.L):
            want = orc.mlp_forward(P[i], X[c, i][ind[c, i]], bf16=True).min() if ind[c, i].any() else np.inf
            assert got[c, i] == pytest.approx(want, abs=1e-12), (c, i)
    assert np.isfinite(got).mean() > 0.5


@pytest.mark.parametrize("k", [0.01, 0.05, 0.2])
def test_query_mlp_fallback_rule_with_constant_network(orc, tiny, tiny_grids, k):
    """A network that outputs the constant k (every weight zero, b4 = k)
    at margin 0.05.  Below the margin (k = 0.01) an in-box pair takes the
    single-precision twin's grid value and a pair outside the box keeps k;
    at the margin itself (k = 0.05, the test is strict) and above it every
    in-domain pair keeps k."""
    T32, dc, dh, pts = _mlp_setup(orc, tiny)
    P = np.zeros((tiny.L, orc.mlp_nparam()))
    P[:, -1] = k
    g32 = [g.astype(np.float32) for g in tiny_grids]
    got = orc.query_mlp(T32, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, g32, pts, P, dc, dh, 0.05)
    ind, _ = _in_domain(T32, dc, dh, pts)
    each = orc.query_f32_each(T32, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, g32, pts).astype(np.float64)
    inbox = np.isfinite(each)
    assert np.all(ind[inbox])                    # the grid box lies inside the domain
    for c in range(T32.shape[0]):
        for i in range(tiny.L):
            if k < 0.05:
                grid_part = each[c, i][inbox[c, i]].min() if inbox[c, i].any() else np.inf
                far_part = k if (ind[c, i] & ~inbox[c, i]).any() else np.inf
                want = min(grid_part, far_part)
            else:
                want = k if ind[c, i].any() else np.inf
            assert got[c, i] == want, (c, i, got[c, i], want)
    if k < 0.05:
        assert (inbox.any(-1) & (got < k)).any()     # some minima come from the grid


# ---------------------------------------------------------------------------
# the core term: the estimate is the network plus the distance to the core box
# ---------------------------------------------------------------------------

_CORE_C = np.array([0.1, -0.2, 0.3])
_CORE_K = np.array([0.2, 0.1, 0.3])
_CORE_H = np.array([1.5, 1.4, 1.6])


@pytest.mark.parametrize("bf16", [False, True])
def test_core_term_closed_forms(orc, bf16):
    """A network that outputs the constant b4 (every weight zero, SiLU(0) =
    0): the estimate is b4 + the distance to the core box, worked out by hand
    for points inside it, on a face, beyond a face, an edge (3-4-5) and a
    corner (3-4-12-13)."""
    P = np.zeros(orc.mlp_nparam())
    c, k = _CORE_C, _CORE_K
    pts = np.array([c,                                              # centre
                    c + [0.1, 0.05, -0.2],                          # inside
                    c + [0.2, 0.0, 0.0],                            # on a face
                    c + [0.2 + 0.05, 0.0, 0.0],                     # beyond a face
                    c + [0.0, -(0.1 + 0.03), 0.3 + 0.04],           # beyond an edge
                    c + [0.2 + 0.03, 0.1 + 0.04, -(0.3 + 0.12)]])   # beyond a corner
    want = np.array([0.0, 0.0, 0.0, 0.05, 0.05, 0.13])
    for b4 in (0.0, 0.25):
        P[-1] = b4
        got = orc.mlp_value(P, pts, c, _CORE_H, k, bf16=bf16)
        assert np.allclose(got, b4 + want, rtol=0, atol=1e-15), (b4, got)
    # without a core box the estimate is the network alone
    assert np.all(orc.mlp_value(P, pts, c, _CORE_H, None, bf16=bf16) == 0.25)


def test_core_term_adds_the_projection_distance(orc):
    """A random network: the estimate equals the network at the normalised
    point plus the distance from the point to its projection onto the box
    (a clamp, formed here independently of the oracle's formula)."""
    P = rand_params(orc, 31, scale=2.0)
    rng = np.random.default_rng(32)
    pts = _CORE_C + rng.uniform(-1.2, 1.2, size=(200, 3)) * _CORE_H
    proj = np.clip(pts, _CORE_C - _CORE_K, _CORE_C + _CORE_K)
    want = orc.mlp_forward(P, (pts - _CORE_C) / _CORE_H) + np.linalg.norm(pts - proj, axis=1)
    got = orc.mlp_value(P, pts, _CORE_C, _CORE_H, _CORE_K)
    assert np.max(np.abs(got - want)) < 1e-12
    assert np.mean(np.linalg.norm(pts - proj, axis=1) > 0) > 0.5      # most points lie outside the box


def test_loss_grad_with_offset_matches_torch_autograd(orc):
    """The loss of the estimate network(x) + D against Y, and its gradient,
    against PyTorch autograd in float64 with the offset added there."""
    P = rand_params(orc, 33, scale=2.0)
    rng = np.random.default_rng(34)
    X = rng.uniform(-1, 1, size=(40, 3))
    D = rng.uniform(0.0, 0.8, size=40)
    Y = rng.uniform(-1, 2, size=40)
    loss, g = orc.mlp_loss_grad(P, X, Y, offset=D)
    net = torch_net(orc, P)
    out = net(torch.tensor(X))[:, 0] + torch.tensor(D)
    tl = torch.nn.functional.l1_loss(out, torch.tensor(Y))
    tl.backward()
    tg = np.concatenate([net[0].weight.grad.numpy().ravel(), net[0].bias.grad.numpy(),
                         net[2].weight.grad.numpy().ravel(), net[2].bias.grad.numpy(),
                         net[4].weight.grad.numpy().ravel(), net[4].bias.grad.numpy(),
                         net[6].weight.grad.numpy().ravel(), net[6].bias.grad.numpy()])
    assert loss == pytest.approx(tl.item(), abs=1e-14)
    assert np.max(np.abs(g - tg)) < 1e-13 * max(1.0, np.abs(tg).max())
    # the offset matters: without it some residual signs differ
    _, g0 = orc.mlp_loss_grad(P, X, Y)
    assert np.max(np.abs(g0 - g)) > 1e-3 * np.abs(tg).max()


@pytest.mark.parametrize("margin", [-np.inf, 0.05])
def test_query_mlp_core_term_with_constant_network(orc, tiny, tiny_grids, margin):
    """A constant network b4 = 0.01 with each link's core box (its mesh's
    bounding box): an in-domain pair's estimate is 0.01 + its distance to
    the box (a clamp, in numpy).  margin -inf: the per-link minimum is the
    smallest estimate; margin 0.05: a pair whose estimate is below the
    margin and whose point is in the grid box takes the single-precision
    twin's grid value instead."""
    import synth
    T32, dc, dh, pts = _mlp_setup(orc, tiny)
    ck = synth.mlp_core(tiny.grid_lo, tiny.grid_hi)
    alo = np.array([m.verts.min(0) for m in tiny.robot.links])
    ahi = np.array([m.verts.max(0) for m in tiny.robot.links])
    assert np.allclose(dc - ck, alo, atol=1e-6) and np.allclose(dc + ck, ahi, atol=1e-6)
    P = np.zeros((tiny.L, orc.mlp_nparam()))
    P[:, -1] = 0.01
    g32 = [g.astype(np.float32) for g in tiny_grids]
    got = orc.query_mlp(T32, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, g32, pts, P, dc, dh, margin, core_k=ck)
    ind, X = _in_domain(T32, dc, dh, pts)
    loc = X * dh[None, :, None, :] + dc[None, :, None, :]
    proj = np.clip(loc, (dc - ck)[None, :, None, :], (dc + ck)[None, :, None, :])
    est = 0.01 + np.linalg.norm(loc - proj, axis=-1)
    each = orc.query_f32_each(T32, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, g32, pts).astype(np.float64)
    if margin > 0:
        est = np.where((est < margin) & np.isfinite(each), each, est)
    want = np.where(ind, est, np.inf).min(-1)
    assert np.max(np.abs(np.where(np.isfinite(want), got - want, 0))) < 1e-9
    assert np.array_equal(np.isfinite(got), np.isfinite(want))
    if margin > 0:
        assert ((got < 0.01) & np.isfinite(got)).any()             # some minima come from the grid


# ---------------------------------------------------------------------------
# the remainder bound: the network's share is B tanh(m / B)
# ---------------------------------------------------------------------------

def test_bounded_share_closed_forms(orc):
    """A constant network b4 = k with bound B: the estimate is E + B tanh(k/B);
    tanh(0.5) = 0.46211715726000974 and tanh(2) = 0.9640275800758169 (tables),
    and a zero network gives E exactly."""
    P = np.zeros(orc.mlp_nparam())
    pts = np.array([_CORE_C, _CORE_C + [0.2 + 0.05, 0.0, 0.0]])       # E = 0 and 0.05
    E = np.array([0.0, 0.05])
    assert np.allclose(orc.mlp_value(P, pts, _CORE_C, _CORE_H, _CORE_K, bound=0.2), E, rtol=0, atol=1e-15)
    P[-1] = 0.1
    got = orc.mlp_value(P, pts, _CORE_C, _CORE_H, _CORE_K, bound=0.2)
    assert np.allclose(got, E + 0.2 * 0.46211715726000974, rtol=0, atol=1e-15)
    P[-1] = -0.4
    got = orc.mlp_value(P, pts, _CORE_C, _CORE_H, _CORE_K, bound=0.2, bf16=True)
    assert np.allclose(got, E - 0.2 * 0.9640275800758169, rtol=0, atol=1e-15)


def test_bounded_share_stays_within_the_bound(orc):
    """A random network with large outputs: every estimate lies within B of
    the core distance, and with B = inf the estimate is the unbounded one."""
    P = rand_params(orc, 35, scale=6.0)
    rng = np.random.default_rng(36)
    pts = _CORE_C + rng.uniform(-1, 1, size=(300, 3)) * _CORE_H
    E = orc.mlp_value(np.zeros_like(P), pts, _CORE_C, _CORE_H, _CORE_K)
    raw = orc.mlp_value(P, pts, _CORE_C, _CORE_H, _CORE_K) - E
    assert np.abs(raw).max() > 1.0                                    # the network does exceed the bound
    got = orc.mlp_value(P, pts, _CORE_C, _CORE_H, _CORE_K, bound=0.15)
    assert np.all(np.abs(got - E) <= 0.15 + 1e-12)                  # (up to the rounding of the sum)
    assert np.allclose(got - E, 0.15 * np.tanh(raw / 0.15), rtol=0, atol=1e-12)


def test_loss_grad_with_bound_matches_torch_autograd(orc):
    """Loss of E + B tanh(net / B) against Y and its gradient, against PyTorch
    autograd in float64 (torch.tanh)."""
    P = rand_params(orc, 37, scale=2.0)
    rng = np.random.default_rng(38)
    X = rng.uniform(-1, 1, size=(40, 3))
    D = rng.uniform(0.0, 0.8, size=40)
    Y = rng.uniform(-0.2, 1.0, size=40)
    B = 0.3
    loss, g = orc.mlp_loss_grad(P, X, Y, offset=D, bound=B)
    net = torch_net(orc, P)
    out = B * torch.tanh(net(torch.tensor(X))[:, 0] / B) + torch.tensor(D)
    tl = torch.nn.functional.l1_loss(out, torch.tensor(Y))
    tl.backward()
    tg = np.concatenate([net[0].weight.grad.numpy().ravel(), net[0].bias.grad.numpy(),
                         net[2].weight.grad.numpy().ravel(), net[2].bias.grad.numpy(),
                         net[4].weight.grad.numpy().ravel(), net[4].bias.grad.numpy(),
                         net[6].weight.grad.numpy().ravel(), net[6].bias.grad.numpy()])
    assert loss == pytest.approx(tl.item(), abs=1e-14)
    assert np.max(np.abs(g - tg)) < 1e-13 * max(1.0, np.abs(tg).max())
    _, g_inf = orc.mlp_loss_grad(P, X, Y, offset=D)
    assert np.max(np.abs(g_inf - g)) > 1e-3 * np.abs(tg).max()        # the bound changes the gradient


def test_query_mlp_bound_with_constant_network(orc, tiny, tiny_grids):
    """A constant network b4 = 0.3 with bound 0.1 and each link's core box:
    every in-domain estimate is E + 0.1 tanh(3) (tanh(3) =
    0.9950547536867305), margin -inf."""
    import synth
    T32, dc, dh, pts = _mlp_setup(orc, tiny)
    ck = synth.mlp_core(tiny.grid_lo, tiny.grid_hi)
    P = np.zeros((tiny.L, orc.mlp_nparam()))
    P[:, -1] = 0.3
    g32 = [g.astype(np.float32) for g in tiny_grids]
    got = orc.query_mlp(T32, tiny.grid_lo, tiny.grid_hi, tiny.grid_n, g32, pts, P, dc, dh, -np.inf, core_k=ck,
                        bounds=np.full(tiny.L, 0.1))
    ind, X = _in_domain(T32, dc, dh, pts)
    loc = X * dh[None, :, None, :] + dc[None, :, None, :]
    proj = np.clip(loc, (dc - ck)[None, :, None, :], (dc + ck)[None, :, None, :])
    est = 0.1 * 0.9950547536867305 + np.linalg.norm(loc - proj, axis=-1)
    want = np.where(ind, est, np.inf).min(-1)
    assert np.array_equal(np.isfinite(got), np.isfinite(want))
    assert np.max(np.abs(np.where(np.isfinite(want), got - want, 0))) < 1e-9
