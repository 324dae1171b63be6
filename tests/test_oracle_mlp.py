"""Pins of the oracle's learned-SDF network (3 -> 128 -> 128 -> 128 -> 1,
SiLU), its L1 loss gradient and its Adam step.

* forward: equal to the same network assembled from PyTorch's CPU Linear
  and SiLU layers in float64 (an independent library implementation);
* gradient: equal to PyTorch autograd of the L1 loss in float64, and to
  central finite differences;
* bfloat16 rounding: equal to PyTorch's float32 -> bfloat16 conversion;
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
