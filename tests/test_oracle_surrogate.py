"""Pins of the FP64 surrogate-network oracle: PyTorch's CPU float64 layers (an independent
library implementation of dense layers and transposed convolution) and finite differences."""
import numpy as np
import torch

from oracle import surrogate as OS


def _torch_net(tp, x):
    """The network from torch's float64 layers; tp maps parameter names to tensors."""
    h = torch.tensor(x)
    hs = []
    for i in range(1, 4):
        h = torch.relu(torch.nn.functional.linear(h, tp[f"W{i}"].T, tp[f"b{i}"]))
        hs.append(h)
    d = h.reshape(-1, 16, 8, 8)
    for i in range(1, 4):
        d = torch.nn.functional.conv_transpose2d(d, tp[f"K{i}"], tp[f"c{i}"], stride=2, padding=1)
        if i < 3:
            d = torch.relu(d)
    a = torch.nn.functional.linear(hs[2], tp["Wa"].T, tp["ba"])
    yb = torch.nn.functional.linear(a, tp["Wb"].T, tp["bb"])
    return d[:, 0] + yb.reshape(-1, 64, 64)


def _torch_forward(p, x):
    return _torch_net({k: torch.tensor(v) for k, v in p.items()}, x)


def test_forward_matches_torch_layers():
    p = OS.init_params(1)
    for k in p:
        if k[0] in "bc":
            p[k] = np.random.default_rng(len(k)).normal(0, 0.1, p[k].shape)
    x = OS.features(np.random.default_rng(2).normal(0, 0.05, (5, 21)), np.linspace(-900, 900, 5))
    y, _ = OS.forward(p, x)
    ref = _torch_forward(p, x).numpy()
    assert y.shape == (5, 64, 64)
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_gradients_match_torch_autograd():
    p = OS.init_params(3)
    rng = np.random.default_rng(4)
    x = OS.features(rng.normal(0, 0.05, (3, 21)), rng.uniform(-1000, 1000, 3))
    target = rng.normal(0, 1, (3, 64, 64))
    loss, g = OS.loss_and_grads(p, x, target)
    tp = {k: torch.tensor(v, requires_grad=True) for k, v in p.items()}
    y = _torch_net(tp, x)
    tl = ((y - torch.tensor(target)) ** 2).mean()
    tl.backward()
    assert abs(loss - tl.item()) < 1e-12 * abs(loss)
    for k in p:
        np.testing.assert_allclose(g[k], tp[k].grad.numpy(), rtol=0, atol=1e-12 * max(1e-30, np.abs(g[k]).max()))


def test_gradient_finite_differences():
    p = OS.init_params(5)
    rng = np.random.default_rng(6)
    x = OS.features(rng.normal(0, 0.05, (2, 21)), rng.uniform(-1000, 1000, 2))
    target = rng.normal(0, 0.5, (2, 64, 64))
    _, g = OS.loss_and_grads(p, x, target)
    for key, idx in [("W1", (3, 17)), ("W3", (100, 7)), ("W2", (900, 1000)), ("b2", (11,)), ("K1", (2, 3, 1, 2)), ("K3", (5, 0, 3, 3)),
                     ("c2", (4,)), ("Wa", (700, 31)), ("ba", (5,)), ("Wb", (200, 2080)), ("bb", (2081,))]:
        h = 1e-6
        pp = {k: v.copy() for k, v in p.items()}
        pm = {k: v.copy() for k, v in p.items()}
        pp[key][idx] += h
        pm[key][idx] -= h
        fd = (OS.loss_and_grads(pp, x, target)[0] - OS.loss_and_grads(pm, x, target)[0]) / (2 * h)
        assert abs(fd - g[key][idx]) < 1e-6 * max(1e-3, abs(g[key][idx])), (key, fd, g[key][idx])


def test_adam_step_closed_form():
    # first Adam step moves every parameter by lr * sign(g) (bias-corrected moments, eps -> 0)
    p = {"a": np.array([1.0, -2.0, 3.0])}
    g = {"a": np.array([0.5, -4.0, 1e-3])}
    m = {"a": np.zeros(3)}
    v = {"a": np.zeros(3)}
    OS.adam_step(p, g, m, v, 1, 0.01, eps=1e-12)
    np.testing.assert_allclose(p["a"], [1.0 - 0.01, -2.0 + 0.01, 3.0 - 0.01], rtol=0, atol=1e-9)
