"""Pins of the U-Net oracle: convolution against torch's CPU conv3d (a library
routine), gradients against torch autograd and central finite differences."""
import numpy as np
import torch

from oracle import unet


def test_conv3d_matches_torch():
    g = np.random.default_rng(0)
    for k in (1, 3):
        x = g.standard_normal((2, 5, 6, 4, 8))
        w = g.standard_normal((7, 5, k, k, k))
        b = g.standard_normal(7)
        ref = torch.nn.functional.conv3d(torch.from_numpy(x), torch.from_numpy(w), torch.from_numpy(b),
                                         padding=k // 2).numpy()
        assert np.abs(unet.conv3d(x, w, b) - ref).max() < 1e-12


def test_conv3d_backward_matches_autograd():
    g = np.random.default_rng(1)
    x = g.standard_normal((2, 3, 4, 6, 4))
    w = g.standard_normal((5, 3, 3, 3, 3))
    b = g.standard_normal(5)
    dy = g.standard_normal((2, 5, 4, 6, 4))
    xt = torch.from_numpy(x).requires_grad_()
    wt = torch.from_numpy(w).requires_grad_()
    bt = torch.from_numpy(b).requires_grad_()
    (torch.nn.functional.conv3d(xt, wt, bt, padding=1) * torch.from_numpy(dy)).sum().backward()
    dx, dw, db = unet.conv3d_backward(x, w, dy)
    assert np.abs(dx - xt.grad.numpy()).max() < 1e-12
    assert np.abs(dw - wt.grad.numpy()).max() < 1e-11
    assert np.abs(db - bt.grad.numpy()).max() < 1e-12


def test_pool_up_adjoint():
    g = np.random.default_rng(2)
    a = g.standard_normal((1, 2, 4, 4, 4))
    c = g.standard_normal((1, 2, 2, 2, 2))
    assert abs((unet.pool(a) * c).sum() - (a * unet.pool_backward(c)).sum()) < 1e-12
    assert abs((unet.up(c) * a).sum() - (c * unet.up_backward(a)).sum()) < 1e-12


def test_network_gradient_finite_differences():
    """Central differences of the masked MSE loss on a tiny input."""
    g = np.random.default_rng(3)
    params = unet.init_params(seed=4)
    x = g.standard_normal((1, 5, 8, 8, 8))
    t = g.standard_normal((1, 3, 8, 8, 8))
    mask = (g.uniform(size=(1, 1, 8, 8, 8)) > 0.2).astype(float)
    y, cache = unet.forward(params, x)
    loss, dy = unet.loss_mse(y, t, mask)
    grads = unet.backward(params, cache, dy)
    eps = 1e-6
    for layer, idx in [(0, (3, 1, 0, 1, 2)), (3, (10, 40, 1, 1, 1)), (4, (5, 100, 2, 0, 1)),
                       (7, (2, 7, 0, 0, 0))]:
        w = params[layer][0]
        old = w[idx]
        w[idx] = old + eps
        lp, _ = unet.loss_mse(unet.forward(params, x)[0], t, mask)
        w[idx] = old - eps
        lm, _ = unet.loss_mse(unet.forward(params, x)[0], t, mask)
        w[idx] = old
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - grads[layer][0][idx]) <= 1e-6 * max(1.0, abs(fd)), (layer, fd, grads[layer][0][idx])
    for layer in (1, 6):
        b = params[layer][1]
        old = b[2]
        b[2] = old + eps
        lp, _ = unet.loss_mse(unet.forward(params, x)[0], t, mask)
        b[2] = old - eps
        lm, _ = unet.loss_mse(unet.forward(params, x)[0], t, mask)
        b[2] = old
        assert abs((lp - lm) / (2 * eps) - grads[layer][1][2]) <= 1e-6


def test_parameter_count():
    n = sum(w.size + b.size for w, b in unet.init_params())
    assert 400_000 < n < 700_000
