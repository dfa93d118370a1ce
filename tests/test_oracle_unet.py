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


def _energy_case(seed, dims=(4, 2, 2)):
    import scipy.sparse.linalg as spla
    from oracle import mesh
    g = np.random.default_rng(seed)
    fixed = mesh.cantilever_fixed(dims).astype(bool)
    E = mesh.simp_modulus(g.uniform(0.2, 1.0, size=dims[0] * dims[1] * dims[2]), 3)
    K = mesh.assemble(dims, E, fixed=fixed)
    f = g.standard_normal(fixed.size)
    f[fixed] = 0.0
    fr = ~fixed
    ustar = np.zeros(fixed.size)
    ustar[fr] = spla.spsolve(K[fr][:, fr].tocsc(), f[fr])
    return K, f, ustar, fixed


def test_energy_score_pins():
    """The score is the relative squared energy-norm error of the best
    multiple of the predicted shape: 0 for the solution's shape at any
    scale, 1 for a zero prediction, and for a random shape the minimum over
    alpha of ||alpha u - u*||_K^2 / ||u*||_K^2 found by a scalar minimiser
    (not the closed form); padding voxels do not enter."""
    from scipy.optimize import minimize_scalar
    dims = (4, 2, 2)
    K, f, ustar, fixed = _energy_case(7, dims)
    c = f @ ustar
    shape = (3, 8, 8, 8)
    ys = unet.dofs_to_output(ustar, dims, shape)
    for scale in (1.0, -3.5, 1e-3):
        s, _ = unet.loss_energy((scale * ys)[None], [K], [f], [c], dims, fixed)
        assert abs(s) < 1e-10
    s, dy = unet.loss_energy(np.zeros((1,) + shape), [K], [f], [c], dims, fixed)
    assert s == 1.0
    g = np.random.default_rng(8)
    y = g.standard_normal((1,) + shape)
    u = unet.output_to_dofs(y[0], dims, fixed)
    err = lambda al: (al * u - ustar) @ (K @ (al * u - ustar)) / c
    best = minimize_scalar(err, bracket=(-1.0, 1.0), tol=1e-12)
    s, _ = unet.loss_energy(y, [K], [f], [c], dims, fixed)
    assert abs(s - best.fun) <= 1e-8
    y2 = y.copy()
    y2[0, :, 5:, :, :] = 123.0               # voxels beyond the node grid
    assert unet.loss_energy(y2, [K], [f], [c], dims, fixed)[0] == s


def test_energy_score_gradient_finite_differences():
    """Central differences of the batch-mean score in y, including a padding
    voxel and a clamped DOF (both zero gradient)."""
    dims = (4, 2, 2)
    cases = [_energy_case(s, dims) for s in (9, 10)]
    Ks = [k for k, _, _, _ in cases]
    fs = [f for _, f, _, _ in cases]
    cs = [f @ u for _, f, u, _ in cases]
    fixed = cases[0][3]
    g = np.random.default_rng(11)
    y = g.standard_normal((2, 3, 8, 8, 8))
    s, dy = unet.loss_energy(y, Ks, fs, cs, dims, fixed)
    s0, _ = unet.loss_energy(y[:1], Ks[:1], fs[:1], cs[:1], dims, fixed)
    s1, _ = unet.loss_energy(y[1:], Ks[1:], fs[1:], cs[1:], dims, fixed)
    assert abs(s - 0.5 * (s0 + s1)) < 1e-14
    eps = 1e-6
    for idx in [(0, 0, 1, 2, 3), (1, 2, 2, 1, 4), (1, 1, 0, 0, 4), (0, 1, 6, 1, 1), (0, 0, 0, 0, 0)]:
        old = y[idx]
        y[idx] = old + eps
        lp = unet.loss_energy(y, Ks, fs, cs, dims, fixed)[0]
        y[idx] = old - eps
        lm = unet.loss_energy(y, Ks, fs, cs, dims, fixed)[0]
        y[idx] = old
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - dy[idx]) <= 1e-6 * max(1e-3, abs(fd)), (idx, fd, dy[idx])
    assert dy[0, 1, 6, 1, 1] == 0.0           # padding voxel
    assert dy[0, 0, 0, 0, 0] == 0.0           # node 0 is clamped
