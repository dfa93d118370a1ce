"""GPU parity and behaviour of the warm-start U-Net (BASELINE extension 4).

Forward and gradients of the device network are compared with the FP64
oracle using the same BF16-rounded weights (the device computes in FP32:
tolerance 1e-4 on outputs, 1e-3 on gradient norms per layer).  Training
must lower the loss, and a trained prediction (energy-optimally scaled) must
not cost PCG-GMG iterations at the same tolerance.
"""
import numpy as np
import pytest

import workloads
from oracle import bf16, unet
from tests.gpu_util import np64, t32, t64

pytestmark = pytest.mark.gpu


def _flat(params):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params])


def _rounded_params(seed):
    params = unet.init_params(seed=seed)
    out = []
    for w, b in params:
        out.append((bf16.round_bf16(w), np.random.default_rng(seed).standard_normal(b.shape) * 0.05))
    return out


def test_forward_matches_oracle():
    from paper_2604_26441_amd import simpgmg
    params = _rounded_params(4)
    net = simpgmg.UNet(seed=1)
    net.set_params(_flat(params))
    x = np.random.default_rng(5).standard_normal((2, 5, 16, 8, 8))
    y = np64(net.forward(t32(x)))
    ref, _ = unet.forward(params, x.astype(np.float32).astype(np.float64))
    assert np.abs(y - ref).max() <= 1e-4 * np.abs(ref).max()


def test_gradients_match_oracle():
    from paper_2604_26441_amd import simpgmg
    params = _rounded_params(6)
    net = simpgmg.UNet(seed=1)
    net.set_params(_flat(params))
    g = np.random.default_rng(7)
    x = g.standard_normal((2, 5, 8, 16, 8)).astype(np.float32).astype(np.float64)
    t = g.standard_normal((2, 3, 8, 16, 8)).astype(np.float32).astype(np.float64)
    mask = (g.uniform(size=(2, 1, 8, 16, 8)) > 0.3).astype(np.float64)
    loss, grads = net.grad(t32(x), t32(t), t32(mask))
    y, cache = unet.forward(params, x)
    lref, dy = unet.loss_mse(y, t, mask)
    gref = unet.backward(params, cache, dy)
    assert abs(loss - lref) <= 1e-5 * abs(lref)
    off = 0
    for (dw, db) in gref:
        gw = grads[off:off + dw.size].reshape(dw.shape)
        off += dw.size
        gb = grads[off:off + db.size]
        off += db.size
        assert np.linalg.norm(gw - dw) <= 1e-3 * np.linalg.norm(dw)
        assert np.linalg.norm(gb - db) <= 1e-3 * max(np.linalg.norm(db), 1e-12)


def test_training_and_warm_start():
    import torch
    from paper_2604_26441_amd import simpgmg
    dims = (16, 8, 8)
    rng = np.random.default_rng(11)
    xs, ts, ms, cases = [], [], [], []
    for k in range(33):
        rho = workloads.grf_rho(dims, seed=500 + k)
        f = workloads.random_face_load(dims, rng)
        o = simpgmg.default_options(*dims, n_levels=3, fine_prec="f64")
        h = simpgmg.setup_hierarchy(o, t64(rho))
        u = t64(np.zeros_like(f))
        res = simpgmg.pcg_solve(h, t64(f), u, rtol=1e-10, maxit=300)
        assert res["status"] == "converged"
        x = simpgmg.unet_input(h, t64(rho), t64(f))
        t, m = simpgmg.unet_target(h, u)
        xs.append(x); ts.append(t); ms.append(m); cases.append((rho, f))
    X, T, M = torch.cat(xs[:32]), torch.cat(ts[:32]), torch.cat(ms[:32])
    net = simpgmg.UNet(seed=3)
    losses = []
    for step in range(160):
        idx = torch.as_tensor(rng.choice(32, size=8, replace=False), device=X.device)
        losses.append(net.train_step(X[idx].contiguous(), T[idx].contiguous(), M[idx].contiguous(), lr=2e-3))
    assert np.mean(losses[-10:]) < 0.5 * np.mean(losses[:10])
    # held-out case: warm start vs zero start at the same tolerance
    rho, f = cases[32]
    o = simpgmg.default_options(*dims, n_levels=3)
    h = simpgmg.setup_hierarchy(o, t64(rho))
    u_cold = t64(np.zeros_like(f))
    cold = simpgmg.pcg_solve(h, t64(f), u_cold, rtol=1e-6, maxit=300, history_cap=512)
    y = net.forward(xs[32])
    u0 = simpgmg.unet_output(h, y)
    alpha = simpgmg.warm_start_scale(h, t64(f), u0)
    assert alpha > 0
    warm = simpgmg.pcg_solve(h, t64(f), u0, rtol=1e-6, maxit=300, history_cap=512)
    assert warm["status"] == "converged" == cold["status"]
    assert warm["history"][0] < 1.0                    # better than the zero start
    assert warm["iters"] <= cold["iters"]
