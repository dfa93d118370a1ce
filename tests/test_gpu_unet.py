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
from oracle import bf16, mesh, unet
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
    """Training on solver-generated pairs lowers the loss; on a case it was
    trained on, the scaled prediction removes part of the initial error in
    the energy norm (the norm the scaled start minimises) and PCG-GMG needs
    no more iterations to the same tolerance; on a held-out case the scale is
    the energy-optimal one, so the start's energy-norm error is never above
    the zero start's.  (A close L2 fit is a much weaker start in the energy
    norm: K weights the fit's high-frequency error.)"""
    import torch
    import scipy.sparse.linalg as spla
    from paper_2604_26441_amd import simpgmg
    dims = (16, 8, 8)
    rng = np.random.default_rng(11)
    fixed = workloads.cantilever_fixed(dims).astype(bool)
    xs, ts, ms, cases = [], [], [], []
    for k in range(9):
        rho = workloads.grf_rho(dims, seed=500 + k) if k % 2 else workloads.uniform_rho(dims)
        f = workloads.random_face_load(dims, rng) if k else workloads.edge_load(dims)
        o = simpgmg.default_options(*dims, n_levels=3, fine_prec="f64")
        h = simpgmg.setup_hierarchy(o, t64(rho))
        u = t64(np.zeros_like(f))
        res = simpgmg.pcg_solve(h, t64(f), u, rtol=1e-8, maxit=500)
        assert res["status"] == "converged"
        x = simpgmg.unet_input(h, t64(rho), t64(f))
        t, m = simpgmg.unet_target(h, u)
        xs.append(x); ts.append(t); ms.append(m); cases.append((rho, f))
    X, T, M = torch.cat(xs[:8]), torch.cat(ts[:8]), torch.cat(ms[:8])
    net = simpgmg.UNet(seed=3)
    losses = []
    for step in range(600):
        losses.append(net.train_step(X, T, M, lr=2e-3))
    assert np.mean(losses[-10:]) < 0.05 * np.mean(losses[:10])

    def starts(k):
        rho, f = cases[k]
        h = simpgmg.setup_hierarchy(simpgmg.default_options(*dims, n_levels=3), t64(rho))
        u_cold = t64(np.zeros_like(f))
        cold = simpgmg.pcg_solve(h, t64(f), u_cold, rtol=1e-6, maxit=500)
        u0 = simpgmg.unet_output(h, net.forward(xs[k]))
        raw = np64(u0)
        alpha = simpgmg.warm_start_scale(h, t64(f), u0)
        x0 = np64(u0)
        warm = simpgmg.pcg_solve(h, t64(f), u0, rtol=1e-6, maxit=500)
        K = mesh.assemble(dims, mesh.simp_modulus(rho, 3), fixed=fixed)
        return f, K, cold, warm, raw, alpha, x0

    # seen case (uniform density, edge load)
    f, K, cold, warm, raw, alpha, x0 = starts(0)
    assert warm["status"] == "converged" == cold["status"]
    fr = ~fixed
    ustar = np.zeros(fixed.size)
    ustar[fr] = spla.spsolve(K[fr][:, fr].tocsc(), f[fr])
    e0 = ustar - x0
    ratio = np.sqrt((e0 @ (K @ e0)) / (ustar @ (K @ ustar)))
    assert ratio < 0.97, ratio
    assert warm["iters"] <= cold["iters"], (warm["iters"], cold["iters"])
    # held-out case: alpha is the energy-optimal scale (checked on the oracle's K)
    f, K, cold, warm, raw, alpha, x0 = starts(8)
    assert warm["status"] == "converged"
    a_ref = (f @ raw) / (raw @ (K @ raw))
    assert abs(alpha - a_ref) <= 1e-9 * abs(a_ref)
    np.testing.assert_allclose(x0, a_ref * raw, rtol=1e-9, atol=1e-300)
    # ||u* - x0||_K^2 - ||u*||_K^2 = x0.K.x0 - 2 f.x0 = -(f.raw)^2 / raw.K.raw <= 0
    assert x0 @ (K @ x0) - 2 * f @ x0 <= 1e-12 * abs(f @ x0)


def test_energy_score_gradients_match_oracle():
    """Energy-norm training score: the device loss and parameter gradients
    against the oracle's score (sparse K of each sample, compliance from a
    direct solve) pushed through the oracle network's backward pass."""
    import torch
    import scipy.sparse.linalg as spla
    from paper_2604_26441_amd import simpgmg
    dims = (16, 8, 8)
    fixed = workloads.cantilever_fixed(dims).astype(bool)
    rng = np.random.default_rng(21)
    rhos = [workloads.grf_rho(dims, seed=700 + k) for k in range(2)]
    fs = [workloads.random_face_load(dims, rng) for _ in range(2)]
    Ks, cs = [], []
    for rho, f in zip(rhos, fs):
        K = mesh.assemble(dims, mesh.simp_modulus(rho, 3), fixed=fixed)
        fr = ~fixed
        us = np.zeros(fixed.size)
        us[fr] = spla.spsolve(K[fr][:, fr].tocsc(), f[fr])
        Ks.append(K)
        cs.append(float(f @ us))
    h = simpgmg.setup_hierarchy(simpgmg.default_options(*dims, n_levels=2), t64(rhos[0]))
    X = torch.cat([simpgmg.unet_input(h, t64(r), t64(f)) for r, f in zip(rhos, fs)])
    params = _rounded_params(12)
    net = simpgmg.UNet(seed=1)
    net.set_params(_flat(params))
    loss, grads = net.energy_step(h, X, t64(np.stack(rhos)), t64(np.stack(fs)), t64(np.array(cs)),
                                  lr=0.0, grads=True)
    x = np64(X)
    y, cache = unet.forward(params, x)
    lref, dy = unet.loss_energy(y, Ks, fs, cs, dims, fixed)
    gref = unet.backward(params, cache, dy)
    assert 0.0 < lref <= 1.0
    assert abs(loss - lref) <= 1e-5 * abs(lref), (loss, lref)
    off = 0
    for (dw, db) in gref:
        gw = grads[off:off + dw.size].reshape(dw.shape)
        off += dw.size
        gb = grads[off:off + db.size]
        off += db.size
        assert np.linalg.norm(gw - dw) <= 1e-3 * np.linalg.norm(dw)
        assert np.linalg.norm(gb - db) <= 1e-3 * max(np.linalg.norm(db), 1e-12)
    # argument checks: a volume smaller than the node grid, a negative rate
    with pytest.raises(simpgmg.SimpGmgError):
        net.energy_step(h, X[:, :, :8].contiguous(), t64(np.stack(rhos)), t64(np.stack(fs)),
                        t64(np.array(cs)))
    with pytest.raises(simpgmg.SimpGmgError):
        net.energy_step(h, X, t64(np.stack(rhos)), t64(np.stack(fs)), t64(np.array(cs)), lr=-1.0)
    # an Adam step on this score lowers it
    l0 = net.energy_step(h, X, t64(np.stack(rhos)), t64(np.stack(fs)), t64(np.array(cs)), lr=1e-3)
    for _ in range(30):
        l1 = net.energy_step(h, X, t64(np.stack(rhos)), t64(np.stack(fs)), t64(np.array(cs)), lr=1e-3)
    assert l1 < l0
