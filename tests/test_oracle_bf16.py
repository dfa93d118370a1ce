"""Pins of the BF16 semantic model (Sec. 3.5, BF16 numerical semantics)."""
import numpy as np
import torch

from oracle import bf16, mesh


def test_round_bf16_matches_torch():
    g = np.random.default_rng(0)
    # random magnitudes plus exact ties between two BF16 neighbours (both parities)
    ties = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 0.5])
    x = np.concatenate([g.standard_normal(10000) * 10.0 ** g.integers(-20, 20, 10000), ties])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(bf16.round_bf16(x), ref)


def test_bf16_model_error_bound():
    dims = (6, 4, 4)
    g = np.random.default_rng(1)
    E = g.uniform(0.1, 1.0, np.prod(dims))
    fixed = mesh.cantilever_fixed(dims)
    u = np.where(fixed, 0, g.standard_normal(fixed.size))
    y = mesh.apply_K_elementwise(dims, E, u, fixed=fixed)
    yb = bf16.apply_K_bf16_model(dims, E, u, fixed)
    K = mesh.assemble(dims, E, fixed=fixed)
    bound = 2.0 ** -8 * (abs(K) @ np.abs(u))
    assert np.all(np.abs(yb - y) <= bound + 1e-300)
    assert np.abs(yb - y).max() > 0
