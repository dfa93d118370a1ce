"""The allocation-free warm-start scaling (sgmg_warm_start_scale_noalloc)
against the entry point it varies (sgmg_warm_start_scale), through the C-ABI.

Both run the same kernels in the same summation order, so the scaled u0 and
alpha must be bitwise equal; alpha is also checked against the oracle's
f.u0 / (u0.K u0) (FP64 sums in another order: 1e-12 relative).  Two calls in
a row share the library's fixed array: the first on a 24x12x12 mesh with the
FP64 matrix-core operator, the second on a smaller 16x8x8 mesh with the
vector-ALU operator (fewer block partials than the first left behind).
"""
import ctypes

import numpy as np
import pytest
import torch

import workloads
from oracle import mesh
from tests.gpu_util import np64, t64

pytestmark = pytest.mark.gpu


def _case(simpgmg, dims, f64_shape, seed):
    rho = np.random.default_rng(seed).uniform(0.1, 1.0, int(np.prod(dims)))
    fixed = workloads.cantilever_fixed(dims).astype(bool)
    f = workloads.edge_load(dims)
    u0 = workloads.random_vector(fixed.size, seed + 1, fixed)
    h = simpgmg.setup_hierarchy(simpgmg.default_options(*dims, n_levels=3), t64(rho))
    simpgmg.set_launch_shape(h, "f64", *f64_shape)
    return h, rho, fixed, f, u0


def test_noalloc_scale_equals_existing_entry_point():
    from paper_2604_26441_amd import simpgmg
    for dims, shape, seed in [((24, 12, 12), (4, 3), 11), ((16, 8, 8), (0, 0), 12),
                              ((20, 10, 10), (1, 3), 14)]:
        h, rho, fixed, f, u0 = _case(simpgmg, dims, shape, seed)
        ua, ub = t64(u0), t64(u0)
        alpha_ref = simpgmg.warm_start_scale(h, t64(f), ua)
        alpha_dev = torch.full((1,), np.nan, dtype=torch.float64, device="cuda:0")
        simpgmg.warm_start_scale_noalloc(h, t64(f), ub, alpha_dev)
        torch.cuda.synchronize()
        alpha = float(alpha_dev.item())
        assert alpha == alpha_ref, (dims, alpha, alpha_ref)
        assert np.array_equal(np64(ua), np64(ub)), dims
        E = mesh.simp_modulus(rho, 3)
        Ku0 = mesh.apply_K_elementwise(dims, E, u0, fixed=fixed)
        alpha_oracle = (f @ u0) / (u0 @ Ku0)
        assert abs(alpha - alpha_oracle) <= 1e-12 * abs(alpha_oracle), (dims, alpha, alpha_oracle)
        assert np.allclose(np64(ub), alpha_oracle * u0, rtol=1e-12, atol=0)
        # without an alpha output the scaling is the same
        uc = t64(u0)
        simpgmg.warm_start_scale_noalloc(h, t64(f), uc)
        assert np.array_equal(np64(uc), np64(ua)), dims
        h.close()


def test_noalloc_scale_rejects_null_arguments():
    from paper_2604_26441_amd import simpgmg
    h, rho, fixed, f, u0 = _case(simpgmg, (16, 8, 8), (0, 0), 13)
    lib = ctypes.CDLL(simpgmg.library_path())
    lib.sgmg_warm_start_scale_noalloc.argtypes = [ctypes.c_void_p] * 5
    u = t64(u0)
    rc = lib.sgmg_warm_start_scale_noalloc(h.handle, None, ctypes.c_void_p(u.data_ptr()), None, None)
    assert rc == -1
    h.close()
