"""Parity at the full size of the timed workload: the 80^3 cantilever
(512,000 elements, 1,594,323 DOF, 4 levels) in the launch configuration the
benchmark uses (launch shapes from the autotuner, the default kernel forms).

Every output of each operator is compared, against the oracle's definitions
applied to the whole vector: the fine K.u by its element loop, the Galerkin
levels by K^{l+1} u = M P^T (M K^l M) P M u composed from the oracle's
prolongation and the level below.  The solve is checked by the oracle's own
residual of the returned solution.  Tolerances are relative to |K| |u|
(entry-wise magnitudes; P has non-negative weights, so P^T |K| P |u| bounds
the Galerkin levels' terms): FP64 1e-13 on the fine level and 1e-12 on the
coarse levels (sums of up to 27 x 9 terms, each itself a sum over the fine
operator), FP32-accurate BF16X3 2e-6.
"""
import numpy as np
import pytest

import workloads
from oracle import hex8, mesh, transfer
from tests.gpu_util import np64, rel_err, t32, t64

pytestmark = pytest.mark.gpu

DIMS = (80, 80, 80)


@pytest.fixture(scope="module")
def field80():
    from paper_2604_26441_amd import simpgmg
    rho = np.random.default_rng(80).uniform(0.05, 1.0, int(np.prod(DIMS)))
    fixed = workloads.cantilever_fixed(DIMS).astype(bool)
    E = mesh.simp_modulus(rho, 3)
    h = simpgmg.setup_hierarchy(simpgmg.default_options(*DIMS, fine_prec="bf16x3"), t64(rho))
    simpgmg.autotune(h)
    return simpgmg, h, fixed, E


def _abs_apply(E, v):
    """|K| v for the fine operator (v >= 0 entry-wise)."""
    ka = np.abs(hex8.ke(0.3))
    dofs = mesh.element_dofs(DIMS)
    fe = (v[dofs] @ ka.T) * E[:, None]
    out = np.zeros_like(v)
    np.add.at(out, dofs.ravel(), fe.ravel())
    return out


def _galerkin(dims, apply_fine, fixed_f, u_c):
    """M_c P^T (M_f K_f M_f) P M_c u_c (Sec. 3.3 definition of the next level)."""
    P = transfer.prolongation(dims)
    fixed_c = transfer.inject_fixed(fixed_f, dims)
    v = P @ np.where(fixed_c, 0.0, u_c)
    v[fixed_f] = 0.0
    w = apply_fine(v)
    w[fixed_f] = 0.0
    y = P.T @ w
    y[fixed_c] = 0.0
    return y


def test_fullsize_fine_operator(field80):
    simpgmg, h, fixed, E = field80
    u = workloads.random_vector(fixed.size, 81, fixed)
    scale = _abs_apply(E, np.abs(u))
    y = t64(np.zeros_like(u))
    simpgmg.apply_K(h, 0, "f64", t64(u), y)
    assert rel_err(np64(y), mesh.apply_K_elementwise(DIMS, E, u, fixed=fixed), scale) < 1e-13
    u32 = u.astype(np.float32).astype(np.float64)
    y3 = t32(np.zeros_like(u))
    simpgmg.apply_K(h, 0, "bf16x3", t32(u32), y3)
    assert rel_err(np64(y3), mesh.apply_K_elementwise(DIMS, E, u32, fixed=fixed), scale) < 2e-6
    assert np.all(np64(y)[fixed] == 0) and np.all(np64(y3)[fixed] == 0)


def test_fullsize_galerkin_levels(field80):
    """Level 1 (68,921 nodes: the LDS-staged kernel) and level 2 (9,261
    nodes: the plane-split kernel)."""
    simpgmg, h, fixed, E = field80
    d1 = transfer.coarse_dims(DIMS)
    fixed1 = transfer.inject_fixed(fixed, DIMS)
    fixed2 = transfer.inject_fixed(fixed1, d1)
    assert h.level_info(1)["dims"] == d1 and h.level_info(2)["dims"] == transfer.coarse_dims(d1)

    def k0(v):
        return mesh.apply_K_elementwise(DIMS, E, v, fixed=fixed)

    def k1(v):
        return _galerkin(DIMS, k0, fixed, v)

    def k1_abs(v):
        return _galerkin(DIMS, lambda w: _abs_apply(E, w), fixed, v)

    cases = [(1, fixed1, k1, k1_abs),
             (2, fixed2, lambda v: _galerkin(d1, k1, fixed1, v),
              lambda v: _galerkin(d1, k1_abs, fixed1, v))]
    for level, fx, ref_apply, abs_apply in cases:
        u = workloads.random_vector(fx.size, 82 + level, fx)
        y = t64(np.zeros_like(u))
        simpgmg.apply_K(h, level, "f64", t64(u), y)
        assert rel_err(np64(y), ref_apply(u), abs_apply(np.abs(u))) < 1e-12, level
        assert np.all(np64(y)[fx] == 0)


def test_fullsize_pcg_solution():
    """The timed solve itself: uniform rho = 0.5, p = 3, edge load, FP32-GMG
    (BF16X3 fine level), rtol 1e-6.  The oracle's residual of the returned u
    must pass rtol and equal the residual the solver reports."""
    from paper_2604_26441_amd import simpgmg
    rho = workloads.uniform_rho(DIMS)
    fixed = workloads.cantilever_fixed(DIMS).astype(bool)
    f = workloads.edge_load(DIMS)
    h = simpgmg.setup_hierarchy(simpgmg.default_options(*DIMS, fine_prec="bf16x3"), t64(rho))
    simpgmg.autotune(h)
    for _ in range(2):                       # a second solve on the same hierarchy
        u = t64(np.zeros_like(f))
        res = simpgmg.pcg_solve(h, t64(f), u, rtol=1e-6, maxit=200)
        assert res["status"] == "converged" and res["iters"] <= 15, res
        x = np64(u)
        r = f - mesh.apply_K_elementwise(DIMS, mesh.simp_modulus(rho, 3), x, fixed=fixed)
        rel = np.linalg.norm(r) / np.linalg.norm(f)
        assert rel < 1e-6
        assert abs(res["rel_res_true"] - rel) < 1e-9


@pytest.mark.parametrize("p", [1, 3])
def test_fullsize_heterogeneous_solves(p):
    """The 60^3 random-field cantilever of the precision study (seed 0) at its
    full size: FP64-GMG, FP32-GMG (BF16X3 fine level) and BF16-GMG (BF16
    fine level, FP32 level 1, flexible PCG) must each return a u whose oracle
    residual passes rtol, with the residual they report."""
    from paper_2604_26441_amd import simpgmg
    dims = (60, 60, 60)
    rho = workloads.grf_rho(dims, 0)
    fixed = workloads.cantilever_fixed(dims).astype(bool)
    f = workloads.edge_load(dims)
    E = mesh.simp_modulus(rho, p)
    variants = {"f64": {}, "bf16x3": {}, "bf16": {"flexible_beta": 1, "level1_prec": "f32"}}
    for prec, kw in variants.items():
        o = simpgmg.default_options(*dims, penal=float(p), fine_prec=prec, **kw)
        h = simpgmg.setup_hierarchy(o, t64(rho))
        u = t64(np.zeros_like(f))
        res = simpgmg.pcg_solve(h, t64(f), u, rtol=1e-6, maxit=500)
        assert res["status"] == "converged", (prec, res)
        r = f - mesh.apply_K_elementwise(dims, E, np64(u), fixed=fixed)
        rel = np.linalg.norm(r) / np.linalg.norm(f)
        assert rel < 1e-6 and abs(res["rel_res_true"] - rel) < 1e-9, (prec, rel, res)


def test_fullsize_100cube_five_levels():
    """The 100^3 cantilever of the warm-start workload (1 M elements, 3.09 M
    DOF) with the automatic depth (5 levels: the 4-level coarsest would have
    6,084 free DOFs, above the dense cutoff), FP32-GMG (BF16X3 fine level):
    the oracle's residual of the returned u passes rtol and equals the
    residual the solver reports."""
    from paper_2604_26441_amd import simpgmg
    dims = (100, 100, 100)
    rho = workloads.uniform_rho(dims)
    fixed = workloads.cantilever_fixed(dims).astype(bool)
    f = workloads.edge_load(dims)
    h = simpgmg.setup_hierarchy(simpgmg.default_options(*dims, n_levels=0, fine_prec="bf16x3"),
                                t64(rho))
    assert h.num_levels() == 5
    u = t64(np.zeros_like(f))
    res = simpgmg.pcg_solve(h, t64(f), u, rtol=1e-6, maxit=200)
    assert res["status"] == "converged", res
    r = f - mesh.apply_K_elementwise(dims, mesh.simp_modulus(rho, 3), np64(u), fixed=fixed)
    rel = np.linalg.norm(r) / np.linalg.norm(f)
    assert rel < 1e-6 and abs(res["rel_res_true"] - rel) < 1e-9, (rel, res)
