"""GPU parity of the restarted flexible GMRES outer solver against the
oracle's (both right-preconditioned by the V-cycle; the device builds its
basis with two classical Gram-Schmidt passes, the oracle with modified
Gram-Schmidt: equal in exact arithmetic, compared to rounding)."""
import numpy as np
import pytest

import workloads
from oracle import krylov, mesh, multigrid
from tests.gpu_util import np64, t64

pytestmark = pytest.mark.gpu


def _case(dims, L, rho, fine_prec="f64", **kw):
    from paper_2604_26441_amd import simpgmg
    fixed = workloads.cantilever_fixed(dims).astype(bool)
    E = mesh.simp_modulus(rho, 3)
    K = mesh.assemble(dims, E, fixed=fixed)
    oh = multigrid.build(dims, E, fixed, multigrid.Options(n_levels=L))
    lams = [lv.lam for lv in oh.levels[:-1]]
    o = simpgmg.default_options(*dims, n_levels=L, fine_prec=fine_prec, **kw)
    h = simpgmg.setup_hierarchy(o, t64(rho), lambda_override=lams)
    return fixed, K, oh, h


def _hist(res):
    h = list(res["history"])
    while h and h[-1] == 0.0:
        h.pop()
    return h


@pytest.mark.parametrize("restart", [32, 4])
def test_fgmres_f64_matches_oracle(restart):
    """Same iterations, same residual history (to rounding), same iterate."""
    from paper_2604_26441_amd import simpgmg
    dims, L = (16, 8, 8), 3
    rho = np.random.default_rng(1).uniform(0.2, 1.0, np.prod(dims))
    fixed, K, oh, h = _case(dims, L, rho)
    f = workloads.edge_load(dims)
    xo, st, it_o, ho = krylov.fgmres(lambda v: K @ v, f, lambda r: multigrid.vcycle(oh, r),
                                     rtol=1e-8, maxit=200, restart=restart)
    u = t64(np.zeros_like(f))
    res = simpgmg.fgmres_solve(h, t64(f), u, rtol=1e-8, maxit=200, restart=restart, history_cap=512)
    assert st == krylov.CONVERGED and res["status"] == "converged"
    assert res["iters"] == it_o
    hg = _hist(res)
    assert len(hg) == len(ho)
    np.testing.assert_allclose(hg, ho, rtol=1e-6, atol=1e-14)
    x = np64(u)
    assert np.linalg.norm(x - xo) <= 1e-7 * np.linalg.norm(xo)
    assert krylov.true_rel_residual(lambda v: K @ v, f, x) < 1e-8


@pytest.mark.parametrize("prec", ["bf16x3", "bf16"])
def test_fgmres_low_precision_smoothing_reaches_fp64_tolerance(prec):
    """FP32-GMG (BF16X3) and the BF16 smoother the paper pairs with FGMRES:
    FP64 true residual below rtol, compliance equal to the direct solve's."""
    import scipy.sparse.linalg as spla
    from paper_2604_26441_amd import simpgmg
    dims, L = (24, 12, 12), 4
    rho = workloads.grf_rho(dims, seed=3)
    fixed, K, oh, h = _case(dims, L, rho, fine_prec=prec)
    f = workloads.edge_load(dims)
    u = t64(np.zeros_like(f))
    res = simpgmg.fgmres_solve(h, t64(f), u, rtol=1e-6, maxit=300, restart=32)
    assert res["status"] == "converged"
    x = np64(u)
    assert krylov.true_rel_residual(lambda v: K @ v, f, x) < 1e-6
    fr = ~fixed
    us = np.zeros(fixed.size)
    us[fr] = spla.spsolve(K[fr][:, fr].tocsc(), f[fr])
    assert abs(f @ x - f @ us) <= 1e-5 * abs(f @ us)
    assert np.all(x[fixed] == 0)


def test_fgmres_statuses_and_warm_start():
    from paper_2604_26441_amd import simpgmg
    dims, L = (16, 8, 8), 3
    rho = workloads.uniform_rho(dims)
    fixed, K, oh, h = _case(dims, L, rho)
    f = workloads.edge_load(dims)
    u = t64(np.zeros_like(f))
    res = simpgmg.fgmres_solve(h, t64(f), u, rtol=1e-12, maxit=3, restart=32)
    assert res["status"] == "maxit" and res["iters"] == 3
    u = t64(np.zeros_like(f))
    res = simpgmg.fgmres_solve(h, t64(np.zeros_like(f)), u)
    assert res["status"] == "converged" and res["iters"] == 0
    # a converged start needs no step
    u = t64(np.zeros_like(f))
    first = simpgmg.fgmres_solve(h, t64(f), u, rtol=1e-8, restart=32)
    again = simpgmg.fgmres_solve(h, t64(f), u, rtol=1e-8, restart=32)
    assert first["status"] == again["status"] == "converged" and again["iters"] == 0
    with pytest.raises(simpgmg.SimpGmgError):
        simpgmg.fgmres_solve(h, t64(f), u, restart=64)
