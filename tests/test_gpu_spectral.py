"""GPU parity of the Lanczos kappa_eff probe against the oracle (through the C-ABI)."""
import numpy as np
import pytest
from scipy.linalg import eigvalsh_tridiagonal

import workloads
from oracle import mesh, multigrid, spectral
from tests.gpu_util import t64

pytestmark = pytest.mark.gpu


def _pair(dims, L, rho, p=3.0):
    from paper_2604_26441_amd import simpgmg
    fixed = workloads.cantilever_fixed(dims).astype(bool)
    E = mesh.simp_modulus(rho, p)
    K = mesh.assemble(dims, E, fixed=fixed)
    oh = multigrid.build(dims, E, fixed, multigrid.Options(n_levels=L, penal=p))
    o = simpgmg.default_options(*dims, n_levels=L, fine_prec="f64", penal=p)
    h = simpgmg.setup_hierarchy(o, t64(rho), lambda_override=[lv.lam for lv in oh.levels[:-1]])
    return K, oh, h, fixed


@pytest.mark.parametrize("dims,L,field,precond,m", [
    ((16, 8, 8), 3, "grf", 2, 30), ((9, 7, 5), 2, "binary", 2, 25),
    ((16, 8, 8), 3, "grf", 1, 20), ((12, 6, 6), 3, "checker", 0, 15)])
def test_lanczos_matches_oracle(dims, L, field, precond, m):
    from paper_2604_26441_amd import simpgmg
    rho = {"grf": workloads.grf_rho(dims, 3, corr_len=2.0),
           "binary": workloads.binary_rho(dims, 0.5, 1e-2, 42),
           "checker": workloads.checkerboard_rho(dims)}[field]
    K, oh, h, fixed = _pair(dims, L, rho)
    g = workloads.random_vector(fixed.size, 0, fixed)
    g /= np.linalg.norm(g)
    M = {2: lambda r: multigrid.vcycle(oh, r), 1: lambda r: oh.levels[0].dinv * r, 0: None}[precond]
    kap, lo, hi, a, b = spectral.kappa_eff(lambda v: K @ v, M, g, m=m)
    res = simpgmg.lanczos(h, t64(g), m=m, precond=precond)
    assert res["steps"] == len(a) == m
    # coefficients of two summation orders drift apart slowly over the steps
    np.testing.assert_allclose(res["alpha"], a, rtol=1e-7)
    np.testing.assert_allclose(res["beta"], b, rtol=1e-6)
    assert res["kappa"] == pytest.approx(kap, rel=1e-7)
    # the library's Sturm bisection on its own coefficients equals LAPACK's
    th = eigvalsh_tridiagonal(np.array(res["alpha"]), np.array(res["beta"][:-1]))
    assert res["theta_min"] == pytest.approx(th[0], rel=1e-12)
    assert res["theta_max"] == pytest.approx(th[-1], rel=1e-12)


def test_lanczos_breakdown_threshold_and_errors():
    from paper_2604_26441_amd import simpgmg
    dims = (8, 4, 4)
    K, oh, h, fixed = _pair(dims, 3, workloads.uniform_rho(dims))
    g = workloads.random_vector(fixed.size, 1, fixed)
    a, b = spectral.lanczos(lambda v: K @ v, lambda r: multigrid.vcycle(oh, r), g, m=10, breakdown=10.0)
    res = simpgmg.lanczos(h, t64(g), m=10, breakdown=10.0)
    assert res["steps"] == len(a) == 1
    assert res["kappa"] == 1.0
    with pytest.raises(simpgmg.SimpGmgError):
        simpgmg.lanczos(h, t64(np.zeros_like(g)), m=5)
