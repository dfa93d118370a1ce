"""GPU parity of the SIMP outer loop (filter, projection, sensitivities, OC
update, full steps) against the oracle, through the C-ABI."""
import numpy as np
import pytest

from oracle import mesh, simp
from tests.gpu_util import np64, t64

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims,rmin,beta", [((9, 7, 5), 1.5, 0.0), ((9, 7, 5), 2.3, 4.0),
                                            ((12, 6, 6), 1.0, 8.0)])
def test_physical_density_matches_oracle(dims, rmin, beta):
    from paper_2604_26441_amd import simpgmg
    rho = np.random.default_rng(1).uniform(0.0, 1.0, int(np.prod(dims)))
    s = simpgmg.Simp(simpgmg.simp_params(*dims, rmin=rmin, beta=beta, eta=0.45))
    out = t64(np.zeros_like(rho))
    s.physical(t64(rho), out)
    ref, _ = simp.physical(dims, rho, rmin, beta, 0.45)
    np.testing.assert_allclose(np64(out), ref, rtol=1e-13, atol=1e-15)


def _hier(dims, rhohat, p=3.0):
    from paper_2604_26441_amd import simpgmg
    o = simpgmg.default_options(*dims, n_levels=3, fine_prec="f64", penal=p)
    return simpgmg.setup_hierarchy(o, t64(rhohat))


@pytest.mark.parametrize("rmin,beta,p", [(1.5, 0.0, 3.0), (2.2, 4.0, 4.5)])
def test_sensitivities_match_oracle(rmin, beta, p):
    from paper_2604_26441_amd import simpgmg
    dims = (12, 6, 6)
    rho = np.random.default_rng(2).uniform(0.2, 1.0, int(np.prod(dims)))
    fixed = mesh.cantilever_fixed(dims)
    f = mesh.edge_load(dims)
    rh, dH = simp.physical(dims, rho, rmin, beta, 0.5)
    u = simp.state_solve(dims, rh, fixed, f, p)
    c_ref, g_ref, gv_ref = simp.design_sensitivity(dims, rh, dH, u, p, rmin)
    s = simpgmg.Simp(simpgmg.simp_params(*dims, rmin=rmin, beta=beta, penal=p))
    h = _hier(dims, rh, p)
    s.physical(t64(rho))
    dc, dv = t64(np.zeros_like(rho)), t64(np.zeros_like(rho))
    c = s.sensitivity(h, t64(u), dc, dv)
    assert c == pytest.approx(c_ref, rel=1e-12)
    # The element energy u_e^T K_e u_e sums 576 products of both signs: in
    # FP64 its rounding error is at most about 48 eps |u_e|^T |K_e| |u_e| (24
    # terms per row sum, 24 row terms; first order), which can exceed eps times
    # the energy itself.  The rest of the chain (p rhohat^(p-1) (E0 - Emin),
    # H', the filter adjoint) has non-negative weights, so the same chain
    # applied to 64 eps |u_e|^T |K_e| |u_e| bounds each side's error.
    from oracle import hex8
    ue = np.abs(u[mesh.element_dofs(dims)])
    e_abs = np.einsum("ei,ij,ej->e", ue, np.abs(hex8.ke(0.3)), ue)
    b = 64 * np.finfo(float).eps * p * rh ** (p - 1) * (1.0 - 1e-9) * e_abs * dH
    if rmin > 1.0:
        b = simp.density_filter_adjoint(dims, rmin, b)
    err = np.abs(np64(dc) - g_ref)
    assert np.all(err <= 2 * b + 1e-14 * np.abs(g_ref)), (err / (b + 1e-300)).max()
    np.testing.assert_allclose(np64(dv), gv_ref, rtol=1e-12)


def test_oc_update_matches_oracle():
    from paper_2604_26441_amd import simpgmg
    dims = (12, 6, 6)
    rmin, beta, p = 1.5, 2.0, 3.0
    rho = np.random.default_rng(3).uniform(0.2, 0.8, int(np.prod(dims)))
    fixed = mesh.cantilever_fixed(dims)
    f = mesh.edge_load(dims)
    rh, dH = simp.physical(dims, rho, rmin, beta, 0.5)
    u = simp.state_solve(dims, rh, fixed, f, p)
    _, g, gv = simp.design_sensitivity(dims, rh, dH, u, p, rmin)
    ref, lam_ref = simp.oc_update(dims, rho, g, gv, 0.4, 0.2, rmin, beta, 0.5)
    s = simpgmg.Simp(simpgmg.simp_params(*dims, rmin=rmin, beta=beta, volfrac=0.4))
    h = _hier(dims, rh, p)
    s.physical(t64(rho))
    s.sensitivity(h, t64(u))
    r = t64(rho)
    res = s.oc_update(r)
    # the bisection stops at a relative width of 1e-9: both sides agree to that
    assert res["lambda"] == pytest.approx(lam_ref, rel=1e-8)
    np.testing.assert_allclose(np64(r), ref, rtol=0, atol=1e-8)
    assert res["volume"] == pytest.approx(0.4 * rho.size, rel=1e-7)
    assert res["max_change"] == pytest.approx(np.abs(ref - rho).max(), rel=1e-7)
    with pytest.raises(simpgmg.SimpGmgError):          # sensitivities are consumed by the update
        s.oc_update(r)


def test_simp_steps_match_oracle_and_check_arguments():
    from paper_2604_26441_amd import simpgmg
    dims = (16, 8, 8)
    fixed = mesh.cantilever_fixed(dims)
    f = mesh.edge_load(dims)
    n = int(np.prod(dims))
    rho_ref = np.full(n, 0.5)
    s = simpgmg.Simp(simpgmg.simp_params(*dims, rmin=1.5, volfrac=0.5))
    h = _hier(dims, rho_ref)
    rho = t64(rho_ref)
    u = t64(np.zeros_like(f))
    fd = t64(f)
    for k in range(3):
        res = s.step(h, rho, fd, u, rtol=1e-11, maxit=300)
        rho_ref, c_ref, _, _ = simp.simp_step(dims, rho_ref, fixed, f, 3.0, 0.5, 0.2, 1.5, 0.0, 0.5)
        assert res["pcg_status"] == "converged"
        assert res["compliance"] == pytest.approx(c_ref, rel=1e-8)
        np.testing.assert_allclose(np64(rho), rho_ref, rtol=0, atol=1e-6)
    o = simpgmg.default_options(*dims, n_levels=3, penal=2.0)
    h2 = simpgmg.setup_hierarchy(o, t64(np.full(n, 0.5)))
    with pytest.raises(simpgmg.SimpGmgError, match="SIMP map"):
        s.step(h2, rho, fd, u)
    s2 = simpgmg.Simp(simpgmg.simp_params(*dims))
    with pytest.raises(simpgmg.SimpGmgError, match="physical"):
        s2.sensitivity(h, u)
    with pytest.raises(simpgmg.SimpGmgError):
        simpgmg.Simp(simpgmg.simp_params(*dims, volfrac=1.5))
