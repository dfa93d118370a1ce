"""Pins of the SIMP outer-loop pieces (Eq. simp_filter and its readings):
filter weights and adjoint, the projection's closed values and derivative,
compliance sensitivities against finite differences of exact solves, and the
OC update's volume constraint, move limits and closed-form cases."""
import numpy as np
import pytest

from oracle import mesh, simp


def test_filter_weights_uniform_field_and_adjoint():
    dims = (5, 5, 5)
    n = 125
    for rmin in (1.5, 2.5):
        assert np.allclose(simp.density_filter(dims, rmin, np.full(n, 0.3)), 0.3, rtol=0, atol=1e-15)
    # interior cone weights for rmin = 1.5: centre 1.5, faces 0.5, edges 1.5 - sqrt 2, corners 0
    W_int = 1.5 + 6 * 0.5 + 12 * (1.5 - np.sqrt(2.0))
    delta = np.zeros(n)
    c = 2 + 5 * (2 + 5 * 2)
    delta[c] = 1.0
    out = simp.density_filter(dims, 1.5, delta)
    assert out[c] == pytest.approx(1.5 / W_int, rel=1e-14)
    assert out[c + 1] == pytest.approx(0.5 / W_int, rel=1e-14)
    assert out[c + 1 + 5] == pytest.approx((1.5 - np.sqrt(2.0)) / W_int, rel=1e-13)
    assert out[c + 1 + 5 + 25] == 0.0
    g = np.random.default_rng(0)
    d2 = (6, 4, 3)
    a, b = g.standard_normal(72), g.standard_normal(72)
    lhs = simp.density_filter(d2, 2.2, a) @ b
    rhs = a @ simp.density_filter_adjoint(d2, 2.2, b)
    assert lhs == pytest.approx(rhs, rel=1e-13)


def test_heaviside_values_and_derivative():
    for beta, eta in ((1.0, 0.5), (8.0, 0.3), (32.0, 0.5)):
        h, _ = simp.heaviside(np.array([0.0, 1.0, eta]), beta, eta)
        den = np.tanh(beta * eta) + np.tanh(beta * (1 - eta))
        assert h[0] == pytest.approx(0.0, abs=1e-15) and h[1] == pytest.approx(1.0, rel=1e-15)
        assert h[2] == pytest.approx(np.tanh(beta * eta) / den, rel=1e-15)
        x = np.linspace(0.05, 0.95, 7)
        e = 1e-6
        fd = (simp.heaviside(x + e, beta, eta)[0] - simp.heaviside(x - e, beta, eta)[0]) / (2 * e)
        np.testing.assert_allclose(simp.heaviside(x, beta, eta)[1], fd, rtol=1e-6, atol=1e-9)
    x = np.linspace(0, 1, 5)
    h, d = simp.heaviside(x, 0.0, 0.5)
    assert np.array_equal(h, x) and np.all(d == 1.0)


def _problem(dims=(4, 2, 2), seed=1):
    g = np.random.default_rng(seed)
    rho = g.uniform(0.3, 1.0, int(np.prod(dims)))
    return rho, mesh.cantilever_fixed(dims), mesh.edge_load(dims)


def test_compliance_is_f_dot_u_and_sensitivity_matches_finite_differences():
    dims = (4, 2, 2)
    rhohat, fixed, f = _problem(dims)
    u = simp.state_solve(dims, rhohat, fixed, f, 3.0)
    c, dc = simp.compliance_sensitivity(dims, rhohat, u, 3.0)
    assert c == pytest.approx(f @ u, rel=1e-12)
    h = 1e-6
    for e in (0, 5, 11, 15):
        rp, rm = rhohat.copy(), rhohat.copy()
        rp[e] += h
        rm[e] -= h
        cp = f @ simp.state_solve(dims, rp, fixed, f, 3.0)
        cm = f @ simp.state_solve(dims, rm, fixed, f, 3.0)
        assert dc[e] == pytest.approx((cp - cm) / (2 * h), rel=1e-6)
    assert np.all(dc < 0)


def test_design_sensitivity_through_filter_and_projection():
    dims = (6, 3, 3)
    rho, fixed, f = _problem(dims, 2)
    rmin, beta, eta, p = 1.8, 4.0, 0.5, 3.0

    def c_of(r):
        rh, _ = simp.physical(dims, r, rmin, beta, eta)
        return f @ simp.state_solve(dims, rh, fixed, f, p)

    rh, dH = simp.physical(dims, rho, rmin, beta, eta)
    u = simp.state_solve(dims, rh, fixed, f, p)
    c, g, gv = simp.design_sensitivity(dims, rh, dH, u, p, rmin)
    h = 1e-6
    for e in (0, 13, 30, 53):
        rp, rm = rho.copy(), rho.copy()
        rp[e] += h
        rm[e] -= h
        assert g[e] == pytest.approx((c_of(rp) - c_of(rm)) / (2 * h), rel=1e-5)
        vp = simp.physical(dims, rp, rmin, beta, eta)[0].sum()
        vm = simp.physical(dims, rm, rmin, beta, eta)[0].sum()
        assert gv[e] == pytest.approx((vp - vm) / (2 * h), rel=1e-6)


def test_oc_volume_constraint_move_limits_and_closed_forms():
    dims = (6, 4, 4)
    n = 96
    g = np.random.default_rng(3)
    rho = g.uniform(0.2, 0.9, n)
    dc = -g.uniform(0.1, 2.0, n)
    dv = np.ones(n)
    new, lam = simp.oc_update(dims, rho, dc, dv, 0.5, 0.2, 1.0, 0.0, 0.5)
    assert new.sum() == pytest.approx(0.5 * n, rel=1e-8)
    assert np.all(new >= np.maximum(0, rho - 0.2) - 1e-15) and np.all(new <= np.minimum(1, rho + 0.2) + 1e-15)
    # uniform sensitivities from a uniform field: the update is uniform at volfrac
    new, lam = simp.oc_update(dims, np.full(n, 0.6), np.full(n, -1.0), dv, 0.5, 0.2, 1.0, 0.0, 0.5)
    np.testing.assert_allclose(new, 0.5, rtol=1e-8)
    assert lam == pytest.approx(1.0 / (0.5 / 0.6) ** 2, rel=1e-7)
    # with the filter and projection the constraint holds on the physical field
    new, _ = simp.oc_update(dims, rho, dc, dv, 0.4, 0.2, 1.5, 2.0, 0.5)
    assert simp.physical(dims, new, 1.5, 2.0, 0.5)[0].sum() == pytest.approx(0.4 * n, rel=1e-8)


def test_simp_steps_lower_compliance_at_fixed_volume():
    dims = (8, 4, 4)
    fixed = mesh.cantilever_fixed(dims)
    f = mesh.edge_load(dims)
    rho = np.full(128, 0.5)
    cs = []
    for _ in range(4):
        rho, c, rh, _ = simp.simp_step(dims, rho, fixed, f, 3.0, 0.5, 0.2, 1.5, 0.0, 0.5)
        cs.append(c)
        assert simp.physical(dims, rho, 1.5, 0.0, 0.5)[0].sum() == pytest.approx(64.0, rel=1e-8)
    assert all(b < a for a, b in zip(cs, cs[1:]))
