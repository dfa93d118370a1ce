"""Pins of the V-cycle (Eq. vcycle, App. D error-propagation operator)."""
import numpy as np
import pytest

from oracle import multigrid, mesh, smoothers, transfer
import workloads


def _hier(dims, L, seed=0, fine="chebyshev", uniform=False):
    g = np.random.default_rng(seed)
    rho = np.full(np.prod(dims), 0.5) if uniform else g.uniform(0.2, 1.0, np.prod(dims))
    E = mesh.simp_modulus(rho, 3)
    fixed = mesh.cantilever_fixed(dims)
    h = multigrid.build(dims, E, fixed, multigrid.Options(n_levels=L, fine_smoother=fine))
    return h


def _dense_V(h):
    fixed = h.levels[0].fixed
    fr = np.where(~fixed)[0]
    M = np.zeros((fr.size, fr.size))
    for k, i in enumerate(fr):
        e = np.zeros(fixed.size)
        e[i] = 1.0
        M[:, k] = multigrid.vcycle(h, e)[fr]
    return M


def _poly_matrix(lev, poly):
    """p(D^-1 K) on free DOFs from the eigen-decomposition of D^-1/2 K D^-1/2."""
    fr = ~lev.fixed
    A = lev.K[fr][:, fr].toarray()
    dh = np.sqrt(lev.d[fr])
    w, V = np.linalg.eigh(A / dh[:, None] / dh[None, :])
    return (V * poly(w)[None, :]) @ V.T / dh[:, None] * dh[None, :], A


def _M_closed_form(h, l=0):
    """Preconditioner matrix from E = p (I - P M_c P^T K) p and M = (I - E) K^-1."""
    lev = h.levels[l]
    o = h.opts
    fr = ~lev.fixed
    if l == len(h.levels) - 1:
        A = lev.K[fr][:, fr].toarray()
        return np.linalg.inv(A + h.coarse_eps * np.eye(A.shape[0]))
    lam = o.lambda_safety * lev.lam
    if l == 0 and o.fine_smoother == "chebyshev":
        poly = lambda w: smoothers.chebyshev_residual_polynomial(w, lam, o.fine_degree, o.cheb_alpha)
    else:
        om = min(o.jacobi_omega_max, 4 / (3 * lam))
        m = o.fine_degree if l == 0 else o.coarse_sweeps
        poly = lambda w: (1 - om * w) ** m
    Pm, A = _poly_matrix(lev, poly)
    coarse = h.levels[l + 1]
    P = transfer.prolongation(lev.dims)[np.where(fr)[0]][:, np.where(~coarse.fixed)[0]].toarray()
    Mc = _M_closed_form(h, l + 1)
    Ecyc = Pm @ (np.eye(A.shape[0]) - P @ Mc @ P.T @ A) @ Pm
    return (np.eye(A.shape[0]) - Ecyc) @ np.linalg.inv(A)


def test_two_and_three_level_match_error_propagation_form():
    for L, fine in [(2, "chebyshev"), (3, "chebyshev"), (3, "jacobi")]:
        h = _hier((4, 2, 4), L, fine=fine)
        M = _dense_V(h)
        Mref = _M_closed_form(h)
        assert np.abs(M - Mref).max() < 1e-9 * np.abs(Mref).max(), (L, fine)


def test_vcycle_symmetric_positive_definite():
    h = _hier((6, 4, 4), 3)
    M = _dense_V(h)
    assert np.abs(M - M.T).max() < 1e-12 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0


def test_stationary_vcycle_contracts():
    h = _hier((8, 4, 4), 3, uniform=True)
    fixed = h.levels[0].fixed
    K = h.levels[0].K
    x = np.where(fixed, 0, np.random.default_rng(0).standard_normal(fixed.size))
    b = np.zeros_like(x)
    n0 = np.sqrt(x @ (K @ x))
    for _ in range(5):
        x = x + multigrid.vcycle(h, b - K @ x)
    assert np.sqrt(x @ (K @ x)) < 0.5 * n0


def test_coarsest_regularisation_value():
    h = _hier((4, 2, 2), 2)
    last = h.levels[-1]
    fr = ~last.fixed
    md = last.K.diagonal()[fr].mean()
    assert h.coarse_eps == max(md * 1e-8, 1e-14)


def test_auto_levels_rule():
    dims = (80, 80, 80)
    fixed = workloads.cantilever_fixed(dims).astype(bool)
    assert multigrid.auto_levels(dims, fixed, 5000) == 4
    assert transfer.free_counts(dims, fixed, 4)[-1] == 3630
    assert multigrid.auto_levels((100, 100, 100), workloads.cantilever_fixed((100,) * 3).astype(bool), 5000) == 5


def _M_closed_form_cycle(h, gamma, l=0):
    """M of the gamma-cycle from the error-propagation form: the coarse level
    (if not the coarsest) is approximated by gamma cycles from zero, whose
    error propagation is E_c^gamma, so M_c^(gamma) = (I - E_c^gamma) K_c^-1."""
    lev = h.levels[l]
    o = h.opts
    fr = ~lev.fixed
    L = len(h.levels) - 1
    if l == L:
        A = lev.K[fr][:, fr].toarray()
        return np.linalg.inv(A + h.coarse_eps * np.eye(A.shape[0]))
    lam = o.lambda_safety * lev.lam
    if l == 0 and o.fine_smoother == "chebyshev":
        poly = lambda w: smoothers.chebyshev_residual_polynomial(w, lam, o.fine_degree, o.cheb_alpha)
    else:
        om = min(o.jacobi_omega_max, 4 / (3 * lam))
        m = o.fine_degree if l == 0 else o.coarse_sweeps
        poly = lambda w: (1 - om * w) ** m
    Pm, A = _poly_matrix(lev, poly)
    coarse = h.levels[l + 1]
    cfr = ~coarse.fixed
    Ac = coarse.K[cfr][:, cfr].toarray()
    Mc = _M_closed_form_cycle(h, gamma, l + 1)
    if l + 1 < L:
        Ec = np.eye(Ac.shape[0]) - Mc @ Ac
        Mc = (np.eye(Ac.shape[0]) - np.linalg.matrix_power(Ec, gamma)) @ np.linalg.inv(Ac)
    P = transfer.prolongation(lev.dims)[np.where(fr)[0]][:, np.where(cfr)[0]].toarray()
    Ecyc = Pm @ (np.eye(A.shape[0]) - P @ Mc @ P.T @ A) @ Pm
    return (np.eye(A.shape[0]) - Ecyc) @ np.linalg.inv(A)


def _dense_cycle(h, gamma):
    fixed = h.levels[0].fixed
    fr = np.where(~fixed)[0]
    M = np.zeros((fr.size, fr.size))
    for k, i in enumerate(fr):
        e = np.zeros(fixed.size)
        e[i] = 1.0
        M[:, k] = multigrid.cycle(h, e, gamma)[fr]
    return M


def test_gamma_one_cycle_is_the_vcycle_and_two_levels_have_no_w():
    h = _hier((8, 4, 4), 3)
    r = workloads.random_vector(h.levels[0].fixed.size, 2, h.levels[0].fixed)
    assert np.array_equal(multigrid.cycle(h, r, 1), multigrid.vcycle(h, r))
    h2 = _hier((8, 4, 4), 2)
    assert np.array_equal(multigrid.cycle(h2, r, 2), multigrid.vcycle(h2, r))


@pytest.mark.parametrize("L,fine", [(3, "chebyshev"), (4, "jacobi")])
def test_w_cycle_matches_error_propagation_form(L, fine):
    h = _hier((8, 8, 8) if L == 4 else (8, 4, 4), L, fine=fine)
    Mw = _dense_cycle(h, 2)
    Mref = _M_closed_form_cycle(h, 2)
    assert np.abs(Mw - Mref).max() <= 1e-9 * np.abs(Mref).max()
    assert np.abs(Mw - Mw.T).max() <= 1e-10 * np.abs(Mw).max()
    # a W-cycle is a better coarse solve than a V-cycle: smaller error propagation
    fr = ~h.levels[0].fixed
    A = h.levels[0].K[fr][:, fr].toarray()
    Mv = _dense_V(h)
    ev = np.abs(np.linalg.eigvals(np.eye(A.shape[0]) - Mv @ A)).max()
    ew = np.abs(np.linalg.eigvals(np.eye(A.shape[0]) - Mw @ A)).max()
    assert ew <= ev + 1e-12
