"""Pins of the oracle's restarted flexible GMRES (Sec. 3.6 describes the
variant: right preconditioning, modified Gram-Schmidt, Givens rotations,
happy breakdown, restart, true-residual acceptance).  Every pin is checked
against something other than the routine itself: a least-squares problem
built by brute force over the Krylov space, exact convergence in n steps,
and closed forms."""
import numpy as np
import pytest

from oracle import krylov


def _spd(n, seed):
    g = np.random.default_rng(seed)
    Q = np.linalg.qr(g.standard_normal((n, n)))[0]
    return Q @ np.diag(np.linspace(1.0, 50.0, n)) @ Q.T


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_minimal_residual_over_preconditioned_krylov_space(k):
    """With a fixed (non-symmetric) preconditioner M, after k steps of one
    cycle x_k = x_0 + M B y with B a basis of K_k(A M, r_0) and y minimising
    ||r_0 - A M B y||: computed by brute force with numpy's lstsq."""
    n = 12
    A = _spd(n, 1)
    g = np.random.default_rng(2)
    Mmat = np.eye(n) + 0.3 * g.standard_normal((n, n))
    f = g.standard_normal(n)
    x0 = g.standard_normal(n)
    x, st, it, _ = krylov.fgmres(lambda v: A @ v, f, lambda v: Mmat @ v, x0=x0, rtol=1e-300,
                                 maxit=k, restart=20)
    assert it == k and st == krylov.MAXIT
    r0 = f - A @ x0
    B = [r0]
    for _ in range(k - 1):
        B.append(A @ (Mmat @ B[-1]))
    B = np.linalg.qr(np.column_stack(B))[0]      # same span, orthonormal columns
    y = np.linalg.lstsq(A @ Mmat @ B, r0, rcond=None)[0]
    xb = x0 + Mmat @ B @ y
    # the power basis of K_k loses digits as k grows (eigenvalues 1..50)
    assert np.allclose(x, xb, rtol=1e-7, atol=1e-8)


def test_flexible_minimises_over_recorded_directions():
    """A preconditioner that changes at every call: the iterate minimises the
    residual over x_0 + span{z_1..z_k} of the z_j actually produced."""
    n, k = 10, 4
    A = _spd(n, 3)
    g = np.random.default_rng(4)
    mats = [np.eye(n) + 0.2 * g.standard_normal((n, n)) for _ in range(k)]
    calls = []

    def M(v):
        out = mats[len(calls) % k] @ v
        calls.append(1)
        return out

    f = g.standard_normal(n)
    rec = []
    x, st, it, _ = krylov.fgmres(lambda v: A @ v, f, M, rtol=1e-300, maxit=k, restart=20, record=rec)
    Z = np.column_stack(rec)
    y = np.linalg.lstsq(A @ Z, f, rcond=None)[0]
    assert np.allclose(x, Z @ y, rtol=1e-9, atol=1e-10)


def test_exact_in_n_steps_and_residual_estimate_is_true_residual():
    """Without restart an n x n system is solved in at most n steps, and each
    step's estimate |g_{j+1}| / ||f|| equals the true relative residual of the
    least-squares iterate after j steps."""
    n = 8
    A = _spd(n, 5)
    f = np.random.default_rng(6).standard_normal(n)
    x, st, it, hist = krylov.fgmres(lambda v: A @ v, f, rtol=1e-12, maxit=n, restart=n)
    assert st == krylov.CONVERGED and it <= n
    assert np.linalg.norm(f - A @ x) / np.linalg.norm(f) < 1e-12
    for j in range(1, 5):
        xj, _, _, hj = krylov.fgmres(lambda v: A @ v, f, rtol=1e-300, maxit=j, restart=n)
        true = np.linalg.norm(f - A @ xj) / np.linalg.norm(f)
        assert abs(hj[-1] - true) <= 1e-12 + 1e-9 * true


def test_restarted_residual_monotone_and_matches_unrestarted_first_cycle():
    n = 30
    A = _spd(n, 7)
    f = np.random.default_rng(8).standard_normal(n)
    x, st, it, hist = krylov.fgmres(lambda v: A @ v, f, rtol=1e-10, maxit=400, restart=5)
    assert st == krylov.CONVERGED
    # non-increasing up to rounding (relative to ||f||: history is ||r|| / ||f||)
    assert all(b <= a + 1e-13 for a, b in zip(hist, hist[1:]))
    x5, _, _, h5 = krylov.fgmres(lambda v: A @ v, f, rtol=1e-300, maxit=5, restart=50)
    assert abs(h5[-1] - hist[5]) <= 1e-12


def test_happy_breakdown_on_an_eigenvector():
    """f an eigenvector of A (M = I): the Krylov space is one-dimensional, the
    second Hessenberg entry vanishes and x = f / lambda after one step."""
    n = 6
    A = _spd(n, 9)
    lam, U = np.linalg.eigh(A)
    f = U[:, 2]
    x, st, it, hist = krylov.fgmres(lambda v: A @ v, f, rtol=1e-13, maxit=50, restart=10)
    assert st == krylov.CONVERGED and it == 1
    assert np.allclose(x, f / lam[2], atol=1e-13)


def test_nonfinite_and_zero_rhs():
    n = 4
    A = np.eye(n)
    x, st, it, _ = krylov.fgmres(lambda v: A @ v, np.zeros(n))
    assert st == krylov.CONVERGED and it == 0 and not x.any()
    x, st, it, _ = krylov.fgmres(lambda v: A @ v * np.nan, np.ones(n), maxit=5)
    assert st == krylov.NONFINITE


def test_gmg_fgmres_matches_direct_solve():
    """Config 0 with the oracle V-cycle as (right) preconditioner: FGMRES(32)
    to 1e-10 reproduces the direct solve of the free-DOF system."""
    import scipy.sparse.linalg as spla
    import workloads
    from oracle import mesh, multigrid
    dims = (16, 8, 8)
    fixed = workloads.cantilever_fixed(dims).astype(bool)
    E = mesh.simp_modulus(workloads.uniform_rho(dims), 3)
    K = mesh.assemble(dims, E, fixed=fixed)
    f = workloads.edge_load(dims)
    h = multigrid.build(dims, E, fixed, multigrid.Options(n_levels=3))
    x, st, it, hist = krylov.fgmres(lambda v: K @ v, f, lambda r: multigrid.vcycle(h, r),
                                    rtol=1e-10, maxit=200, restart=32)
    assert st == krylov.CONVERGED and it < 60
    fr = ~fixed
    us = np.zeros(fixed.size)
    us[fr] = spla.spsolve(K[fr][:, fr].tocsc(), f[fr])
    assert np.linalg.norm(x - us) <= 1e-8 * np.linalg.norm(us)
