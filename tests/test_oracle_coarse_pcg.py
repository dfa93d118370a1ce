"""Pins of the iterative coarsest solve: above the dense cutoff the coarsest
level is solved by a fixed number of Jacobi-PCG steps (Sec. 3.2; Table
repro_defaults: 80 steps past 5000 coarse DOFs).  The steps are pinned to
conjugate-gradient theory, not to a second copy of the iteration: after k
steps from zero, preconditioned CG minimises the K-energy error over the
Krylov space span{z, (D^-1 K) z, ..., (D^-1 K)^(k-1) z} with z = D^-1 r.
"""
import numpy as np
import pytest

from oracle import multigrid, mesh


def _hier(dims, L, iters, seed=0):
    g = np.random.default_rng(seed)
    E = mesh.simp_modulus(g.uniform(0.2, 1.0, int(np.prod(dims))), 3)
    fixed = mesh.cantilever_fixed(dims)
    return multigrid.build(dims, E, fixed,
                           multigrid.Options(n_levels=L, dense_max=0, coarse_pcg_iters=iters))


def _rhs(h, seed=1):
    last = h.levels[-1]
    r = np.random.default_rng(seed).standard_normal(last.fixed.size)
    r[last.fixed] = 0.0
    return r


def _krylov_energy_min(h, r, k):
    """x in the k-dimensional preconditioned Krylov space minimising ||x - K^-1 r||_K."""
    last = h.levels[-1]
    fr = ~last.fixed
    A = last.K[fr][:, fr].toarray()
    dinv = last.dinv[fr]
    w = dinv * r[fr]
    W = np.empty((w.size, k))
    for j in range(k):
        W[:, j] = w
        w = dinv * (A @ w)
    Q, _ = np.linalg.qr(W)                   # same span, well conditioned
    y = np.linalg.solve(Q.T @ A @ Q, Q.T @ r[fr])
    x = np.zeros_like(r)
    x[fr] = Q @ y
    return x


def test_dense_cutoff_switches_to_pcg():
    h = _hier((4, 2, 2), 2, 5)
    assert h.coarse_chol is None
    h2 = multigrid.build((4, 2, 2), np.ones(16), mesh.cantilever_fixed((4, 2, 2)),
                         multigrid.Options(n_levels=2))
    assert h2.coarse_chol is not None


def test_one_step_is_the_optimal_multiple_of_the_jacobi_direction():
    h = _hier((6, 4, 4), 2, 1)
    r = _rhs(h)
    last = h.levels[-1]
    z = last.dinv * r
    Kz = last.K @ z
    x = multigrid.coarse_solve(h, r)
    np.testing.assert_allclose(x, (r @ z) / (z @ Kz) * z, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("k", [2, 3, 5])
def test_k_steps_minimise_energy_over_krylov_space(k):
    h = _hier((6, 4, 4), 2, k)
    r = _rhs(h)
    x = multigrid.coarse_solve(h, r)
    ref = _krylov_energy_min(h, r, k)
    np.testing.assert_allclose(x, ref, rtol=0, atol=1e-9 * np.abs(ref).max())


def test_many_steps_reach_the_exact_coarse_solution():
    h = _hier((6, 4, 4), 2, 400)
    r = _rhs(h)
    last = h.levels[-1]
    fr = ~last.fixed
    x = multigrid.coarse_solve(h, r)
    exact = np.linalg.solve(last.K[fr][:, fr].toarray(), r[fr])
    np.testing.assert_allclose(x[fr], exact, rtol=0, atol=1e-9 * np.abs(exact).max())
    assert np.all(x[~fr] == 0.0)


def test_zero_right_hand_side_returns_zero():
    h = _hier((4, 2, 2), 2, 80)
    x = multigrid.coarse_solve(h, np.zeros(h.levels[-1].fixed.size))
    assert np.all(x == 0.0)


def test_vcycle_with_converged_pcg_matches_dense_coarsest():
    """With enough steps the V-cycle with the iterative coarsest solve equals
    the one with the dense solve up to the dense solve's eps regularisation."""
    dims = (8, 4, 4)
    g = np.random.default_rng(3)
    E = mesh.simp_modulus(g.uniform(0.2, 1.0, int(np.prod(dims))), 3)
    fixed = mesh.cantilever_fixed(dims)
    hd = multigrid.build(dims, E, fixed, multigrid.Options(n_levels=3))
    hi = multigrid.build(dims, E, fixed, multigrid.Options(n_levels=3, dense_max=0,
                                                           coarse_pcg_iters=400))
    r = g.standard_normal(fixed.size)
    r[fixed] = 0.0
    zd = multigrid.vcycle(hd, r)
    zi = multigrid.vcycle(hi, r)
    np.testing.assert_allclose(zi, zd, rtol=0, atol=1e-6 * np.abs(zd).max())
