"""Pins of diagonal, power iteration, Chebyshev and Jacobi (Sec. 3.4, 3.5, App. D)."""
import json
import os

import numpy as np

from oracle import mesh, rng, smoothers

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")))


def _small_system(dims=(4, 3, 3), seed=0):
    g = np.random.default_rng(seed)
    E = g.uniform(0.05, 1.0, np.prod(dims))
    fixed = mesh.cantilever_fixed(dims)
    K = mesh.assemble(dims, E, fixed=fixed)
    d, dinv = smoothers.diagonal(K, fixed)
    free = ~fixed
    A = K[free][:, free].toarray()
    Dh = np.sqrt(d[free])
    w, V = np.linalg.eigh(A / Dh[:, None] / Dh[None, :])     # D^-1/2 K D^-1/2
    return K, fixed, d, dinv, free, w, V, Dh


def test_splitmix64_published_first_output():
    # first output of SplitMix64 seeded with 0 (reference implementation value)
    assert int(rng.splitmix64(0, 1)[0]) == 0xE220A8397B1DCDAF
    u = rng.uniform_pm1(123, 100000)
    assert u.min() >= -1 and u.max() < 1 and abs(u.mean()) < 0.01


def test_chebyshev_band_factor_paper_value():
    g = GOLD["chebyshev_band_factor"]
    lmb = np.linspace(g["alpha"], 1.0, 20001)
    p = smoothers.chebyshev_residual_polynomial(lmb, 1.0, g["degree"], g["alpha"])
    assert abs(np.abs(p).max() - g["value_about"]) < g["abs_tol"]
    # and the exact 1 / T_2(31/29)
    assert abs(np.abs(p).max() - 1.0 / (2 * (31 / 29) ** 2 - 1)) < 1e-12


def test_chebyshev_error_polynomial():
    """Error after nu steps = p_nu(D^-1 K) e_0 in the eigenbasis (closed form)."""
    K, fixed, d, dinv, free, w, V, Dh = _small_system()
    lam = w.max() * 1.02
    g = np.random.default_rng(1)
    xs = np.zeros(fixed.size)
    xs[free] = g.standard_normal(free.sum())
    b = K @ xs
    for degree in (1, 2, 3, 4):
        for x0 in (None, np.where(fixed, 0, g.standard_normal(fixed.size))):
            x = smoothers.chebyshev(lambda v: K @ v, b, dinv, lam, degree, 1 / 30, x0)
            e0 = (xs if x0 is None else xs - x0)[free] * Dh
            pred = V @ (smoothers.chebyshev_residual_polynomial(w, lam, degree, 1 / 30) * (V.T @ e0))
            assert np.abs((xs - x)[free] * Dh - pred).max() < 1e-11 * np.abs(e0).max()


def test_jacobi_error_polynomial():
    K, fixed, d, dinv, free, w, V, Dh = _small_system(seed=2)
    g = np.random.default_rng(3)
    xs = np.where(fixed, 0, g.standard_normal(fixed.size))
    b = K @ xs
    omega = smoothers.jacobi_omega(w.max(), 0.5)
    for m in (1, 2, 3):
        x = smoothers.jacobi(lambda v: K @ v, b, dinv, omega, m)
        e0 = xs[free] * Dh
        pred = V @ ((1 - omega * w) ** m * (V.T @ e0))
        assert np.abs((xs - x)[free] * Dh - pred).max() < 1e-11 * np.abs(e0).max()


def test_power_iteration_lower_bound_and_monotone():
    K, fixed, d, dinv, free, w, V, Dh = _small_system(dims=(6, 4, 4), seed=4)
    ests = [smoothers.power_lambda(lambda v: K @ v, d, dinv, fixed, it, 0) for it in (2, 5, 10, 20, 200)]
    assert all(e <= w.max() * (1 + 1e-12) for e in ests)
    assert all(b >= a - 1e-12 for a, b in zip(ests, ests[1:]))
    assert abs(ests[-1] - w.max()) < 2e-3 * w.max()


def test_power_iteration_floor():
    K, fixed, d, dinv, free, w, V, Dh = _small_system()
    assert smoothers.power_lambda(lambda v: 0 * v, d, dinv, fixed, 3, 0) == smoothers.LAMBDA_FLOOR


def test_diagonal_floor_and_fixed():
    K, fixed, d, dinv, free, w, V, Dh = _small_system()
    assert np.all(dinv[fixed] == 0) and np.all(d[free] > 0)
    assert np.allclose(dinv[free] * K.diagonal()[free], 1.0)
