"""Pins of the Lanczos kappa_eff probe (Sec. 4 E5/E10, Eq. kappa_bound):
against dense eigenvalues of M K, Cauchy interlacing of the Ritz values,
CG's Lanczos connection and the breakdown on an eigenvector."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import mesh, multigrid, spectral


def _system(dims, L=2, seed=0):
    g = np.random.default_rng(seed)
    E = mesh.simp_modulus(g.uniform(0.2, 1.0, int(np.prod(dims))), 3)
    fixed = mesh.cantilever_fixed(dims)
    K = mesh.assemble(dims, E, fixed=fixed)
    h = multigrid.build(dims, E, fixed, multigrid.Options(n_levels=L))
    return K, h, fixed


def _start(fixed, seed=5):
    v = np.random.default_rng(seed).standard_normal(fixed.size)
    v[fixed] = 0.0
    return v / np.linalg.norm(v)


def _dense_M(h, fixed):
    fr = np.where(~fixed)[0]
    M = np.empty((fr.size, fr.size))
    for k, i in enumerate(fr):
        e = np.zeros(fixed.size)
        e[i] = 1.0
        M[:, k] = multigrid.vcycle(h, e)[fr]
    return M


def test_identity_preconditioner_full_run_gives_extreme_eigenvalues_of_K():
    K, _, fixed = _system((4, 2, 2))
    fr = ~fixed
    lam = np.linalg.eigvalsh(K[fr][:, fr].toarray())
    # without reorthogonalisation the small end (kappa(K) ~ 2.5e3) needs about 2n steps
    kap, lo, hi, a, b = spectral.kappa_eff(lambda v: K @ v, None, _start(fixed), m=3 * int(fr.sum()))
    assert lo == pytest.approx(lam[0], rel=1e-9)
    assert hi == pytest.approx(lam[-1], rel=1e-9)
    assert kap == pytest.approx(lam[-1] / lam[0], rel=1e-8)


def test_vcycle_full_run_gives_kappa_of_MK():
    dims = (6, 4, 4)
    K, h, fixed = _system(dims)
    fr = ~fixed
    M = _dense_M(h, fixed)
    M = 0.5 * (M + M.T)
    # M K x = lam x  <=>  K x = lam M^-1 x
    lam = sla.eigh(K[fr][:, fr].toarray(), np.linalg.inv(M), eigvals_only=True)
    kap, lo, hi, _, _ = spectral.kappa_eff(lambda v: K @ v, lambda r: multigrid.vcycle(h, r),
                                           _start(fixed), m=int(fr.sum()) + 20)
    assert lo == pytest.approx(lam[0], rel=1e-7)
    assert hi == pytest.approx(lam[-1], rel=1e-7)
    assert kap == pytest.approx(lam[-1] / lam[0], rel=1e-7)
    assert kap < 10.0                          # a working V-cycle: kappa_eff is small


def test_ritz_values_interlace_and_kappa_grows_with_steps():
    dims = (6, 4, 4)
    K, h, fixed = _system(dims, seed=1)
    fr = ~fixed
    M = _dense_M(h, fixed)
    lam = sla.eigh(K[fr][:, fr].toarray(), np.linalg.inv(0.5 * (M + M.T)), eigvals_only=True)
    a, b = spectral.lanczos(lambda v: K @ v, lambda r: multigrid.vcycle(h, r), _start(fixed, 2), m=30)
    assert len(a) == 30
    prev = 1.0
    for k in range(1, 31):
        th = spectral.ritz_values(a[:k], b[:k])
        assert th[0] >= lam[0] * (1 - 1e-9) and th[-1] <= lam[-1] * (1 + 1e-9)
        kap = th[-1] / th[0]
        assert kap >= prev * (1 - 1e-12)
        prev = kap


def test_lanczos_connection_with_cg_coefficients():
    """T from the Lanczos recurrence equals T from PCG's step lengths and
    beta ratios (diag 1/al_j + be_{j-1}/al_{j-1}, off-diag sqrt(be_j)/al_j)."""
    K, h, fixed = _system((8, 4, 4), L=3, seed=2)
    g = _start(fixed, 3)
    M = lambda r: multigrid.vcycle(h, r)
    a, b = spectral.lanczos(lambda v: K @ v, M, g, m=12)
    r = g.copy()
    z = M(r)
    p = z.copy()
    rz = r @ z
    al, be = [], []
    for _ in range(12):
        q = K @ p
        alpha = rz / (p @ q)
        r = r - alpha * q
        z = M(r)
        rz_new = r @ z
        al.append(alpha)
        be.append(rz_new / rz)
        p = z + be[-1] * p
        rz = rz_new
    diag = [1 / al[0]] + [1 / al[j] + be[j - 1] / al[j - 1] for j in range(1, 12)]
    off = [np.sqrt(be[j]) / al[j] for j in range(11)]
    np.testing.assert_allclose(a, diag, rtol=1e-9)
    np.testing.assert_allclose(b[:11], off, rtol=1e-8)


def test_breakdown_on_an_eigenvector_and_scale_invariance():
    K, _, fixed = _system((4, 2, 2), seed=3)
    fr = np.where(~fixed)[0]
    lam, X = np.linalg.eigh(K[fr][:, fr].toarray())
    g = np.zeros(fixed.size)
    g[fr] = X[:, 7]
    a, b = spectral.lanczos(lambda v: K @ v, None, g, m=10)
    assert len(a) == 1 and a[0] == pytest.approx(lam[7], rel=1e-12)
    kap, *_ = spectral.kappa_eff(lambda v: K @ v, None, g, m=10)
    assert kap == 1.0
    g2 = _start(fixed, 4)
    a1, b1 = spectral.lanczos(lambda v: K @ v, None, g2, m=8)
    a2, b2 = spectral.lanczos(lambda v: K @ v, None, 1e3 * g2, m=8)
    np.testing.assert_allclose(a2, a1, rtol=1e-12)
    np.testing.assert_allclose(b2, b1, rtol=1e-12)


def test_breakdown_rule_does_not_depend_on_start_length():
    K, h, fixed = _system((6, 4, 4), seed=4)
    M = lambda r: multigrid.vcycle(h, r)
    g = _start(fixed, 6)
    a1, _ = spectral.lanczos(lambda v: K @ v, M, g, m=40, breakdown=0.18)
    a2, _ = spectral.lanczos(lambda v: K @ v, M, 1e-6 * g, m=40, breakdown=0.18)
    assert 1 < len(a1) < 40 and len(a2) == len(a1)
