"""Pins of the outer PCG (Sec. 3.6) and the M1-style direct-solve agreement (Sec. 4.2)."""
import numpy as np
import scipy.sparse.linalg as spla

from oracle import krylov, mesh, multigrid
import workloads


def _system(dims=(8, 4, 4), seed=0):
    g = np.random.default_rng(seed)
    E = mesh.simp_modulus(g.uniform(0.3, 1.0, np.prod(dims)), 3)
    fixed = mesh.cantilever_fixed(dims)
    K = mesh.assemble(dims, E, fixed=fixed)
    f = mesh.edge_load(dims)
    return dims, E, fixed, K, f


def _direct(K, f, fixed):
    fr = ~fixed
    u = np.zeros_like(f)
    u[fr] = spla.spsolve(K[fr][:, fr].tocsc(), f[fr])
    return u


def test_cg_matches_scipy_iterates():
    dims, E, fixed, K, f = _system()
    fr = np.where(~fixed)[0]
    A = K[fr][:, fr]
    ours, ref = [], []
    krylov.pcg(lambda v: K @ v, f, None, rtol=1e-30, maxit=12, callback=lambda x: ours.append(x[fr].copy()))
    spla.cg(A, f[fr], rtol=1e-30, maxiter=12, callback=lambda x: ref.append(x.copy()))
    for a, b in zip(ours, ref):
        assert np.abs(a - b).max() < 1e-9 * np.abs(b).max()


def test_jacobi_pcg_matches_scipy_iterates():
    dims, E, fixed, K, f = _system(seed=1)
    fr = np.where(~fixed)[0]
    A = K[fr][:, fr]
    dinv = 1 / A.diagonal()
    ours, ref = [], []
    dfull = np.zeros_like(f)
    dfull[fr] = dinv
    krylov.pcg(lambda v: K @ v, f, lambda r: dfull * r, rtol=1e-30, maxit=12,
               callback=lambda x: ours.append(x[fr].copy()))
    Mop = spla.LinearOperator(A.shape, matvec=lambda v: dinv * v)
    spla.cg(A, f[fr], rtol=1e-30, maxiter=12, M=Mop, callback=lambda x: ref.append(x.copy()))
    for a, b in zip(ours, ref):
        assert np.abs(a - b).max() < 1e-9 * np.abs(b).max()


def test_gmg_pcg_agrees_with_direct_solve():
    """Analogue of validation check M1: residual below 1e-10 and direct-solve agreement."""
    dims, E, fixed, K, f = _system((16, 8, 8), seed=2)
    h = multigrid.build(dims, E, fixed, multigrid.Options(n_levels=3))
    x, st, it, hist = krylov.pcg(lambda v: K @ v, f, lambda r: multigrid.vcycle(h, r), rtol=1e-10, maxit=200)
    assert st == krylov.CONVERGED
    assert krylov.true_rel_residual(lambda v: K @ v, f, x) < 1e-10
    u = _direct(K, f, fixed)
    assert np.linalg.norm(x - u) < 1e-8 * np.linalg.norm(u)


def test_compliance_monotone_and_bounded():
    dims, E, fixed, K, f = _system(seed=3)
    u = _direct(K, f, fixed)
    h = multigrid.build(dims, E, fixed, multigrid.Options(n_levels=2))
    comp = []
    krylov.pcg(lambda v: K @ v, f, lambda r: multigrid.vcycle(h, r), rtol=1e-12, maxit=100,
               callback=lambda x: comp.append(f @ x))
    assert all(b >= a - 1e-14 * abs(f @ u) for a, b in zip(comp, comp[1:]))
    assert max(comp) <= (f @ u) * (1 + 1e-12)


def test_config0_iteration_counts():
    dims = (16, 8, 8)
    fixed = mesh.cantilever_fixed(dims)
    E = mesh.simp_modulus(workloads.uniform_rho(dims), 3)
    K = mesh.assemble(dims, E, fixed=fixed)
    f = mesh.edge_load(dims)
    h = multigrid.build(dims, E, fixed, multigrid.Options(n_levels=3))
    x, st, it, _ = krylov.pcg(lambda v: K @ v, f, lambda r: multigrid.vcycle(h, r), rtol=1e-6, maxit=200)
    assert st == krylov.CONVERGED and it <= 30
    x, st, itj, _ = krylov.pcg(lambda v: K @ v, f, lambda r: h.levels[0].dinv * r, rtol=1e-6, maxit=2000)
    assert st == krylov.CONVERGED and itj > 3 * it


def test_failure_statuses():
    dims, E, fixed, K, f = _system()
    _, st, it, _ = krylov.pcg(lambda v: K @ v, f, None, rtol=1e-6, maxit=1)
    assert st == krylov.MAXIT and it == 1
    fn = f.copy()
    fn[-1] = np.nan
    _, st, _, _ = krylov.pcg(lambda v: K @ v, fn, None, rtol=1e-6, maxit=5)
    assert st == krylov.NONFINITE
    _, st, _, _ = krylov.pcg(lambda v: K @ v, f, lambda r: -r, rtol=1e-6, maxit=5)
    assert st == krylov.BREAKDOWN
    x0 = _direct(K, f, fixed)
    _, st, it, _ = krylov.pcg(lambda v: K @ v, f, None, x0=x0, rtol=1e-6, maxit=5)
    assert st == krylov.CONVERGED and it == 0
