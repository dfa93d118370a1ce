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


def _directions(K, f, precond, flexible, maxit):
    """Steps d_k = x_{k+1} - x_k of the oracle PCG (each a multiple of p_k)."""
    xs = [np.zeros_like(f)]
    krylov.pcg(lambda v: K @ v, f, precond, rtol=1e-30, maxit=maxit, flexible=flexible,
               callback=lambda x: xs.append(x.copy()))
    return [b - a for a, b in zip(xs, xs[1:])]


def test_flexible_beta_equals_fletcher_reeves_with_a_fixed_preconditioner():
    """Sec. 3.6 reading of beta: with a fixed SPD preconditioner z_{k+1}.r_k = 0
    in exact arithmetic, so the Polak-Ribiere (flexible) beta equals the
    Fletcher-Reeves one and both runs give the same iterates up to rounding."""
    dims, E, fixed, K, f = _system(seed=4)
    h = multigrid.build(dims, E, fixed, multigrid.Options(n_levels=2))
    M = lambda r: multigrid.vcycle(h, r)
    fr, pr = [], []
    krylov.pcg(lambda v: K @ v, f, M, rtol=1e-30, maxit=8, callback=lambda x: fr.append(x.copy()))
    krylov.pcg(lambda v: K @ v, f, M, rtol=1e-30, maxit=8, flexible=True,
               callback=lambda x: pr.append(x.copy()))
    assert len(fr) == len(pr) == 8
    for a, b in zip(fr, pr):
        assert np.abs(a - b).max() <= 1e-9 * np.abs(a).max()


def test_flexible_beta_keeps_consecutive_directions_conjugate():
    """With a preconditioner that changes every step (the BF16 V-cycle is not a
    fixed linear map), beta = z_{k+1}.(r_{k+1} - r_k) / z_k.r_k equals
    -z_{k+1}.K p_k / p_k.K p_k (because r_{k+1} - r_k = -alpha_k K p_k), so
    p_{k+1} is K-orthogonal to p_k whatever the preconditioner: the defining
    property of flexible CG.  Fletcher-Reeves loses it, which shows that the
    check discriminates."""
    dims, E, fixed, K, f = _system(seed=5)
    free = ~fixed
    g = np.random.default_rng(7)
    scales = [np.where(free, g.uniform(0.2, 5.0, f.size), 0.0) for _ in range(12)]
    d = K.diagonal()
    dinv = np.where(free, 1.0 / np.where(free, d, 1.0), 0.0)

    def varying():
        k = [0]

        def M(r):
            s = scales[k[0] % len(scales)]
            k[0] += 1
            return s * dinv * r
        return M

    def worst(dirs):
        w = 0.0
        for a, b in zip(dirs, dirs[1:]):
            Ka, Kb = K @ a, K @ b
            w = max(w, abs(b @ Ka) / np.sqrt((a @ Ka) * (b @ Kb)))
        return w

    flex = _directions(K, f, varying(), True, 10)
    fr = _directions(K, f, varying(), False, 10)
    assert len(flex) == 10
    assert worst(flex) < 1e-10
    assert worst(fr) > 1e-3


def _rule_trip(hist, w):
    """First iteration k >= w at which the best of the last w relative residuals
    is not 1% below the best before them (reading of the stagnation class)."""
    for k in range(w, len(hist)):
        h = hist[:k + 1]
        if min(h[-w:]) > 0.99 * min(h[:-w]):
            return k
    return None


def test_stagnation_status_at_the_first_qualifying_iteration():
    """Sec. 3.6 lists stagnant residual histories among the failure classes.
    Jacobi-PCG on the uniform 16x8x8 cantilever has a 2-norm residual that
    reaches a minimum and then rises for several iterations.  The residual
    history is recomputed from scipy's CG iterates (a library routine), and
    the oracle must stop with STAGNATED exactly where the window rule first
    holds on that history, with the same history up to that point."""
    dims = (16, 8, 8)
    fixed = mesh.cantilever_fixed(dims)
    E = mesh.simp_modulus(workloads.uniform_rho(dims), 3)
    K = mesh.assemble(dims, E, fixed=fixed)
    f = mesh.edge_load(dims)
    fr = np.where(~fixed)[0]
    A = K[fr][:, fr]
    dinv = 1.0 / A.diagonal()
    ref = [1.0]
    Mop = spla.LinearOperator(A.shape, matvec=lambda v: dinv * v)
    nf = np.linalg.norm(f[fr])
    spla.cg(A, f[fr], rtol=1e-30, maxiter=60, M=Mop,
            callback=lambda x: ref.append(float(np.linalg.norm(f[fr] - A @ x)) / nf))
    dfull = np.zeros_like(f)
    dfull[fr] = dinv
    for w in (3, 5, 8):
        k = _rule_trip(ref, w)
        assert k is not None and k < 60
        x, st, it, hist = krylov.pcg(lambda v: K @ v, f, lambda r: dfull * r, rtol=1e-12,
                                     maxit=200, stag_window=w)
        assert st == krylov.STAGNATED and it == k
        np.testing.assert_allclose(hist, ref[:k + 1], rtol=1e-8)
    # without the window the same run goes on to the cap
    _, st, it, _ = krylov.pcg(lambda v: K @ v, f, lambda r: dfull * r, rtol=1e-30, maxit=40)
    assert st == krylov.MAXIT and it == 40


def test_spectrum_margin_reading_on_a_random_field_cantilever():
    """Reading of the smoother spectrum margin (Sec. 3.4 targets [alpha lam, lam]
    with lam the power-iteration estimate of Sec. 3.5; no margin is printed).
    On a 48x24x24 random-field cantilever (the batch workload's system with
    seed 1010, rho in [1e-3, 1], p = 3) 20 power steps land more than 10%
    below lambda_max(D^-1 K): with the literal interval (1.0) or a 1.1 margin
    degree-2 Chebyshev amplifies the unresolved top of the spectrum, the
    V-cycle stops being positive definite and PCG breaks down (p.q <= 0 or
    r.z <= 0); with 1.3 the interval covers lambda_max and PCG converges."""
    dims = (48, 24, 24)
    rho = workloads.grf_rho(dims, 1010)
    E = mesh.simp_modulus(rho, 3)
    fixed = workloads.cantilever_fixed(dims).astype(bool)
    K = mesh.assemble(dims, E, fixed=fixed)
    f = workloads.edge_load(dims)
    h = multigrid.build(dims, E, fixed, multigrid.Options(n_levels=4))
    lev = h.levels[0]
    # lambda_max(D^-1 K) on the free DOFs: largest eigenvalue of the
    # symmetric D^-1/2 K D^-1/2 (ARPACK, a library routine)
    fr = np.where(~fixed)[0]
    s = 1.0 / np.sqrt(lev.d[fr])
    A = K[fr][:, fr]
    op = spla.LinearOperator(A.shape, matvec=lambda v: s * (A @ (s * v)), dtype=np.float64)
    lam_max = float(spla.eigsh(op, k=1, which="LA", tol=1e-8, return_eigenvectors=False)[0])
    assert lev.lam < lam_max / 1.1 and 1.3 * lev.lam > lam_max
    out = {}
    for safety in (1.0, 1.1, 1.3):
        h.opts.lambda_safety = safety
        _, st, it, _ = krylov.pcg(lambda v: K @ v, f, lambda r: multigrid.vcycle(h, r), rtol=1e-6,
                                  maxit=200)
        out[safety] = (st, it)
    assert out[1.0][0] == krylov.BREAKDOWN and out[1.1][0] == krylov.BREAKDOWN
    assert out[1.3][0] == krylov.CONVERGED and out[1.3][1] <= 40
