"""Galerkin geometric multigrid hierarchy and V-cycle (oracle, FP64).

Test infrastructure only.

Follows Sec. 3.2 (Eq. vcycle): pre-smooth from zero, restrict the residual with
R = P^T, recurse, prolong and correct, post-smooth from the corrected iterate
with the same right-hand side; the coarsest level is solved by dense Cholesky
of K_L + eps I (n_L <= 5000, eps = max(mean diag * 1e-8, 1e-14), Sec. 4.1)
or by a fixed number of PCG steps (Table repro_defaults: 80).  Level 0 uses
the Chebyshev (or damped-Jacobi) smoother of degree nu = 2, levels 1..L-1 use
damped Jacobi with 2 pre and 2 post sweeps (Table repro_defaults; reading).
Reading: the smoothers use 1.3 times the power-iteration estimate as the
upper end of the spectrum.  The estimate approaches lambda_max from below
(about 8% low after 20 steps on a uniform 20^3 cantilever, 20% low on a
48x24x24 random-field cantilever with rho in [1e-3, 1]), and degree-2
Chebyshev amplifies eigenvalues above its interval, which makes PCG break
down; the margin is an option (1.0 gives the literal form).
Level 0 is the assembled fine operator here, which the matrix-free action
equals exactly (Eq. mf_matvec).
"""
from dataclasses import dataclass, field
import numpy as np
import scipy.sparse as sp

from . import mesh, transfer, galerkin, smoothers


@dataclass
class Options:
    nu: float = 0.3
    E0: float = 1.0
    Emin: float = 1e-9
    penal: float = 3.0
    n_levels: int = 4
    fine_smoother: str = "chebyshev"      # or "jacobi"
    fine_degree: int = 2
    coarse_sweeps: int = 2
    cheb_alpha: float = 1.0 / 30.0
    jacobi_omega_max: float = 0.5
    power_iters_fine: int = 20
    power_iters_coarse: int = 10
    dense_max: int = 5000
    coarse_pcg_iters: int = 80
    seed: int = 0
    lambda_safety: float = 1.3            # smoothers use lambda_safety * estimate (reading)
    lambdas: list = None                  # optional override of the raw estimates


@dataclass
class Level:
    dims: tuple
    fixed: np.ndarray
    K: sp.csr_matrix
    d: np.ndarray = None
    dinv: np.ndarray = None
    lam: float = None                     # raw power-iteration estimate (floored)


@dataclass
class Hierarchy:
    opts: Options
    levels: list = field(default_factory=list)
    coarse_free: np.ndarray = None
    coarse_chol: np.ndarray = None
    coarse_eps: float = None


def auto_levels(dims, fixed, dense_max=5000, max_levels=6):
    """Fewest levels whose coarsest free-DOF count is <= dense_max (capped)."""
    for L in range(2, max_levels + 1):
        d = transfer.level_dims(dims, L)[-1]
        if min(d) < 1:
            return L - 1
        if transfer.free_counts(dims, fixed, L)[-1] <= dense_max:
            return L
    return max_levels


def build(dims, E, fixed, opts: Options):
    h = Hierarchy(opts=opts)
    fixed = np.asarray(fixed, dtype=bool)
    K0 = mesh.assemble(dims, E, opts.nu, fixed=fixed)
    h.levels.append(Level(tuple(dims), fixed, K0))
    for l in range(1, opts.n_levels):
        fine = h.levels[-1]
        cd = transfer.coarse_dims(fine.dims)
        cf = transfer.inject_fixed(fine.fixed, fine.dims)
        if l == 1:
            Kc = galerkin.galerkin_level1_local(fine.dims, E, fine.fixed, cf, opts.nu)
        else:
            Kc = galerkin.galerkin_explicit(fine.K, fine.dims, fine.fixed, cf)
        h.levels.append(Level(cd, cf, Kc))
    for l, lev in enumerate(h.levels):
        lev.d, lev.dinv = smoothers.diagonal(lev.K, lev.fixed)
    for l, lev in enumerate(h.levels[:-1]):
        if opts.lambdas is not None:
            lev.lam = float(opts.lambdas[l])
        else:
            iters = opts.power_iters_fine if l == 0 else opts.power_iters_coarse
            lev.lam = smoothers.power_lambda(lambda v, K=lev.K: K @ v, lev.d, lev.dinv,
                                             lev.fixed, iters, opts.seed + l)
    last = h.levels[-1]
    free = np.where(~last.fixed)[0]
    h.coarse_free = free
    A = last.K[free][:, free].toarray()
    h.coarse_eps = max(float(np.mean(np.diag(A))) * 1e-8, 1e-14) if free.size else 0.0
    if free.size <= opts.dense_max:
        h.coarse_chol = np.linalg.cholesky(A + h.coarse_eps * np.eye(free.size))
    return h


def coarse_solve(h, r):
    last = h.levels[-1]
    z = np.zeros_like(r)
    rf = r[h.coarse_free]
    if h.coarse_chol is not None:
        Lc = h.coarse_chol
        y = np.linalg.solve(Lc, rf)          # forward (triangular)
        z[h.coarse_free] = np.linalg.solve(Lc.T, y)
        return z
    # fixed-count Jacobi-PCG on K_L (reading of "fixed-count PCG")
    A = last.K
    x = np.zeros_like(r)
    res = r.copy()
    zz = last.dinv * res
    p = zz.copy()
    rz = res @ zz
    for _ in range(h.opts.coarse_pcg_iters):
        q = A @ p
        pq = p @ q
        if pq <= 0 or rz == 0:
            break
        a = rz / pq
        x += a * p
        res -= a * q
        zz = last.dinv * res
        rz_new = res @ zz
        p = zz + (rz_new / rz) * p
        rz = rz_new
    return x


def _smooth(h, l, b, x0):
    lev = h.levels[l]
    o = h.opts
    A = lambda v, K=lev.K: K @ v
    if l == 0 and o.fine_smoother == "chebyshev":
        return smoothers.chebyshev(A, b, lev.dinv, o.lambda_safety * lev.lam, o.fine_degree,
                                   o.cheb_alpha, x0)
    sweeps = o.fine_degree if l == 0 else o.coarse_sweeps
    omega = smoothers.jacobi_omega(o.lambda_safety * lev.lam, o.jacobi_omega_max)
    return smoothers.jacobi(A, b, lev.dinv, omega, sweeps, x0)


def restrict(h, l, r_fine):
    """M_{l+1} P^T M_l r."""
    fine, coarse = h.levels[l], h.levels[l + 1]
    P = transfer.prolongation(fine.dims)
    rc = P.T @ np.where(fine.fixed, 0.0, r_fine)
    rc[coarse.fixed] = 0.0
    return rc


def prolong(h, l, e_coarse):
    """M_l P M_{l+1} e."""
    fine, coarse = h.levels[l], h.levels[l + 1]
    P = transfer.prolongation(fine.dims)
    e = P @ np.where(coarse.fixed, 0.0, e_coarse)
    e[fine.fixed] = 0.0
    return e


def vcycle(h, r, l=0):
    """z = V^l(r) of Eq. vcycle."""
    L = len(h.levels) - 1
    if l == L:
        return coarse_solve(h, r)
    K = h.levels[l].K
    x = _smooth(h, l, r, None)
    rc = restrict(h, l, r - K @ x)
    ec = vcycle(h, rc, l + 1)
    x = x + prolong(h, l, ec)
    return _smooth(h, l, r, x)


def cycle(h, r, gamma=1, l=0, x0=None):
    """Multigrid cycle with cycle index gamma (Sec. 4 E6(c): V-cycle gamma = 1,
    W-cycle gamma = 2; Trottenberg, Oosterlee and Schueller, Multigrid,
    Sec. 2.4): pre-smooth from x0 (zero if None), restrict the residual,
    approximate the coarse residual equation by gamma cycles of the coarser
    level, each starting from the previous one's result (the coarsest level
    is solved once: a second solve adds nothing), prolong, post-smooth.
    gamma = 1 from zero is the V-cycle of Eq. vcycle."""
    L = len(h.levels) - 1
    if l == L:
        return coarse_solve(h, r)
    K = h.levels[l].K
    x = _smooth(h, l, r, x0)
    rc = restrict(h, l, r - K @ x)
    if l + 1 == L:
        ec = coarse_solve(h, rc)
    else:
        ec = None
        for _ in range(gamma):
            ec = cycle(h, rc, gamma, l + 1, ec)
    x = x + prolong(h, l, ec)
    return _smooth(h, l, r, x)
