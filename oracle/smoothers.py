"""Diagonal, power iteration, Chebyshev-Jacobi and damped-Jacobi smoothers (oracle, FP64).

Test infrastructure only.

* Power iteration: Sec. 3.5 (spectral-radius estimation): a fixed number of
  iterations (20 fine, 10 coarse) for lambda_max(D^-1 K), floored at 1e-6
  (Sec. 4.1 safeguards).  Reading: start vector uniform on [-1,1) from
  SplitMix64 (seed + level) on free DOFs; k-th step forms w = K x, takes the
  D-inner-product Rayleigh quotient (x.w)/(x.Dx), then x <- D^-1 w / ||D^-1 w||_2;
  the quotient of the last step is returned (exactly N products with K).
* Chebyshev: Sec. 3.4 targets [alpha*lam, lam] of D^-1 K and cites Saad,
  "Iterative Methods for Sparse Linear Systems", Ch. 12 (Chebyshev
  acceleration).  The printed algorithm's seed/recurrence is garbled, so the
  three-term Chebyshev acceleration of that chapter is used: theta = centre,
  delta = half-width, sigma1 = theta/delta, rho_0 = 1/sigma1,
  d_0 = D^-1 r_0 / theta, rho_{k+1} = 1/(2 sigma1 - rho_k),
  d_{k+1} = rho_{k+1} rho_k d_k + (2 rho_{k+1}/delta) D^-1 r_{k+1}.
* Damped Jacobi: x <- x + omega D^-1 (b - K x), omega = min(omega_max, 4/(3 lam))
  (omega_max = 0.5 from Table repro_defaults; the 4/(3 lam) rule is a reading).
"""
import numpy as np

from .rng import uniform_pm1

LAMBDA_FLOOR = 1e-6


def diagonal(K, fixed):
    """D = diag(K) on free DOFs, floored at 1e-30 * max D; D^-1 is 0 on fixed DOFs."""
    fixed = np.asarray(fixed, dtype=bool)
    d = K.diagonal().astype(np.float64).copy()
    free = ~fixed
    dmax = d[free].max() if free.any() else 1.0
    d[free] = np.maximum(d[free], 1e-30 * dmax)
    dinv = np.zeros_like(d)
    dinv[free] = 1.0 / d[free]
    d[fixed] = 0.0
    return d, dinv


def power_lambda(apply_K, d, dinv, fixed, iters, seed):
    """Estimate lambda_max(D^-1 K) with exactly ``iters`` products with K."""
    fixed = np.asarray(fixed, dtype=bool)
    x = uniform_pm1(seed, d.size)
    x[fixed] = 0.0
    x /= np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        w = apply_K(x)
        lam = float(x @ w) / float(x @ (d * x))
        y = dinv * w
        ny = np.linalg.norm(y)
        if not ny > 0:                     # K x = 0: nothing left to iterate on
            break
        x = y / ny
    return lam if lam > LAMBDA_FLOOR else LAMBDA_FLOOR


def chebyshev(apply_K, b, dinv, lam, degree, alpha, x0=None):
    """Degree-``degree`` Chebyshev-Jacobi smoothing of K x = b on [alpha*lam, lam]."""
    theta = 0.5 * lam * (1.0 + alpha)
    delta = 0.5 * lam * (1.0 - alpha)
    sigma1 = theta / delta
    if x0 is None:
        x = np.zeros_like(b)
        r = b.copy()
    else:
        x = x0.copy()
        r = b - apply_K(x)
    d = dinv * r / theta
    rho = 1.0 / sigma1
    for k in range(degree):
        x = x + d
        if k == degree - 1:
            break
        r = b - apply_K(x)
        rho_new = 1.0 / (2.0 * sigma1 - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (dinv * r)
        rho = rho_new
    return x


def jacobi_omega(lam, omega_max):
    return min(omega_max, 4.0 / (3.0 * lam))


def jacobi(apply_K, b, dinv, omega, sweeps, x0=None):
    """``sweeps`` damped-Jacobi sweeps for K x = b."""
    if x0 is None:
        x = omega * dinv * b
        start = 1
    else:
        x = x0.copy()
        start = 0
    for _ in range(start, sweeps):
        x = x + omega * dinv * (b - apply_K(x))
    return x


def chebyshev_residual_polynomial(lmb, lam, degree, alpha):
    """Closed form of the Chebyshev error factor p(l) = T_k((theta - l)/delta) / T_k(theta/delta)."""
    theta = 0.5 * lam * (1.0 + alpha)
    delta = 0.5 * lam * (1.0 - alpha)
    T = np.polynomial.chebyshev.Chebyshev.basis(degree)
    return T((theta - np.asarray(lmb)) / delta) / T(theta / delta)
