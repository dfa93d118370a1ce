"""Lanczos probe of the effective condition number of the preconditioned
operator M K (oracle, FP64).

Test infrastructure only.

The robustness and BF16 spectral-proxy screens (Sec. 4: E5, E10; the
conditional bound of App. bound, Eq. kappa_bound) measure
kappa_eff = lambda_max(M K) / lambda_min(M K) for the frozen V-cycle M by a
Lanczos process started from a normalised Gaussian vector (Table
repro_defaults).  M is SPD (symmetric pre/post smoothing, Galerkin coarse
operators), so M K is self-adjoint in the M^-1 inner product, and the
textbook preconditioned Lanczos process (Saad, Iterative Methods for Sparse
Linear Systems, Sec. 9.2 with the M^-1 inner product) tridiagonalises it
while applying only M and K: each basis vector v_j is carried together with
w_j = M^-1 v_j.

    r_1 = g,  z_1 = M r_1,  b_1 = sqrt(r_1 . z_1),  v_1 = z_1 / b_1,  w_1 = r_1 / b_1
    step j:  s = K v_j,  a_j = s . v_j,
             r_{j+1} = s - a_j w_j - b_j w_{j-1}      (b_1 w_0 := 0),
             z_{j+1} = M r_{j+1},  b_{j+1} = sqrt(r_{j+1} . z_{j+1}),
             v_{j+1} = z_{j+1} / b_{j+1},  w_{j+1} = r_{j+1} / b_{j+1}.

T_m = tridiag(b_2..b_m; a_1..a_m; b_2..b_m); its eigenvalues (Ritz values)
lie in [lambda_min, lambda_max] of M K and move outwards as m grows, so
kappa_m = theta_max / theta_min is a lower estimate of kappa_eff.

Readings (the paper gives neither): no reorthogonalisation; m steps (50 by
default), ending earlier when b_{j+1} <= breakdown * max_i<=j |a_i| (an
invariant subspace, measured against the spectral scale, so that the rule
does not depend on the length of g) or when r . z is not positive (M not SPD
to rounding); the start
vector is the caller's (a seeded Gaussian on the free DOFs: the paper's
CuPy draw cannot be reproduced).
"""
import numpy as np
from scipy.linalg import eigvalsh_tridiagonal


def lanczos(apply_A, precond, g, m=50, breakdown=1e-12):
    """Returns (alpha, beta): alpha[j] = a_{j+1}, beta[j] = b_{j+2} (the norm
    after step j; beta[:-1] are the off-diagonals of T).  len(alpha) is the
    number of steps taken."""
    M = precond if precond is not None else (lambda v: v.copy())
    r = np.array(g, dtype=np.float64)
    z = M(r)
    rz = float(r @ z)
    if not rz > 0.0:
        return np.zeros(0), np.zeros(0)
    b1 = np.sqrt(rz)
    v, w = z / b1, r / b1
    w_prev = np.zeros_like(w)
    b = 0.0
    amax = 0.0
    alpha, beta = [], []
    for _ in range(m):
        s = apply_A(v)
        a = float(s @ v)
        r = s - a * w - b * w_prev
        z = M(r)
        rz = float(r @ z)
        alpha.append(a)
        amax = max(amax, abs(a))
        bn = np.sqrt(rz) if rz > 0.0 else 0.0
        beta.append(bn)
        if not bn > breakdown * amax:
            break
        w_prev, w, v, b = w, r / bn, z / bn, bn
    return np.array(alpha), np.array(beta)


def ritz_values(alpha, beta):
    """Eigenvalues of T (ascending)."""
    k = len(alpha)
    if k == 0:
        return np.zeros(0)
    if k == 1:
        return np.array(alpha[:1], dtype=np.float64)
    return eigvalsh_tridiagonal(np.asarray(alpha, dtype=np.float64),
                                np.asarray(beta[:k - 1], dtype=np.float64))


def kappa_eff(apply_A, precond, g, m=50, breakdown=1e-12):
    """(kappa, theta_min, theta_max, alpha, beta) from m Lanczos steps."""
    alpha, beta = lanczos(apply_A, precond, g, m, breakdown)
    th = ritz_values(alpha, beta)
    if th.size == 0:
        return float("nan"), float("nan"), float("nan"), alpha, beta
    return float(th[-1] / th[0]), float(th[0]), float(th[-1]), alpha, beta
