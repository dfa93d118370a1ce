"""Preconditioned conjugate gradients with true-residual acceptance (oracle, FP64).

Test infrastructure only.

Follows Sec. 3.6: left-preconditioned CG (Saad, Alg. 9.1) with the frozen
V-cycle (or D^-1, or nothing) as preconditioner; convergence is
||f - K x||_2 / ||f||_2 < rtol checked on the true residual; iteration caps,
stagnation and non-finite iterates are failures.  Readings: the recursive
residual triggers the true-residual check, a failed check replaces r by the
true residual and restarts the recurrence (beta = 0); stagnation (opt-in, window w, the paper's Jacobi-PCG runs reach
the cap rather than stop early) = the best relative residual of the last w
iterations is not 1% below the best before them; beta is Fletcher-Reeves, or
Polak-Ribiere (flexible) on request.
"""
import numpy as np

CONVERGED, MAXIT, STAGNATED, NONFINITE, BREAKDOWN = 0, 1, 2, 3, 4


def pcg(apply_A, f, precond=None, x0=None, rtol=1e-6, maxit=200, flexible=False,
        stag_window=0, callback=None):
    """Returns (x, status, iters, history) with history[k] = ||r_k|| / ||f||."""
    M = precond if precond is not None else (lambda v: v.copy())
    nf = float(np.linalg.norm(f))
    if nf == 0.0:
        return np.zeros_like(f), CONVERGED, 0, [0.0]
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64)
    r = f - apply_A(x) if x0 is not None else f.copy()
    hist = [float(np.linalg.norm(r)) / nf]
    if not np.isfinite(hist[0]):
        return x, NONFINITE, 0, hist
    if hist[0] < rtol:
        return x, CONVERGED, 0, hist
    z = M(r)
    rz = float(r @ z)
    if not np.isfinite(rz):
        return x, NONFINITE, 0, hist
    if rz <= 0:
        return x, BREAKDOWN, 0, hist
    p = z.copy()
    for it in range(1, maxit + 1):
        q = apply_A(p)
        pq = float(p @ q)
        if not np.isfinite(pq):
            return x, NONFINITE, it - 1, hist
        if pq <= 0:
            return x, BREAKDOWN, it - 1, hist
        alpha = rz / pq
        x = x + alpha * p
        if callback is not None:
            callback(x)
        r_old = r
        r = r - alpha * q
        rel = float(np.linalg.norm(r)) / nf
        if not np.isfinite(rel):
            hist.append(rel)
            return x, NONFINITE, it, hist
        if rel < rtol:
            rt = f - apply_A(x)
            rel_true = float(np.linalg.norm(rt)) / nf
            if rel_true < rtol:
                hist.append(rel)
                return x, CONVERGED, it, hist
            r = rt
            rel = rel_true
            restart = True
        else:
            restart = False
        hist.append(rel)
        if stag_window and it >= stag_window:
            if min(hist[-stag_window:]) > 0.99 * min(hist[:-stag_window]):
                return x, STAGNATED, it, hist
        z = M(r)
        rz_new = float(r @ z)
        if not np.isfinite(rz_new):
            return x, NONFINITE, it, hist
        if rz_new <= 0:
            return x, BREAKDOWN, it, hist
        if restart:
            beta = 0.0
        elif flexible:
            beta = float(z @ (r - r_old)) / rz
        else:
            beta = rz_new / rz
        p = z + beta * p
        rz = rz_new
    return x, MAXIT, maxit, hist


def true_rel_residual(apply_A, f, x):
    return float(np.linalg.norm(f - apply_A(x))) / float(np.linalg.norm(f))
