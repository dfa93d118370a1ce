"""Preconditioned Krylov solvers with true-residual acceptance (oracle, FP64):
CG (pcg) and restarted flexible GMRES (fgmres).

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


def fgmres(apply_A, f, precond=None, x0=None, rtol=1e-6, maxit=200, restart=32,
           breakdown=1e-14, record=None):
    """Restarted right-preconditioned flexible GMRES (Sec. 3.6, outer solver of
    the BF16 and large-scale runs).  Each cycle starts from the true residual
    r = f - A x, beta = ||r||, v_1 = r / beta; step j stores z_j = M(v_j)
    (M may change between calls: the minimisation is over span{z_j}),
    w = A z_j, orthogonalises w against v_1..v_j by modified Gram-Schmidt,
    h_{j+1,j} = ||w||, and updates the QR factorisation of the Hessenberg
    matrix with one new Givens rotation, so |g_{j+1}| is the residual norm of
    the cycle's least-squares iterate.  A new Hessenberg entry below
    `breakdown` (absolute) ends the cycle (happy breakdown), as does the
    estimate reaching rtol or the cycle reaching `restart` steps; then
    x += Z y with R y = g (least squares if R is singular).  Acceptance is on
    the true residual at the start of the next cycle.

    Returns (x, status, iters, history): iters counts Arnoldi steps (products
    with A of preconditioned vectors); history holds the true relative
    residual at each cycle start and the estimate after each step.  `record`
    (a list, optional) receives the z_j of every step."""
    M = precond if precond is not None else (lambda v: v.copy())
    nf = float(np.linalg.norm(f))
    if nf == 0.0:
        return np.zeros_like(f), CONVERGED, 0, [0.0]
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64)
    it = 0
    hist = []
    while True:
        r = f - apply_A(x)
        beta = float(np.linalg.norm(r))
        rel = beta / nf
        hist.append(rel)
        if not np.isfinite(rel):
            return x, NONFINITE, it, hist
        if rel < rtol:
            return x, CONVERGED, it, hist
        if it >= maxit:
            return x, MAXIT, it, hist
        m = restart
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k = 0
        for j in range(m):
            if it >= maxit:
                break
            z = M(V[j])
            Z.append(z)
            if record is not None:
                record.append(z.copy())
            w = apply_A(z)
            for i in range(j + 1):                  # modified Gram-Schmidt
                H[i, j] = float(w @ V[i])
                w = w - H[i, j] * V[i]
            hnext = float(np.linalg.norm(w))
            H[j + 1, j] = hnext
            it += 1
            k = j + 1
            for i in range(j):                      # earlier rotations on column j
                a, b = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * b
                H[i + 1, j] = -sn[i] * a + cs[i] * b
            a, b = H[j, j], H[j + 1, j]
            d = float(np.hypot(a, b))
            cs[j], sn[j] = (a / d, b / d) if d > 0.0 else (1.0, 0.0)
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            est = abs(g[j + 1]) / nf
            hist.append(est)
            if not np.isfinite(est):
                return x, NONFINITE, it, hist
            if hnext < breakdown or est < rtol:
                break
            V.append(w / hnext)
        R = H[:k, :k]
        try:
            if np.any(np.diag(R) == 0.0):
                raise np.linalg.LinAlgError
            y = np.linalg.solve(np.triu(R), g[:k])
        except np.linalg.LinAlgError:
            y = np.linalg.lstsq(np.triu(R), g[:k], rcond=None)[0]
        x = x + np.column_stack(Z[:k]) @ y
