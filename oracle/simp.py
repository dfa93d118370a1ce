"""SIMP outer-loop pieces (oracle, FP64): density filter, Heaviside
projection, compliance sensitivities, the optimality-criteria (OC) update
with volume bisection, and a plain driver.

Test infrastructure only.

The paper (Sec. 3.1, Eq. simp_filter) fixes the chain of densities: design
rho, filtered rho~ = F rho, physical rhohat = H_{beta,eta}(rho~), modulus
E_e = Emin + (E0 - Emin) rhohat_e^p, one frozen field per linear solve, the
filter applied once per SIMP update; and (Sec. 3.5) a spectral-radius
estimate refreshed only when max_e E_e moves by more than 10 %.  The filter,
projection and OC parameters are in a companion paper that is not available,
so the standard textbook forms are the readings here:

  * F: linear density filter with cone weights w(e, i) = max(0, rmin - d(e, i))
    over element centres inside the mesh, normalised per output element:
    rho~_e = sum_i w(e, i) rho_i / W_e with W_e = sum_i w(e, i)
    (Bruns and Tortorelli 2001; Bourdin 2001).  Its adjoint is
    (F^T g)_i = sum_e w(e, i) g_e / W_e.
  * H_{beta,eta}(x) = (tanh(beta eta) + tanh(beta (x - eta)))
                      / (tanh(beta eta) + tanh(beta (1 - eta)))
    (Wang, Lazarov and Sigmund 2011); beta = 0 means no projection.
  * Compliance c = f . u = sum_e E_e u_e^T K_e u_e and its derivative
    dc/drhohat_e = -p (E0 - Emin) rhohat_e^(p-1) u_e^T K_e u_e (the adjoint of
    the self-adjoint compliance problem); volume V = sum_e rhohat_e.  Both are
    carried back to rho through H' and F^T.
  * OC update (Bendsoe and Sigmund, Topology Optimization, Sec. 1.2):
    rho_new = clamp(rho sqrt(max(-dc, 0) / (lam dv)), max(0, rho - move),
    min(1, rho + move)), with lam found by bisection on [0, 1e9] so that the
    physical volume of rho_new equals volfrac * n_el; the bisection stops when
    (l2 - l1) / (l1 + l2) <= tol (1e-9 here, tighter than the usual 1e-3, so
    that the volume constraint holds to rounding) or after 200 halvings.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import hex8, mesh


def filter_matrix(dims, rmin):
    """Sparse W (n_el x n_el) of cone weights over element centres, and the
    row sums.  Element index ex + nx (ey + ny ez)."""
    nx, ny, nz = dims
    r = int(np.ceil(rmin)) - 1
    rows, cols, vals = [], [], []
    for ez in range(nz):
        for ey in range(ny):
            for ex in range(nx):
                e = ex + nx * (ey + ny * ez)
                for dz in range(-r, r + 1):
                    for dy in range(-r, r + 1):
                        for dx in range(-r, r + 1):
                            jx, jy, jz = ex + dx, ey + dy, ez + dz
                            if not (0 <= jx < nx and 0 <= jy < ny and 0 <= jz < nz):
                                continue
                            w = rmin - np.sqrt(dx * dx + dy * dy + dz * dz)
                            if w > 0:
                                rows.append(e)
                                cols.append(jx + nx * (jy + ny * jz))
                                vals.append(w)
    n = nx * ny * nz
    W = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    return W, np.asarray(W.sum(axis=1)).ravel()


def density_filter(dims, rmin, rho):
    W, ws = filter_matrix(dims, rmin)
    return (W @ rho) / ws


def density_filter_adjoint(dims, rmin, g):
    W, ws = filter_matrix(dims, rmin)
    return W.T @ (g / ws)


def heaviside(x, beta, eta):
    """(H(x), H'(x)); beta = 0: identity."""
    x = np.asarray(x, dtype=np.float64)
    if beta == 0:
        return x.copy(), np.ones_like(x)
    den = np.tanh(beta * eta) + np.tanh(beta * (1.0 - eta))
    t = np.tanh(beta * (x - eta))
    return (np.tanh(beta * eta) + t) / den, beta * (1.0 - t * t) / den


def physical(dims, rho, rmin, beta, eta):
    """(rhohat, H'(rho~)) from the design field (rmin <= 1: no filter)."""
    rt = density_filter(dims, rmin, rho) if rmin > 1.0 else np.array(rho, dtype=np.float64)
    return heaviside(rt, beta, eta)


def element_energy(dims, u, nu=0.3):
    """u_e^T K_e u_e per element (unit modulus)."""
    Ke = hex8.ke(nu)
    ue = np.asarray(u, dtype=np.float64)[mesh.element_dofs(dims)]
    return np.einsum("ei,ij,ej->e", ue, Ke, ue)


def compliance_sensitivity(dims, rhohat, u, p, E0=1.0, Emin=1e-9, nu=0.3):
    """(c, dc/drhohat) with c = sum_e E_e u_e^T K_e u_e."""
    ce = element_energy(dims, u, nu)
    E = mesh.simp_modulus(rhohat, p, E0, Emin)
    dc = -p * (E0 - Emin) * np.asarray(rhohat) ** (p - 1) * ce
    return float(E @ ce), dc


def oc_update(dims, rho, dc, dv, volfrac, move, rmin, beta, eta, tol=1e-9, max_halvings=200):
    """One OC step on the design field.  dc, dv are derivatives with respect
    to rho (already carried through H' and F^T).  Returns (rho_new, lam)."""
    rho = np.asarray(rho, dtype=np.float64)
    target = volfrac * rho.size
    lo_b = np.maximum(0.0, rho - move)
    hi_b = np.minimum(1.0, rho + move)
    ratio = np.maximum(-dc, 0.0) / np.maximum(dv, 1e-300)
    l1, l2 = 0.0, 1e9
    new = rho
    for _ in range(max_halvings):
        lmid = 0.5 * (l1 + l2)
        new = np.clip(rho * np.sqrt(ratio / lmid), lo_b, hi_b)
        vol = float(physical(dims, new, rmin, beta, eta)[0].sum())
        if vol > target:
            l1 = lmid
        else:
            l2 = lmid
        if (l2 - l1) <= tol * (l1 + l2):
            break
    return new, lmid


def state_solve(dims, rhohat, fixed, f, p, nu=0.3, E0=1.0, Emin=1e-9):
    """Exact u of K(E(rhohat)) u = f on the free DOFs."""
    E = mesh.simp_modulus(rhohat, p, E0, Emin)
    K = mesh.assemble(dims, E, nu, fixed=fixed)
    fr = ~np.asarray(fixed, dtype=bool)
    u = np.zeros_like(f)
    u[fr] = spla.spsolve(K[fr][:, fr].tocsc(), f[fr])
    return u


def design_sensitivity(dims, rhohat, dH, u, p, rmin, E0=1.0, Emin=1e-9, nu=0.3):
    """(c, dc/drho, dV/drho): the compliance and volume derivatives carried
    from rhohat through H' and the filter adjoint."""
    c, dc_hat = compliance_sensitivity(dims, rhohat, u, p, E0, Emin, nu)
    g = dH * dc_hat
    gv = dH.copy()
    if rmin > 1.0:
        g = density_filter_adjoint(dims, rmin, g)
        gv = density_filter_adjoint(dims, rmin, gv)
    return c, g, gv


def simp_step(dims, rho, fixed, f, p, volfrac, move, rmin, beta, eta, nu=0.3, E0=1.0,
              Emin=1e-9):
    """One SIMP iteration with an exact state solve: physical density,
    K(E) u = f on the free DOFs, compliance and sensitivities, OC update.
    Returns (rho_new, compliance, rhohat, u)."""
    rhohat, dH = physical(dims, rho, rmin, beta, eta)
    u = state_solve(dims, rhohat, fixed, f, p, nu, E0, Emin)
    c, g, gv = design_sensitivity(dims, rhohat, dH, u, p, rmin, E0, Emin, nu)
    rho_new, _ = oc_update(dims, rho, g, gv, volfrac, move, rmin, beta, eta)
    return rho_new, c, rhohat, u
