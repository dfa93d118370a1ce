"""Galerkin coarse operators (oracle, FP64).

Test infrastructure only.

Follows Sec. 3.3: level 1 by element-local aggregation,
K^1 = sum_e E_e (P_e)^T K_e P_e (Eq. galerkin_level1), and deeper levels by
sparse triple products K^{l+1} = R^l K^l P^l.  Both act on the free-DOF
subspace: with M the free selector of a level,
K^{l+1} = M_{l+1} P^T (M_l K^l M_l) P M_{l+1}.
"""
import numpy as np
import scipy.sparse as sp

from . import hex8
from .mesh import element_dofs, node_id, n_nodes
from .transfer import coarse_dims, prolongation

# 1D local pattern of a fine element inside its coarse element, indexed by
# (fine element index - 2 * coarse element index) in {0, 1, 2}; rows: fine
# local node dx in {0,1}; columns: coarse local node in {0,1}.  Pattern 2 only
# occurs for the last fine element of an odd axis (trailing node reading).
PATTERNS_1D = {
    0: np.array([[1.0, 0.0], [0.5, 0.5]]),
    1: np.array([[0.5, 0.5], [0.0, 1.0]]),
    2: np.array([[0.0, 1.0], [0.0, 1.0]]),
}


def galerkin_explicit(K, dims, fixed_fine, fixed_coarse):
    """M_c P^T (M_f K M_f) P M_c by explicit sparse products."""
    P = prolongation(dims)
    mf = sp.diags((~np.asarray(fixed_fine, dtype=bool)).astype(float))
    mc = sp.diags((~np.asarray(fixed_coarse, dtype=bool)).astype(float))
    Kc = (mc @ P.T @ (mf @ K @ mf) @ P @ mc).tocsr()
    Kc.sum_duplicates()
    Kc.eliminate_zeros()
    return Kc


def local_prolongation(pattern):
    """24x24 P_e for a pattern triple: rows fine local DOFs, cols coarse local DOFs."""
    Pe = np.zeros((24, 24))
    for a, (dx, dy, dz) in enumerate(hex8.NODE_OFFSETS):
        for b, (cx, cy, cz) in enumerate(hex8.NODE_OFFSETS):
            w = (PATTERNS_1D[pattern[0]][dx, cx] * PATTERNS_1D[pattern[1]][dy, cy]
                 * PATTERNS_1D[pattern[2]][dz, cz])
            for c in range(3):
                Pe[3 * a + c, 3 * b + c] = w
    return Pe


def galerkin_level1_local(dims, E, fixed_fine, fixed_coarse, nu=0.3):
    """K^1 = M_c sum_e E_e P_e^T (M_e K_e M_e) P_e M_c, scattered into coarse DOFs."""
    nx, ny, nz = dims
    cdims = coarse_dims(dims)
    cx, cy, cz = cdims
    Ke = hex8.ke(nu)
    fixed_fine = np.asarray(fixed_fine, dtype=bool)
    E = np.asarray(E, dtype=np.float64)
    fdofs = element_dofs(dims)                       # (n_el, 24)
    cdofs_all = element_dofs(cdims)                  # (n_cel, 24)
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    cex = np.minimum(ex // 2, cx - 1)
    cey = np.minimum(ey // 2, cy - 1)
    cez = np.minimum(ez // 2, cz - 1)
    pat = np.stack([ex - 2 * cex, ey - 2 * cey, ez - 2 * cez], axis=1)
    ce = cex + cx * (cey + cy * cez)
    cdofs = cdofs_all[ce]                            # coarse DOFs of the parent
    elem_masked = fixed_fine[fdofs].any(axis=1)
    rows, cols, vals = [], [], []
    patterns = {tuple(p) for p in pat.tolist()}
    for p in sorted(patterns):
        Pe = local_prolongation(p)
        G = Pe.T @ Ke @ Pe
        sel = np.where((pat == p).all(axis=1) & ~elem_masked)[0]
        if sel.size:
            rows.append(np.repeat(cdofs[sel], 24, axis=1).ravel())
            cols.append(np.tile(cdofs[sel], (1, 24)).ravel())
            vals.append((E[sel, None] * G.ravel()[None, :]).ravel())
        for e in np.where((pat == p).all(axis=1) & elem_masked)[0]:
            m = (~fixed_fine[fdofs[e]]).astype(float)
            Gm = Pe.T @ (m[:, None] * Ke * m[None, :]) @ Pe
            rows.append(np.repeat(cdofs[e], 24))
            cols.append(np.tile(cdofs[e], 24))
            vals.append(E[e] * Gm.ravel())
    n = 3 * n_nodes(cdims)
    K1 = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(n, n)).tocsr()
    K1.sum_duplicates()
    mc = sp.diags((~np.asarray(fixed_coarse, dtype=bool)).astype(float))
    K1 = (mc @ K1 @ mc).tocsr()
    K1.eliminate_zeros()
    return K1


def stencil_blocks(K, dims):
    """Dense view of a 27-point block operator: S[n, o, 3, 3], o = (ox+1)+3(oy+1)+9(oz+1).

    Used by tests to check that a Galerkin level has the structured 27-point
    block pattern; entries outside the stencil raise.
    """
    nx, ny, nz = dims
    Nn = n_nodes(dims)
    S = np.zeros((Nn, 27, 3, 3))
    Kc = K.tocoo()
    rn, cn = Kc.row // 3, Kc.col // 3
    ri = np.stack(np.unravel_index(rn, (nz + 1, ny + 1, nx + 1)), axis=1)[:, ::-1]
    ci = np.stack(np.unravel_index(cn, (nz + 1, ny + 1, nx + 1)), axis=1)[:, ::-1]
    off = ci - ri
    if np.abs(off).max(initial=0) > 1:
        raise ValueError("operator is not a 27-point block stencil")
    o = (off[:, 0] + 1) + 3 * (off[:, 1] + 1) + 9 * (off[:, 2] + 1)
    np.add.at(S, (rn, o, Kc.row % 3, Kc.col % 3), Kc.data)
    return S
