"""Trilinear prolongation, injection of Dirichlet masks, level sizes (oracle).

Test infrastructure only.

Follows Sec. 3.3 (Eq. trilinear_weights, Eq. vector_prolongation): 2:1
coarsening per axis, 1D weights in {1, 1/2, 0}; P = P_s (x) I_3, R = P^T.
A coarse DOF is free iff the fine DOF at node (2i,2j,2k) is free.

Readings (the paper only says "2:1 in each direction"):
  * n_coarse = floor(n_fine / 2) elements per axis (the level sizes quoted in
    Sec. 3.3 and Sec. 4.1 for the 216k mesh require the floor);
  * when n_fine is odd, the trailing fine node 2*n_c + 1 takes weight 1 from
    the last coarse node n_c (keeps the partition of unity).
"""
import numpy as np
import scipy.sparse as sp

from .mesh import n_nodes


def coarse_dims(dims):
    return tuple(n // 2 for n in dims)


def weights_1d(nf):
    """(nf+1, nc+1) matrix W with W[i_f, i_c] = 1D interpolation weight."""
    nc = nf // 2
    W = np.zeros((nf + 1, nc + 1))
    for i in range(nf + 1):
        if i % 2 == 0:
            W[i, i // 2] = 1.0
        elif i < 2 * nc:
            W[i, (i - 1) // 2] = 0.5
            W[i, (i + 1) // 2] = 0.5
        else:                       # trailing node of an odd fine axis
            W[i, nc] = 1.0
    return W


def scalar_prolongation(dims):
    """P_s: (Nn_fine, Nn_coarse), node order x fastest."""
    nx, ny, nz = dims
    Px, Py, Pz = (sp.csr_matrix(weights_1d(n)) for n in (nx, ny, nz))
    return sp.kron(Pz, sp.kron(Py, Px)).tocsr()


def prolongation(dims):
    """Vector P = P_s (x) I_3 on interleaved DOFs."""
    return sp.kron(scalar_prolongation(dims), sp.identity(3)).tocsr()


def inject_fixed(fixed_fine, dims):
    """Coarse fixed mask by injection from fine node (2i, 2j, 2k)."""
    nx, ny, nz = dims
    cx, cy, cz = coarse_dims(dims)
    ff = np.asarray(fixed_fine, dtype=bool).reshape(nz + 1, ny + 1, nx + 1, 3)
    return ff[0:2 * cz + 1:2, 0:2 * cy + 1:2, 0:2 * cx + 1:2, :].reshape(-1).copy()


def level_dims(dims, n_levels):
    out = [tuple(dims)]
    for _ in range(n_levels - 1):
        out.append(coarse_dims(out[-1]))
    return out


def free_counts(dims, fixed, n_levels):
    """Free-DOF count per level for a given fine mask."""
    counts = []
    d, f = tuple(dims), np.asarray(fixed, dtype=bool)
    for lvl in range(n_levels):
        counts.append(int((~f).sum()))
        if lvl + 1 < n_levels:
            f = inject_fixed(f, d)
            d = coarse_dims(d)
    return counts
