"""Structured hex8 cantilever mesh, SIMP moduli, assembly (oracle, FP64).

Test infrastructure only.

Follows Sec. 3.1: E_e = Emin + (E0 - Emin) rho_e^p (Eq. simp_filter, filter and
projection not applied: the standalone solver studies prescribe E_e directly),
K = sum_e E_e K_e (Eq. state_eq), free-DOF system K_ff u_f = f_f.

Numbering (reading, the paper does not state it): node (i,j,k) has index
i + (nx+1)*(j + (ny+1)*k) (x fastest); DOF = 3*node + c (xyz interleaved, as
P = P_s (x) I_3 in Eq. vector_prolongation implies); element (ex,ey,ez) has
index ex + nx*(ey + ny*ez).  Cantilever: every DOF of the x = 0 face is fixed;
a unit -z load is spread equally over the nodes (nx, j, 0), j = 0..ny.
"""
import numpy as np
import scipy.sparse as sp

from . import hex8


def n_nodes(dims):
    nx, ny, nz = dims
    return (nx + 1) * (ny + 1) * (nz + 1)


def node_id(i, j, k, dims):
    nx, ny, _ = dims
    return i + (nx + 1) * (j + (ny + 1) * k)


def element_nodes(dims):
    """(n_el, 8) global node index of local node a = dx + 2dy + 4dz of each element."""
    nx, ny, nz = dims
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    out = np.empty((ex.size, 8), dtype=np.int64)
    for a, (dx, dy, dz) in enumerate(hex8.NODE_OFFSETS):
        out[:, a] = node_id(ex + dx, ey + dy, ez + dz, dims)
    return out


def element_dofs(dims):
    en = element_nodes(dims)
    return (3 * en[:, :, None] + np.arange(3)[None, None, :]).reshape(en.shape[0], 24)


def cantilever_fixed(dims):
    """Boolean mask over all DOFs: True where the DOF is clamped (node on x = 0)."""
    nx, ny, nz = dims
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    fixed_node = (i.ravel() == 0)
    return np.repeat(fixed_node, 3)


def edge_load(dims):
    """Unit total -z force spread equally over nodes (nx, j, 0), j = 0..ny."""
    nx, ny, nz = dims
    f = np.zeros(3 * n_nodes(dims))
    for j in range(ny + 1):
        f[3 * node_id(nx, j, 0, dims) + 2] = -1.0 / (ny + 1)
    return f


def simp_modulus(rho, p, E0=1.0, Emin=1e-9):
    """Eq. simp_filter with the physical density given directly."""
    rho = np.asarray(rho, dtype=np.float64)
    return Emin + (E0 - Emin) * rho ** p


def assemble(dims, E, nu=0.3, fixed=None):
    """Global K = sum_e E_e K_e as CSR (FP64).

    With ``fixed`` given, rows and columns of fixed DOFs are zeroed, i.e. the
    returned matrix is M K M with M the free-DOF selector (fixed DOFs carry
    zero rows: the full-length vector form of K_ff).
    """
    Ke = hex8.ke(nu)
    dofs = element_dofs(dims)
    n = 3 * n_nodes(dims)
    rows = np.repeat(dofs, 24, axis=1).ravel()
    cols = np.tile(dofs, (1, 24)).ravel()
    vals = (np.asarray(E, dtype=np.float64)[:, None] * Ke.ravel()[None, :]).ravel()
    K = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    K.sum_duplicates()
    if fixed is not None:
        m = sp.diags((~np.asarray(fixed, dtype=bool)).astype(np.float64))
        K = (m @ K @ m).tocsr()
        K.eliminate_zeros()
    return K


def apply_K_elementwise(dims, E, u, nu=0.3, fixed=None):
    """y = M (sum_e E_e K_e) M u by an explicit element loop (gather, 24x24 product, scatter)."""
    Ke = hex8.ke(nu)
    dofs = element_dofs(dims)
    u = np.array(u, dtype=np.float64)
    if fixed is not None:
        u[np.asarray(fixed, dtype=bool)] = 0.0
    ue = u[dofs]                                   # (n_el, 24)
    fe = (ue @ Ke.T) * np.asarray(E, dtype=np.float64)[:, None]
    y = np.zeros_like(u)
    np.add.at(y, dofs.ravel(), fe.ravel())
    if fixed is not None:
        y[np.asarray(fixed, dtype=bool)] = 0.0
    return y


def rigid_body_modes(dims):
    """(3*Nn, 6) translations and infinitesimal rotations evaluated at the nodes."""
    nx, ny, nz = dims
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    x, y, z = i.ravel().astype(float), j.ravel().astype(float), k.ravel().astype(float)
    Nn = x.size
    R = np.zeros((3 * Nn, 6))
    for c in range(3):
        R[c::3, c] = 1.0
    # rotation about x: (0, -z, y); about y: (z, 0, -x); about z: (-y, x, 0)
    R[1::3, 3], R[2::3, 3] = -z, y
    R[0::3, 4], R[2::3, 4] = z, -x
    R[0::3, 5], R[1::3, 5] = -y, x
    return R
