"""Pins of the Galerkin hierarchy (Sec. 3.3, Eq. galerkin_level1, Sec. 3.8)."""
import numpy as np

from oracle import galerkin, mesh, transfer


def _setup(dims, E, fixed):
    K = mesh.assemble(dims, E, fixed=fixed)
    fc = transfer.inject_fixed(fixed, dims)
    return K, fc


def test_local_aggregation_equals_explicit_product():
    rng = np.random.default_rng(5)
    for dims in [(4, 4, 2), (6, 4, 4), (5, 3, 7)]:           # even and odd axes
        E = rng.uniform(1e-3, 1.0, np.prod(dims))
        fixed = mesh.cantilever_fixed(dims)
        K, fc = _setup(dims, E, fixed)
        Kx = galerkin.galerkin_explicit(K, dims, fixed, fc)
        Kl = galerkin.galerkin_level1_local(dims, E, fixed, fc)
        assert abs(Kx - Kl).max() <= 1e-14 * abs(Kx).max()


def test_local_aggregation_general_mask():
    """A mask that is not injection-consistent (odd high face clamped) still matches."""
    dims = (5, 4, 3)
    rng = np.random.default_rng(6)
    E = rng.uniform(0.1, 1.0, np.prod(dims))
    nx = dims[0]
    i = np.arange(mesh.n_nodes(dims)) % (nx + 1)
    fixed = np.repeat((i == 0) | (i == nx), 3)
    K, fc = _setup(dims, E, fixed)
    Kx = galerkin.galerkin_explicit(K, dims, fixed, fc)
    Kl = galerkin.galerkin_level1_local(dims, E, fixed, fc)
    assert abs(Kx - Kl).max() <= 1e-14 * abs(Kx).max()


def test_nested_spaces_uniform_modulus_closed_form():
    """Trilinear P embeds the coarse FE space: with E constant on coarse elements,
    P^T K_h P equals the coarse-mesh assembly with element size 2 (K_e scales
    linearly with h in 3D), and two coarsenings give size 4."""
    dims = (8, 4, 4)
    fixed = mesh.cantilever_fixed(dims)
    E = np.full(np.prod(dims), 0.37)
    K, fc = _setup(dims, E, fixed)
    K1 = galerkin.galerkin_level1_local(dims, E, fixed, fc)
    cd = transfer.coarse_dims(dims)
    ref1 = mesh.assemble(cd, np.full(np.prod(cd), 2 * 0.37), fixed=fc)
    assert abs(K1 - ref1).max() <= 1e-14 * abs(ref1).max()
    fc2 = transfer.inject_fixed(fc, cd)
    K2 = galerkin.galerkin_explicit(K1, cd, fc, fc2)
    cd2 = transfer.coarse_dims(cd)
    ref2 = mesh.assemble(cd2, np.full(np.prod(cd2), 4 * 0.37), fixed=fc2)
    assert abs(K2 - ref2).max() <= 1e-14 * abs(ref2).max()


def test_piecewise_coarse_modulus_closed_form():
    """E constant on each coarse element (random per coarse element)."""
    dims = (6, 4, 4)
    cd = transfer.coarse_dims(dims)
    rng = np.random.default_rng(2)
    Ec = rng.uniform(0.01, 1.0, np.prod(cd))
    nx, ny, nz = dims
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    E = Ec[(ex // 2 + cd[0] * (ey // 2 + cd[1] * (ez // 2))).ravel()]
    fixed = mesh.cantilever_fixed(dims)
    K, fc = _setup(dims, E, fixed)
    K1 = galerkin.galerkin_level1_local(dims, E, fixed, fc)
    ref = mesh.assemble(cd, 2 * Ec, fixed=fc)
    assert abs(K1 - ref).max() <= 1e-14 * abs(ref).max()


def test_stencil_structure_symmetry_spd():
    dims = (6, 6, 4)
    rng = np.random.default_rng(7)
    E = rng.uniform(1e-3, 1.0, np.prod(dims))
    fixed = mesh.cantilever_fixed(dims)
    K, fc = _setup(dims, E, fixed)
    K1 = galerkin.galerkin_level1_local(dims, E, fixed, fc)
    S = galerkin.stencil_blocks(K1, transfer.coarse_dims(dims))   # raises if not 27-point
    assert S.shape[1] == 27
    assert abs(K1 - K1.T).max() <= 1e-15 * abs(K1).max()
    free = ~fc
    np.linalg.cholesky(K1[free][:, free].toarray())
