"""Pins of numbering, boundary conditions and assembly (Sec. 3.1, Table e7)."""
import json
import os

import numpy as np
import scipy.sparse.linalg as spla

import workloads
from oracle import mesh, transfer

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")))


def test_free_dof_counts_table_e7():
    for row in GOLD["free_dofs"]:
        dims = tuple(row["dims"])
        assert np.prod(dims) == row["n_elem"]
        assert int((~mesh.cantilever_fixed(dims)).sum()) == row["n_free"]


def test_level_sizes_216k():
    g = GOLD["level_sizes_216k"]
    dims = tuple(g["dims"])
    counts = transfer.free_counts(dims, mesh.cantilever_fixed(dims), 4)
    assert abs(counts[1] - g["level1_about"]) <= g["level1_rel_tol"] * g["level1_about"]
    assert abs(counts[3] - g["level3_about"]) <= g["level3_rel_tol"] * g["level3_about"]


def test_workload_inputs_match_oracle_reading():
    for dims in [(16, 8, 8), (5, 3, 4)]:
        assert np.array_equal(workloads.cantilever_fixed(dims).astype(bool), mesh.cantilever_fixed(dims))
        assert np.array_equal(workloads.edge_load(dims), mesh.edge_load(dims))
        assert abs(mesh.edge_load(dims).sum() + 1.0) < 1e-15


def test_assembly_symmetric_and_rigid_body_kernel():
    dims = (4, 3, 2)
    E = np.random.default_rng(0).uniform(0.1, 1.0, np.prod(dims))
    K = mesh.assemble(dims, E)
    assert abs(K - K.T).max() < 1e-15
    R = mesh.rigid_body_modes(dims)
    assert np.abs(K @ R).max() < 1e-13 * abs(K).max()


def test_patch_test_uniform_strain():
    """Uniform modulus + linear field: all interior nodal forces vanish."""
    dims = (4, 4, 3)
    K = mesh.assemble(dims, np.ones(np.prod(dims)))
    nx, ny, nz = dims
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    X = np.stack([i.ravel(), j.ravel(), k.ravel()], 1).astype(float)
    G = np.array([[0.3, -1.0, 0.2], [0.5, 0.1, -0.7], [0.0, 0.4, 1.1]])
    u = (X @ G.T).ravel()
    y = (K @ u).reshape(-1, 3)
    interior = (i.ravel() > 0) & (i.ravel() < nx) & (j.ravel() > 0) & (j.ravel() < ny) \
        & (k.ravel() > 0) & (k.ravel() < nz)
    assert np.abs(y[interior]).max() < 1e-13


def test_elementwise_apply_equals_assembled():
    dims = (5, 3, 4)
    rng = np.random.default_rng(1)
    E = rng.uniform(1e-3, 1.0, np.prod(dims))
    fixed = mesh.cantilever_fixed(dims)
    u = rng.standard_normal(fixed.size)
    u[fixed] = 0
    K = mesh.assemble(dims, E, fixed=fixed)
    assert np.abs(K @ u - mesh.apply_K_elementwise(dims, E, u, fixed=fixed)).max() < 1e-13


def test_free_system_spd():
    dims = (4, 2, 2)
    fixed = mesh.cantilever_fixed(dims)
    K = mesh.assemble(dims, mesh.simp_modulus(np.full(16, 0.5), 3), fixed=fixed)
    free = ~fixed
    np.linalg.cholesky(K[free][:, free].toarray())


def test_simp_map():
    assert mesh.simp_modulus(np.array([0.0]), 3)[0] == 1e-9
    assert mesh.simp_modulus(np.array([1.0]), 3)[0] == 1.0
    assert abs(mesh.simp_modulus(np.array([0.5]), 3)[0] - (1e-9 + 0.125 * (1 - 1e-9))) < 1e-17
