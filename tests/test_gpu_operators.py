"""GPU parity of the operators against the oracle (through the C-ABI).

Sizes span several 256-node tiles with ragged tails; one odd-dimension mesh
exercises the trailing-node coarsening.  Tolerances: FP64 1e-13 and FP32 2e-6
relative to |K||u| entry-wise magnitudes (FP32 unit roundoff 6e-8 times
<= 216 accumulated terms).
"""
import numpy as np
import pytest

import workloads
from oracle import galerkin, mesh, multigrid, smoothers
from tests.gpu_util import np64, rel_err, t32, t64

pytestmark = pytest.mark.gpu

CASES = [((16, 8, 8), 3, 0), ((24, 12, 12), 4, 1), ((9, 7, 5), 3, 2)]


def _inputs(dims, seed):
    g = np.random.default_rng(seed)
    rho = g.uniform(0.05, 1.0, np.prod(dims))
    fixed = workloads.cantilever_fixed(dims).astype(bool)
    return rho, fixed


def _gpu_h(dims, L, rho, **kw):
    from paper_2604_26441_amd import simpgmg
    o = simpgmg.default_options(*dims, n_levels=L, **kw)
    return simpgmg.setup_hierarchy(o, t64(rho))


@pytest.mark.parametrize("dims,L,seed", CASES)
def test_fine_apply_f64_f32(dims, L, seed):
    from paper_2604_26441_amd import simpgmg
    rho, fixed = _inputs(dims, seed)
    E = mesh.simp_modulus(rho, 3)
    K = mesh.assemble(dims, E, fixed=fixed)
    h = _gpu_h(dims, L, rho)
    u = workloads.random_vector(fixed.size, seed + 10, fixed)
    ref = K @ u
    scale = abs(K) @ np.abs(u)
    y = t64(np.zeros_like(u))
    simpgmg.apply_K(h, 0, "f64", t64(u), y)
    assert rel_err(np64(y), ref, scale) < 1e-13
    y32 = t32(np.zeros_like(u))
    simpgmg.apply_K(h, 0, "f32", t32(u), y32)
    ref32 = K @ u.astype(np.float32).astype(np.float64)
    assert rel_err(np64(y32), ref32, scale) < 2e-6
    assert np.all(np64(y)[fixed] == 0) and np.all(np64(y32)[fixed] == 0)


@pytest.mark.parametrize("dims,L,seed", CASES)
def test_galerkin_levels_and_diagonals(dims, L, seed):
    rho, fixed = _inputs(dims, seed)
    E = mesh.simp_modulus(rho, 3)
    oh = multigrid.build(dims, E, fixed, multigrid.Options(n_levels=L, lambdas=[1.0] * (L - 1)))
    h = _gpu_h(dims, L, rho)
    assert h.num_levels() == L
    for l in range(L):
        info = h.level_info(l)
        assert info["dims"] == oh.levels[l].dims
        assert info["n_free"] == int((~oh.levels[l].fixed).sum())
        d = h.diagonal(l)
        assert np.abs(d - oh.levels[l].d).max() <= 1e-13 * np.abs(oh.levels[l].d).max()
    for l in range(1, L):
        S = h.stencil(l)                                       # [27,3,3,nn]
        ref = galerkin.stencil_blocks(oh.levels[l].K, oh.levels[l].dims)   # [nn,27,3,3]
        ref = np.transpose(ref, (1, 2, 3, 0))
        assert np.abs(S - ref).max() <= 1e-13 * np.abs(ref).max(), l


@pytest.mark.parametrize("form", [0, 1, 2, 3])
@pytest.mark.parametrize("dims,L,seed", CASES)
def test_stencil_apply(dims, L, seed, form):
    """form 1: LDS-staged 27-offset kernel, 2: plane-split kernel, 0: chosen
    by level size (the plane-split kernel at these sizes), 3: level 1 from
    the child moduli of its elements (rows next to Dirichlet DOFs and odd-axis
    ends from the stencil), the other levels as 0."""
    from paper_2604_26441_amd import simpgmg
    rho, fixed = _inputs(dims, seed)
    E = mesh.simp_modulus(rho, 3)
    oh = multigrid.build(dims, E, fixed, multigrid.Options(n_levels=L, lambdas=[1.0] * (L - 1)))
    h = _gpu_h(dims, L, rho, stencil_form=form)
    for l in range(1, L):
        K = oh.levels[l].K
        u = workloads.random_vector(K.shape[0], seed + l, oh.levels[l].fixed)
        y = t64(np.zeros_like(u))
        simpgmg.apply_K(h, l, "f64", t64(u), y)
        assert rel_err(np64(y), K @ u, abs(K) @ np.abs(u)) < 1e-13


@pytest.mark.parametrize("dims", [(20, 12, 10), (21, 9, 11)])
def test_level1_element_products_with_scattered_dirichlet(dims):
    """Level 1 from the child moduli (stencil_form 3) with Dirichlet DOFs
    inside the mesh, single components included, and (second mesh) odd
    axes: every row against the oracle's Galerkin operator, and the same
    level applied from the stored stencil."""
    import torch
    from paper_2604_26441_amd import simpgmg
    rho, _ = _inputs(dims, 17)
    g = np.random.default_rng(18)
    fixed = workloads.cantilever_fixed(dims).astype(bool)
    fixed |= g.uniform(size=fixed.size) < 0.01
    E = mesh.simp_modulus(rho, 3)
    oh = multigrid.build(dims, E, fixed, multigrid.Options(n_levels=3, lambdas=[1.0] * 2))
    fd = torch.as_tensor(fixed.astype(np.uint8), device="cuda:0")
    h3 = simpgmg.setup_hierarchy(simpgmg.default_options(*dims, n_levels=3, stencil_form=3),
                                 t64(rho), fixed_dof=fd)
    h0 = simpgmg.setup_hierarchy(simpgmg.default_options(*dims, n_levels=3), t64(rho), fixed_dof=fd)
    K = oh.levels[1].K
    u = workloads.random_vector(K.shape[0], 19, oh.levels[1].fixed)
    y3, y0 = t64(np.zeros_like(u)), t64(np.zeros_like(u))
    simpgmg.apply_K(h3, 1, "f64", t64(u), y3)
    simpgmg.apply_K(h0, 1, "f64", t64(u), y0)
    scale = abs(K) @ np.abs(u)
    assert rel_err(np64(y3), K @ u, scale) < 1e-13
    assert rel_err(np64(y3), np64(y0), scale) < 1e-13
    assert np.all(np64(y3)[oh.levels[1].fixed] == 0)
    # the default form holds the products too; pinning them (any chunk
    # length) gives the same bits as the form that asks for them
    for planes in (1, 4):
        simpgmg.set_launch_shape(h0, "level1", 1, planes)
        y1 = t64(np.zeros_like(u))
        simpgmg.apply_K(h0, 1, "f64", t64(u), y1)
        assert np.array_equal(np64(y1), np64(y3)), planes
    simpgmg.set_launch_shape(h0, "level1", 0, 0)
    y1 = t64(np.zeros_like(u))
    simpgmg.apply_K(h0, 1, "f64", t64(u), y1)
    assert np.array_equal(np64(y1), np64(y0))
    with pytest.raises(simpgmg.SimpGmgError):
        simpgmg.set_launch_shape(h0, "level1", 1, 0)
    h2 = simpgmg.setup_hierarchy(simpgmg.default_options(*dims, n_levels=3, stencil_form=1),
                                 t64(rho), fixed_dof=fd)
    with pytest.raises(simpgmg.SimpGmgError):     # form 1 keeps no element products
        simpgmg.set_launch_shape(h2, "level1", 1, 2)


@pytest.mark.parametrize("dims,L,seed", CASES)
def test_power_iteration_lambdas(dims, L, seed):
    rho, fixed = _inputs(dims, seed)
    E = mesh.simp_modulus(rho, 3)
    oh = multigrid.build(dims, E, fixed, multigrid.Options(n_levels=L))
    h = _gpu_h(dims, L, rho)
    for l in range(L - 1):
        lam = h.level_info(l)["lambda"]
        assert abs(lam - oh.levels[l].lam) <= 1e-10 * oh.levels[l].lam, (l, lam, oh.levels[l].lam)


MFMA_CASES = [((16, 8, 8), 0), ((9, 7, 5), 1), ((31, 6, 20), 2), ((24, 12, 12), 3)]


@pytest.mark.parametrize("dims,seed", MFMA_CASES)
def test_fine_apply_mfma_bf16x3_and_bf16(dims, seed):
    """MFMA K.u: BF16X3 is FP32-accurate; BF16 equals the BF16 semantic model
    (input rounded to BF16, exact element matrix, FP32 accumulation); FP64 is
    FP64-accurate."""
    from oracle import bf16
    from paper_2604_26441_amd import simpgmg
    rho, fixed = _inputs(dims, seed)
    E = mesh.simp_modulus(rho, 3)
    K = mesh.assemble(dims, E, fixed=fixed)
    h = _gpu_h(dims, 2, rho)
    u = workloads.random_vector(fixed.size, seed + 20, fixed).astype(np.float32).astype(np.float64)
    scale = abs(K) @ np.abs(u)
    y3 = t32(np.zeros_like(u))
    simpgmg.apply_K(h, 0, "bf16x3", t32(u), y3)
    assert rel_err(np64(y3), K @ u, scale) < 2e-6
    y1 = t32(np.zeros_like(u))
    simpgmg.apply_K(h, 0, "bf16", t32(u), y1)
    ref1 = bf16.apply_K_bf16_model(dims, E, u, fixed)
    assert rel_err(np64(y1), ref1, scale) < 2e-6
    assert rel_err(np64(y1), K @ u, scale) < 2.0 ** -8
    assert np.all(np64(y3)[fixed] == 0) and np.all(np64(y1)[fixed] == 0)
    # BF16X2: two round-to-nearest terms carry the input to about 2^-17 (a
    # dropped term would leave 2^-9)
    y2 = t32(np.zeros_like(u))
    simpgmg.apply_K(h, 0, "bf16x2", t32(u), y2)
    e2 = rel_err(np64(y2), K @ u, scale)
    assert e2 < 2.0 ** -15 and np.all(np64(y2)[fixed] == 0)
    # FP64 operator on the FP64 matrix cores, same tiles (two shapes), and
    # the sum-factorised vector-ALU tiles (two chunk lengths)
    u64 = workloads.random_vector(fixed.size, seed + 30, fixed)
    for shape in ((4, 2), (8, 5), (1, 2), (1, 7)):
        simpgmg.set_launch_shape(h, "f64", *shape)
        y64 = t64(np.zeros_like(u64))
        simpgmg.apply_K(h, 0, "f64", t64(u64), y64)
        assert rel_err(np64(y64), K @ u64, abs(K) @ np.abs(u64)) < 1e-13, shape
        assert np.all(np64(y64)[fixed] == 0)


def test_fine_apply_deterministic():
    """Owner-computes scatter: two applications are bitwise identical."""
    from paper_2604_26441_amd import simpgmg
    dims = (24, 12, 12)
    rho, fixed = _inputs(dims, 9)
    h = _gpu_h(dims, 2, rho)
    u = t32(workloads.random_vector(fixed.size, 9, fixed))
    for prec in ("bf16x3", "bf16", "f32"):
        a, b = t32(np.zeros(fixed.size)), t32(np.zeros(fixed.size))
        simpgmg.apply_K(h, 0, prec, u, a)
        simpgmg.apply_K(h, 0, prec, u, b)
        assert np.array_equal(np64(a), np64(b)), prec


def test_sf64_chunk_length_keeps_results_bitwise():
    """FP64 sum-factorised tiles: the chunk length moves work between waves
    only (every node sums its eight elements in one order), on a mesh with
    ragged tiles in every axis; one chunk length also against the oracle's
    assembled K."""
    from paper_2604_26441_amd import simpgmg
    dims = (31, 7, 20)
    rho, fixed = _inputs(dims, 13)
    h = _gpu_h(dims, 2, rho)
    u = workloads.random_vector(fixed.size, 14, fixed)
    out = []
    for planes in (1, 3, 32):
        simpgmg.set_launch_shape(h, "f64", 1, planes)
        y = t64(np.zeros(fixed.size))
        simpgmg.apply_K(h, 0, "f64", t64(u), y)
        out.append(np64(y))
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])
    K = mesh.assemble(dims, mesh.simp_modulus(rho, 3), fixed=fixed)
    assert rel_err(out[0], K @ u, abs(K) @ np.abs(u)) < 1e-13


def test_bf16_family_chunk_lengths_keep_results_bitwise():
    """BF16 and BF16X3 MFMA tiles: every candidate chunk length of the
    autotuner, odd ones included (3 planes; 6 against a mesh of 20 node
    planes leaves a short last chunk), gives the bits of the default shape:
    a chunk moves work between waves only."""
    from paper_2604_26441_amd import simpgmg
    dims = (31, 6, 19)
    rho, fixed = _inputs(dims, 21)
    h = _gpu_h(dims, 2, rho)
    u = t32(workloads.random_vector(fixed.size, 22, fixed))
    for prec in ("bf16", "bf16x3"):
        ref = None
        for rows in (4, 8):
            for planes in (2, 3, 4, 6, 8, 16, 32):
                simpgmg.set_launch_shape(h, prec, rows, planes)
                y = t32(np.zeros(fixed.size))
                simpgmg.apply_K(h, 0, prec, u, y)
                if ref is None:
                    ref = np64(y)
                assert np.array_equal(np64(y), ref), (prec, rows, planes)


def test_autotune_keeps_results_bitwise():
    """The tuned launch shape moves work between workgroups only."""
    from paper_2604_26441_amd import simpgmg
    dims = (31, 6, 20)
    rho, fixed = _inputs(dims, 11)
    h = _gpu_h(dims, 2, rho)
    u = t32(workloads.random_vector(fixed.size, 12, fixed))
    before = {}
    u64 = t64(np64(u))
    simpgmg.set_launch_shape(h, "f64", 4, 3)
    for prec in ("bf16", "bf16x3", "f64"):
        y = t64(np.zeros(fixed.size)) if prec == "f64" else t32(np.zeros(fixed.size))
        simpgmg.apply_K(h, 0, prec, u64 if prec == "f64" else u, y)
        before[prec] = np64(y)
    z = simpgmg.autotune(h)
    zc = (2, 3, 4, 6, 8, 16, 32)
    assert all(r in (4, 8) and p in zc for r, p in z[:2])
    assert z[2] == (0, 0) or (z[2][0] in (1, 4, 8) and z[2][1] in zc)
    if z[2][0] in (0, 1):                   # the tuner chose a vector-ALU kernel:
        simpgmg.set_launch_shape(h, "f64", 8, 16)   # compare another MFMA shape
    for prec in ("bf16", "bf16x3", "f64"):
        y = t64(np.zeros(fixed.size)) if prec == "f64" else t32(np.zeros(fixed.size))
        simpgmg.apply_K(h, 0, prec, u64 if prec == "f64" else u, y)
        assert np.array_equal(np64(y), before[prec]), prec
