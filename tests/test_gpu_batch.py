"""GPU parity of the persistent batched solve (BASELINE extension 2).

Each item of one persistent launch must reproduce the single-system solve of
the same hierarchy with FP32 vector-ALU smoothing (same operators, same
algorithm; only dot-product summation order differs): equal status, equal
iteration count (+-1), FP64 true residual below rtol, solutions within the
solver tolerance.  The oracle's own solve fixes the expected compliance.
"""
import numpy as np
import pytest

import workloads
from oracle import krylov, mesh, multigrid
from tests.gpu_util import np64, t64

pytestmark = pytest.mark.gpu


def _systems():
    dims = [(16, 8, 8), (20, 10, 10), (12, 6, 6), (24, 12, 12)]
    rhos = [workloads.grf_rho(d, seed=100 + i) for i, d in enumerate(dims)]
    return dims, rhos


def test_batch_matches_single_solves_and_oracle():
    import torch
    from paper_2604_26441_amd import simpgmg
    dims, rhos = _systems()
    opts = [simpgmg.default_options(*d, n_levels=0, dense_max=1000, fine_prec="f32") for d in dims]
    b = simpgmg.setup_batch(opts, [t64(r) for r in rhos])
    rng = np.random.default_rng(7)
    item_sys, fs = [], []
    for s, d in enumerate(dims):
        for k in range(1 + s % 3):                       # 1..3 load cases per system
            item_sys.append(s)
            fs.append(workloads.random_face_load(d, rng) if k else workloads.edge_load(d))
    us = [t64(np.zeros_like(f)) for f in fs]
    res, ms = simpgmg.pcg_solve_batch(b, item_sys, [t64(f) for f in fs], us, rtol=1e-6, maxit=300)
    assert ms > 0 and b.block_size() in (256, 512)
    for i, (s, f) in enumerate(zip(item_sys, fs)):
        h = b.hierarchy(s)
        u1 = t64(np.zeros_like(f))
        single = simpgmg.pcg_solve(h, t64(f), u1, rtol=1e-6, maxit=300)
        assert res[i]["status"] == "converged" == single["status"], (i, res[i], single)
        assert abs(res[i]["iters"] - single["iters"]) <= 1
        assert res[i]["rel_res_true"] < 1e-6
        xb, xs = np64(us[i]), np64(u1)
        assert np.linalg.norm(xb - xs) <= 1e-5 * np.linalg.norm(xs)
    # oracle, for every item: the FP64 true residual of the returned u with the
    # oracle's assembled operator, and its compliance against the direct solve
    import scipy.sparse.linalg as spla
    for s, d in enumerate(dims):
        fixed = workloads.cantilever_fixed(d).astype(bool)
        K = mesh.assemble(d, mesh.simp_modulus(rhos[s], 3), fixed=fixed)
        fr = ~fixed
        lu = spla.splu(K[fr][:, fr].tocsc())
        for i in [i for i, q in enumerate(item_sys) if q == s]:
            ustar = np.zeros(fixed.size)
            ustar[fr] = lu.solve(fs[i][fr])
            x = np64(us[i])
            assert krylov.true_rel_residual(lambda v: K @ v, fs[i], x) < 1e-6, (s, i)
            assert abs(fs[i] @ x - fs[i] @ ustar) <= 1e-5 * abs(fs[i] @ ustar), (s, i)


def test_batch_graph_replays_agree():
    """The captured launch replayed three times (host work in between) gives
    the same results as the first, eager-tuned, solve."""
    from paper_2604_26441_amd import simpgmg
    dims, rhos = _systems()
    opts = [simpgmg.default_options(*d, n_levels=0, dense_max=1000, fine_prec="f32") for d in dims]
    b = simpgmg.setup_batch(opts, [t64(r) for r in rhos])
    fs = [workloads.edge_load(d) for d in dims]
    first = None
    for rep in range(3):
        us = [t64(np.zeros_like(f)) for f in fs]
        res, _ = simpgmg.pcg_solve_batch(b, list(range(len(dims))), [t64(f) for f in fs], us)
        xs = [np64(u) for u in us]
        if first is None:
            first = (res, xs)
        else:
            assert [r["iters"] for r in res] == [r["iters"] for r in first[0]]
            for a, c in zip(xs, first[1]):
                assert np.array_equal(a, c)


@pytest.mark.parametrize("workers", [1, 3])
def test_concurrent_batch_equals_single_solves(workers):
    """Worker threads with their own streams: every item bitwise equal to a
    lone single solve on the same hierarchy (items of one system in order)."""
    from paper_2604_26441_amd import simpgmg
    dims, rhos = _systems()
    opts = [simpgmg.default_options(*d, n_levels=0, dense_max=1000, fine_prec="f32") for d in dims]
    b = simpgmg.setup_batch(opts, [t64(r) for r in rhos])
    rng = np.random.default_rng(11)
    item_sys, fs = [], []
    for s, d in enumerate(dims):
        for k in range(1 + (s + 1) % 3):
            item_sys.append(s)
            fs.append(workloads.random_face_load(d, rng) if k else workloads.edge_load(d))
    us = [t64(np.zeros_like(f)) for f in fs]
    res, ms = simpgmg.pcg_solve_batch_concurrent(b, item_sys, [t64(f) for f in fs], us,
                                                 rtol=1e-6, maxit=300, workers=workers)
    assert ms > 0
    for i, (s, f) in enumerate(zip(item_sys, fs)):
        h = b.hierarchy(s)
        u1 = t64(np.zeros_like(f))
        r1 = simpgmg.pcg_solve(h, t64(f), u1, rtol=1e-6, maxit=300)
        assert res[i]["status"] == r1["status"] == "converged"
        assert res[i]["iters"] == r1["iters"]
        assert np.array_equal(np64(us[i]), np64(u1))
    with pytest.raises(simpgmg.SimpGmgError):
        simpgmg.pcg_solve_batch_concurrent(b, item_sys, [t64(f) for f in fs], us, workers=0)


def test_batch_config3_every_item_meets_the_oracle():
    """The whole batch workload (32 systems 2m x m x m, m in 8..24, up to the
    48 x 24 x 24 system; random-field rho, p = 3; 1-4 random face loads each):
    one persistent launch, the concurrent and the stage-batched solves (FP32
    fine levels), and the stage-batched solve with BF16X3 fine levels on the
    matrix cores, by host loop and in one graph launch (bitwise equal); every
    item converged with the oracle's FP64 true residual of
    its u below rtol (matrix-free element loop of the oracle)."""
    from paper_2604_26441_amd import simpgmg
    dims, rhos, item_sys, fs = workloads.batch_config()
    assert max(d[0] for d in dims) == 48
    opts = [simpgmg.default_options(*d, n_levels=0, dense_max=1000, fine_prec="f32") for d in dims]
    b = simpgmg.setup_batch(opts, [t64(r) for r in rhos])
    us = [t64(np.zeros_like(f)) for f in fs]
    res, _ = simpgmg.pcg_solve_batch(b, item_sys, [t64(f) for f in fs], us, rtol=1e-6, maxit=300)
    uc = [t64(np.zeros_like(f)) for f in fs]
    resc, _ = simpgmg.pcg_solve_batch_concurrent(b, item_sys, [t64(f) for f in fs], uc,
                                                 rtol=1e-6, maxit=300, workers=4)
    ug = [t64(np.zeros_like(f)) for f in fs]
    resg, _ = simpgmg.pcg_solve_batch(b, item_sys, [t64(f) for f in fs], ug, rtol=1e-6, maxit=300,
                                      staged=True)
    # the FP32 staged solve in one graph launch: bitwise the host-loop one
    ugg = [t64(np.zeros_like(f)) for f in fs]
    resgg, _, nl = simpgmg.pcg_solve_batch_graph(b, item_sys, [t64(f) for f in fs], ugg,
                                                 rtol=1e-6, maxit=300, steps=128)
    assert nl == 1
    _same_results(resg, ug, resgg, ugg)
    b.close()
    # the staged solve again with BF16X3 fine levels (MFMA level 0, tuned shapes)
    opts = [simpgmg.default_options(*d, n_levels=0, dense_max=1000, fine_prec="bf16x3") for d in dims]
    b = simpgmg.setup_batch(opts, [t64(r) for r in rhos])
    um = [t64(np.zeros_like(f)) for f in fs]
    resm, _ = simpgmg.pcg_solve_batch(b, item_sys, [t64(f) for f in fs], um, rtol=1e-6, maxit=300,
                                      staged=True)
    # and in one graph launch (iteration control on the device): bitwise the staged solve
    uq = [t64(np.zeros_like(f)) for f in fs]
    resq, _, nl = simpgmg.pcg_solve_batch_graph(b, item_sys, [t64(f) for f in fs], uq, rtol=1e-6,
                                                maxit=300, steps=128)
    assert nl == 1
    _same_results(resm, um, resq, uq)
    for i, (s, f) in enumerate(zip(item_sys, fs)):
        d = dims[s]
        fixed = workloads.cantilever_fixed(d).astype(bool)
        E = mesh.simp_modulus(rhos[s], 3)
        for r, u in ((res[i], us[i]), (resc[i], uc[i]), (resg[i], ug[i]), (resm[i], um[i]),
                     (resq[i], uq[i])):
            assert r["status"] == "converged", (i, d, r)
            x = np64(u)
            rel = np.linalg.norm(f - mesh.apply_K_elementwise(d, E, x, fixed=fixed)) / np.linalg.norm(f)
            assert rel < 1e-6, (i, d, rel)
            assert abs(rel - r["rel_res_true"]) < 1e-9, (i, d, rel, r)


def test_staged_batch_matches_persistent_batch_and_oracle():
    """The stage-batched solve (one launch per stage over all items, two
    graphs replayed from a host loop): every item converged, iterations within
    one of the persistent launch's (same operators, per-item reductions in
    another order), the oracle's true residual below rtol and equal to the
    one reported, solutions within the solver tolerance of the persistent
    launch's; a second solve with the same item set replays the graphs."""
    from paper_2604_26441_amd import simpgmg
    dims, rhos = _systems()
    opts = [simpgmg.default_options(*d, n_levels=0, dense_max=1000, fine_prec="f32") for d in dims]
    b = simpgmg.setup_batch(opts, [t64(r) for r in rhos])
    rng = np.random.default_rng(9)
    item_sys, fs = [], []
    for s, d in enumerate(dims):
        for k in range(1 + (s + 2) % 3):
            item_sys.append(s)
            fs.append(workloads.random_face_load(d, rng) if k else workloads.edge_load(d))
    up = [t64(np.zeros_like(f)) for f in fs]
    rp, _ = simpgmg.pcg_solve_batch(b, item_sys, [t64(f) for f in fs], up, rtol=1e-6, maxit=300)
    for rep in range(2):
        us = [t64(np.zeros_like(f)) for f in fs]
        rs, ms = simpgmg.pcg_solve_batch(b, item_sys, [t64(f) for f in fs], us, rtol=1e-6,
                                         maxit=300, staged=True)
        assert ms > 0
        for i, (s, f) in enumerate(zip(item_sys, fs)):
            d = dims[s]
            assert rs[i]["status"] == "converged" == rp[i]["status"], (i, rs[i], rp[i])
            assert abs(rs[i]["iters"] - rp[i]["iters"]) <= 1, (i, rs[i], rp[i])
            fixed = workloads.cantilever_fixed(d).astype(bool)
            x = np64(us[i])
            Kx = mesh.apply_K_elementwise(d, mesh.simp_modulus(rhos[s], 3), x, fixed=fixed)
            rel = np.linalg.norm(f - Kx) / np.linalg.norm(f)
            assert rel < 1e-6 and abs(rel - rs[i]["rel_res_true"]) < 1e-9, (i, rel, rs[i])
            xp = np64(up[i])
            assert np.linalg.norm(x - xp) <= 1e-5 * np.linalg.norm(xp), i


def test_staged_batch_mfma_level0_matches_single_solves_and_oracle():
    """With every system's fine level in BF16X3, the staged solve runs level 0
    on the batched MFMA operator (launch shape tuned on the item set, odd and
    ragged meshes (ragged against the 15-element tiles) with 1-3 load cases).  Each item against the single solve of
    its hierarchy, which runs the same BF16X3 operator one mesh at a time:
    same status, iterations within one (per-item reductions in another
    order), solutions within the solver tolerance; and against the oracle:
    true residual below rtol and equal to the one reported.  A second solve
    replays the graphs."""
    from paper_2604_26441_amd import simpgmg
    dims = [(16, 8, 8), (20, 10, 10), (12, 6, 6), (30, 14, 14), (22, 12, 10)]
    rhos = [workloads.grf_rho(d, seed=300 + i) for i, d in enumerate(dims)]
    opts = [simpgmg.default_options(*d, n_levels=0, dense_max=1000, fine_prec="bf16x3") for d in dims]
    b = simpgmg.setup_batch(opts, [t64(r) for r in rhos])
    rng = np.random.default_rng(13)
    item_sys, fs = [], []
    for s, d in enumerate(dims):
        for k in range(1 + s % 3):
            item_sys.append(s)
            fs.append(workloads.random_face_load(d, rng) if k else workloads.edge_load(d))
    singles = []
    for s, f in zip(item_sys, fs):
        u = t64(np.zeros_like(f))
        r = simpgmg.pcg_solve(b.hierarchy(s), t64(f), u, rtol=1e-6, maxit=300)
        singles.append((r, np64(u)))
    for rep in range(2):
        us = [t64(np.zeros_like(f)) for f in fs]
        rs, ms = simpgmg.pcg_solve_batch(b, item_sys, [t64(f) for f in fs], us, rtol=1e-6,
                                         maxit=300, staged=True)
        assert ms > 0
        for i, (s, f) in enumerate(zip(item_sys, fs)):
            d = dims[s]
            r1, x1 = singles[i]
            assert rs[i]["status"] == "converged" == r1["status"], (i, rs[i], r1)
            assert abs(rs[i]["iters"] - r1["iters"]) <= 1, (i, rs[i], r1)
            fixed = workloads.cantilever_fixed(d).astype(bool)
            x = np64(us[i])
            Kx = mesh.apply_K_elementwise(d, mesh.simp_modulus(rhos[s], 3), x, fixed=fixed)
            rel = np.linalg.norm(f - Kx) / np.linalg.norm(f)
            assert rel < 1e-6 and abs(rel - rs[i]["rel_res_true"]) < 1e-9, (i, rel, rs[i])
            assert np.linalg.norm(x - x1) <= 1e-5 * np.linalg.norm(x1), i


def test_staged_batch_edge_cases():
    """Zero right-hand side (u = 0 at once), a start at the solution
    (converged at iteration 0), maxit 0, and argument checks."""
    from paper_2604_26441_amd import simpgmg
    dims, rhos = _systems()
    opts = [simpgmg.default_options(*d, n_levels=0, dense_max=1000, fine_prec="f32") for d in dims[:2]]
    b = simpgmg.setup_batch(opts, [t64(r) for r in rhos[:2]])
    f0 = workloads.edge_load(dims[0])
    f1 = workloads.edge_load(dims[1])
    u1 = t64(np.zeros_like(f1))
    simpgmg.pcg_solve(b.hierarchy(1), t64(f1), u1, rtol=1e-10, maxit=300)
    fs = [np.zeros_like(f0), f1]
    us = [t64(np.ones_like(f0) * (1 - workloads.cantilever_fixed(dims[0]))), u1]
    res, _ = simpgmg.pcg_solve_batch(b, [0, 1], [t64(f) for f in fs], us, rtol=1e-6, staged=True)
    assert res[0]["status"] == "converged" and np.all(np64(us[0]) == 0)
    assert res[1]["status"] == "converged" and res[1]["iters"] == 0
    us = [t64(np.zeros_like(f0)), t64(np.zeros_like(f1))]
    res, _ = simpgmg.pcg_solve_batch(b, [0, 1], [t64(f0), t64(f1)], us, rtol=1e-6, maxit=0,
                                     staged=True)
    assert [r["status"] for r in res] == ["maxit", "maxit"] and all(r["iters"] == 0 for r in res)
    assert all(abs(r["rel_res_true"] - 1.0) < 1e-12 for r in res)
    for kw in ({"maxit": -1}, {"rtol": 0.0}):
        with pytest.raises(simpgmg.SimpGmgError):
            simpgmg.pcg_solve_batch(b, [0, 1], [t64(f0), t64(f1)], us, staged=True, **kw)


def _graph_case(dims, seed, prec):
    from paper_2604_26441_amd import simpgmg
    rhos = [workloads.grf_rho(d, seed=seed + i) for i, d in enumerate(dims)]
    opts = [simpgmg.default_options(*d, n_levels=0, dense_max=1000, fine_prec=prec) for d in dims]
    b = simpgmg.setup_batch(opts, [t64(r) for r in rhos])
    rng = np.random.default_rng(seed)
    item_sys, fs = [], []
    for s, d in enumerate(dims):
        for k in range(1 + s % 3):
            item_sys.append(s)
            fs.append(workloads.random_face_load(d, rng) if k else workloads.edge_load(d))
    return b, rhos, item_sys, fs


def _same_results(ra, ua, rb, ub):
    for i in range(len(ra)):
        assert ra[i] == rb[i], (i, ra[i], rb[i])
        assert np.array_equal(np64(ua[i]), np64(ub[i])), i


def test_graph_batch_bitwise_equals_staged_and_passes_oracle():
    """The one-launch solve (iteration control on the device) takes the same
    decisions as the staged solve's host loop, item by item, so every item's
    status, iterations, residuals and u are bitwise equal to the staged
    solve's; with 128 steps per launch the whole solve is one launch, with 4
    steps it takes several and stays bitwise equal.  The oracle's FP64 true
    residual of every returned u is below rtol and equal to the reported one.
    BF16X3 fine levels (MFMA level 0) on odd and ragged meshes, 1-3 load
    cases per system."""
    from paper_2604_26441_amd import simpgmg
    dims = [(16, 8, 8), (20, 10, 10), (12, 6, 6), (30, 14, 14), (22, 12, 10)]
    b, rhos, item_sys, fs = _graph_case(dims, 500, "bf16x3")
    ft = [t64(f) for f in fs]
    us = [t64(np.zeros_like(f)) for f in fs]
    rs, _ = simpgmg.pcg_solve_batch(b, item_sys, ft, us, rtol=1e-6, maxit=300, staged=True)
    assert all(r["status"] == "converged" for r in rs)
    its = max(r["iters"] for r in rs)
    assert 4 < its <= 128
    for steps in (128, 4, 128):
        ug = [t64(np.zeros_like(f)) for f in fs]
        rg, ms, nl = simpgmg.pcg_solve_batch_graph(b, item_sys, ft, ug, rtol=1e-6, maxit=300,
                                                   steps=steps)
        assert ms > 0 and nl == -(-its // steps), (steps, nl, its)
        _same_results(rs, us, rg, ug)
    for i, (s, f) in enumerate(zip(item_sys, fs)):
        d = dims[s]
        fixed = workloads.cantilever_fixed(d).astype(bool)
        x = np64(ug[i])
        Kx = mesh.apply_K_elementwise(d, mesh.simp_modulus(rhos[s], 3), x, fixed=fixed)
        rel = np.linalg.norm(f - Kx) / np.linalg.norm(f)
        assert rel < 1e-6 and abs(rel - rg[i]["rel_res_true"]) < 1e-9, (i, rel, rg[i])


def test_graph_batch_edge_cases_match_staged():
    """Zero right-hand side (u = 0), a start at the solution (converged at
    iteration 0), maxit 0, a maxit that stops the items mid-solve (status
    maxit, the true residual from the final prologue) over several launches:
    each bitwise equal to the staged solve; argument checks on steps."""
    from paper_2604_26441_amd import simpgmg
    dims = [(16, 8, 8), (20, 10, 10)]
    b, rhos, _, _ = _graph_case(dims, 100, "f32")
    f0 = workloads.edge_load(dims[0])
    f1 = workloads.edge_load(dims[1])
    u1 = t64(np.zeros_like(f1))
    simpgmg.pcg_solve(b.hierarchy(1), t64(f1), u1, rtol=1e-10, maxit=300)
    start0 = np.ones_like(f0) * (1 - workloads.cantilever_fixed(dims[0]))
    cases = [([np.zeros_like(f0), f1], [start0, np64(u1)], {"rtol": 1e-6}),
             ([f0, f1], [np.zeros_like(f0), np.zeros_like(f1)], {"rtol": 1e-6, "maxit": 0}),
             ([f0, f1], [np.zeros_like(f0), np.zeros_like(f1)], {"rtol": 1e-12, "maxit": 5})]
    for fs, u0, kw in cases:
        ft = [t64(f) for f in fs]
        us = [t64(u.copy()) for u in u0]
        rs, _ = simpgmg.pcg_solve_batch(b, [0, 1], ft, us, staged=True, **kw)
        ug = [t64(u.copy()) for u in u0]
        rg, _, nl = simpgmg.pcg_solve_batch_graph(b, [0, 1], ft, ug, steps=2, **kw)
        _same_results(rs, us, rg, ug)
        assert nl == (3 if kw.get("maxit") == 5 else 1), (kw, nl)
    assert rg[0]["status"] == rg[1]["status"] == "maxit" and rg[0]["iters"] == 5
    assert rg[0]["rel_res_true"] > 1e-12
    for steps in (0, 3, 1026):
        with pytest.raises(simpgmg.SimpGmgError):
            simpgmg.pcg_solve_batch_graph(b, [0, 1], ft, ug, steps=steps)
