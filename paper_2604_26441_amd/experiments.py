"""Experiment drivers for the solver (GPU), printing one JSON record per run.

  python -m paper_2604_26441_amd.experiments sizes   # uniform cantilevers 40^3/60^3/80^3:
                                                     # FP32-GMG vs FP64-GMG vs Jacobi-PCG
  python -m paper_2604_26441_amd.experiments kernels # fine K.u and level-1 stencil timings
  python -m paper_2604_26441_amd.experiments e1 | spectral_proxy | robustness
                                                     # binary-contrast and stress screens

Timing protocol: 2 warm-up solves, then 5 timed solves (HIP events inside
sgmg_pcg_solve); setup is timed separately with host clocks around a
synchronised setup call.
"""
import json
import sys
import time

import numpy as np
import torch

import workloads
from . import simpgmg


def _schedule(kw):
    """Eq. prec_schedule: the BF16 path runs level 1 in FP32 (levels >= 2
    stay FP64); FP32-GMG keeps every level >= 1 in FP64."""
    if kw.get("fine_prec") == "bf16":
        kw.setdefault("level1_prec", "f32")
    return kw


def _solve(dims, precond=2, maxit=200, trials=5, warmup=2, **kw):
    dev = "cuda:0"
    rho = torch.tensor(workloads.uniform_rho(dims), dtype=torch.float64, device=dev)
    f = torch.tensor(workloads.edge_load(dims), dtype=torch.float64, device=dev)
    o = simpgmg.default_options(*dims, **_schedule(kw))
    h = simpgmg.setup_hierarchy(o, rho)      # launch shapes and the level-1 form, untimed
    simpgmg.autotune(h)
    h.close()
    times, setups, res = [], [], None
    for k in range(warmup + trials):
        t0 = time.perf_counter()
        h = simpgmg.setup_hierarchy(o, rho)
        torch.cuda.synchronize()
        su = (time.perf_counter() - t0) * 1e3
        u = torch.zeros_like(f)
        res = simpgmg.pcg_solve(h, f, u, rtol=1e-6, maxit=maxit, precond=precond)
        if k >= warmup:
            times.append(res["solve_ms"])
            setups.append(su)
        h.close()
    return {"solve_ms_mean": float(np.mean(times)), "solve_ms_std": float(np.std(times)),
            "setup_ms_mean": float(np.mean(setups)), "iters": res["iters"], "status": res["status"],
            "rel_res_true": res["rel_res_true"]}


def sizes():
    for n in (40, 60, 80):
        dims = (n, n, n)
        rec = {"dims": dims}
        rec["fp32_gmg_bf16x3"] = _solve(dims, fine_prec="bf16x3")
        rec["fp32_gmg_f32valu"] = _solve(dims, fine_prec="f32")
        rec["fp64_gmg"] = _solve(dims, fine_prec="f64")
        rec["bf16_gmg_flex"] = _solve(dims, fine_prec="bf16", flexible_beta=1)
        rec["jacobi_pcg_cap200"] = _solve(dims, precond=1, maxit=200, fine_prec="f64")
        rec["jacobi_pcg_to_1e-6"] = _solve(dims, precond=1, maxit=20000, fine_prec="f64", trials=1, warmup=0)
        print(json.dumps(rec), flush=True)


def hetero(n=60, seeds=9, maxit=500):
    """Heterogeneous 60^3 cantilevers (GRF rho, correlation length 4
    elements, logistic map to [1e-3, 1]) for p in {1, 2, 3} and 9 seeds:
    FP64-GMG, FP32-GMG (BF16X3 fine operator), FP32-GMG on the FP32 vector
    ALU and BF16-GMG (flexible PCG) to rtol 1e-6, cap 500; errors against an
    FP64-GMG solve to 1e-10 of the same system (compliance and solution)."""
    dev = "cuda:0"
    dims = (n, n, n)
    f = torch.tensor(workloads.edge_load(dims), dtype=torch.float64, device=dev)
    variants = {"fp64_gmg": {"fine_prec": "f64"}, "fp32_gmg_bf16x3": {"fine_prec": "bf16x3"},
                "fp32_gmg_f32valu": {"fine_prec": "f32"},
                "bf16_gmg_flex": {"fine_prec": "bf16", "flexible_beta": 1}}
    tuned = False
    for p in (1, 2, 3):
        for seed in range(seeds):
            rho = torch.tensor(workloads.grf_rho(dims, seed), dtype=torch.float64, device=dev)
            h = simpgmg.setup_hierarchy(simpgmg.default_options(*dims, penal=float(p), fine_prec="f64"), rho)
            uref = torch.zeros_like(f)
            ref = simpgmg.pcg_solve(h, f, uref, rtol=1e-10, maxit=4000)
            h.close()
            cref = float(f @ uref)
            rec = {"p": p, "seed": seed, "ref": {"status": ref["status"], "iters": ref["iters"],
                                                  "rel_res_true": ref["rel_res_true"]}}
            for name, kw in variants.items():
                h = simpgmg.setup_hierarchy(simpgmg.default_options(*dims, penal=float(p),
                                                                    **_schedule(dict(kw))), rho)
                if not tuned and kw["fine_prec"] in ("bf16", "bf16x3"):
                    simpgmg.autotune(h)
                    tuned = True
                for _ in range(2):
                    u = torch.zeros_like(f)
                    r = simpgmg.pcg_solve(h, f, u, rtol=1e-6, maxit=maxit)
                c = float(f @ u)
                rec[name] = {"status": r["status"], "iters": r["iters"], "solve_ms": round(r["solve_ms"], 3),
                             "rel_res_true": r["rel_res_true"],
                             "compliance_rel_err": abs(c - cref) / abs(cref),
                             "u_rel_err": float(torch.linalg.norm(u - uref) / torch.linalg.norm(uref))}
                h.close()
            print(json.dumps(rec), flush=True)


def hetero_oracle(maxit=500):
    """The precision schedules on the heterogeneous 60^3 cases whose oracle
    reference solves are stored in tests/golden/config2_oracle.json (the
    oracle's FP64 PCG-GMG to rtol 1e-10, written by
    tests/golden/make_config2_reference.py): per schedule and case, the
    iterations beside the oracle's at rtol 1e-6, the compliance error
    |f.u - c*| / c* and the energy-norm error ||u - u*||_K / ||u*||_K from
    u.K u - 2 f.u + c* (K u* = f, c* = f.u*), with K u from the library's FP64
    fine operator."""
    import os
    dev = "cuda:0"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    G = json.load(open(os.path.join(root, "tests", "golden", "config2_oracle.json")))
    dims = tuple(G["dims"])
    f = torch.tensor(workloads.edge_load(dims), dtype=torch.float64, device=dev)
    schedules = {"fp64_gmg": {"fine_prec": "f64"}, "fp32_gmg_bf16x3": {"fine_prec": "bf16x3"},
                 "bf16_gmg_flex": {"fine_prec": "bf16", "flexible_beta": 1}}
    for case in G["cases"]:
        p, seed, cstar = case["p"], case["seed"], case["compliance"]
        rho = torch.tensor(workloads.grf_rho(dims, seed), dtype=torch.float64, device=dev)
        rec = {"p": p, "seed": seed, "oracle_iters": case["iters_rtol_1e-6"]}
        for name, kw in schedules.items():
            h = simpgmg.setup_hierarchy(simpgmg.default_options(*dims, penal=float(p),
                                                                **_schedule(dict(kw))), rho)
            u = torch.zeros_like(f)
            r = simpgmg.pcg_solve(h, f, u, rtol=1e-6, maxit=maxit)
            y = torch.empty_like(u)
            simpgmg.apply_K(h, 0, "f64", u, y)
            h.close()
            c = float(torch.dot(f, u))
            # ||u - u*||_K^2 / c*; below about 4e-16 (relative error 2e-8)
            # the rounding of the three terms decides its sign
            e2 = (float(torch.dot(u, y)) - 2.0 * c + cstar) / cstar
            rec[name] = {"status": r["status"], "iters": r["iters"],
                         "compliance_rel_err": abs(c - cstar) / abs(cstar),
                         "energy_sq_rel": e2}
        print(json.dumps(rec), flush=True)


EPS_BF16 = 2.0 ** -8      # BF16 unit roundoff (8-bit significand, round to nearest)


def _kappa(h, dims, steps=(20, 50)):
    """Lanczos kappa_eff of the V-cycle-preconditioned fine operator after
    each number of steps in `steps`, start vector a normalised Gaussian
    (seed 0) on the free DOFs."""
    fixed = workloads.cantilever_fixed(dims)
    g = workloads.random_vector(fixed.size, 0, fixed)
    g /= np.linalg.norm(g)
    gd = torch.tensor(g, dtype=torch.float64, device="cuda:0")
    return {f"kappa_eff_{m}": simpgmg.lanczos(h, gd, m=m)["kappa"] for m in steps}


def _fgmres_run(dims, rho, p, f, fine_prec, restart, maxit):
    o = simpgmg.default_options(*dims, penal=float(p), **_schedule({"fine_prec": fine_prec}))
    h = simpgmg.setup_hierarchy(o, rho)
    u = torch.zeros_like(f)
    r = simpgmg.fgmres_solve(h, f, u, rtol=1e-6, maxit=maxit, restart=restart)
    return h, u, r


def e1(maxit=200):
    """Binary-contrast sweep (Sec. 4, E1): 40^3, 60^3, 80^3 cantilevers, each
    element solid with probability V_f in {0.2, 0.5, 0.8} else void at 1e-2
    (Bernoulli, seed 42), p in {1.5, 3, 4.5}; FP64-GMG PCG, rtol 1e-6, cap 200."""
    dev = "cuda:0"
    for n in (40, 60, 80):
        dims = (n, n, n)
        f = torch.tensor(workloads.edge_load(dims), dtype=torch.float64, device=dev)
        for vf in (0.2, 0.5, 0.8):
            rho = torch.tensor(workloads.binary_rho(dims, vf, 1e-2, 42), dtype=torch.float64, device=dev)
            for p in (1.5, 3.0, 4.5):
                h = simpgmg.setup_hierarchy(simpgmg.default_options(*dims, penal=p, fine_prec="f64"), rho)
                u = torch.zeros_like(f)
                r = simpgmg.pcg_solve(h, f, u, rtol=1e-6, maxit=maxit)
                h.close()
                print(json.dumps({"n": n, "vf": vf, "p": p, "status": r["status"], "iters": r["iters"],
                                  "rel_res_true": r["rel_res_true"],
                                  "solve_ms": round(r["solve_ms"], 3)}), flush=True)


def spectral_proxy(maxit=500):
    """BF16 spectral-proxy grid (Sec. 4, E5): 40^3 and 60^3 binary fields
    (V_f in {0.2, 0.5, 0.8}, void 1e-2, seed 42) for p in {1.5, 3, 4.5}:
    kappa_eff of the FP64 hierarchy by Lanczos (50 steps), eps_BF16 * kappa,
    then FGMRES (restart 32, cap 500, rtol 1e-6) with the BF16 and the FP64
    hierarchy and their compliance difference."""
    dev = "cuda:0"
    for n in (40, 60):
        dims = (n, n, n)
        f = torch.tensor(workloads.edge_load(dims), dtype=torch.float64, device=dev)
        for vf in (0.2, 0.5, 0.8):
            rho = torch.tensor(workloads.binary_rho(dims, vf, 1e-2, 42), dtype=torch.float64, device=dev)
            for p in (1.5, 3.0, 4.5):
                rec = {"n": n, "vf": vf, "p": p}
                comp = {}
                for prec in ("f64", "bf16"):
                    h, u, r = _fgmres_run(dims, rho, p, f, prec, 32, maxit)
                    if prec == "f64":
                        kap = _kappa(h, dims)
                        rec.update(kap, eps_kappa=EPS_BF16 * kap["kappa_eff_50"])
                    h.close()
                    comp[prec] = float(f @ u)
                    rec[prec] = {"status": r["status"], "iters": r["iters"],
                                 "rel_res_true": r["rel_res_true"], "solve_ms": round(r["solve_ms"], 3)}
                rec["compliance_rel_diff"] = abs(comp["bf16"] - comp["f64"]) / abs(comp["f64"])
                print(json.dumps(rec), flush=True)


def robustness(n=40, maxit=500):
    """The ten stress configurations of Sec. 4 (E10) on the 40^3 (64k)
    cantilever with the FP64 hierarchy: FGMRES restart 50, cap 500, rtol
    1e-6, and kappa_eff by Lanczos (50 steps)."""
    dev = "cuda:0"
    dims = (n, n, n)
    f = torch.tensor(workloads.edge_load(dims), dtype=torch.float64, device=dev)
    for label, rho_np, p in workloads.robustness_suite(dims):
        rho = torch.tensor(rho_np, dtype=torch.float64, device=dev)
        h, u, r = _fgmres_run(dims, rho, p, f, "f64", 50, maxit)
        kap = _kappa(h, dims)
        h.close()
        print(json.dumps({"config": label, "p": p, "status": r["status"], "iters": r["iters"],
                          "rel_res_true": r["rel_res_true"], "solve_ms": round(r["solve_ms"], 3),
                          **kap}), flush=True)


def _timed(dims, rho, f, solver="pcg", restart=32, maxit=500, trials=3, **kw):
    """Setup once, then `trials` solves after one warm-up: mean solve ms
    (HIP events inside the solver), iterations, status, true residual."""
    h = simpgmg.setup_hierarchy(simpgmg.default_options(*dims, **_schedule(dict(kw))), rho)
    ms = []
    for k in range(trials + 1):
        u = torch.zeros_like(f)
        r = (simpgmg.pcg_solve(h, f, u, rtol=1e-6, maxit=maxit) if solver == "pcg" else
             simpgmg.fgmres_solve(h, f, u, rtol=1e-6, maxit=maxit, restart=restart))
        if k:
            ms.append(r["solve_ms"])
    h.close()
    return {"status": r["status"], "iters": r["iters"], "rel_res_true": r["rel_res_true"],
            "solve_ms": round(float(np.mean(ms)), 3), "solve_ms_std": round(float(np.std(ms)), 3)}


def ablations(n=60):
    """Sec. 4 E6 on the 60^3 (216k) cantilever, rho = 0.5, p = 3, PCG rtol
    1e-6: (a) fine precision FP64 / FP32; (b) depth 2..5 with level 1 in FP64
    or FP32 (FP32 fine level); (c) V- vs W-cycle; (d) Chebyshev vs Jacobi
    (degree 2); then the high-contrast smoother screen (binary fields, void
    1e-2, seed 42, p = 3, 40^3 and 60^3, V_f 0.5 / 0.2; FP64-GMG with
    FGMRES restart 32, cap 500) for Chebyshev and Jacobi of degree 2 and 4."""
    dev = "cuda:0"
    dims = (n, n, n)
    rho = torch.tensor(workloads.uniform_rho(dims), dtype=torch.float64, device=dev)
    f = torch.tensor(workloads.edge_load(dims), dtype=torch.float64, device=dev)
    runs = [("a", {"fine_prec": "f64"}), ("a", {"fine_prec": "f32"})]
    runs += [("b", {"fine_prec": "f32", "n_levels": L, "level1_prec": p1})
             for L in (2, 3, 4, 5) for p1 in ("f64", "f32")]
    runs += [("c", {"fine_prec": "f32", "cycle_gamma": g}) for g in (1, 2)]
    runs += [("d", {"fine_prec": "f32", "fine_smoother": sm}) for sm in (0, 1)]
    for tag, kw in runs:
        print(json.dumps({"ablation": tag, **kw, **_timed(dims, rho, f, **kw)}), flush=True)
    for m in (40, 60):
        d2 = (m, m, m)
        f2 = torch.tensor(workloads.edge_load(d2), dtype=torch.float64, device=dev)
        for vf in (0.5, 0.2):
            r2 = torch.tensor(workloads.binary_rho(d2, vf, 1e-2, 42), dtype=torch.float64, device=dev)
            for sm, deg in ((0, 2), (0, 4), (1, 2), (1, 4)):
                kw = {"fine_prec": "f64", "fine_smoother": sm, "fine_degree": deg}
                print(json.dumps({"screen": "high_contrast", "n": m, "vf": vf,
                                  "smoother": "chebyshev" if sm == 0 else "jacobi", "degree": deg,
                                  **_timed(d2, r2, f2, solver="fgmres", trials=1, **kw)}), flush=True)


def sensitivity(n=60):
    """Sec. 4 E6 sensitivity surface on the 60^3 cantilever (rho = 0.5,
    p = 3): Chebyshev degree {1, 2, 4} x depth {3, 4} x FGMRES restart
    {16, 32, 50}, FP32-GMG (BF16X3 fine K.u) and BF16-GMG, rtol 1e-6, cap 500."""
    dev = "cuda:0"
    dims = (n, n, n)
    rho = torch.tensor(workloads.uniform_rho(dims), dtype=torch.float64, device=dev)
    f = torch.tensor(workloads.edge_load(dims), dtype=torch.float64, device=dev)
    h = simpgmg.setup_hierarchy(simpgmg.default_options(*dims, fine_prec="bf16x3"), rho)
    simpgmg.autotune(h)
    h.close()
    for prec in ("bf16x3", "bf16"):
        for deg in (1, 2, 4):
            for L in (3, 4):
                for rs in (16, 32, 50):
                    kw = {"fine_prec": prec, "fine_degree": deg, "n_levels": L}
                    print(json.dumps({"restart": rs, **kw,
                                      **_timed(dims, rho, f, solver="fgmres", restart=rs, **kw)}),
                          flush=True)


def simp_schedule(steps=30, rtol=1e-5, cap=1000):
    """The auxiliary 30-step fixed-penalty OC schedule (App. e3_aux): p = 3,
    volume fraction 0.5 from the uniform design, density filter rmin 1.5, no
    projection, move 0.2, linear solves to rtol 1e-5 with a 1000-iteration
    cap, warm-started from the previous state; FP32-GMG PCG against
    Jacobi-PCG on the cantilever (60^3), the torsion bar (30x10x10) and the
    MBB half-beam (30x5x10).  Wall time of the whole schedule (host clock,
    synchronised; the hierarchy is set up once before it), cap hits, and
    the compliance at every step."""
    dev = "cuda:0"
    benches = [("cantilever-216k", (60, 60, 60), None, None, 4),
               ("torsion-3k", (30, 10, 10), None, "torsion", 0),
               ("mbb-1.5k", (30, 5, 10), "mbb", "mbb", 0)]
    for name, dims, fix_kind, load_kind, levels in benches:
        n = dims[0] * dims[1] * dims[2]
        fixed = None if fix_kind is None else torch.tensor(workloads.mbb_fixed(dims), device=dev)
        f_np = {None: workloads.edge_load, "torsion": workloads.torsion_load,
                "mbb": workloads.mbb_load}[load_kind](dims)
        f = torch.tensor(f_np, dtype=torch.float64, device=dev)
        rec = {"bench": name, "dims": dims}
        for solver, precond, prec in (("fp32_gmg", 2, "bf16x3"), ("jacobi_pcg", 1, "f64")):
            o = simpgmg.default_options(*dims, n_levels=levels, fine_prec=prec)
            rho = torch.full((n,), 0.5, dtype=torch.float64, device=dev)
            h = simpgmg.setup_hierarchy(o, rho, fixed_dof=fixed)
            if prec == "bf16x3":
                simpgmg.autotune(h)
            s = simpgmg.Simp(simpgmg.simp_params(*dims, volfrac=0.5, rmin=1.5))
            u = torch.zeros_like(f)
            comp, iters, caps = [], [], 0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(steps):
                r = s.step(h, rho, f, u, rtol=rtol, maxit=cap, precond=precond)
                comp.append(r["compliance"])
                iters.append(r["pcg_iters"])
                caps += r["pcg_status"] != "converged"
            torch.cuda.synchronize()
            rec[solver] = {"wall_s": round(time.perf_counter() - t0, 4), "cap_hits": caps,
                           "iters": iters, "compliance": comp}
            s.close()
            h.close()
        c0g, c0j = rec["fp32_gmg"]["compliance"][0], rec["jacobi_pcg"]["compliance"][0]
        rec["step0_compliance_rel_diff"] = abs(c0g - c0j) / abs(c0j)
        rec["time_ratio_jacobi_over_gmg"] = rec["jacobi_pcg"]["wall_s"] / rec["fp32_gmg"]["wall_s"]
        print(json.dumps(rec), flush=True)


def large(trials=5, warmup=2):
    """The paper's large-scale table (Table e7) like for like: 2:1:1 boxes
    100x50x25 (125k), 160x80x40 (512k), 200x100x50 (1M) with uniform modulus
    E_e = 0.5, FP32-GMG (fine K.u BF16X3 on MFMA), 4 levels, restarted FGMRES
    (restart 50), rtol 1e-6; setup and solve wall times, iterations, the
    device-memory delta of the setup; PCG on the same systems beside it."""
    dev = "cuda:0"
    for dims in ((100, 50, 25), (160, 80, 40), (200, 100, 50)):
        nel = dims[0] * dims[1] * dims[2]
        E = torch.full((nel,), 0.5, dtype=torch.float64, device=dev)
        f = torch.tensor(workloads.edge_load(dims), dtype=torch.float64, device=dev)
        o = simpgmg.default_options(*dims, n_levels=4, fine_prec="bf16x3", input_is_modulus=1)
        h = simpgmg.setup_hierarchy(o, E)
        simpgmg.autotune(h)
        nfc = h.level_info(3)["n_free"]
        h.close()
        rec = {"dims": dims, "elements": nel, "coarsest_free_dofs": nfc,
               "coarsest_solve": "dense" if nfc <= o.dense_max else f"pcg{o.coarse_pcg_iters}"}
        for solver in ("fgmres50", "pcg"):
            setups, solves, its, st, mem = [], [], [], [], []
            for k in range(warmup + trials):
                torch.cuda.synchronize()
                free0 = torch.cuda.mem_get_info()[0]
                t0 = time.perf_counter()
                h = simpgmg.setup_hierarchy(o, E)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                free1 = torch.cuda.mem_get_info()[0]
                u = torch.zeros_like(f)
                if solver == "pcg":
                    r = simpgmg.pcg_solve(h, f, u, rtol=1e-6, maxit=500)
                else:
                    r = simpgmg.fgmres_solve(h, f, u, rtol=1e-6, maxit=500, restart=50)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                if k >= warmup:
                    setups.append((t1 - t0) * 1e3)
                    solves.append((t2 - t1) * 1e3)
                    its.append(r["iters"])
                    st.append(r["status"])
                    mem.append((free0 - free1) / 2**20)
                h.close()
            rec[solver] = {"setup_ms_mean": float(np.mean(setups)), "setup_ms_std": float(np.std(setups)),
                           "solve_ms_mean": float(np.mean(solves)), "solve_ms_std": float(np.std(solves)),
                           "iters": its[-1], "status": st[-1], "rel_res_true": r["rel_res_true"],
                           "setup_mem_MiB": float(np.mean(mem))}
        print(json.dumps(rec), flush=True)


def kernels():
    dev = "cuda:0"
    for n in (40, 60, 80, 128):
        dims = (n, n, n)
        o = simpgmg.default_options(*dims, n_levels=0)     # fewest levels with n_L <= 5000
        rho = torch.tensor(workloads.uniform_rho(dims), dtype=torch.float64, device=dev)
        h = simpgmg.setup_hierarchy(o, rho)
        fixed = torch.tensor(workloads.cantilever_fixed(dims), device=dev).bool()
        rec = {"dims": dims, "mfma_shape_bf16_bf16x3": simpgmg.autotune(h)}
        for prec in ("f64", "f32", "bf16x3", "bf16"):
            dt = torch.float64 if prec == "f64" else torch.float32
            u = torch.ones(fixed.numel(), dtype=dt, device=dev).masked_fill_(fixed, 0)
            y = torch.empty_like(u)
            for _ in range(5):
                simpgmg.apply_K(h, 0, prec, u, y)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(200):
                simpgmg.apply_K(h, 0, prec, u, y)
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / 200
            es = 8 if prec == "f64" else 4
            byts = 2 * fixed.numel() * es + n ** 3 * es
            rec[f"ku_{prec}_us"] = round(us, 2)
            rec[f"ku_{prec}_GBs"] = round(byts / us / 1e3, 1)
        info = h.level_info(1)
        d = info["dims"]
        n1 = 3 * (d[0] + 1) * (d[1] + 1) * (d[2] + 1)
        u1 = torch.ones(n1, dtype=torch.float64, device=dev)
        y1 = torch.empty_like(u1)
        for _ in range(5):
            simpgmg.apply_K(h, 1, "f64", u1, y1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(100):
            simpgmg.apply_K(h, 1, "f64", u1, y1)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / 100
        nn1 = n1 // 3
        rec["l1_stencil_f64_us"] = round(us, 2)
        rec["l1_stencil_f64_GBs"] = round((243 * 8 * nn1 + 2 * 8 * n1) / us / 1e3, 1)
        h.close()
        print(json.dumps(rec), flush=True)


def _graph_runs(b, item_sys, ft, sres, steps=128, reps=4):
    """The staged solve in one graph launch per `steps` iterations (the first
    run captures the graphs): mean wall time of the later runs, launches, and
    whether every item's result equals the staged solve's `sres`."""
    runs, res, nl = [], None, 0
    for rep in range(reps):
        us = [torch.zeros_like(f) for f in ft]
        res, ms, nl = simpgmg.pcg_solve_batch_graph(b, item_sys, ft, us, rtol=1e-6, maxit=300,
                                                    steps=steps)
        runs.append(ms)
    return {"graph_steps": steps, "graph_ms_runs": runs, "graph_ms": float(np.mean(runs[1:])),
            "graph_launches": nl, "graph_equals_staged": res == sres}


def batch_graph(precs=("bf16x3", "f32"), steps=128):
    """The 84-item batch (as batch()) with BF16X3 and FP32 fine levels: the
    staged solve by host loop and in one graph launch of `steps` steps."""
    dev = "cuda:0"
    dims, rhos, item_sys, fs = workloads.batch_config()
    ft = [torch.tensor(f, dtype=torch.float64, device=dev) for f in fs]
    for prec in precs:
        opts = [simpgmg.default_options(*d, n_levels=0, dense_max=1000, fine_prec=prec) for d in dims]
        b = simpgmg.setup_batch(opts, [torch.tensor(r, dtype=torch.float64, device=dev) for r in rhos])
        rec = {"fine_prec": prec, "n_items": len(item_sys)}
        sruns = []
        for rep in range(4):
            us = [torch.zeros_like(f) for f in ft]
            sres, ms = simpgmg.pcg_solve_batch(b, item_sys, ft, us, rtol=1e-6, maxit=300, staged=True)
            sruns.append(ms)
        rec["staged_ms"] = float(np.mean(sruns[1:]))
        rec["max_iters"] = max(r["iters"] for r in sres)
        t0 = time.perf_counter()
        rec.update(_graph_runs(b, item_sys, ft, sres, steps=steps))
        rec["graph_wall_s_incl_capture"] = time.perf_counter() - t0
        rec["max_rel_res_true"] = max(r["rel_res_true"] for r in sres)
        print(json.dumps(rec), flush=True)
        b.close()


def batch():
    """32 uneven cantilevers (2m x m x m, m in 8..24), random-field rho, p = 3,
    1-4 face load cases each, FP32 smoothing, rtol 1e-6: one persistent launch
    and the stage-batched solve against the same items solved one after
    another with sgmg_pcg_solve, from
    2, 4, 8 Python threads with a stream each, and by the library's concurrent
    batch solve with 2-16 native workers."""
    dev = "cuda:0"
    dims, rhos, item_sys, fs = workloads.batch_config()
    opts = [simpgmg.default_options(*d, n_levels=0, dense_max=1000, fine_prec="f32") for d in dims]
    t0 = time.perf_counter()
    b = simpgmg.setup_batch(opts, [torch.tensor(r, dtype=torch.float64, device=dev) for r in rhos])
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    ft = [torch.tensor(f, dtype=torch.float64, device=dev) for f in fs]
    rec = {"n_systems": len(dims), "n_items": len(item_sys),
           "elements_total": int(sum(d[0] * d[1] * d[2] for d in dims)), "setup_ms": setup_ms}
    runs = []
    for rep in range(4):                                   # first run includes autotuning
        us = [torch.zeros_like(f) for f in ft]
        res, ms = simpgmg.pcg_solve_batch(b, item_sys, ft, us, rtol=1e-6, maxit=300)
        runs.append(ms)
    rec["batched_ms_runs"] = runs
    rec["batched_ms"] = float(np.mean(runs[1:]))
    # stage-batched: one launch per stage over all items (first run captures
    # the graphs)
    sruns = []
    for rep in range(4):
        us = [torch.zeros_like(f) for f in ft]
        sres, ms = simpgmg.pcg_solve_batch(b, item_sys, ft, us, rtol=1e-6, maxit=300, staged=True)
        sruns.append(ms)
    rec["staged_ms_runs"] = sruns
    rec["staged_ms"] = float(np.mean(sruns[1:]))
    rec["staged_all_converged"] = all(r["status"] == "converged" for r in sres)
    rec["staged_iters"] = [r["iters"] for r in sres]
    rec["staged_max_rel_res_true"] = max(r["rel_res_true"] for r in sres)
    rec.update(_graph_runs(b, item_sys, ft, sres))
    rec["block_size"] = b.block_size()
    rec["batched_all_converged"] = all(r["status"] == "converged" for r in res)
    rec["batched_iters"] = [r["iters"] for r in res]
    rec["batched_max_rel_res_true"] = max(r["rel_res_true"] for r in res)
    hs = [b.hierarchy(s) for s in range(len(dims))]
    tot, its, ok = [], [], True
    for rep in range(2):                                   # first pass captures the graphs
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = []
        for s, f in zip(item_sys, ft):
            u = torch.zeros_like(f)
            r = simpgmg.pcg_solve(hs[s], f, u, rtol=1e-6, maxit=300)
            its.append(r["iters"])
            ok = ok and r["status"] == "converged"
        torch.cuda.synchronize()
        tot.append((time.perf_counter() - t0) * 1e3)
    rec["sequential_f32_ms"] = tot[-1]
    rec["sequential_iters"] = its
    rec["sequential_all_converged"] = ok
    rec["speedup_vs_sequential"] = rec["sequential_f32_ms"] / rec["batched_ms"]
    # the same solves from host threads, one stream each (systems spread by
    # total elements x items, largest first; a system's items stay on one
    # stream since they share its hierarchy)
    import threading
    for nthreads in (2, 4, 8):
        work = {}
        for i, sidx in enumerate(item_sys):
            work.setdefault(sidx, []).append(i)
        order = sorted(work, key=lambda q: -dims[q][0] * dims[q][1] * dims[q][2] * len(work[q]))
        lanes, load = [[] for _ in range(nthreads)], [0] * nthreads
        for q in order:
            k = load.index(min(load))
            lanes[k].append(q)
            load[k] += dims[q][0] * dims[q][1] * dims[q][2] * len(work[q])
        streams = [torch.cuda.Stream() for _ in range(nthreads)]
        status = []

        def run(k):
            with torch.cuda.stream(streams[k]):
                for q in lanes[k]:
                    for i in work[q]:
                        u = torch.zeros_like(ft[i])
                        r = simpgmg.pcg_solve(hs[q], ft[i], u, rtol=1e-6, maxit=300, stream=streams[k])
                        status.append(r["status"])
                streams[k].synchronize()
        times = []
        for rep in range(2):
            status.clear()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            th = [threading.Thread(target=run, args=(k,)) for k in range(nthreads)]
            for t in th:
                t.start()
            for t in th:
                t.join()
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        rec[f"streams{nthreads}_ms"] = times[-1]
        rec[f"streams{nthreads}_all_converged"] = all(x == "converged" for x in status) and len(status) == len(item_sys)
    # the library's concurrent batch solve (native worker threads, a stream each)
    for nw in (2, 4, 8, 16):
        times = []
        for rep in range(3):
            us = [torch.zeros_like(f) for f in ft]
            res, ms = simpgmg.pcg_solve_batch_concurrent(b, item_sys, ft, us, rtol=1e-6, maxit=300,
                                                         workers=nw)
            times.append(ms)
        rec[f"concurrent{nw}_ms"] = float(np.median(times))
        rec[f"concurrent{nw}_all_converged"] = all(r["status"] == "converged" for r in res)
    print(json.dumps(rec), flush=True)
    # the same items with the fine level in BF16X3 on the matrix cores (the
    # FP32-GMG schedule of the single solves): staged, sequential, concurrent
    b.close()
    opts = [simpgmg.default_options(*d, n_levels=0, dense_max=1000, fine_prec="bf16x3") for d in dims]
    b = simpgmg.setup_batch(opts, [torch.tensor(r, dtype=torch.float64, device=dev) for r in rhos])
    rec2 = {"fine_prec": "bf16x3"}
    sruns = []
    for rep in range(4):                                   # first run tunes the shape, captures
        us = [torch.zeros_like(f) for f in ft]
        sres, ms = simpgmg.pcg_solve_batch(b, item_sys, ft, us, rtol=1e-6, maxit=300, staged=True)
        sruns.append(ms)
    rec2["staged_ms_runs"] = sruns
    rec2["staged_ms"] = float(np.mean(sruns[1:]))
    rec2["staged_all_converged"] = all(r["status"] == "converged" for r in sres)
    rec2["staged_iters"] = [r["iters"] for r in sres]
    rec2["staged_max_rel_res_true"] = max(r["rel_res_true"] for r in sres)
    rec2.update(_graph_runs(b, item_sys, ft, sres))
    hs = [b.hierarchy(q) for q in range(len(dims))]
    tot = []
    for rep in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for q, f in zip(item_sys, ft):
            u = torch.zeros_like(f)
            simpgmg.pcg_solve(hs[q], f, u, rtol=1e-6, maxit=300)
        torch.cuda.synchronize()
        tot.append((time.perf_counter() - t0) * 1e3)
    rec2["sequential_ms"] = tot[-1]
    for nw in (4, 8):
        times = []
        for rep in range(3):
            us = [torch.zeros_like(f) for f in ft]
            res, ms = simpgmg.pcg_solve_batch_concurrent(b, item_sys, ft, us, rtol=1e-6, maxit=300,
                                                         workers=nw)
            times.append(ms)
        rec2[f"concurrent{nw}_ms"] = float(np.median(times))
        rec2[f"concurrent{nw}_all_converged"] = all(r["status"] == "converged" for r in res)
    print(json.dumps(rec2), flush=True)


def train_warm_start(n_train=2000, train_seconds=120.0, batch_size=8, lr=1e-3, seed=2024,
                     progress=True, loss="energy"):
    """U-Net trained on solver-generated 32^3 random-field pairs (GRF seeds
    10000+, p = 3, random face loads, FP32-GMG-PCG to 1e-8).  loss "energy":
    the library's energy-norm score (the squared energy-norm error the
    scaled prediction leaves, relative to the zero start's); "mse": the
    masked MSE against u / max|u|.  Returns the network and a record of the
    data generation and training."""
    dev = "cuda:0"
    rng = np.random.default_rng(seed)
    dims = (32, 32, 32)
    t0 = time.perf_counter()
    X, T, M, R, F, C = [], [], [], [], [], []
    iters = []
    h_keep = None
    for k in range(n_train):
        rho = torch.tensor(workloads.grf_rho(dims, 10000 + k), dtype=torch.float64, device=dev)
        f = torch.tensor(workloads.random_face_load(dims, rng), dtype=torch.float64, device=dev)
        h = simpgmg.setup_hierarchy(simpgmg.default_options(*dims, n_levels=0), rho)
        u = torch.zeros_like(f)
        res = simpgmg.pcg_solve(h, f, u, rtol=1e-8, maxit=500)
        iters.append(res["iters"])
        X.append(simpgmg.unet_input(h, rho, f))
        t, m = simpgmg.unet_target(h, u)
        T.append(t)
        M.append(m)
        R.append(rho)
        F.append(f)
        C.append(torch.dot(f, u).reshape(1))            # compliance f.u*, the score's scale
        if h_keep is None:
            h_keep = h                                  # the mesh and clamps of every sample
        else:
            h.close()
        if progress and (k + 1) % 250 == 0:
            print(json.dumps({"pairs": k + 1, "s": round(time.perf_counter() - t0, 1)}), flush=True)
    X, T, M = torch.cat(X), torch.cat(T), torch.cat(M)
    R, F, C = torch.stack(R), torch.stack(F), torch.cat(C)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    net = simpgmg.UNet(seed=0)
    t0 = time.perf_counter()
    losses, steps = [], 0
    while time.perf_counter() - t0 < train_seconds:
        idx = torch.as_tensor(rng.choice(n_train, size=batch_size, replace=False), device=dev)
        if loss == "energy":
            losses.append(net.energy_step(h_keep, X[idx].contiguous(), R[idx].contiguous(),
                                          F[idx].contiguous(), C[idx].contiguous(), lr=lr))
        else:
            losses.append(net.train_step(X[idx].contiguous(), T[idx].contiguous(),
                                         M[idx].contiguous(), lr=lr))
        steps += 1
        if progress and steps % 500 == 0:
            print(json.dumps({"step": steps, "loss": float(np.mean(losses[-50:]))}), flush=True)
    train_s = time.perf_counter() - t0
    h_keep.close()
    rec = {"loss": loss, "n_train": n_train, "train_pairs_gen_s": round(gen_s, 2),
           "train_solve_iters_mean": float(np.mean(iters)), "train_steps": steps,
           "train_s": round(train_s, 2), "batch": batch_size,
           "loss_first10": float(np.mean(losses[:10])), "loss_last10": float(np.mean(losses[-10:])),
           "params": simpgmg.UNet.num_params()}
    return net, rec


def warm_vs_cold(net, h, rho, f, rtol=1e-6, maxit=500, reps=3):
    """Zero start against the scaled network start on hierarchy h (same
    tolerance); warm time includes input assembly, inference and scaling."""
    for _ in range(2):                                     # warm-up (graph capture)
        u = torch.zeros_like(f)
        simpgmg.pcg_solve(h, f, u, rtol=rtol, maxit=maxit)
    net.forward(simpgmg.unet_input(h, rho, f))             # warm-up (activation buffers)
    cold_ms, warm_ms, net_ms = [], [], []
    for _ in range(reps):
        u = torch.zeros_like(f)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cold = simpgmg.pcg_solve(h, f, u, rtol=rtol, maxit=maxit)
        torch.cuda.synchronize()
        cold_ms.append((time.perf_counter() - t1) * 1e3)
        t1 = time.perf_counter()
        x = simpgmg.unet_input(h, rho, f)
        u0 = simpgmg.unet_output(h, net.forward(x))
        alpha = simpgmg.warm_start_scale(h, f, u0)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        warm = simpgmg.pcg_solve(h, f, u0, rtol=rtol, maxit=maxit, history_cap=1)
        torch.cuda.synchronize()
        warm_ms.append((time.perf_counter() - t1) * 1e3)
        net_ms.append((t2 - t1) * 1e3)
    # the prediction's energy-norm score on this case (compliance of the cold
    # solution as the scale): the squared energy-norm error of the scaled
    # start relative to the zero start's
    c = torch.dot(f, u).reshape(1)
    score = net.energy_step(h, x, rho.reshape(1, -1), f.reshape(1, -1), c, lr=0.0)
    return {"energy_score": score, "energy_err_ratio": float(np.sqrt(max(score, 0.0))),
            "cold_iters": cold["iters"], "cold_status": cold["status"],
            "cold_ms": round(float(np.mean(cold_ms)), 3),
            "warm_iters": warm["iters"], "warm_status": warm["status"],
            "warm_rel_res_true": warm["rel_res_true"],
            "warm_ms_total": round(float(np.mean(warm_ms)), 3),
            "warm_ms_network": round(float(np.mean(net_ms)), 3),
            "warm_initial_rel_res": warm["history"][0], "alpha": alpha}


def warmstart(n_train=2000, train_seconds=120.0, loss="energy"):
    """Learned warm start: the network of train_warm_start (trained on the
    given loss), then 100^3 uniform and random-field cantilevers (edge load)
    solved by FP32-GMG-PCG to 1e-6 from zero and from the scaled prediction.
    Command line: warmstart [energy|mse] [training seconds]."""
    dev = "cuda:0"
    if len(sys.argv) > 2 and sys.argv[1] == "warmstart":
        loss = sys.argv[2]
        if len(sys.argv) > 3:
            train_seconds = float(sys.argv[3])
    net, rec = train_warm_start(n_train, train_seconds, loss=loss)
    rec["tests"] = []
    n = 100
    tdims = (n, n, n)
    cases = [("uniform", workloads.uniform_rho(tdims))] + \
            [(f"grf{s}", workloads.grf_rho(tdims, s)) for s in range(5)]
    f = torch.tensor(workloads.edge_load(tdims), dtype=torch.float64, device=dev)
    for name, rho_np in cases:
        rho = torch.tensor(rho_np, dtype=torch.float64, device=dev)
        h = simpgmg.setup_hierarchy(simpgmg.default_options(*tdims, n_levels=0), rho)
        simpgmg.autotune(h)
        r = {"case": name, **warm_vs_cold(net, h, rho, f)}
        rec["tests"].append(r)
        h.close()
        print(json.dumps(r), flush=True)
    print(json.dumps(rec), flush=True)


def batchprof(fine_prec="bf16x3", reps=3):
    """Workload for a kernel trace of the stage-batched solve: the config-3
    batch (32 systems, 84 load cases) with the given fine-level precision,
    solved reps times after set-up (the first solve tunes the launch shapes
    and captures the graphs).  Command line: batchprof [bf16x3|f32]."""
    dev = "cuda:0"
    if len(sys.argv) > 2 and sys.argv[1] == "batchprof":
        fine_prec = sys.argv[2]
    dims, rhos, item_sys, fs = workloads.batch_config()
    opts = [simpgmg.default_options(*d, n_levels=0, dense_max=1000, fine_prec=fine_prec) for d in dims]
    b = simpgmg.setup_batch(opts, [torch.tensor(r, dtype=torch.float64, device=dev) for r in rhos])
    ft = [torch.tensor(f, dtype=torch.float64, device=dev) for f in fs]
    for rep in range(reps + 1):
        us = [torch.zeros_like(f) for f in ft]
        res, ms = simpgmg.pcg_solve_batch(b, item_sys, ft, us, rtol=1e-6, maxit=300, staged=True)
        print(json.dumps({"fine_prec": fine_prec, "rep": rep, "ms": round(ms, 3),
                          "converged": sum(r["status"] == "converged" for r in res),
                          "max_iters": max(r["iters"] for r in res)}), flush=True)


def unetprof():
    """Workload for a kernel trace of the warm-start network: 13 forward
    passes at 1 x 5 x 104^3 (the 100^3 mesh's padded node grid), then 13
    MSE training steps at 8 x 5 x 32^3, with the wall time of the last 10 of
    each."""
    dev = "cuda:0"
    net = simpgmg.UNet(seed=0)
    g = torch.Generator(device=dev).manual_seed(0)
    rec = {}
    x = torch.randn((1, 5, 104, 104, 104), dtype=torch.float32, device=dev, generator=g)
    for k in range(13):
        if k == 3:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        net.forward(x)
    torch.cuda.synchronize()
    rec["forward_104cube_ms"] = round((time.perf_counter() - t0) / 10 * 1e3, 3)
    x = torch.randn((8, 5, 32, 32, 32), dtype=torch.float32, device=dev, generator=g)
    t = torch.randn((8, 3, 32, 32, 32), dtype=torch.float32, device=dev, generator=g)
    for k in range(13):
        if k == 3:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        net.train_step(x, t, None, lr=1e-4)
    torch.cuda.synchronize()
    rec["train_step_8x32cube_ms"] = round((time.perf_counter() - t0) / 10 * 1e3, 3)
    print(json.dumps(rec), flush=True)


TRAFFIC_SHAPES = [(r, z) for r in (4, 8) for z in (2, 4, 8, 16, 32)]


def traffic(n=80, reps=20):
    """Workload for HBM-traffic counters: the 80^3 fine K.u in BF16X3 for
    every launch shape the autotuner can pick (TRAFFIC_SHAPES, in this order,
    reps launches each), then BF16 and FP64 at shape (4, 4), the
    level-1 stencil apply, and a plain device copy of 1 GiB (the calibration
    kernel: its FETCH_SIZE / WRITE_SIZE per dispatch are compared with the
    1 GiB it moves; at that size the 8 x 4 MiB of L2 cannot hold a useful
    part of the source)."""
    dev = "cuda:0"
    dims = (n, n, n)
    rho = torch.tensor(workloads.uniform_rho(dims), dtype=torch.float64, device=dev)
    h = simpgmg.setup_hierarchy(simpgmg.default_options(*dims, n_levels=4), rho)
    simpgmg.set_launch_shape(h, "bf16", 4, 4)           # no autotuning: the dispatch order
    simpgmg.set_launch_shape(h, "f64", 4, 4)            # of the K.u launches is fixed
    fixed = torch.tensor(workloads.cantilever_fixed(dims), device=dev).bool()
    u32 = torch.ones(fixed.numel(), dtype=torch.float32, device=dev).masked_fill_(fixed, 0)
    u64 = u32.double()
    y32, y64 = torch.empty_like(u32), torch.empty_like(u64)
    for r, z in TRAFFIC_SHAPES:
        simpgmg.set_launch_shape(h, "bf16x3", r, z)
        for _ in range(reps):
            simpgmg.apply_K(h, 0, "bf16x3", u32, y32)
    for prec, u, y in (("bf16", u32, y32), ("f64", u64, y64)):
        for _ in range(reps):
            simpgmg.apply_K(h, 0, prec, u, y)
    info = h.level_info(1)
    d = info["dims"]
    n1 = 3 * (d[0] + 1) * (d[1] + 1) * (d[2] + 1)
    u1 = torch.ones(n1, dtype=torch.float64, device=dev)
    y1 = torch.empty_like(u1)
    for _ in range(reps):
        simpgmg.apply_K(h, 1, "f64", u1, y1)
    a = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(4):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"dims": dims, "reps": reps, "copy_bytes": a.numel() * 4,
                      "bf16x3_shapes": TRAFFIC_SHAPES, "level1_nodes": n1 // 3}), flush=True)


def l1prof(reps=20):
    """Workload for counter profiles of the level-1 Galerkin operator from
    the element products: on the 80^3 and 128^3 cantilevers (rho = 0.5, the
    bench's 4 levels), reps STORE applications of level 1 at each chunk
    length in L1PROF_PLANES (3 and 8 planes: the tuned lengths at 80^3 and
    128^3), random input; then a 1 GiB device copy 4 times (the counter
    calibration, as in kuprof)."""
    dev = "cuda:0"
    for n in (80, 128):
        rho = torch.full((n * n * n,), 0.5, dtype=torch.float64, device=dev)
        h = simpgmg.setup_hierarchy(simpgmg.default_options(n, n, n), rho)
        m = 3 * (n // 2 + 1) ** 3
        g = torch.Generator(device=dev).manual_seed(n)
        u = torch.randn(m, dtype=torch.float64, device=dev, generator=g)
        y = torch.empty_like(u)
        for planes in L1PROF_PLANES:
            simpgmg.set_launch_shape(h, "level1", 1, planes)
            for _ in range(reps):
                simpgmg.apply_K(h, 1, "f64", u, y)
        torch.cuda.synchronize()
        h.close()
        print(json.dumps({"n": n, "reps": reps, "planes": L1PROF_PLANES}), flush=True)
    a = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(4):
        b.copy_(a)
    torch.cuda.synchronize()


L1PROF_PLANES = (3, 8)


def kuprof(reps=20):
    """Workload for counter profiles of the BF16-family fine K.u: on the 80^3
    and 256^3 cantilevers (rho = 0.5; the 256^3 one with 2 levels, only its
    level 0 is used), BF16 and then BF16X3 STORE launches, reps per launch
    shape the autotuner can pick (TRAFFIC_SHAPES, in this order), all-ones
    input on free DOFs; then a 1 GiB device copy 4 times (the counter
    calibration: its FETCH_SIZE / WRITE_SIZE per dispatch are compared with
    the 1 GiB it moves)."""
    dev = "cuda:0"
    for n in (80, 256):
        dims = (n, n, n)
        rho = torch.tensor(workloads.uniform_rho(dims), dtype=torch.float64, device=dev)
        h = simpgmg.setup_hierarchy(simpgmg.default_options(*dims, n_levels=2 if n > 128 else 4), rho)
        fixed = torch.tensor(workloads.cantilever_fixed(dims), device=dev).bool()
        u = torch.ones(fixed.numel(), dtype=torch.float32, device=dev).masked_fill_(fixed, 0)
        y = torch.empty_like(u)
        for prec in ("bf16", "bf16x3"):
            for rows, planes in TRAFFIC_SHAPES:
                simpgmg.set_launch_shape(h, prec, rows, planes)
                for _ in range(reps):
                    simpgmg.apply_K(h, 0, prec, u, y)
        torch.cuda.synchronize()
        h.close()
        print(json.dumps({"n": n, "reps": reps, "shapes": TRAFFIC_SHAPES}), flush=True)
    a = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(4):
        b.copy_(a)
    torch.cuda.synchronize()


if __name__ == "__main__":
    if len(sys.argv) > 2 and sys.argv[1] == "batch_graph":     # batch_graph PRECS [STEPS]
        batch_graph(tuple(sys.argv[2].split(",")), int(sys.argv[3]) if len(sys.argv) > 3 else 128)
        sys.exit(0)
    {"sizes": sizes, "hetero": hetero, "hetero_oracle": hetero_oracle, "large": large, "kernels": kernels, "batch": batch, "batch_graph": batch_graph,
     "e1": e1, "spectral_proxy": spectral_proxy, "robustness": robustness,
     "ablations": ablations, "sensitivity": sensitivity, "simp_schedule": simp_schedule,
     "warmstart": warmstart, "traffic": traffic, "kuprof": kuprof, "l1prof": l1prof,
     "batchprof": batchprof,
     "unetprof": unetprof}[sys.argv[1]]()
