"""Benchmark: FP32-GMG PCG solve of the 80^3 hex8 SIMP cantilever on one MI355X.

One step = setup_hierarchy + pcg_solve (cold start) of the 512k-element
cantilever (rho = 0.5, p = 3, x = 0 clamped, unit -z edge load), 4 levels,
rtol 1e-6 on the FP64 true residual, cap 200.  ``value`` is the mean solve
time in ms (HIP events around the solve on the solver's stream).  The line
also carries the roofline of the dominant kernel, timed with HIP events on
the stream it runs on, and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK = 78.6      # TFLOP/s without packed FP32 (256 CU x 64 lanes x 2 x 2.4 GHz)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=80, help="elements per axis of the cube")
    ap.add_argument("--fine-prec", default=os.environ.get("SGMG_FINE_PREC", "bf16x3"))
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ku256", action="store_true", help="skip the 256^3 K.u roofline")
    ap.add_argument("--no-compare", action="store_true", help="skip FP64-GMG and Jacobi-PCG comparisons")
    ap.add_argument("--warm-pairs", type=int, default=300,
                    help="solver-generated 32^3 training pairs for the warm-start comparison (0: skip)")
    ap.add_argument("--warm-train-s", type=float, default=20.0)
    return ap.parse_args()


PROFILE = os.path.join(ROOT, "profiles", "fine_ku_counters_256cube.md")
KU_SOURCE = os.path.join(ROOT, "paper_2604_26441_amd", "csrc", "kernels_mfma.hip")


def measured_profile(prec, shape):
    """Calibrated HBM bytes per launch and matrix-core busy fraction of the
    BF16-family fine K.u at 256^3 for the given precision and launch shape,
    from the committed rocprofv3 counter summary; None if the kernel source
    changed since the counters were taken or the row is missing."""
    import hashlib
    try:
        text = open(PROFILE).read()
        src = hashlib.sha1(open(KU_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    if shape is None or f"kernel_source_sha1: {src}" not in text:
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if (len(cells) >= 9 and cells[0] == "256^3" and cells[1] == prec and cells[2].isdigit()
                and (int(cells[2]), int(cells[3])) == tuple(shape)):
            return {"traffic": int(cells[6]), "mfma_util": float(cells[8])}
    return None


def oracle_solve(dims, levels, maxit=200):
    """The oracle's setup and PCG-GMG solve (rtol 1e-6) of the rho = 0.5
    cantilever of the given shape, on the calling thread; returns the timings
    (ms), the iterate, the outcome and the hierarchy."""
    import workloads
    from oracle import krylov, mesh, multigrid
    t0 = time.perf_counter()
    rho = workloads.uniform_rho(dims)
    fixed = workloads.cantilever_fixed(dims).astype(bool)
    f = workloads.edge_load(dims)
    E = mesh.simp_modulus(rho, 3)
    oh = multigrid.build(dims, E, fixed, multigrid.Options(n_levels=levels))
    t1 = time.perf_counter()
    K = oh.levels[0].K
    M = lambda r: multigrid.vcycle(oh, r)
    xo, st, it, _ = krylov.pcg(lambda v: K @ v, f, M, rtol=1e-6, maxit=maxit)
    t2 = time.perf_counter()
    return (t1 - t0) * 1e3, (t2 - t1) * 1e3, xo, st, it, oh, f


def cpu_baseline(n, gpu_u, gpu_iters, small):
    """The oracle (FP64 PCG-GMG on assembled SciPy CSR, 4 levels, the same
    Chebyshev / Jacobi smoothing and rtol 1e-6) solving the same n^3
    cantilever on one host thread: setup and the full solve timed
    separately.  Afterwards, untimed, the oracle's iterate is refined to rtol
    1e-10 and the GPU solution's errors against that reference are
    reported.  ``small`` lists the smaller meshes (shape, levels, GPU
    record) on which the oracle's setup and solve are timed the same way and
    set beside the GPU's."""
    import platform
    from threadpoolctl import threadpool_limits
    from oracle import krylov, multigrid
    dims = (n, n, n)
    others = []
    with threadpool_limits(limits=1):
        for sdims, lv, g in small:
            su, so, _, st, it, _, _ = oracle_solve(sdims, lv)
            others.append({"mesh": "x".join(map(str, sdims)), "levels": lv,
                           "setup_ms": round(su, 1), "solve_ms": round(so, 1), "iters": it,
                           "status": st, "gpu": g})
        su, so, xo, st, it, oh, f = oracle_solve(dims, 4)
        K = oh.levels[0].K
        M = lambda r: multigrid.vcycle(oh, r)
        xr, st_r, it_r, _ = krylov.pcg(lambda v: K @ v, f, M, x0=xo, rtol=1e-10, maxit=200)
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    base = {"value": round(so, 1), "unit": "ms", "cores": 1, "kind": "oracle",
            "sample": f"the whole oracle solve of the same {n}^3 cantilever to rtol 1e-6 "
                      f"({it} iterations, status {st}; GPU: {gpu_iters}), setup timed apart",
            "setup_ms": round(su, 1), "iters": it, "cpu": cpu,
            "nproc": os.cpu_count(), "host": platform.node(), "other_sizes": others}

    def errs(u):
        d = u - xr
        c, cr = float(f @ u), float(f @ xr)
        return {"compliance_rel": abs(c - cr) / abs(cr),
                "u_rel": float(np.linalg.norm(d) / np.linalg.norm(xr)),
                "energy_rel": float(np.sqrt(max(d @ (K @ d), 0.0) / (xr @ (K @ xr))))}
    err = {"reference": f"oracle PCG-GMG refined to rtol 1e-10 ({it + it_r} iterations)",
           "gpu": errs(gpu_u), "oracle_rtol_1e-6": errs(xo)}
    return base, err


def ku_roofline(n, prec, reps, tune=True):
    """The fine K.u (STORE) in the smoother precision on an n^3 cantilever
    (2-level hierarchy: only level 0 is used) at its fastest launch shape
    (the autotuner ranks shapes by a smoothing step, so the STORE form's
    shapes with 8 rows are timed here as well), timed with HIP events around
    reps back-to-back launches on the stream they run on; algorithmic bytes =
    read u + write y + read E/s."""
    import torch
    import workloads
    from paper_2604_26441_amd import simpgmg
    dev = torch.device("cuda:0")
    dims = (n, n, n)
    rho = torch.tensor(workloads.uniform_rho(dims), dtype=torch.float64, device=dev)
    h = simpgmg.setup_hierarchy(simpgmg.default_options(*dims, n_levels=2 if n > 128 else 4,
                                                        fine_prec=prec), rho)
    shape = simpgmg.autotune(h) if tune else None
    p = simpgmg.PRECISIONS[prec]
    dt = torch.float64 if p == simpgmg.F64 else torch.float32
    fixed = torch.tensor(workloads.cantilever_fixed(dims), device=dev).bool()
    uk = torch.ones(3 * (n + 1) ** 3, dtype=dt, device=dev).masked_fill_(fixed, 0)
    yk = torch.empty_like(uk)
    stream = torch.cuda.current_stream()
    if tune and prec in ("bf16", "bf16x3"):
        q = 1 if prec == "bf16x3" else 0
        best = None
        for cand in {tuple(shape[q]), (8, 8), (8, 16), (8, 32)}:
            simpgmg.set_launch_shape(h, prec, *cand)
            for _ in range(20):
                simpgmg.apply_K(h, 0, p, uk, yk)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(30):
                simpgmg.apply_K(h, 0, p, uk, yk)
            e1.record(stream)
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1)
            if best is None or t < best[0]:
                best = (t, cand)
        simpgmg.set_launch_shape(h, prec, *best[1])
        shape = list(shape)
        shape[q] = best[1]
    # steady state: the first launches on freshly allocated buffers of this
    # size run up to 20 % slower (clocks and address translation warming up)
    for _ in range(100):
        simpgmg.apply_K(h, 0, p, uk, yk)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        simpgmg.apply_K(h, 0, p, uk, yk)
    ev1.record(stream)
    torch.cuda.synchronize()
    us = ev0.elapsed_time(ev1) * 1e3 / reps
    es = 8 if p == simpgmg.F64 else 4
    nodes, nel = (n + 1) ** 3, n ** 3
    byts = 2 * 3 * nodes * es + nel * es
    h.close()
    return {"mesh": f"{n}^3", "us": round(us, 3), "bytes": byts, "GBs": round(byts / us / 1e3, 1),
            "GFLOPs": round(2 * 24 * 24 * nel / us / 1e3, 1),
            "shape": shape[1 if prec == "bf16x3" else 0] if shape else None}


def gpu_solve(dims, levels, fine_prec, reps=3):
    """Setup and PCG-GMG solve (rtol 1e-6, cap 200) of the rho = 0.5
    cantilever of the given shape on the GPU: one untimed warm-up, then the
    mean over reps of the setup wall time and of the solve time the library
    reports."""
    import torch
    import workloads
    from paper_2604_26441_amd import simpgmg
    dev = torch.device("cuda:0")
    rho = torch.tensor(workloads.uniform_rho(dims), dtype=torch.float64, device=dev)
    f = torch.tensor(workloads.edge_load(dims), dtype=torch.float64, device=dev)
    o = simpgmg.default_options(*dims, n_levels=levels, fine_prec=fine_prec)
    su, so = [], []
    for k in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = simpgmg.setup_hierarchy(o, rho)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        u = torch.zeros_like(f)
        res = simpgmg.pcg_solve(h, f, u, rtol=1e-6, maxit=200)
        h.close()
        if k:
            su.append((t1 - t0) * 1e3)
            so.append(res["solve_ms"])
    return {"setup_ms": round(float(np.mean(su)), 3), "solve_ms": round(float(np.mean(so)), 3),
            "iters": res["iters"], "status": res["status"], "fine_prec": fine_prec}


def progress(msg):
    """A progress line on stderr (stdout carries only the result line)."""
    print(f"bench.py: {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU; use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads
    from paper_2604_26441_amd import simpgmg

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = args.n
    dims = (n, n, n)
    rho = torch.tensor(workloads.uniform_rho(dims), dtype=torch.float64, device=dev)
    f = torch.tensor(workloads.edge_load(dims), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def opts(**kw):
        kw.setdefault("n_levels", args.levels)
        return simpgmg.default_options(*dims, **kw)

    def step(o, precond=2, maxit=200):
        t0 = time.perf_counter()
        h = simpgmg.setup_hierarchy(o, rho)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        u = torch.zeros_like(f)
        res = simpgmg.pcg_solve(h, f, u, rtol=1e-6, maxit=maxit, precond=precond)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        res["u"] = u
        return h, res, (t1 - t0) * 1e3, (t2 - t1) * 1e3

    o32 = opts(fine_prec=args.fine_prec)
    tuned = None
    if args.fine_prec in ("bf16", "bf16x3"):
        h = simpgmg.setup_hierarchy(o32, rho)      # launch-shape autotuning, untimed
        tuned = simpgmg.autotune(h)
        h.close()
    for _ in range(args.warmup):
        h, res, _, _ = step(o32)
        h.close()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    solve_ms, setup_ms, iters, status, relres = [], [], [], [], []
    for k in range(args.steps):
        h, res, su, _ = step(o32)
        solve_ms.append(res["solve_ms"])
        setup_ms.append(su)
        iters.append(res["iters"])
        status.append(res["status"])
        relres.append(res["rel_res_true"])
        last_u = res["u"]
        if k != args.steps - 1:
            h.close()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t_start) * 1e3
    progress(f"{args.steps} timed solves done, {float(np.mean(solve_ms)):.3f} ms each")

    # the fine K.u in the smoother precision on the bench mesh: 200
    # back-to-back launches on torch's current stream (the stream the library
    # launches on), HIP events around them; then the same launches one at a
    # time with 1 GiB written between them (the 256 MiB last-level cache holds
    # none of the operands when a launch starts)
    prec = simpgmg.PRECISIONS[args.fine_prec]
    dt = torch.float64 if prec == simpgmg.F64 else torch.float32
    fixed = torch.tensor(workloads.cantilever_fixed(dims), device=dev).bool()
    uk = torch.ones(3 * (n + 1) ** 3, dtype=dt, device=dev).masked_fill_(fixed, 0)
    yk = torch.empty_like(uk)
    for _ in range(5):
        simpgmg.apply_K(h, 0, prec, uk, yk)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.kernel_reps):
        simpgmg.apply_K(h, 0, prec, uk, yk)
    ev1.record(stream)
    torch.cuda.synchronize()
    ku_us = ev0.elapsed_time(ev1) * 1e3 / args.kernel_reps
    flush = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device=dev)
    cold = []
    for k in range(20):
        flush.fill_(float(k))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        simpgmg.apply_K(h, 0, prec, uk, yk)
        e1.record(stream)
        torch.cuda.synchronize()
        cold.append(e0.elapsed_time(e1) * 1e3)
    del flush
    ku_cold_us = float(np.mean(cold))
    es = 8 if prec == simpgmg.F64 else 4
    nodes, nel = (n + 1) ** 3, n ** 3
    ku_bytes = 2 * 3 * nodes * es + nel * es          # read u, write y, read E
    ku_flop = 2 * 24 * 24 * nel
    achieved = ku_bytes / (ku_us * 1e-6) / 1e9
    h.close()
    ku_big = ku_roofline(256, args.fine_prec, 200) if not args.no_ku256 else None

    progress("K.u timings done")
    extra = {}
    if not args.no_compare:
        h, r64, su64, _ = step(opts(fine_prec="f64"))
        h.close()
        h, rj, suj, _ = step(opts(fine_prec="f64"), precond=1, maxit=200)
        h.close()
        extra = {"fp64_gmg": {"solve_ms": round(r64["solve_ms"], 3), "iters": r64["iters"],
                              "status": r64["status"]},
                 "jacobi_pcg_cap200": {"solve_ms": round(rj["solve_ms"], 3), "iters": rj["iters"],
                                       "status": rj["status"], "rel_res_true": rj["rel_res_true"]}}

    if args.warm_pairs > 0:
        progress("warm-start training")
        # learned warm start on the same solve: network trained here on
        # solver-generated 32^3 random-field pairs, then zero start vs scaled
        # prediction, same tolerance
        from paper_2604_26441_amd import experiments
        net, rec = experiments.train_warm_start(args.warm_pairs, args.warm_train_s, progress=False)
        h = simpgmg.setup_hierarchy(o32, rho)
        extra["warm_start"] = {"train": rec, **experiments.warm_vs_cold(net, h, rho, f)}
        h.close()
        net.close()

    prof = measured_profile(args.fine_prec, ku_big["shape"]) if ku_big else None

    mean_solve = float(np.mean(solve_ms))
    line = {
        "metric": "PCG-GMG solve ms at 512k elems @1e-6 rel-res; K·u HBM GB/s; iters vs warm-start",
        "value": round(mean_solve, 3),
        "unit": "ms",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f64": "f64", "bf16": "bf16", "bf16x3": "f32"}[args.fine_prec],
        "data": "synthetic",
        "config": {"workload": f"hex8 SIMP cantilever {n}x{n}x{n} ({nel} elements), rho=0.5, p=3, "
                               f"FP32-GMG-PCG, {args.levels} levels, Chebyshev deg 2, rtol 1e-6, cap 200",
                   "fine_prec": args.fine_prec, "mfma_shape_bf16_bf16x3": tuned},
        "solve_ms_std": round(float(np.std(solve_ms)), 3),
        "setup_ms": round(float(np.mean(setup_ms)), 3),
        "iters": iters, "status": status, "rel_res_true": relres,
        "ku": {"kernel": "fine K.u (sgmg_apply_K level 0)", "mesh": f"{n}^3", "us": round(ku_us, 3),
               "GBs": round(achieved, 1), "GFLOPs": round(ku_flop / (ku_us * 1e-6) / 1e9, 1),
               "cold_us": round(ku_cold_us, 3),
               "cold_GBs": round(ku_bytes / (ku_cold_us * 1e-6) / 1e9, 1),
               "note": "the 14.8 MB working set stays in the 8 x 4 MiB L2 and 256 MiB MALL between "
                       "back-to-back launches; cold_* flush the MALL with a 1 GiB write first"},
        **extra,
    }
    if ku_big:
        a = ku_big["GBs"]
        line["roofline"] = {"bound": "hbm", "achieved": a, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": round(a / HBM_PEAK_GBS, 4),
                            "traffic": prof["traffic"] if prof else None,
                            "kernel": f"fine K.u {args.fine_prec}", "mesh": ku_big["mesh"],
                            "us": ku_big["us"], "bytes_per_launch": ku_big["bytes"],
                            "shape": ku_big["shape"],
                            "mfma_util": prof["mfma_util"] if prof else None,
                            "note": "256^3 cantilever (16.8 M elements, 474 MB per launch): beyond "
                                    "the caches, so HBM-bound; the bench mesh's figure is under ku"}
    if not args.no_cpu_baseline:
        u_host = last_u.cpu().numpy()
        progress("oracle timings (one host thread)")
        small = []
        for sdims, lv in (((16, 8, 8), 3), ((40, 40, 40), 4), ((60, 60, 60), 4)):
            g = gpu_solve(sdims, lv, args.fine_prec)
            small.append((sdims, lv, g))
        line["cpu_baseline"], line["error_vs_oracle"] = cpu_baseline(n, u_host, iters[-1], small)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
