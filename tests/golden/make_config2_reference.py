"""Writes tests/golden/config2_oracle.json: the oracle's reference solutions
of the heterogeneous 60^3 cantilevers of the precision study (Sec. 3.5 and
Sec. 4 M7/M8: errors of the reduced-precision solves are measured against an
FP64 solve).

For each penalisation p in {1, 2, 3} and seed in {0, 1}: rho from the seeded
Gaussian random field of workloads.grf_rho, the x = 0 face clamped, the unit
edge load; the oracle's FP64 PCG-GMG (4 levels, Chebyshev degree 2 on level
0, Jacobi 2 + 2 below, dense coarsest Cholesky) to rtol 1e-6 (its iteration
count is recorded) and then, continuing from that iterate, to rtol 1e-10.
Stored per case: the compliance c* = f . u* of the 1e-10 solve, u*^T K u*
(equal to c* up to the solve's residual), ||u*||_2, and the iterations.
The energy-norm error of any u follows from these without u*:
||u - u*||_K^2 = u^T K u - 2 f . u + c*, since K u* = f.

Calls only oracle/ and workloads/ (seeded inputs).  Run from the repository
root:  python tests/golden/make_config2_reference.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import krylov, mesh, multigrid  # noqa: E402

DIMS = (60, 60, 60)
CASES = [(p, seed) for p in (1, 2, 3) for seed in (0, 1)]


def main():
    out = {"_source": "Reference solves of the oracle (FP64 PCG-GMG, rtol 1e-10) for the "
                      "precision study of Sec. 3.5 and Sec. 4 (M7/M8 compare reduced-precision "
                      "compliance with FP64); written by tests/golden/make_config2_reference.py",
           "dims": list(DIMS), "cases": []}
    f = workloads.edge_load(DIMS)
    fixed = workloads.cantilever_fixed(DIMS).astype(bool)
    for p, seed in CASES:
        t0 = time.time()
        rho = workloads.grf_rho(DIMS, seed)
        E = mesh.simp_modulus(rho, p)
        oh = multigrid.build(DIMS, E, fixed, multigrid.Options(n_levels=4, penal=float(p)))
        K = oh.levels[0].K
        M = lambda r: multigrid.vcycle(oh, r)
        x6, st6, it6, _ = krylov.pcg(lambda v: K @ v, f, M, rtol=1e-6, maxit=500)
        xs, st, it, _ = krylov.pcg(lambda v: K @ v, f, M, x0=x6, rtol=1e-10, maxit=500)
        rec = {"p": p, "seed": seed, "compliance": float(f @ xs), "uKu": float(xs @ (K @ xs)),
               "u_norm": float(np.linalg.norm(xs)), "iters_rtol_1e-6": it6, "status_rtol_1e-6": st6,
               "iters_refine_to_1e-10": it, "status_1e-10": st,
               "rel_res_true": krylov.true_rel_residual(lambda v: K @ v, f, xs)}
        out["cases"].append(rec)
        print(json.dumps(rec), f"{time.time() - t0:.1f}s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config2_oracle.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
