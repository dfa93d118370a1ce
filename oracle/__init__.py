"""CPU FP64 oracle for the matrix-free Galerkin GMG-PCG solver.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import, call or execute anything in this
package; the product library never does, and the product never falls back to
it.  It shares no code with the HIP path.

Modules: hex8 (element stiffness), mesh (numbering, BCs, SIMP map, assembly),
transfer (trilinear P, injection), galerkin (level-1 local aggregation and
explicit triple products), smoothers (diagonal, power iteration, Chebyshev,
damped Jacobi), multigrid (hierarchy, V-cycle, coarsest solve), krylov (PCG,
FGMRES),
bf16 (BF16 semantic model), rng (SplitMix64), unet (conv3d reference),
spectral (Lanczos kappa_eff probe of M K), simp (density filter, Heaviside
projection, compliance sensitivities, OC update).

Parity status: every function is pinned by tests/test_oracle_*.py against
closed forms, invariants, printed values of the paper or library routines.
"""
