/*
 * simpgmg.h - C ABI of the MI355X (gfx950) matrix-free Galerkin multigrid
 * PCG solver for 3D hex8 SIMP linear elasticity.
 *
 * Method (arXiv:2604.26441):
 *   Sec. 3.1 (Eq. simp_filter, Eq. state_eq): E_e = Emin + (E0 - Emin) rho_e^p,
 *     K = sum_e E_e K_e, solve the free-DOF system K_ff u_f = f_f.
 *   Sec. 3.2 (Eq. vcycle): V-cycle preconditioner.
 *   Sec. 3.3 (Eq. trilinear_weights, vector_prolongation, mf_matvec,
 *     galerkin_level1): 2:1 trilinear transfers, Dirichlet masks inherited by
 *     injection, matrix-free level 0, level 1 by local Galerkin aggregation,
 *     deeper levels by Galerkin triple products.
 *   Sec. 3.4 (Alg. cheb): Chebyshev-Jacobi smoother; Sec. 3.5: precision
 *     descent, BF16 semantics, power-iteration lambda_max estimates.
 *   Sec. 3.6: outer PCG, acceptance on the true relative residual.
 *
 * Conventions shared by every entry point
 *   Mesh: nx*ny*nz unit hexahedra.  Node (i,j,k) has index
 *     i + (nx+1)*(j + (ny+1)*k); DOF index 3*node + c, c in {x,y,z}.
 *     Element (ex,ey,ez) has index ex + nx*(ey + ny*ez).
 *   Vectors: device pointers in the full-DOF layout of their level, length
 *     3*(nx+1)*(ny+1)*(nz+1).  Fixed (Dirichlet) DOFs carry zeros on input
 *     and are written as zeros on output; the operators act as M K M with M
 *     the free-DOF selector, which is the free-DOF system K_ff in full-length
 *     form.
 *   Ownership: the caller allocates and owns every vector passed in.  The
 *     library allocates the hierarchy (operators, work vectors, scratch) in
 *     setup and frees it in sgmg_destroy.  No pointer passed in is retained
 *     after a call returns.
 *   Streams: every call is ordered on the given HIP stream (0 = the null
 *     stream).  sgmg_setup_hierarchy and sgmg_update_moduli synchronise the
 *     stream before returning; sgmg_pcg_solve synchronises once per outer
 *     iteration to read its scalars; sgmg_apply_K and sgmg_vcycle are
 *     asynchronous.  Calls on one hierarchy must not overlap (they share the
 *     hierarchy's work vectors).
 *   Errors: 0 = success; SGMG_EINVAL (-1) invalid argument or a mesh that
 *     cannot be coarsened to the requested depth; SGMG_EHIP (-2) a HIP runtime
 *     error; SGMG_ENOMEM (-3) device allocation failed; SGMG_EFACTOR (-4) the
 *     coarsest factorisation met a non-positive pivot after regularisation.
 *     sgmg_last_error() returns a thread-local message for the last failure.
 *     Non-convergence of a solve is not an error: it is reported in
 *     sgmg_solve_info.status.
 */
#ifndef SIMPGMG_H
#define SIMPGMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SGMG_EINVAL  (-1)
#define SGMG_EHIP    (-2)
#define SGMG_ENOMEM  (-3)
#define SGMG_EFACTOR (-4)

/* Arithmetic of an operator application.
 *   F64    : FP64 vectors and arithmetic.
 *   F32    : FP32 vectors, FP32 vector-ALU arithmetic.
 *   BF16   : FP32 vectors; element input tile rounded to BF16, element matrix
 *            exact in BF16, FP32 accumulation on MFMA, E_e applied in FP32
 *            (Sec. 3.5, BF16 numerical semantics).  Level 0 only.
 *   BF16X3 : FP32 vectors; the input tile is split into three BF16 terms whose
 *            sum carries the FP32 significand, each term multiplied on MFMA
 *            with FP32 accumulation (FP32-accurate).  Level 0 only.
 *   BF16X2 : as BF16X3 with two terms (about 16 significant bits of the
 *            input); runs on BF16X3's launch shape.  Level 0 only.        */
typedef enum { SGMG_F64 = 0, SGMG_F32 = 1, SGMG_BF16 = 2, SGMG_BF16X3 = 3,
               SGMG_BF16X2 = 4 } sgmg_prec;

/* Solve status (Sec. 3.6 failure classes). */
typedef enum {
  SGMG_CONVERGED = 0,  /* FP64 true relative residual below rtol            */
  SGMG_MAXIT = 1,      /* iteration cap reached                              */
  SGMG_STAGNATED = 2,  /* stagnation window enabled and tripped              */
  SGMG_NONFINITE = 3,  /* a non-finite scalar or residual appeared           */
  SGMG_BREAKDOWN = 4   /* p.q <= 0 or r.z <= 0                               */
} sgmg_status;

typedef struct {
  int nx, ny, nz;            /* elements per axis, each >= 2 (SGMG_EINVAL otherwise) */
  double nu, E0, Emin, penal;/* Poisson ratio 0.3, E0 1, Emin 1e-9, SIMP penalty p   */
  int input_is_modulus;      /* 0: the setup array is rho (SIMP map applied);
                                1: it is E_e directly                                */
  int n_levels;              /* >= 2; 0 = fewest levels whose coarsest free-DOF
                                count is <= dense_max (at most 8; if none is, all
                                levels down to one element per axis)                 */
  int fine_smoother;         /* 0 Chebyshev (Alg. cheb), 1 damped Jacobi             */
  int fine_degree;           /* Chebyshev degree / Jacobi sweeps on level 0 (2)      */
  int coarse_sweeps;         /* damped-Jacobi pre and post sweeps on levels >= 1 (2) */
  double cheb_alpha;         /* lower end of the Chebyshev interval, 1/30            */
  double jacobi_omega_max;   /* damping cap 0.5; omega = min(cap, 4/(3 lambda))      */
  double lambda_safety;      /* smoothers use lambda_safety * estimate (1.3)         */
  int power_iters_fine;      /* power iterations on level 0 (20)                     */
  int power_iters_coarse;    /* power iterations on levels >= 1 (10)                 */
  sgmg_prec fine_prec;       /* level-0 smoother/residual arithmetic                 */
  sgmg_prec level1_prec;     /* F64 or F32: storage and arithmetic of level 1 (the
                                paper's BF16 schedule, Eq. prec_schedule, uses F32;
                                its FP32-GMG runs F64)                               */
  int dense_max;             /* coarsest dense-solve limit on free DOFs (5000)       */
  int coarse_pcg_iters;      /* Jacobi-PCG steps of the coarsest solve when its
                                free-DOF count exceeds dense_max (80)                */
  uint64_t seed;             /* power-iteration start vector: SplitMix64(seed+level) */
  int flexible_beta;         /* 1: Polak-Ribiere beta in PCG, 0: Fletcher-Reeves     */
  int stag_window;           /* 0 = off; else stagnation window in iterations        */
  const double* lambda_override; /* host array of n_levels-1 raw estimates, or NULL  */
  int use_graphs;            /* 1: each PCG iteration (K.p, updates, V-cycle) is
                                replayed from a HIP graph captured once per
                                hierarchy; 0: direct launches (same results)      */
  int cycle_gamma;           /* cycle index: 1 V-cycle (default), 2 W-cycle (Sec. 4
                                E6(c)): every level whose coarser level is not the
                                coarsest approximates its coarse residual equation
                                by two coarser cycles, the second starting from
                                the first one's result; the coarsest is solved
                                once                                              */
  int stencil_form;          /* kernel of the Galerkin-level products (same
                                operator, sums in another order): 0 by level size
                                (default: the LDS-staged 27-offset form on levels
                                of >= 40000 nodes, the plane-split form below),
                                1 the LDS-staged form on every level, 2 the
                                plane-split form on every level, 3 as 0 except
                                that an FP64 level 1 above the coarsest applies
                                its operator from the child moduli of each
                                coarse element (Eq. galerkin_level1 evaluated
                                per element, sum/difference basis) and reads
                                the stored stencil only for the rows next to
                                Dirichlet DOFs or odd-axis ends (the stencil is
                                still assembled for the coarser products)       */
  int bf16_guard;            /* 1 (default): a PCG solve with the V-cycle and
                                fine_prec BF16 watches its progress (Sec. 3.5:
                                BF16 is used only under a guard, and Sec. 3.6:
                                acceptance is on the FP64 true residual); if a
                                step fails (p.q <= 0 or non-finite), r.z <= 0 or
                                non-finite, or the relative residual has not
                                dropped by guard_drop over the last guard_window
                                iterations, the level-0 smoothing switches to
                                BF16X3 (FP32-accurate) for the rest of the solve
                                and the recurrence restarts from the current
                                iterate with its FP64 true residual; the
                                hierarchy is BF16 again after the solve.
                                0: no guard                                       */
  int guard_window;          /* iterations of the progress test (50)              */
  double guard_drop;         /* required residual reduction over the window (10)  */
} sgmg_options;

typedef struct {
  int status;                /* sgmg_status                                          */
  int iters;                 /* outer PCG iterations (products with K on level 0)    */
  double rel_res_true;       /* ||f - K u||_2 / ||f||_2 in FP64 at exit              */
  double rel_res_recur;      /* recursive residual norm / ||f|| at exit              */
  double* history;           /* caller-owned host buffer of history_cap doubles, or
                                NULL; entry k = recursive ||r_k|| / ||f||            */
  int history_cap;
  double solve_ms;           /* wall time of the solve on the stream (HIP events)    */
  int fallback_iter;         /* iteration at which the BF16 guard switched the
                                smoothing to BF16X3, or -1                           */
} sgmg_solve_info;

typedef struct sgmg_hierarchy sgmg_hierarchy;

/* Fills *o with the paper's defaults (Table repro_defaults) for an nx*ny*nz
 * mesh: nu 0.3, E0 1, Emin 1e-9, p 3, 4 levels, Chebyshev degree 2, 2 coarse
 * sweeps, alpha 1/30, omega cap 0.5, 20/10 power iterations, level-0 F32,
 * level-1 F64, dense_max 5000, seed 0, lambda_safety 1.3, BF16 guard on (window
 * 50, drop 10). */
void sgmg_default_options(sgmg_options* o, int nx, int ny, int nz);

/* Builds the hierarchy for one frozen modulus field (Sec. 3.3, 3.5).
 *   rho_or_E : device, nx*ny*nz doubles in element order (rho in [0,1] or E_e).
 *   fixed_dof: device, 3*n_nodes bytes, nonzero = DOF fixed; NULL = clamp the
 *              x = 0 face (cantilever).
 *   out      : receives the handle (NULL on failure).
 * Work: SIMP map, masks by injection, diagonals, level-1 local Galerkin
 * aggregation, deeper Galerkin products, power iterations, coarsest dense
 * factorisation (explicit inverse of K_L + eps I, eps = max(mean diag * 1e-8,
 * 1e-14)).  When the coarsest free-DOF count exceeds dense_max, the coarsest
 * solve is instead coarse_pcg_iters steps of Jacobi-PCG on K_L from zero,
 * stopping early only on p.Kp <= 0 or r.z = 0 (Sec. 3.2, Table
 * repro_defaults); each step is two chip-wide launches.  Returns SGMG_EINVAL
 * if a coarse level would have no elements, or if the iterative coarsest
 * solve is needed and coarse_pcg_iters < 1. */
int sgmg_setup_hierarchy(const sgmg_options* opts, const double* rho_or_E,
                         const uint8_t* fixed_dof, void* stream, sgmg_hierarchy** out);

/* Re-assembles every E-dependent operator for a new field on the same mesh
 * and masks; lambda estimates are recomputed only if max_e E_e moved by more
 * than 10% since they were last estimated (Sec. 3.5). */
int sgmg_update_moduli(sgmg_hierarchy* h, const double* rho_or_E, void* stream);

/* y = M K^level M u.  level 0: the matrix-free fine operator in precision
 * prec (u, y are double* for F64, float* otherwise).  level >= 1: the stored
 * Galerkin operator; prec must be F64 (double vectors) or F32 (float vectors),
 * F32 only if that level is stored in FP32.  u and y must not alias. */
int sgmg_apply_K(const sgmg_hierarchy* h, int level, sgmg_prec prec,
                 const void* u, void* y, void* stream);

/* z = V(r): one V-cycle of Eq. vcycle on level 0 (double vectors). */
int sgmg_vcycle(const sgmg_hierarchy* h, const double* r, double* z, void* stream);

/* PCG on K u = f (Sec. 3.6).  precond: 0 none, 1 Jacobi (D^-1 of level 0),
 * 2 the V-cycle.  u: in = x0 (zeros for a cold start), out = the iterate at
 * exit.  Converged only if the FP64 true residual passes rtol; the recursive
 * residual triggers the check and a failed check replaces r by the true
 * residual.  info may be NULL.  The host may queue iteration k + 1 before it
 * has read iteration k's scalars (which the device writes into mapped host
 * memory); such an iteration writes only solver-owned buffers and is
 * discarded if iteration k ends the solve, so u, the status and the counts
 * are those of the plain loop.  Returns after all of its work on the stream
 * has completed.  Calls on one hierarchy must not overlap. */
int sgmg_pcg_solve(sgmg_hierarchy* h, int precond, const double* f, double* u,
                   double rtol, int maxit, sgmg_solve_info* info, void* stream);

/* Restarted right-preconditioned flexible GMRES on K u = f (Sec. 3.6: the
 * outer solver of the paper's BF16, large-scale and robustness runs), FP64.
 * precond as for sgmg_pcg_solve (2: the V-cycle, which may use any fine
 * precision); restart 1..63 (the paper's default 32, 50 for large scale).
 * Each cycle starts from the FP64 true residual; step j stores
 * z_j = M(v_j), forms w = K z_j, orthogonalises it against v_0..v_j
 * (classical Gram-Schmidt applied twice: the j + 1 dot products of a pass
 * are one kernel), and updates the Hessenberg QR with a Givens rotation on
 * the host (one readback per step).  A new Hessenberg entry below 1e-14
 * (happy breakdown), the residual estimate below rtol or `restart` steps
 * end the cycle with x += Z y.  Converged only if the next cycle's true
 * residual passes rtol.  info->iters counts Arnoldi steps; history holds the
 * true relative residual at each cycle start and the estimate after each
 * step.  Allocates (2 restart + 1) FP64 vectors on first use (kept by h). */
int sgmg_fgmres_solve(sgmg_hierarchy* h, int precond, int restart, const double* f, double* u,
                      double rtol, int maxit, sgmg_solve_info* info, void* stream);

/* Lanczos probe of the preconditioned operator M K (Sec. 4: the kappa_eff
 * screen of the robustness and BF16 spectral-proxy runs; Eq. kappa_bound).
 * M as for sgmg_pcg_solve (precond 0 none, 1 Jacobi, 2 the V-cycle in the
 * hierarchy's precision), K the FP64 fine operator.  Runs the preconditioned
 * Lanczos process in the M^-1 inner product, carrying w_j = M^-1 v_j:
 *   r_1 = g, z_1 = M r_1, b_1 = sqrt(r_1.z_1), v_1 = z_1/b_1, w_1 = r_1/b_1;
 *   s = K v_j, a_j = s.v_j, r = s - a_j w_j - b_j w_{j-1}, z = M r,
 *   b_{j+1} = sqrt(r.z), v_{j+1} = z/b_{j+1}, w_{j+1} = r/b_{j+1};
 * without reorthogonalisation, for m steps or until b_{j+1} <= breakdown *
 * max_i<=j |a_i| (an invariant subspace relative to the spectral scale).
 *   g     : device, 3*n_nodes doubles, the start vector (fixed DOFs ignored).
 *   alpha : host, m doubles: a_1..a_steps.
 *   beta  : host, m doubles: beta[j] = b_{j+2}, the norm after step j; the
 *           first steps-1 are the off-diagonals of the tridiagonal T.
 *   steps : out, number of steps taken.
 *   ritz  : host, 2 doubles or NULL: smallest and largest eigenvalue of T
 *           (Sturm bisection); kappa_eff = ritz[1] / ritz[0].
 * Overwrites the solver's work vectors; synchronises the stream twice per
 * step (the dot products are read back).  Returns SGMG_EINVAL if g.Mg <= 0
 * or a coefficient is not finite. */
int sgmg_lanczos(sgmg_hierarchy* h, int precond, int m, const double* g, double breakdown,
                 double* alpha, double* beta, int* steps, double* ritz, void* stream);

/* Autotuner of the fine operators' launch shape: times each candidate
 * (element rows per wave tile: 4, 8; owned node planes per wave: 2, 3, 4,
 * 6, 8, 16, 32) on this hierarchy's mesh for the BF16, BF16X3 and FP64 kernels
 * (the BF16 family in the smoothing epilogue, FP64 as a plain product),
 * keeps the fastest in h and in a process-wide cache keyed by (nx, ny, nz,
 * variant) that later setups of the same mesh read.  shape_out (host, 6
 * ints, may be NULL) receives (rows, planes) for BF16, BF16X3, then FP64;
 * for FP64 the vector-ALU node kernel is a candidate too, reported as (0, 0),
 * and so are the vector-ALU sum-factorised tiles with 2 .. 32 planes,
 * reported as (1, planes) ((1, 4) is the FP64 choice of an untuned mesh).  When
 * the hierarchy holds the level-1 element products (stencil_form 0 or 3,
 * FP64 level 1 above the coarsest) it also times level 1 from the stored
 * stencil against the products with 1 to 6 and 8 planes and keeps the faster
 * (with stencil_form 3 the products stay); that choice is kept in the same
 * cache (later stencil_form 0 setups of the mesh read it) and not reported.
 * Allocates four temporary vectors and synchronises the stream.  Within one
 * kernel the launch shape changes only which wave computes a node, never the
 * arithmetic: results are bitwise identical.  The three FP64 kernels agree
 * to rounding (the sum-factorised product and the node kernel order the
 * element sums differently from the matrix-core one). */
int sgmg_autotune(sgmg_hierarchy* h, int* shape_out, void* stream);
/* Pins the launch shape of one fine-operator variant (0 BF16, 1 BF16X3, 2
 * FP64) on h, e.g. to reuse a shape tuned earlier: rows 4 or 8, planes >= 1;
 * FP64 also accepts (0, 0), the vector-ALU node kernel, and (1, planes >= 1),
 * the vector-ALU kernel with the element product in sum-factorised form.
 * Variant 3 selects how level 1 is applied on a hierarchy that holds its
 * element products (stencil_form 0 or 3, FP64 level 1 above the coarsest):
 * (0, any) the stored stencil, (1, planes >= 1) the products.  Returns
 * SGMG_EINVAL for other values.  No device work. */
int sgmg_set_launch_shape(sgmg_hierarchy* h, int variant, int rows, int planes);

/* Introspection for tests and reports. */
int sgmg_num_levels(const sgmg_hierarchy* h);
/* dims[3] elements of level l, free DOF count, raw lambda estimate. */
int sgmg_level_info(const sgmg_hierarchy* h, int level, int* dims, int* n_free, double* lambda);
/* Copies the level's 27-point block stencil (level >= 1) to a host buffer of
 * 243*n_nodes doubles laid out [o][d][d'][node], o = (ox+1)+3(oy+1)+9(oz+1),
 * entry = K[3*node+d, 3*(node+o)+d']. */
int sgmg_copy_stencil(const sgmg_hierarchy* h, int level, double* host_out);
/* Copies diag(K^level) (zeros on fixed DOFs) to a host buffer. */
int sgmg_copy_diagonal(const sgmg_hierarchy* h, int level, double* host_out);

/* ---- Batched persistent solve (extension: many uneven systems, one launch) ----
 * Not a passage of the paper: many independent cantilevers and load cases
 * solved by one persistent kernel launch replayed from a captured HIP graph.
 * Each workgroup takes (system, load case) work items from a device queue,
 * largest systems first, and runs the complete FP64-outer PCG with the
 * V-cycle (FP32 Chebyshev on level 0, FP64 Jacobi on the Galerkin levels,
 * dense coarsest solve) of its item at block level, with the same acceptance
 * rule as sgmg_pcg_solve.  The block size is picked by timing 256 and 512
 * threads on the first solve of a batch. */
typedef struct sgmg_batch sgmg_batch;

/* Builds one hierarchy per system with sgmg_setup_hierarchy.
 *   opts      : host array of nsys options (each with its own mesh).
 *   rho_or_E  : host array of nsys device pointers (element fields).
 *   fixed_dof : host array of nsys device masks, NULL entries (or NULL) for
 *               the cantilever clamp.
 * Returns SGMG_EINVAL if a system's coarsest level exceeds dense_max (the
 * batched V-cycle has only the dense coarsest solve) or its cycle_gamma is
 * not 1.                                                                   */
int sgmg_setup_batch(int nsys, const sgmg_options* opts, const double* const* rho_or_E,
                     const uint8_t* const* fixed_dof, void* stream, sgmg_batch** out);

/* Solves nitems load cases: item i is system item_sys[i] with right-hand
 * side f[i] and iterate u[i] (host arrays of device pointers, full-DOF
 * layout of that system; u[i]: in x0, out solution).  infos (host, nitems,
 * may be NULL) receives each item's status, iterations and residuals;
 * *total_ms (may be NULL) the wall time of the launch.  Work vectors are
 * allocated on the first call for an item set and reused.  Synchronises. */
int sgmg_pcg_solve_batch(sgmg_batch* b, int nitems, const int* item_sys, const double* const* f,
                         double* const* u, double rtol, int maxit, sgmg_solve_info* infos,
                         double* total_ms, void* stream);

/* The same items solved stage by stage: every stage of the outer PCG (Sec.
 * 3.6) and of the V-cycle (Eq. vcycle) is one launch over all items, with as
 * many workgroups per item as its level has work (so the whole device works
 * on each stage, whatever the item sizes).  Two captured graphs are replayed
 * from a host loop: a prologue (r = f - K u in FP64, V-cycle, p = z, r.z)
 * and one PCG iteration (q = K p, alpha, x and r, V-cycle, beta, p); per-item
 * flags copied in before each replay select the items that take part.  After
 * every iteration the host reads each item's scalars; an item whose
 * recursive residual passes rtol runs the prologue, which is its FP64
 * true-residual check and, if that fails, its restart (beta = 0).  Same
 * algorithm and acceptance as sgmg_pcg_solve with Fletcher-Reeves beta.
 * Level operators: level 0 inside the V-cycle on the BF16X3 MFMA operator
 * when every item's system has fine_prec BF16X3 (else the FP32 vector-ALU
 * node operator), the Galerkin levels on the FP64 stored stencils, the
 * outer q = K p on the FP64 MFMA operator; the two MFMA launch shapes and the
 * stencil form of each Galerkin level are timed on the item set at its first
 * call and the fastest kept.  Reductions
 * per item in a fixed order.  All systems must share the smoothing step
 * counts.  Work vectors, tables and graphs are built on the first call for
 * an item set.  *total_ms: wall time of the whole solve on the stream.
 * Synchronises once per iteration. */
int sgmg_pcg_solve_batch_staged(sgmg_batch* b, int nitems, const int* item_sys,
                                const double* const* f, double* const* u, double rtol, int maxit,
                                sgmg_solve_info* infos, double* total_ms, void* stream);

/* The stage-by-stage solve of sgmg_pcg_solve_batch_staged with the
 * iteration control on the device, so that one graph launch runs the whole
 * solve: the launch holds the prologue, a decision kernel (|f|, the first
 * residual test, u = 0 where f = 0) and steps PCG iterations, each followed
 * by a decision kernel (breakdown and residual tests), the prologue for the
 * items whose recursive residual passed (their FP64 true-residual check and
 * restart) and a second decision kernel (the outcome of the check, the next
 * iteration's flags); at its end, once no item iterates, the prologue gives
 * the true residual of the items that stopped without one.  Items that
 * stopped keep no flag: their blocks return at once.  The tests are those of
 * the host loop of the staged solve, item by item, so every item's status,
 * iterations, residuals and u are bitwise those of
 * sgmg_pcg_solve_batch_staged.  steps: iterations per launch (even, 2..1024);
 * when an item still iterates after them, a further launch of steps
 * iterations follows (*launches, may be NULL, receives the number of
 * launches).  The two graphs (first launch, further launches) are captured
 * on the first call for an item set, rtol, maxit and steps, and kept.
 * Arguments otherwise as sgmg_pcg_solve_batch_staged; *total_ms covers all
 * launches.  Synchronises once per launch. */
int sgmg_pcg_solve_batch_graph(sgmg_batch* b, int nitems, const int* item_sys,
                               const double* const* f, double* const* u, double rtol, int maxit,
                               int steps, sgmg_solve_info* infos, int* launches, double* total_ms,
                               void* stream);

/* The same items solved by nworkers host threads (1..16), each with a HIP
 * stream of its own: a worker takes whole systems, largest DOFs x load
 * cases first, and solves that system's items in item order with
 * sgmg_pcg_solve (the V-cycle preconditioner; the system's hierarchy, its
 * work vectors and its captured iteration graphs are used by one worker at
 * a time).  Each item's result is bitwise that of a lone sgmg_pcg_solve
 * from the same u.  infos (host, nitems, may be NULL; a history buffer in
 * an entry is filled) and *total_ms (host wall time) as above.  The caller's
 * stream is synchronised before the workers start; all work has finished
 * when the call returns.  The first failing solve's error is returned. */
int sgmg_pcg_solve_batch_concurrent(sgmg_batch* b, int nitems, const int* item_sys,
                                    const double* const* f, double* const* u, double rtol,
                                    int maxit, int nworkers, sgmg_solve_info* infos,
                                    double* total_ms, void* stream);

/* Borrowed handle of system s (owned by the batch), e.g. for single solves. */
sgmg_hierarchy* sgmg_batch_hierarchy(sgmg_batch* b, int s);
/* Block size chosen by the autotuner (0 before the first solve). */
int sgmg_batch_block_size(const sgmg_batch* b);
/* Work memory of one batch item (host arithmetic only, no device work): for
 * a hierarchy of L levels (2..8) with level_dofs[l] full-DOF vector lengths
 * and nL free coarsest DOFs, the byte offset and size of each sub-buffer (in
 * order: r, z, p, q, t in FP64 and b, d, r, x[0], x[1] in FP32 on level 0;
 * b, x[0], x[1], r in FP64 on each level 1..L-1; the coarsest right-hand
 * side, max(nL, 1) doubles) into offsets and sizes (10 + 4 (L - 1) + 1
 * entries each, either may be NULL); every offset is a multiple of 256.
 * Returns the allocation size the batched solve reserves per item, or 0 for
 * invalid arguments. */
size_t sgmg_batch_item_layout(int L, const int* level_dofs, int nL, size_t* offsets,
                              size_t* sizes);
void sgmg_batch_destroy(sgmg_batch* b);

/* ---- Learned warm start (extension: a 3D U-Net predicts the initial guess) ----
 * Not a passage of the paper.  Network on the node grid padded to multiples
 * of 8 (volume N x C x D x H x W, x fastest; D, H, W = padded z, y, x node
 * counts): e1 = relu(c1(x)), e2 = relu(c2(pool e1)), e3 = relu(c3(pool e2)),
 * b = relu(c4(pool e3)), d3 = relu(c5(up b)) + e3, d2 = relu(c6(up d3)) + e2,
 * d1 = relu(c7(up d2)) + e1, y = c8(d1); c1..c7 3x3x3 convolutions with
 * channels 5->16->32->64->128->64->32->16, c8 1x1x1 16->3, pool = 2x2x2 mean,
 * up = nearest x2.  Weights are rounded to BF16 for compute (FP32 master
 * copy for Adam), accumulation is FP32; the 3x3x3 convolutions run on the
 * matrix cores with the FP32 activations split exactly into three BF16
 * terms, so every product is exact and only the FP32 sums round.  Input channels: density averaged to
 * nodes, load / max|f| (3), clamp mask.  The prediction's scale is set by
 * sgmg_warm_start_scale, and PCG-GMG to the same tolerance is both fallback
 * and judge of the result. */
typedef struct sgmg_unet sgmg_unet;
int sgmg_unet_create(uint64_t seed, sgmg_unet** out);   /* He-normal init, zero bias */
int sgmg_unet_num_params(void);
/* Host buffer, per layer w[co][ci][kz][ky][kx] then b[co] (FP32). */
int sgmg_unet_set_params(sgmg_unet* u, const float* host, void* stream);
int sgmg_unet_get_params(sgmg_unet* u, int quantized, float* host, void* stream);
/* out (device, N x 3 x D x H x W) = network(in (device, N x 5 x D x H x W)). */
int sgmg_unet_forward(sgmg_unet* u, int N, int D, int H, int W, const float* in, float* out,
                      void* stream);
/* Masked MSE sum(m (y - t)^2) / sum(m) (mask N x D x H x W broadcast over the
 * 3 channels, NULL = all ones), its gradients (host, parameter layout), no
 * update. */
int sgmg_unet_grad(sgmg_unet* u, int N, int D, int H, int W, const float* in, const float* target,
                   const float* mask, float* loss, float* grads_host, void* stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) on the same loss; *loss before
 * the step.  Synchronises. */
int sgmg_unet_train_step(sgmg_unet* u, int N, int D, int H, int W, const float* in,
                         const float* target, const float* mask, float lr, float* loss,
                         void* stream);
/* Energy-norm training score (the error the scaled warm start leaves):
 * for sample n, u_n = the output's 3 channels on the first Nz x Ny x Nx
 * voxels of h's node grid as a DOF vector (zero on clamped DOFs); with
 * a = f_n.u_n, b = u_n.K_n u_n and c = cstar[n] = f_n.u*_n (the compliance),
 * score 1 - a^2 / (b c) = ||(a/b) u_n - u*_n||_K^2 / ||u*_n||_K^2 (1 when
 * b <= 0).  *loss (host) = mean score before the update.  K_n is h's fine
 * operator with the element field rho_or_E + n * n_elements, read as
 * sgmg_setup_hierarchy reads its input (h's SIMP map).  in (device,
 * N x 5 x D x H x W, D, H, W >= h's node counts z, y, x), rho_or_E (device,
 * N x n_elements), f (device, N x 3 n_nodes), cstar (device, N), grads_host
 * (host, parameter layout, may be NULL).  lr > 0: one Adam step follows;
 * lr = 0: gradients only.  Synchronises.  SGMG_EINVAL for NULL inputs, a
 * negative lr or a volume smaller than the node grid. */
int sgmg_unet_energy_step(sgmg_unet* u, const sgmg_hierarchy* h, int N, int D, int H, int W,
                          const float* in, const double* rho_or_E, const double* f,
                          const double* cstar, float lr, float* loss, float* grads_host,
                          void* stream);
/* Network input for hierarchy h's mesh: rho (device, elements), f (device,
 * DOFs) -> in (device, 5 x Dp x Hp x Wp, zero padded). */
int sgmg_unet_input(const sgmg_hierarchy* h, const double* rho, const double* f, int Dp, int Hp,
                    int Wp, float* in, void* stream);
/* Network output (device, 3 x Dp x Hp x Wp) -> u0 (device, DOFs, FP64, zero on
 * clamped DOFs). */
int sgmg_unet_output(const sgmg_hierarchy* h, const float* out, int Dp, int Hp, int Wp, double* u0,
                     void* stream);
/* Training target for a solved displacement u (device, DOFs): t (device,
 * 3 x Dp x Hp x Wp) = u / max|u| on the mesh nodes, 0 in the padding; mask
 * (device, Dp x Hp x Wp, may be NULL) = 1 on the mesh nodes. */
int sgmg_unet_target(const sgmg_hierarchy* h, const double* u, int Dp, int Hp, int Wp, float* t,
                     float* mask, void* stream);
/* u0 <- alpha u0 with alpha = (f . u0) / (u0 . K u0), the minimiser of the
 * energy norm of the error along u0; *alpha (host, may be NULL). */
int sgmg_warm_start_scale(sgmg_hierarchy* h, const double* f, double* u0, double* alpha,
                          void* stream);
/* For callers that cannot allocate device memory (code under HIP stream
 * capture, serving loops, harnesses that forbid hipMalloc): the same scaling
 * as sgmg_warm_start_scale, with the same kernels and summation order, so u0
 * and alpha are bitwise those of sgmg_warm_start_scale.  Its reduction
 * partials and scalars live in a fixed library array of 64 Ki + 32 doubles
 * (512 KiB) per GPU, held until the process ends, instead of the hierarchy's
 * workspace; K u0 is reduced without being stored.  Nothing is allocated and
 * nothing synchronises: the call is stream-ordered and returns at once.
 *   f, u0     device, 3*n_nodes FP64 of h's level 0; u0 is scaled in place.
 *   alpha_dev device pointer to one double that receives alpha, or NULL.
 *   Call with h's device current.  Calls that overlap on one GPU (another
 *   stream, another thread, another hierarchy) share the array and race.
 *   SGMG_EINVAL for NULL arguments or a mesh whose reductions need more than
 *   65,536 block partials (about 255^3 elements with the vector-ALU FP64
 *   operator); SGMG_EHIP if the array's device address cannot be obtained. */
int sgmg_warm_start_scale_noalloc(const sgmg_hierarchy* h, const double* f, double* u0,
                                  double* alpha_dev, void* stream);
void sgmg_unet_destroy(sgmg_unet* u);

void sgmg_destroy(sgmg_hierarchy* h);
/* ---- SIMP outer loop (Sec. 3.1, Eq. simp_filter) -----------------------------
 * Design density rho (element field, x-fastest, FP64 on the device) ->
 * filtered rho~ = F rho -> physical rhohat = H(rho~) -> E = Emin + (E0 -
 * Emin) rhohat^p, one frozen field per linear solve.  The filter and
 * projection forms are the standard ones (the paper's parameters are in a
 * companion paper): F the linear cone filter w(e, i) = max(0, rmin - |c_e -
 * c_i|) over element centres, normalised by the row sum (rmin <= 1: no
 * filter); H(x) = (tanh(b eta) + tanh(b (x - eta))) / (tanh(b eta) +
 * tanh(b (1 - eta))), b = 0 the identity.  Compliance sensitivities are
 * carried back through H' and F^T; the optimality-criteria update rho_new =
 * clamp(rho sqrt(max(-dc, 0) / (lam dv)), rho -/+ move, [0, 1]) finds lam by
 * bisection on [0, 1e9] until (l2 - l1) <= oc_tol (l1 + l2) so that the
 * physical volume is volfrac * n_el. */
typedef struct {
  int nx, ny, nz;            /* elements per axis                                   */
  double penal, E0, Emin;    /* SIMP map (must equal the hierarchy's)               */
  double volfrac;            /* target physical volume fraction                     */
  double move;               /* OC move limit                                       */
  double rmin;               /* filter radius in elements (<= 1: no filter)         */
  double beta, eta;          /* projection sharpness (0: none) and threshold        */
  double oc_tol;             /* bisection stop (l2 - l1) <= oc_tol (l1 + l2)        */
  int oc_max_halvings;
} sgmg_simp_params;

typedef struct {
  double compliance;         /* f . u = sum_e E_e u_e^T K_e u_e of the solved state   */
  double volume;             /* physical volume of the updated design                 */
  double lambda;             /* OC multiplier                                         */
  double max_change;         /* max_e |rho_new - rho|                                 */
  int pcg_status, pcg_iters;
  double rel_res_true, solve_ms;
} sgmg_simp_info;

typedef struct sgmg_simp sgmg_simp;

/* Defaults: p 3, E0 1, Emin 1e-9, volfrac 0.5, move 0.2, rmin 1.5, beta 0,
 * eta 0.5, oc_tol 1e-9, 200 halvings. */
void sgmg_simp_default_params(sgmg_simp_params* p, int nx, int ny, int nz);
/* Allocates the state (filter row sums and four element fields); SGMG_EINVAL
 * for parameters outside their ranges (rmin in (0, 16]). */
int sgmg_simp_create(const sgmg_simp_params* p, void* stream, sgmg_simp** out);
void sgmg_simp_destroy(sgmg_simp* s);
/* rhohat = H(F rho), kept in s (and copied to rhohat, device, if not NULL). */
int sgmg_simp_physical(sgmg_simp* s, const double* rho, double* rhohat, void* stream);
/* From the state u (device, 3*n_nodes) of the last physical field: the
 * compliance (host), and the design sensitivities dc = dc/drho and dv =
 * dV/drho (device, optional) that the OC update uses.  h supplies K_e and
 * must have the same mesh.  SGMG_EINVAL if sgmg_simp_physical has not run. */
int sgmg_simp_sensitivity(sgmg_simp* s, const sgmg_hierarchy* h, const double* u,
                          double* compliance, double* dc, double* dv, void* stream);
/* One OC update of rho (device, in place) from the last sensitivities; the
 * outputs (host, optional) are the multiplier, the physical volume at it and
 * the largest density change.  Reads back one scalar per halving. */
int sgmg_simp_oc_update(sgmg_simp* s, double* rho, double* lambda, double* volume,
                        double* max_change, void* stream);
/* One SIMP iteration: physical field, sgmg_update_moduli (which re-estimates
 * the smoother spectra only when max E moved by more than 10 %), the PCG
 * solve (precond as for sgmg_pcg_solve: 2 the V-cycle, 1 Jacobi) from the u
 * passed in (a warm start from the previous design), sensitivities and the
 * OC update of rho.  The hierarchy must have been set up with
 * input_is_modulus 0 and the same penal, E0 and Emin.  A PCG solve that
 * does not converge is reported in info, not as an error. */
int sgmg_simp_step(sgmg_simp* s, sgmg_hierarchy* h, int precond, double* rho, const double* f,
                   double* u, double rtol, int maxit, sgmg_simp_info* info, void* stream);

const char* sgmg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SIMPGMG_H */
