// Host interface of the stage-batched PCG-GMG kernels (kernels_bstage.hip).
#pragma once
#include "batch.hpp"

namespace sgmg {

// Per-item device scalars, kBsScalars doubles per item.
enum BsScalar {
  kBsFF = 0,      // f.f
  kBsRR = 1,      // r.r of the last update (prologue: of the true residual)
  kBsPQ = 2,      // p.q
  kBsAlpha = 3,   // rz / p.q (0 when p.q is not positive and finite)
  kBsRZ = 4,      // r.z of the current search direction
  kBsRZNew = 5,   // r.z of the last V-cycle
  kBsBeta = 6,
  kBsScalars = 8
};

// A stage grid: entry b = (item, local block) of workgroup b; the entries of
// one item are contiguous, starting at start[item], count[item] of them.
struct BsTable {
  const int2* blk = nullptr;
  int n = 0;
  const int* start = nullptr;
  const int* count = nullptr;
};

struct BsArgs {
  const BSys* sys;
  const BItem* items;
};

int bs_threads();
int bs_coarse_rows();
void bs_fine64_res(const BsArgs& a, const BsTable& t, const int* flags, double* part, hipStream_t s);
void bs_fine64_store_dot(const BsArgs& a, const BsTable& t, const int* flags, double* part,
                         hipStream_t s);
void bs_finalize(const BsTable& t, int nitems, int nv, const double* part, const int* flags,
                 int what, double* scal, hipStream_t s);
void bs_update_xr(const BsArgs& a, const BsTable& t, const int* flags, const double* scal,
                  double* part, hipStream_t s);
void bs_entry(const BsArgs& a, const BsTable& t, const int* flags, hipStream_t s);
void bs_dot_rz(const BsArgs& a, const BsTable& t, const int* flags, int set_p, double* part,
               hipStream_t s);
void bs_update_p(const BsArgs& a, const BsTable& t, const int* flags, const double* scal,
                 hipStream_t s);
void bs_smooth0(const BsArgs& a, const BsTable& t, const int* flags, int post, int k, int cin,
                int last, hipStream_t s);
void bs_resid0(const BsArgs& a, const BsTable& t, const int* flags, int cin, hipStream_t s);
void bs_restrict(const BsArgs& a, const BsTable& t, const int* flags, int l, hipStream_t s);
void bs_coarse(const BsArgs& a, const BsTable& tg, const BsTable& tm, const int* flags,
               hipStream_t s);
void bs_prolong(const BsArgs& a, const BsTable& t, const int* flags, int l, int cfine, int ccoarse,
                hipStream_t s);
// Level 0 on the BF16X3 MFMA operator: the tile grid of a mesh for launch
// shape (rows, zchunk) as (ntx, nty, ntiles, blocks), and the stage launch
// (mode EPI_SMOOTH with post / k / last as bs_smooth0, or EPI_RESID) over a
// table of (item, block) entries with geo[item] = that item's grid.
int4 bs_mfma_geometry(const Grid& g, int rows, int zchunk);
// Galerkin level l on the row-split stencil form: blocks of a level grid, and
// the stage launch (mode EPI_SMOOTH: damped-Jacobi step, or EPI_RESID) over a
// table of (item, block) entries.
int bs_stencil_blocks(const Grid& g);
void bs_stencil(const BsArgs& a, const BsTable& t, const int* flags, int l, int mode, int cin,
                hipStream_t s);
// The same stages on the LDS-staged stencil form (one block per 64 nodes).
int bs_stencil_s_blocks(const Grid& g);
void bs_stencil_s(const BsArgs& a, const BsTable& t, const int* flags, int l, int mode, int cin,
                  hipStream_t s);
void bs_fine_mfma(const BsArgs& a, const BsTable& t, const int4* geo, const int* flags, int rows,
                  int zchunk, int mode, int post, int k, int cin, int last, hipStream_t s);
// The outer FP64 q = K p on the FP64 MFMA operator (rows 4 or 8) or the
// vector-ALU sum/difference-basis operator (rows 1, tiles of rows 4), with
// the p.q block partials in part (one per table entry).
void bs_fine_mfma64_store_dot(const BsArgs& a, const BsTable& t, const int4* geo, const int* flags,
                              int rows, int zchunk, double* part, hipStream_t s);
void bs_fine_sf64_store_dot(const BsArgs& a, const BsTable& t, const int4* geo, const int* flags,
                            int zchunk, double* part, hipStream_t s);

// Device-side iteration control of the one-launch solve: per item the
// status (-1 while iterating, else the sgmg_status), the iteration count, |f|,
// the recurrence and the true relative residual (-1 until computed), a flag
// for f = 0 (u is then zeroed), and the iteration index in two slots (slot
// s & 1 is current in step s; the step's last kernel writes the other).
struct BsLoop {
  int* status;
  int* iters;
  double* nf;
  double* rel;
  double* rel_true;
  int* zero;
  int* it;
};
// Sets every item up for the prologue (flags [0, n) = 1, [n, 2n) = 0).
void bs_loop_init(int n, int* flags, const BsLoop& lp, hipStream_t s);
// After the prologue: |f|, the first residual test, the flags of iteration 1.
void bs_decide_start(int n, const double* scal, int* flags, const BsLoop& lp, double rtol,
                     int maxit, hipStream_t s);
// u = 0 for the items with f = 0 (over the level-0 vector table).
void bs_zero_u(const BsArgs& a, const BsTable& t, const BsLoop& lp, hipStream_t s);
// After an iteration (step parity cur): breakdown and residual tests; the
// items whose recurrence residual passed get the prologue flag (the true-
// residual check and restart).
void bs_decide_iter(int n, const double* scal, int* flags, const BsLoop& lp, int cur, double rtol,
                    int maxit, hipStream_t s);
// After the (flag-gated) prologue: the checked items' outcome, the flags of
// the next iteration and the next iteration index.
void bs_decide_check(int n, const double* scal, int* flags, const BsLoop& lp, int cur, double rtol,
                     int maxit, hipStream_t s);
// After the last step of a launch: when no item is still iterating, the
// prologue flag of every item without a true residual; the iteration flags
// stay set for the next launch (one block).
void bs_decide_final(int n, int* flags, const BsLoop& lp, hipStream_t s);
// After that prologue: those items' true relative residual.
void bs_final_rel(int n, const double* scal, int* flags, const BsLoop& lp, hipStream_t s);

}  // namespace sgmg
