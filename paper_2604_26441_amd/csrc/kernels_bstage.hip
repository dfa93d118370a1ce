// Stage-batched PCG-GMG over many systems and load cases: every stage of the
// outer PCG (Sec. 3.6) and of the V-cycle (Eq. vcycle) is one launch over all
// items.  A stage's grid is a table of (item, local block) pairs, so each
// item gets as many workgroups as its level has work and the whole chip works
// on every stage.  Items carry an active flag: the blocks of an inactive item
// return at once.  Arithmetic per node is that of the persistent batched
// solver (the shared node bodies of node_ops.hpp), reductions are per item,
// in a fixed order (block partials, then one block per item).
#include "batch.hpp"
#include "bstage.hpp"
#include "node_ops.hpp"

namespace sgmg {

namespace {

constexpr int kB = 256;   // threads per block in every stage kernel

struct Slot {             // the table entry of this block
  int item, lb;
};

__device__ inline bool active_block(const int2* __restrict__ tab, const int* __restrict__ flags,
                                    Slot& s) {
  const int2 e = tab[blockIdx.x];
  s.item = e.x;
  s.lb = e.y;
  return flags[s.item] != 0;
}

template <int NV>
__device__ inline void block_partials(const double (&v)[NV], double* __restrict__ part) {
  __shared__ double lds[16 * NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double t = block_sum(v[k], lds + 16 * k);
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * NV + k] = t;
  }
}

// ---------------------------------------------------------------------------
// FP64 fine operator over level-0 nodes.  RES: r = f - K u with partials
// (f.f, r.r); STORE_DOT: q = K p with partial p.q.
constexpr int kRes = 0, kStoreDot = 1;

template <int MODE>
__global__ __launch_bounds__(kB) void k_bs_fine64(const BSys* __restrict__ sys,
                                                  const BItem* __restrict__ items,
                                                  const int2* __restrict__ tab,
                                                  const int* __restrict__ flags,
                                                  double* __restrict__ part) {
  Slot sl;
  if (!active_block(tab, flags, sl)) return;
  const BItem& I = items[sl.item];
  const BSys& S = sys[I.sys];
  const BLevel& V = S.lev[0];
  const int node = sl.lb * kB + threadIdx.x;
  double a = 0.0, b = 0.0;
  if (node < V.g.Nn) {
    const double* x = MODE == kRes ? I.u : I.p;
    double acc[3], xo[3];
    fine_node_Ku<double>(V.g, S.E64, S.ke64, x, node, acc, xo);
    const unsigned fx = V.fixn[node];
    const size_t base = 3 * (size_t)node;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const bool fixed = (fx >> c) & 1u;
      if (MODE == kRes) {
        const double fv = I.f[base + c];
        const double rv = fixed ? 0.0 : fv - acc[c];
        I.r[base + c] = rv;
        a += fv * fv;
        b += rv * rv;
      } else {
        const double y = fixed ? 0.0 : acc[c];
        I.q[base + c] = y;
        a += xo[c] * y;
      }
    }
  }
  if (MODE == kRes) {
    const double v[2] = {a, b};
    block_partials<2>(v, part);
  } else {
    const double v[1] = {a};
    block_partials<1>(v, part);
  }
}

// ---------------------------------------------------------------------------
// Per-item totals: one block per item adds its blocks' partials in order.
// WHAT: 0 (f.f, r.r) -> ff, rr (prologue); 1 p.q -> alpha = rz / p.q (0 when
// p.q is not positive and finite, so x and r stay); 2 r.r -> rr; 3 r.z ->
// beta = r.z / rz_old, rz_old = r.z (iteration); 4 r.z -> rz_old (prologue).
__global__ __launch_bounds__(kB) void k_bs_finalize(const int* __restrict__ start,
                                                    const int* __restrict__ count, int nv,
                                                    const double* __restrict__ part,
                                                    const int* __restrict__ flags, int what,
                                                    double* __restrict__ scal) {
  __shared__ double lds[32];
  const int it = blockIdx.x;
  if (!flags[it]) return;
  double tot[2] = {0.0, 0.0};
  for (int k = 0; k < nv; ++k) {
    double v = 0.0;
    for (int j = threadIdx.x; j < count[it]; j += kB) v += part[(size_t)(start[it] + j) * nv + k];
    tot[k] = block_sum(v, lds + 16 * k);
  }
  if (threadIdx.x != 0) return;
  double* sc = scal + (size_t)it * kBsScalars;
  if (what == 0) {
    sc[kBsFF] = tot[0];
    sc[kBsRR] = tot[1];
  } else if (what == 1) {
    const double pq = tot[0];
    sc[kBsPQ] = pq;
    sc[kBsAlpha] = (pq > 0.0 && isfinite(pq)) ? sc[kBsRZ] / pq : 0.0;
  } else if (what == 2) {
    sc[kBsRR] = tot[0];
  } else if (what == 3) {
    const double rz = tot[0];
    sc[kBsRZNew] = rz;
    sc[kBsBeta] = rz / sc[kBsRZ];
    sc[kBsRZ] = rz;
  } else {
    sc[kBsRZNew] = tot[0];
    sc[kBsRZ] = tot[0];
  }
}

// ---------------------------------------------------------------------------
// Level-0 vector stages over DOFs.
__device__ inline void vcycle_entry(const BSys& S, const BItem& I, size_t i, double r) {
  const BLevel& V = S.lev[0];
  const double c0 = V.cheb ? 1.0 / V.theta : V.omega;
  const float bv = (float)r;
  I.b0[i] = bv;
  const float xv = (float)c0 * V.dinv32[i] * bv;
  I.x0[0][i] = xv;
  I.d0[i] = xv;
}

// x += alpha p, r -= alpha q (partial r.r), and the V-cycle entry from r.
__global__ __launch_bounds__(kB) void k_bs_update_xr(const BSys* __restrict__ sys,
                                                     const BItem* __restrict__ items,
                                                     const int2* __restrict__ tab,
                                                     const int* __restrict__ flags,
                                                     const double* __restrict__ scal,
                                                     double* __restrict__ part) {
  Slot sl;
  if (!active_block(tab, flags, sl)) return;
  const BItem& I = items[sl.item];
  const BSys& S = sys[I.sys];
  const double alpha = scal[(size_t)sl.item * kBsScalars + kBsAlpha];
  const size_t i = (size_t)sl.lb * kB + threadIdx.x;
  double rr = 0.0;
  if (i < (size_t)S.lev[0].g.n) {
    I.u[i] += alpha * I.p[i];
    const double rv = I.r[i] - alpha * I.q[i];
    I.r[i] = rv;
    rr = rv * rv;
    vcycle_entry(S, I, i, rv);
  }
  const double v[1] = {rr};
  block_partials<1>(v, part);
}

// V-cycle entry from r (prologue).
__global__ __launch_bounds__(kB) void k_bs_entry(const BSys* __restrict__ sys,
                                                 const BItem* __restrict__ items,
                                                 const int2* __restrict__ tab,
                                                 const int* __restrict__ flags) {
  Slot sl;
  if (!active_block(tab, flags, sl)) return;
  const BItem& I = items[sl.item];
  const BSys& S = sys[I.sys];
  const size_t i = (size_t)sl.lb * kB + threadIdx.x;
  if (i < (size_t)S.lev[0].g.n) vcycle_entry(S, I, i, I.r[i]);
}

// Partial r.z; with set_p also p = z (prologue).
__global__ __launch_bounds__(kB) void k_bs_dot_rz(const BSys* __restrict__ sys,
                                                  const BItem* __restrict__ items,
                                                  const int2* __restrict__ tab,
                                                  const int* __restrict__ flags, int set_p,
                                                  double* __restrict__ part) {
  Slot sl;
  if (!active_block(tab, flags, sl)) return;
  const BItem& I = items[sl.item];
  const BSys& S = sys[I.sys];
  const size_t i = (size_t)sl.lb * kB + threadIdx.x;
  double rz = 0.0;
  if (i < (size_t)S.lev[0].g.n) {
    const double z = I.z[i];
    rz = I.r[i] * z;
    if (set_p) I.p[i] = z;
  }
  const double v[1] = {rz};
  block_partials<1>(v, part);
}

// p = z + beta p.
__global__ __launch_bounds__(kB) void k_bs_update_p(const BSys* __restrict__ sys,
                                                    const BItem* __restrict__ items,
                                                    const int2* __restrict__ tab,
                                                    const int* __restrict__ flags,
                                                    const double* __restrict__ scal) {
  Slot sl;
  if (!active_block(tab, flags, sl)) return;
  const BItem& I = items[sl.item];
  const BSys& S = sys[I.sys];
  const double beta = scal[(size_t)sl.item * kBsScalars + kBsBeta];
  const size_t i = (size_t)sl.lb * kB + threadIdx.x;
  if (i < (size_t)S.lev[0].g.n) I.p[i] = I.z[i] + beta * I.p[i];
}

// ---------------------------------------------------------------------------
// V-cycle stages.  cin / cout: ping-pong buffer of the level's iterate read
// and written.  MODE: EPI_SMOOTH (step k, pre or post) or EPI_RESID.
template <int MODE>
__global__ __launch_bounds__(kB) void k_bs_apply0(const BSys* __restrict__ sys,
                                                  const BItem* __restrict__ items,
                                                  const int2* __restrict__ tab,
                                                  const int* __restrict__ flags, int post, int k,
                                                  int cin, int last) {
  Slot sl;
  if (!active_block(tab, flags, sl)) return;
  const BItem& I = items[sl.item];
  const BSys& S = sys[I.sys];
  const BLevel& V = S.lev[0];
  const int node = sl.lb * kB + threadIdx.x;
  if (node >= V.g.Nn) return;
  Epi<float> ep{};
  ep.mode = MODE;
  ep.b = I.b0;
  if (MODE == EPI_RESID) {
    ep.out = I.r0;
  } else {
    double c1 = 0.0, c2 = 0.0;
    smooth_coef(V, post != 0, k, c1, c2);
    ep.out = I.x0[1 - cin];
    ep.dinv = V.dinv32;
    ep.d = I.d0;
    ep.c1 = c1;
    ep.c2 = c2;
    ep.store_d = 1;
    ep.out64 = last ? I.z : nullptr;
  }
  float acc[3], xo[3];
  fine_node_Ku<float>(V.g, S.E32, S.ke32, I.x0[cin], node, acc, xo);
  const double y[3] = {(double)acc[0], (double)acc[1], (double)acc[2]};
  epilogue3(ep, node, V.fixn[node], xo, y);
}

// Restriction of level l's residual to level l + 1 over the coarse nodes,
// with the first Jacobi step of level l + 1 from zero unless it is the item's
// coarsest level.
__global__ __launch_bounds__(kB) void k_bs_restrict(const BSys* __restrict__ sys,
                                                    const BItem* __restrict__ items,
                                                    const int2* __restrict__ tab,
                                                    const int* __restrict__ flags, int l) {
  Slot sl;
  if (!active_block(tab, flags, sl)) return;
  const BItem& I = items[sl.item];
  const BSys& S = sys[I.sys];
  const BLevel& V = S.lev[l];
  const BLevel& W = S.lev[l + 1];
  // thread per coarse DOF: the 27 fine values are read unconditionally at
  // clamped indices and weighted (zero weights outside the fine grid), in
  // the order of the node-level definition (z, y, x)
  const int q = sl.lb * kB + threadIdx.x;
  if (q >= 3 * W.g.Nn) return;
  const int Ic = q / 3, k = q - 3 * Ic;
  const int Ix = Ic % W.g.Nx, t = Ic / W.g.Nx, Iy = t % W.g.Ny, Iz = t / W.g.Ny;
  double wx[3], wy[3], wz[3];
  int ix[3], iy[3], iz[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int fx = 2 * Ix - 1 + j, fy = 2 * Iy - 1 + j, fz = 2 * Iz - 1 + j;
    wx[j] = fx >= 0 && fx < V.g.Nx ? w1d(fx, Ix, V.g.nx) : 0.0;
    wy[j] = fy >= 0 && fy < V.g.Ny ? w1d(fy, Iy, V.g.ny) : 0.0;
    wz[j] = fz >= 0 && fz < V.g.Nz ? w1d(fz, Iz, V.g.nz) : 0.0;
    ix[j] = min(max(fx, 0), V.g.Nx - 1);
    iy[j] = min(max(fy, 0), V.g.Ny - 1);
    iz[j] = min(max(fz, 0), V.g.Nz - 1);
  }
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const size_t row = (size_t)V.g.Nx * (iy[b] + (size_t)V.g.Ny * iz[c]);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const size_t f = 3 * (row + ix[a]) + k;
        const double r = l == 0 ? (double)I.r0[f] : I.lr[l][f];
        acc += wx[a] * (wy[b] * wz[c]) * r;
      }
    }
  const bool first = l + 1 < S.L - 1;
  const size_t dof = 3 * (size_t)Ic + k;
  const double v = (W.fixn[Ic] >> k) & 1u ? 0.0 : acc;
  I.lb[l + 1][dof] = v;
  if (first) I.lx[l + 1][0][dof] = W.omega * W.dinv64[dof] * v;
}

// Coarsest level (each item's own): gather the free right-hand side.
__global__ __launch_bounds__(kB) void k_bs_coarse_gather(const BSys* __restrict__ sys,
                                                         const BItem* __restrict__ items,
                                                         const int2* __restrict__ tab,
                                                         const int* __restrict__ flags) {
  Slot sl;
  if (!active_block(tab, flags, sl)) return;
  const BItem& I = items[sl.item];
  const BSys& S = sys[I.sys];
  const int j = sl.lb * kB + threadIdx.x;
  if (j < S.nL) I.rc[j] = I.lb[S.L - 1][S.free_idx[j]];
}

// x_c = Ainv r_c: a block does kCoarseRows rows of one item, one wave per row
// at a time, coalesced along the row, fixed-order wave sums.
constexpr int kCoarseRows = 16;

__global__ __launch_bounds__(kB) void k_bs_coarse_symv(const BSys* __restrict__ sys,
                                                       const BItem* __restrict__ items,
                                                       const int2* __restrict__ tab,
                                                       const int* __restrict__ flags) {
  Slot sl;
  if (!active_block(tab, flags, sl)) return;
  const BItem& I = items[sl.item];
  const BSys& S = sys[I.sys];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double* xc = I.lx[S.L - 1][0];
  for (int rr = w; rr < kCoarseRows; rr += kB / 64) {
    const int i = sl.lb * kCoarseRows + rr;
    if (i >= S.nL) break;
    const double* row = S.Ainv + (size_t)i * S.nL;
    double s = 0.0;
    for (int j = lane; j < S.nL; j += 64) s += row[j] * I.rc[j];
    s = wave_sum(s);
    if (lane == 0) xc[S.free_idx[i]] = s;
  }
}

// Prolongation and correction of level l from level l + 1.  ccoarse: buffer
// of level l + 1's iterate when l + 1 is not the item's coarsest (the
// coarsest solve writes buffer 0); cfine: level l's buffer.
__global__ __launch_bounds__(kB) void k_bs_prolong(const BSys* __restrict__ sys,
                                                   const BItem* __restrict__ items,
                                                   const int2* __restrict__ tab,
                                                   const int* __restrict__ flags, int l,
                                                   int cfine, int ccoarse) {
  Slot sl;
  if (!active_block(tab, flags, sl)) return;
  const BItem& I = items[sl.item];
  const BSys& S = sys[I.sys];
  const BLevel& V = S.lev[l];
  const BLevel& W = S.lev[l + 1];
  const int i = sl.lb * kB + threadIdx.x;
  if (i >= V.g.Nn) return;
  const double* ec = I.lx[l + 1][l + 1 == S.L - 1 ? 0 : ccoarse];
  double acc[3];
  prolong_node<double>(V.g, W.g, ec, i, acc);
  const unsigned fx = V.fixn[i];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    if ((fx >> q) & 1u) continue;
    const size_t b = 3 * (size_t)i + q;
    if (l == 0) I.x0[cfine][b] = (float)((double)I.x0[cfine][b] + acc[q]);
    else I.lx[l][cfine][b] += acc[q];
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.  A table's grid is its entry count.
void bs_fine64_res(const BsArgs& a, const BsTable& t, const int* flags, double* part, hipStream_t s) {
  if (t.n) k_bs_fine64<kRes><<<t.n, kB, 0, s>>>(a.sys, a.items, t.blk, flags, part);
}
void bs_fine64_store_dot(const BsArgs& a, const BsTable& t, const int* flags, double* part,
                         hipStream_t s) {
  if (t.n) k_bs_fine64<kStoreDot><<<t.n, kB, 0, s>>>(a.sys, a.items, t.blk, flags, part);
}
void bs_finalize(const BsTable& t, int nitems, int nv, const double* part, const int* flags,
                 int what, double* scal, hipStream_t s) {
  k_bs_finalize<<<nitems, kB, 0, s>>>(t.start, t.count, nv, part, flags, what, scal);
}
void bs_update_xr(const BsArgs& a, const BsTable& t, const int* flags, const double* scal,
                  double* part, hipStream_t s) {
  if (t.n) k_bs_update_xr<<<t.n, kB, 0, s>>>(a.sys, a.items, t.blk, flags, scal, part);
}
void bs_entry(const BsArgs& a, const BsTable& t, const int* flags, hipStream_t s) {
  if (t.n) k_bs_entry<<<t.n, kB, 0, s>>>(a.sys, a.items, t.blk, flags);
}
void bs_dot_rz(const BsArgs& a, const BsTable& t, const int* flags, int set_p, double* part,
               hipStream_t s) {
  if (t.n) k_bs_dot_rz<<<t.n, kB, 0, s>>>(a.sys, a.items, t.blk, flags, set_p, part);
}
void bs_update_p(const BsArgs& a, const BsTable& t, const int* flags, const double* scal,
                 hipStream_t s) {
  if (t.n) k_bs_update_p<<<t.n, kB, 0, s>>>(a.sys, a.items, t.blk, flags, scal);
}
void bs_smooth0(const BsArgs& a, const BsTable& t, const int* flags, int post, int k, int cin,
                int last, hipStream_t s) {
  if (t.n) k_bs_apply0<EPI_SMOOTH><<<t.n, kB, 0, s>>>(a.sys, a.items, t.blk, flags, post, k, cin, last);
}
void bs_resid0(const BsArgs& a, const BsTable& t, const int* flags, int cin, hipStream_t s) {
  if (t.n) k_bs_apply0<EPI_RESID><<<t.n, kB, 0, s>>>(a.sys, a.items, t.blk, flags, 0, 0, cin, 0);
}
void bs_restrict(const BsArgs& a, const BsTable& t, const int* flags, int l, hipStream_t s) {
  if (t.n) k_bs_restrict<<<t.n, kB, 0, s>>>(a.sys, a.items, t.blk, flags, l);
}
void bs_coarse(const BsArgs& a, const BsTable& tg, const BsTable& tm, const int* flags,
               hipStream_t s) {
  if (tg.n) k_bs_coarse_gather<<<tg.n, kB, 0, s>>>(a.sys, a.items, tg.blk, flags);
  if (tm.n) k_bs_coarse_symv<<<tm.n, kB, 0, s>>>(a.sys, a.items, tm.blk, flags);
}
void bs_prolong(const BsArgs& a, const BsTable& t, const int* flags, int l, int cfine, int ccoarse,
                hipStream_t s) {
  if (t.n) k_bs_prolong<<<t.n, kB, 0, s>>>(a.sys, a.items, t.blk, flags, l, cfine, ccoarse);
}

int bs_threads() { return kB; }
int bs_coarse_rows() { return kCoarseRows; }

// ---------------------------------------------------------------------------
// Device-side iteration control (the one-launch solve).  The tests are those
// of the host loop of sgmg_pcg_solve_batch_staged, item by item, so that the
// same stages run for the same items in the same order.
namespace {

__global__ void k_bs_loop_init(int n, int* __restrict__ flags, BsLoop lp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    lp.it[0] = 1;
    lp.it[1] = 1;
  }
  if (i >= n) return;
  flags[i] = 1;
  flags[n + i] = 0;
  lp.status[i] = -1;
  lp.iters[i] = 0;
  lp.nf[i] = 0.0;
  lp.rel[i] = 0.0;
  lp.rel_true[i] = -1.0;
  lp.zero[i] = 0;
}

__global__ void k_bs_decide_start(int n, const double* __restrict__ scal, int* __restrict__ flags,
                                  BsLoop lp, double rtol, int maxit) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* sc = scal + (size_t)i * kBsScalars;
  const double nf = sqrt(sc[kBsFF]);
  lp.nf[i] = nf;
  int st = -1;
  if (nf == 0.0) {                              // f = 0: the solution is u = 0
    lp.zero[i] = 1;
    st = SGMG_CONVERGED;
    lp.rel[i] = 0.0;
    lp.rel_true[i] = 0.0;
  } else {
    const double rel = sqrt(sc[kBsRR]) / nf;
    lp.rel[i] = rel;
    const double rz = sc[kBsRZ];
    if (!isfinite(rel)) st = SGMG_NONFINITE;
    else if (rel < rtol) { st = SGMG_CONVERGED; lp.rel_true[i] = rel; }
    else if (maxit == 0) st = SGMG_MAXIT;
    else if (!isfinite(rz)) st = SGMG_NONFINITE;
    else if (rz <= 0.0) st = SGMG_BREAKDOWN;
  }
  lp.status[i] = st;
  flags[i] = 0;
  flags[n + i] = st < 0;
}

__global__ __launch_bounds__(kB) void k_bs_zero_u(const BItem* __restrict__ items,
                                                  const BSys* __restrict__ sys,
                                                  const int2* __restrict__ tab, BsLoop lp) {
  Slot sl;
  if (!active_block(tab, lp.zero, sl)) return;
  const BItem& I = items[sl.item];
  const size_t i = (size_t)sl.lb * kB + threadIdx.x;
  if (i < (size_t)sys[I.sys].lev[0].g.n) I.u[i] = 0.0;
}

__global__ void k_bs_decide_iter(int n, const double* __restrict__ scal, int* __restrict__ flags,
                                 BsLoop lp, int cur, double rtol, int maxit) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int it = lp.it[cur];
  int check = 0;
  if (flags[n + i]) {
    const double* sc = scal + (size_t)i * kBsScalars;
    int st = -1, its = it;
    const double pq = sc[kBsPQ];
    if (!isfinite(pq)) { st = SGMG_NONFINITE; its = it - 1; }
    else if (pq <= 0.0) { st = SGMG_BREAKDOWN; its = it - 1; }
    else {
      const double rel = sqrt(sc[kBsRR]) / lp.nf[i];
      lp.rel[i] = rel;
      const double rz = sc[kBsRZNew];
      if (!isfinite(rel)) st = SGMG_NONFINITE;
      else if (rel < rtol) check = 1;             // true-residual check
      else if (!isfinite(rz)) st = SGMG_NONFINITE;
      else if (rz <= 0.0) st = SGMG_BREAKDOWN;
      else if (it == maxit) st = SGMG_MAXIT;
    }
    lp.iters[i] = its;
    lp.status[i] = st;
  }
  flags[n + i] = 0;
  flags[i] = check;
}

__global__ void k_bs_decide_check(int n, const double* __restrict__ scal, int* __restrict__ flags,
                                  BsLoop lp, int cur, double rtol, int maxit) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int it = lp.it[cur];
  if (i == 0) lp.it[cur ^ 1] = it + 1;
  if (i >= n) return;
  if (flags[i]) {
    const double* sc = scal + (size_t)i * kBsScalars;
    const double rt = sqrt(sc[kBsRR]) / lp.nf[i];
    int st = -1;
    if (rt < rtol) {
      st = SGMG_CONVERGED;
      lp.rel_true[i] = rt;
    } else {
      lp.rel[i] = rt;
      const double rz = sc[kBsRZ];
      if (!isfinite(rz)) st = SGMG_NONFINITE;
      else if (rz <= 0.0) st = SGMG_BREAKDOWN;
      else if (it == maxit) st = SGMG_MAXIT;
    }
    lp.status[i] = st;
  }
  flags[i] = 0;
  flags[n + i] = lp.status[i] < 0;
}

__global__ __launch_bounds__(256) void k_bs_decide_final(int n, int* __restrict__ flags,
                                                          BsLoop lp) {
  __shared__ int active;
  if (threadIdx.x == 0) active = 0;
  __syncthreads();
  int a = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) a |= lp.status[i] < 0;
  if (a) active = 1;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    flags[i] = !active && lp.rel_true[i] < 0.0;
    flags[n + i] = lp.status[i] < 0;      // kept for the next launch's first step
  }
}

__global__ void k_bs_final_rel(int n, const double* __restrict__ scal, int* __restrict__ flags,
                               BsLoop lp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !flags[i]) return;
  const double nf = lp.nf[i];
  lp.rel_true[i] = sqrt(scal[(size_t)i * kBsScalars + kBsRR]) / (nf > 0.0 ? nf : 1.0);
  flags[i] = 0;
}

}  // namespace

void bs_decide_final(int n, int* flags, const BsLoop& lp, hipStream_t s) {
  k_bs_decide_final<<<1, 256, 0, s>>>(n, flags, lp);
}
void bs_final_rel(int n, const double* scal, int* flags, const BsLoop& lp, hipStream_t s) {
  k_bs_final_rel<<<div_up(n, 256), 256, 0, s>>>(n, scal, flags, lp);
}
void bs_loop_init(int n, int* flags, const BsLoop& lp, hipStream_t s) {
  k_bs_loop_init<<<div_up(n, 256), 256, 0, s>>>(n, flags, lp);
}
void bs_decide_start(int n, const double* scal, int* flags, const BsLoop& lp, double rtol,
                     int maxit, hipStream_t s) {
  k_bs_decide_start<<<div_up(n, 256), 256, 0, s>>>(n, scal, flags, lp, rtol, maxit);
}
void bs_zero_u(const BsArgs& a, const BsTable& t, const BsLoop& lp, hipStream_t s) {
  if (t.n) k_bs_zero_u<<<t.n, kB, 0, s>>>(a.items, a.sys, t.blk, lp);
}
void bs_decide_iter(int n, const double* scal, int* flags, const BsLoop& lp, int cur, double rtol,
                    int maxit, hipStream_t s) {
  k_bs_decide_iter<<<div_up(n, 256), 256, 0, s>>>(n, scal, flags, lp, cur, rtol, maxit);
}
void bs_decide_check(int n, const double* scal, int* flags, const BsLoop& lp, int cur, double rtol,
                     int maxit, hipStream_t s) {
  k_bs_decide_check<<<div_up(n, 256), 256, 0, s>>>(n, scal, flags, lp, cur, rtol, maxit);
}

}  // namespace sgmg
