// Coarsest level (Sec. 3.2, Sec. 4.1): dense K_L + eps I on the free DOFs,
// explicit inverse by a blocked in-place Gauss-Jordan sweep (no pivoting:
// the matrix is SPD), and the per-cycle solve as a gather-GEMV-scatter.
#include "kernels.hpp"

namespace sgmg {

constexpr int kNB = 64;       // Gauss-Jordan panel width

__global__ void k_dense_assemble(Grid g, const double* __restrict__ S,
                                 const int* __restrict__ free_idx, int nf, double* __restrict__ A) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)nf * nf) return;
  const int i = (int)(t / nf), j = (int)(t % nf);
  const int di = free_idx[i], dj = free_idx[j];
  const int ni = di / 3, nj = dj / 3, d = di % 3, e = dj % 3;
  const int ix = ni % g.Nx, iy = (ni / g.Nx) % g.Ny, iz = ni / (g.Nx * g.Ny);
  const int jx = nj % g.Nx, jy = (nj / g.Nx) % g.Ny, jz = nj / (g.Nx * g.Ny);
  const int ox = jx - ix, oy = jy - iy, oz = jz - iz;
  double v = 0.0;
  if (ox >= -1 && ox <= 1 && oy >= -1 && oy <= 1 && oz >= -1 && oz <= 1) {
    const int o = (ox + 1) + 3 * (oy + 1) + 9 * (oz + 1);
    v = S[(size_t)(o * 9 + 3 * d + e) * g.Nn + ni];
  }
  A[t] = v;
}

void launch_dense_assemble(const Grid& g, const double* S, const int* free_idx, int nf, double* A,
                           hipStream_t s) {
  k_dense_assemble<<<div_up((long)nf * nf, 256), 256, 0, s>>>(g, S, free_idx, nf, A);
}

__global__ void k_dense_diag_sum(const double* __restrict__ A, int nf, RedWs ws, double* out) {
  double s = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nf; i += gridDim.x * blockDim.x)
    s += A[(size_t)i * nf + i];
  const double v[1] = {s};
  grid_sum<1>(v, ws);
}

void launch_dense_diag_sum(const double* A, int nf, RedWs ws, double* out, hipStream_t s) {
  k_dense_diag_sum<<<1, 256, 0, s>>>(A, nf, ws, out);
  launch_finalize(ws, 1, 1, out, s);
}

// eps = max(mean diag * 1e-8, 1e-14) added to the diagonal (Sec. 4.1).
__global__ void k_dense_add_diag(double* __restrict__ A, int nf, const double* __restrict__ dsum,
                                 double* __restrict__ eps_out) {
  const double eps = fmax(*dsum / nf * 1e-8, 1e-14);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && eps_out) *eps_out = eps;
  if (i < nf) A[(size_t)i * nf + i] += eps;
}

void launch_dense_add_diag(double* A, int nf, const double* mean_diag_sum, hipStream_t s,
                           double* eps_out) {
  k_dense_add_diag<<<div_up(nf, 256), 256, 0, s>>>(A, nf, mean_diag_sum, eps_out);
}

// --- blocked Gauss-Jordan sweep --------------------------------------------
// For pivot block K: Q = A_KK^-1; A_KJ <- Q A_KJ (J != K);
// A_IJ <- A_IJ - A_IK(old) A_KJ(new) (I, J != K); A_IK <- -A_IK(old) Q.
// After all blocks A holds its inverse.

__global__ void k_gj_copy_col(const double* __restrict__ A, int n, int k0, int nb,
                              double* __restrict__ C) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)n * kNB) return;
  const int i = (int)(t / kNB), c = (int)(t % kNB);
  C[t] = c < nb ? A[(size_t)i * n + k0 + c] : 0.0;
}

// Inverse of the nb x nb pivot block by in-place Gauss-Jordan (SPD: no
// pivoting), four waves: lane r of wave w keeps columns 16w .. 16w + 15 of
// row r in registers.  The 16 steps whose pivot column a wave owns are
// unrolled, so every register index is a compile-time constant.  At step p
// the owner wave publishes column p and lane p of every wave publishes its
// part of row p in LDS; after a block barrier every lane updates its 16
// entries:
//   r == p : a_pc <- a_pc / a_pp (c != p),  a_pp <- 1 / a_pp
//   r != p : a_rc <- a_rc - (a_rp / a_pp) a_pc (c != p),  a_rp <- -a_rp / a_pp
// (the same operations, in the same precision, as one lane per row would
// do).  The block is zero-padded to 64 x 64 with a unit diagonal, so padded
// rows and columns stay decoupled.
__global__ __launch_bounds__(256) void k_gj_pivot(double* __restrict__ A, int n, int k0, int nb,
                                                  double* __restrict__ Q, int* __restrict__ flag) {
  __shared__ double colp[2][kNB];   // column p (double-buffered over steps)
  __shared__ double rowp[2][kNB];   // row p
  const int r = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c0 = 16 * w;
  double v[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const int col = c0 + c;
    v[c] = (r < nb && col < nb) ? A[(size_t)(k0 + r) * n + k0 + col] : (r == col ? 1.0 : 0.0);
  }
  bool bad = false;
  for (int pw = 0; pw < 4; ++pw) {
#pragma unroll
    for (int sp = 0; sp < 16; ++sp) {
      const int p = 16 * pw + sp, buf = sp & 1;
      if (w == pw) colp[buf][r] = v[sp];
      if (r == p) {
#pragma unroll
        for (int c = 0; c < 16; ++c) rowp[buf][c0 + c] = v[c];
      }
      __syncthreads();
      const double pv = colp[buf][p];
      bad |= !(pv > 0.0);
      const double inv = 1.0 / pv;
      const bool me = r == p;
      const double g = colp[buf][r] * inv;            // a_rp / a_pp
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const double rc = rowp[buf][c0 + c];
        const double upd = me ? rc * inv : __builtin_fma(-g, rc, v[c]);
        v[c] = (w == pw && c == sp) ? (me ? inv : -g) : upd;
      }
    }
  }
  if (bad && threadIdx.x == 0) *flag = 1;
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const int col = c0 + c;
    const bool in = r < nb && col < nb;
    const double x = in ? v[c] : 0.0;
    Q[r * kNB + col] = x;
    if (in) A[(size_t)(k0 + r) * n + k0 + col] = x;
  }
}

// A_KJ <- Q A_KJ for every column j outside the panel (Q staged in LDS).
__global__ __launch_bounds__(256) void k_gj_rowpanel(double* __restrict__ A, int n, int k0, int nb,
                                                     const double* __restrict__ Q) {
  // 64 columns per block: Q and the block's 64 x 64 piece of the panel rows
  // are staged in LDS (Q zero-padded past nb), then each thread forms a
  // 4 x 4 register tile (rows tr + 16 q, columns tc + 16 w) over the 64
  // products in order
  __shared__ double Qs[kNB][kNB + 1];
  __shared__ double Vs[kNB][kNB + 1];
  const int j0 = blockIdx.x * 64;
  for (int e = threadIdx.x; e < kNB * kNB; e += 256) {
    const int r = e / kNB, c = e % kNB, j = j0 + c;
    Qs[r][c] = (r < nb && c < nb) ? Q[r * kNB + c] : 0.0;
    Vs[r][c] = (r < nb && j < n) ? A[(size_t)(k0 + r) * n + j] : 0.0;
  }
  __syncthreads();
  const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;
  double acc[4][4] = {};
  for (int t = 0; t < kNB; ++t) {
    double a[4], b[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      a[q] = Qs[tr + 16 * q][t];
      b[q] = Vs[t][tc + 16 * q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int w = 0; w < 4; ++w) acc[q][w] += a[q] * b[w];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = tr + 16 * q;
    if (r >= nb) continue;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int j = j0 + tc + 16 * w;
      if (j < n && !(j >= k0 && j < k0 + nb)) A[(size_t)(k0 + r) * n + j] = acc[q][w];
    }
  }
}

// Rank-nb update of all rows outside the panel: A_IJ -= C_I R_J with R_J =
// A_KJ (new) for columns outside the panel and R_J = -Q for the panel's own
// columns, which receive -C_I Q (stored, not subtracted).  A 128 x 128
// output tile per 256-thread block on the FP64 matrix cores
// (v_mfma_f64_16x16x4_f64): each wave owns a 64 x 64 quarter as 4 x 4 MFMA
// tiles, K streamed through LDS in chunks of 16 (4 k-steps of 4).  Operand
// layouts: A lane l = (row l % 16, k l / 16), B lane l = (k l / 16, column
// l % 16); result register i of lane l = (row 4 i + l / 16, column l % 16).
constexpr int kUpdTile = 128, kUpdK = 16;
typedef double f64x4_gj __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_gj_update(double* __restrict__ A, int n, int k0, int nb,
                                                   const double* __restrict__ C,
                                                   const double* __restrict__ Q) {
  __shared__ double Cs[kUpdTile][kUpdK + 1];
  __shared__ double Rs[kUpdK][kUpdTile + 1];
  const int i0 = blockIdx.y * kUpdTile, j0 = blockIdx.x * kUpdTile;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wr = (wv >> 1) * 64, wc = (wv & 1) * 64;
  const int lr = lane & 15, lk = lane >> 4;
  f64x4_gj acc[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int w = 0; w < 4; ++w) acc[q][w] = f64x4_gj{0.0, 0.0, 0.0, 0.0};
  for (int t0 = 0; t0 < nb; t0 += kUpdK) {
    // staging: every load at a clamped, valid address, all issued before
    // the first LDS store, the value selected afterwards
    constexpr int kPer = kUpdTile * kUpdK / 256;
    double cv[kPer], av[kPer], qv[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int r = e / kUpdK, c = e % kUpdK;
      cv[u] = C[(size_t)min(i0 + r, n - 1) * kNB + min(t0 + c, nb - 1)];
      const int rr = e / kUpdTile, cc = e % kUpdTile;
      const int t = min(t0 + rr, nb - 1), j = min(j0 + cc, n - 1);
      av[u] = A[(size_t)(k0 + t) * n + j];
      qv[u] = Q[t * kNB + min(max(j - k0, 0), nb - 1)];
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int r = e / kUpdK, c = e % kUpdK;
      Cs[r][c] = (i0 + r < n && t0 + c < nb) ? cv[u] : 0.0;
      const int rr = e / kUpdTile, cc = e % kUpdTile;
      const int t = t0 + rr, j = j0 + cc;
      double v = 0.0;
      if (t < nb && j < n) v = (j >= k0 && j < k0 + nb) ? -qv[u] : av[u];   // -C Q | A_KJ (new)
      Rs[rr][cc] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kUpdK; kk += 4) {
      double a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = Cs[wr + 16 * q + lr][kk + lk];
        b[q] = Rs[kk + lk][wc + 16 * q + lr];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int w = 0; w < 4; ++w)
          acc[q][w] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b[w], acc[q][w], 0, 0, 0);
    }
    __syncthreads();
  }
  // read-modify-write of the tile: all old values are loaded first (at
  // clamped, valid addresses), then the stores are masked
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double old[4][4];
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int i = min(i0 + wr + 16 * q + 4 * ii + lk, n - 1);
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int j = min(j0 + wc + 16 * w + lr, n - 1);
        old[ii][w] = A[(size_t)i * n + j];
      }
    }
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int i = i0 + wr + 16 * q + 4 * ii + lk;
      const bool row_ok = i < n && !(i >= k0 && i < k0 + nb);
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int j = j0 + wc + 16 * w + lr;
        if (!row_ok || j >= n) continue;
        const bool panel_col = j >= k0 && j < k0 + nb;
        A[(size_t)i * n + j] = panel_col ? acc[q][w][ii] : old[ii][w] - acc[q][w][ii];
      }
    }
  }
}

int dense_spd_inverse(double* A, int n, double* scratch, int* d_flag, hipStream_t s) {
  double* C = scratch;                       // n * kNB
  double* Q = scratch + (size_t)n * kNB;     // kNB * kNB
  for (int k0 = 0; k0 < n; k0 += kNB) {
    const int nb = (n - k0) < kNB ? (n - k0) : kNB;
    k_gj_copy_col<<<div_up((long)n * kNB, 256), 256, 0, s>>>(A, n, k0, nb, C);
    k_gj_pivot<<<1, 256, 0, s>>>(A, n, k0, nb, Q, d_flag);
    k_gj_rowpanel<<<div_up(n, 64), 256, 0, s>>>(A, n, k0, nb, Q);
    dim3 grid(div_up(n, kUpdTile), div_up(n, kUpdTile));
    k_gj_update<<<grid, 256, 0, s>>>(A, n, k0, nb, C, Q);
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Symmetric form of the coarsest solve.  The explicit inverse of the SPD
// matrix K_L + eps I is symmetric, so only its upper triangle is read per
// cycle: it is packed once per factorisation into 64 x 64 tiles (I, J),
// I <= J, tile t(I, J) = I nb - I (I - 1) / 2 + (J - I), each tile row-major
// and zero-padded past nf.  A cycle reads every stored coefficient once:
//   pass 1, one workgroup per tile: row sums A_IJ x_J (towards y_I) and, off
//           the diagonal, column sums A_IJ^T x_I (towards y_J), written as
//           per-tile partials;
//   pass 2, per output block I: y_I = the sum over J of the column partial
//           of tile (J, I) for J < I and the row partial of tile (I, J) for
//           J >= I, in a fixed order.
// x is gathered through the free-DOF list inside pass 1, and y is scattered
// by pass 2, so no separate gather launch remains.  Fixed summation order:
// deterministic.
constexpr int kTile = 64;

int sym_tiles(int nf) {
  const int nb = div_up(nf, kTile);
  return nb * (nb + 1) / 2;
}

__device__ inline int tile_index(int I, int J, int nb) { return I * nb - I * (I - 1) / 2 + (J - I); }

// Inverse of tile_index: the block row from the quadratic's root, corrected
// by at most a step either way against rounding.
__device__ inline void tile_ij(int t, int nb, int& I, int& J) {
  const double b = 2.0 * nb + 1.0;
  int i = (int)((b - sqrt(b * b - 8.0 * t)) * 0.5);
  i = max(0, min(i, nb - 1));
  while (i > 0 && tile_index(i, i, nb) > t) --i;
  while (i + 1 < nb && tile_index(i + 1, i + 1, nb) <= t) ++i;
  I = i;
  J = i + (t - tile_index(i, i, nb));
}

__global__ __launch_bounds__(256) void k_dense_pack(const double* __restrict__ A, int nf, int nb,
                                                   double* __restrict__ P) {
  int I, J;
  tile_ij(blockIdx.x, nb, I, J);
  double* T = P + (size_t)blockIdx.x * kTile * kTile;
  for (int e = threadIdx.x; e < kTile * kTile; e += 256) {
    const int a = e / kTile, b = e % kTile;
    const int i = I * kTile + a, j = J * kTile + b;
    T[e] = (i < nf && j < nf) ? A[(size_t)i * nf + j] : 0.0;
  }
}

__global__ __launch_bounds__(256) void k_dense_symv_tiles(const double* __restrict__ P, int nf,
                                                         int nb, const int* __restrict__ free_idx,
                                                         const double* __restrict__ r,
                                                         double* __restrict__ prow,
                                                         double* __restrict__ pcol) {
  __shared__ double tile[kTile][kTile + 1];
  __shared__ double xs[2][kTile];
  __shared__ double red[4][kTile];
  const int t = blockIdx.x;
  int I, J;
  tile_ij(t, nb, I, J);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const double* T = P + (size_t)t * kTile * kTile;
  double v[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = T[(w + 4 * k) * kTile + lane];
  if (w < 2) {
    const int i = (w == 0 ? I : J) * kTile + lane;
    xs[w][lane] = i < nf ? r[free_idx[i]] : 0.0;
  }
  __syncthreads();
  // column partial over this wave's 16 rows (towards y_J)
  double pc = 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    pc += v[k] * xs[0][w + 4 * k];
    tile[w + 4 * k][lane] = v[k];
  }
  red[w][lane] = pc;
  __syncthreads();
  if (w == 0 && I != J)
    pcol[(size_t)t * kTile + lane] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
  __syncthreads();
  // row partial: lane = row, this wave's 16 columns (towards y_I)
  double pr = 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) pr += tile[lane][16 * w + k] * xs[1][16 * w + k];
  red[w][lane] = pr;
  __syncthreads();
  if (w == 0)
    prow[(size_t)t * kTile + lane] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

// One block of 4 waves per output block I: wave w adds the partials of
// J = w, w + 4, ... (tile indices in closed form, loads independent), then
// the four wave sums are added in a fixed order.
__global__ __launch_bounds__(256) void k_dense_symv_sum(int nf, int nb,
                                                       const int* __restrict__ free_idx,
                                                       const double* __restrict__ prow,
                                                       const double* __restrict__ pcol,
                                                       double* __restrict__ z) {
  __shared__ double red[4][kTile];
  const int I = blockIdx.x, a = threadIdx.x & 63, w = threadIdx.x >> 6;
  double y0 = 0.0, y1 = 0.0;
  int J = w;
  for (; J + 4 < nb; J += 8) {
    const int J1 = J + 4;
    y0 += J < I ? pcol[(size_t)tile_index(J, I, nb) * kTile + a]
                : prow[(size_t)tile_index(I, J, nb) * kTile + a];
    y1 += J1 < I ? pcol[(size_t)tile_index(J1, I, nb) * kTile + a]
                 : prow[(size_t)tile_index(I, J1, nb) * kTile + a];
  }
  if (J < nb)
    y0 += J < I ? pcol[(size_t)tile_index(J, I, nb) * kTile + a]
                : prow[(size_t)tile_index(I, J, nb) * kTile + a];
  red[w][a] = y0 + y1;
  __syncthreads();
  if (w == 0) {
    const int i = I * kTile + a;
    if (i < nf) z[free_idx[i]] = (red[0][a] + red[1][a]) + (red[2][a] + red[3][a]);
  }
}

void launch_dense_pack(const double* A, int nf, double* P, hipStream_t s) {
  if (nf <= 0) return;
  k_dense_pack<<<sym_tiles(nf), 256, 0, s>>>(A, nf, div_up(nf, kTile), P);
}

void launch_dense_symv(const double* P, const int* free_idx, int nf, const double* r,
                       double* partials, double* z, hipStream_t s) {
  if (nf <= 0) return;
  const int nb = div_up(nf, kTile), nt = sym_tiles(nf);
  double* prow = partials;
  double* pcol = partials + (size_t)nt * kTile;
  k_dense_symv_tiles<<<nt, 256, 0, s>>>(P, nf, nb, free_idx, r, prow, pcol);
  k_dense_symv_sum<<<nb, 256, 0, s>>>(nf, nb, free_idx, prow, pcol, z);
}

}  // namespace sgmg
