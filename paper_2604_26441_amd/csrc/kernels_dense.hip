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

__global__ __launch_bounds__(256) void k_gj_pivot(double* __restrict__ A, int n, int k0, int nb,
                                                  double* __restrict__ Q, int* __restrict__ flag) {
  __shared__ double P[kNB][kNB + 1];
  constexpr int kPer = kNB * kNB / 256;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int t = threadIdx.x + 256 * q, r = t / kNB, c = t % kNB;
    P[r][c] = (r < nb && c < nb) ? A[(size_t)(k0 + r) * n + k0 + c] : 0.0;
  }
  __syncthreads();
  for (int piv = 0; piv < nb; ++piv) {
    const double pv = P[piv][piv];
    if (!(pv > 0.0) && threadIdx.x == 0) *flag = 1;
    const double inv = 1.0 / pv;
    double nv[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int t = threadIdx.x + 256 * q, r = t / kNB, c = t % kNB;
      double v = P[r][c];
      if (r < nb && c < nb) {
        if (r == piv && c == piv) v = inv;
        else if (r == piv) v = inv * P[piv][c];
        else if (c == piv) v = -P[r][piv] * inv;
        else v = P[r][c] - P[r][piv] * inv * P[piv][c];
      }
      nv[q] = v;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int t = threadIdx.x + 256 * q;
      P[t / kNB][t % kNB] = nv[q];
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int t = threadIdx.x + 256 * q, r = t / kNB, c = t % kNB;
    const double v = (r < nb && c < nb) ? P[r][c] : 0.0;
    Q[t] = v;
    if (r < nb && c < nb) A[(size_t)(k0 + r) * n + k0 + c] = v;
  }
}

// A_KJ <- Q A_KJ for every column j outside the panel (Q staged in LDS).
__global__ __launch_bounds__(64) void k_gj_rowpanel(double* __restrict__ A, int n, int k0, int nb,
                                                    const double* __restrict__ Q) {
  __shared__ double Qs[kNB * kNB];
  for (int t = threadIdx.x; t < kNB * kNB; t += 64) Qs[t] = Q[t];
  __syncthreads();
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n || (j >= k0 && j < k0 + nb)) return;
  double v[kNB];
#pragma unroll
  for (int t = 0; t < kNB; ++t) v[t] = t < nb ? A[(size_t)(k0 + t) * n + j] : 0.0;
  for (int r = 0; r < nb; ++r) {
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < kNB; ++t) s += Qs[r * kNB + t] * v[t];
    A[(size_t)(k0 + r) * n + j] = s;
  }
}

// Rank-nb update of all rows outside the panel, 64x64 output tile per block.
__global__ __launch_bounds__(256) void k_gj_update(double* __restrict__ A, int n, int k0, int nb,
                                                   const double* __restrict__ C,
                                                   const double* __restrict__ Q) {
  __shared__ double Cs[64][kNB + 1];
  __shared__ double Rs[kNB][64 + 1];
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  for (int t = threadIdx.x; t < 64 * kNB; t += 256) {
    const int r = t / kNB, c = t % kNB;
    const int i = i0 + r;
    Cs[r][c] = (i < n) ? C[(size_t)i * kNB + c] : 0.0;
  }
  for (int t = threadIdx.x; t < kNB * 64; t += 256) {
    const int r = t / 64, c = t % 64;
    const int j = j0 + c;
    double v = 0.0;
    if (r < nb && j < n) {
      if (j >= k0 && j < k0 + nb) v = -Q[r * kNB + (j - k0)];   // A_IK <- -C Q
      else v = A[(size_t)(k0 + r) * n + j];                     // A_KJ (new)
    }
    Rs[r][c] = v;
  }
  __syncthreads();
  const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;
  double acc[4][4] = {};
  for (int t = 0; t < nb; ++t) {
    double a[4], b[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) { a[q] = Cs[tr + 16 * q][t]; b[q] = Rs[t][tc + 16 * q]; }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int w = 0; w < 4; ++w) acc[q][w] += a[q] * b[w];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = i0 + tr + 16 * q;
    if (i >= n || (i >= k0 && i < k0 + nb)) continue;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int j = j0 + tc + 16 * w;
      if (j >= n) continue;
      double* dst = A + (size_t)i * n + j;
      if (j >= k0 && j < k0 + nb) *dst = acc[q][w];
      else *dst -= acc[q][w];
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
    k_gj_rowpanel<<<div_up(n, 64), 64, 0, s>>>(A, n, k0, nb, Q);
    dim3 grid(div_up(n, 64), div_up(n, 64));
    k_gj_update<<<grid, 256, 0, s>>>(A, n, k0, nb, C, Q);
  }
  return 0;
}

// z[free] = Ainv rc with rc = r[free]; fixed entries of z are left untouched
// (they are zero in the level's buffer).
__global__ void k_dense_gather(const double* __restrict__ r, const int* __restrict__ free_idx,
                               int nf, double* __restrict__ rc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nf) rc[i] = r[free_idx[i]];
}

// One wave per row of the explicit inverse (4 rows per block): each lane
// streams the row with stride 64 and four independent partial sums, then a
// fixed-order wave reduction.  No block barrier (a wave past the last row
// simply exits).
__global__ __launch_bounds__(256) void k_dense_gemv(const double* __restrict__ Ainv,
                                                    const double* __restrict__ rc,
                                                    const int* __restrict__ free_idx, int nf,
                                                    double* __restrict__ z) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= nf) return;
  const double* row = Ainv + (size_t)i * nf;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int j = lane;
  for (; j + 192 < nf; j += 256) {
    s0 += row[j] * rc[j];
    s1 += row[j + 64] * rc[j + 64];
    s2 += row[j + 128] * rc[j + 128];
    s3 += row[j + 192] * rc[j + 192];
  }
  for (; j < nf; j += 64) s0 += row[j] * rc[j];
  const double s = wave_sum((s0 + s1) + (s2 + s3));
  if (lane == 0) z[free_idx[i]] = s;
}

void launch_dense_solve(const double* Ainv, const int* free_idx, int nf, const double* r,
                        double* rc, double* z, hipStream_t s) {
  k_dense_gather<<<div_up(nf, 256), 256, 0, s>>>(r, free_idx, nf, rc);
  k_dense_gemv<<<div_up(nf, 4), 256, 0, s>>>(Ainv, rc, free_idx, nf, z);
}

}  // namespace sgmg
