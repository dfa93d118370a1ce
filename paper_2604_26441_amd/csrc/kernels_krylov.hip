// Basis kernels of the restarted flexible GMRES outer solver (Sec. 3.6):
// block-of-columns dot products and updates over the Arnoldi basis V (FP64,
// column c at V + c * n), deterministic two-stage reductions.
#include "kernels.hpp"

namespace sgmg {

constexpr int kKryBlock = 256;
constexpr int kKryGrid = 1024;     // grid-stride, fixed grid: fixed summation order
constexpr int kKryMaxCols = 64;

static int kry_grid(int n) {
  const int g = div_up(n, kKryBlock);
  return g < kKryGrid ? (g ? g : 1) : kKryGrid;
}

// Wave partial of one column sum into LDS; after a barrier, finish_partials
// adds the waves' values of every column (thread c: column c).
__device__ inline void wave_partial(double a, int c, double (*lds)[kKryBlock / 64]) {
  const double t = wave_sum(a);
  if ((threadIdx.x & 63) == 0) lds[c][threadIdx.x >> 6] = t;
}
__device__ inline void finish_partials(int ncols, double (*lds)[kKryBlock / 64], double* partials) {
  __syncthreads();
  if ((int)threadIdx.x < ncols) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < kKryBlock / 64; ++k) t += lds[threadIdx.x][k];
    partials[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
  }
}

// partials of h[c] = V_c . w, c < ncols
__global__ __launch_bounds__(kKryBlock) void k_basis_dots(const double* __restrict__ V, int ncols,
                                                         const double* __restrict__ w, int n,
                                                         double* __restrict__ partials) {
  __shared__ double lds[kKryMaxCols][kKryBlock / 64];
  for (int c = 0; c < ncols; ++c) {
    double a = 0.0;
    const double* v = V + (size_t)c * n;
    for (int i = blockIdx.x * kKryBlock + threadIdx.x; i < n; i += gridDim.x * kKryBlock)
      a += v[i] * w[i];
    wave_partial(a, c, lds);
  }
  finish_partials(ncols, lds, partials);
}

// w -= V h (h on the device, ncols entries), then the partials of either
// V_c . w (next_dots != 0, ncols sums) or w . w (one sum).  Each thread
// updates its rows first and then re-reads them per column (row-local).
__global__ __launch_bounds__(kKryBlock) void k_basis_update(double* __restrict__ w,
                                                           const double* __restrict__ V, int ncols,
                                                           const double* __restrict__ h, int n,
                                                           int next_dots,
                                                           double* __restrict__ partials) {
  __shared__ double lds[kKryMaxCols][kKryBlock / 64];
  __shared__ double hs[kKryMaxCols];
  if ((int)threadIdx.x < ncols) hs[threadIdx.x] = h[threadIdx.x];
  __syncthreads();
  double ww = 0.0;
  for (int i = blockIdx.x * kKryBlock + threadIdx.x; i < n; i += gridDim.x * kKryBlock) {
    double x = w[i];
    for (int c = 0; c < ncols; ++c) x -= hs[c] * V[(size_t)c * n + i];
    w[i] = x;
    ww += x * x;
  }
  if (!next_dots) {
    wave_partial(ww, 0, lds);
    finish_partials(1, lds, partials);
    return;
  }
  for (int c = 0; c < ncols; ++c) {
    double a = 0.0;
    const double* v = V + (size_t)c * n;
    for (int i = blockIdx.x * kKryBlock + threadIdx.x; i < n; i += gridDim.x * kKryBlock)
      a += v[i] * w[i];
    wave_partial(a, c, lds);
  }
  finish_partials(ncols, lds, partials);
}

// v = w / sqrt(*nrm2) (v may alias w)
__global__ void k_scale_inv_sqrt(const double* __restrict__ w, double* v, const double* nrm2, int n) {
  const double a = 1.0 / sqrt(*nrm2);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    v[i] = w[i] * a;
}

// x += Z y (y on the device, k entries)
__global__ void k_basis_combine(double* __restrict__ x, const double* __restrict__ Z, int k,
                                const double* __restrict__ y, int n) {
  __shared__ double ys[kKryMaxCols];
  if ((int)threadIdx.x < k) ys[threadIdx.x] = y[threadIdx.x];
  __syncthreads();
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double a = x[i];
    for (int c = 0; c < k; ++c) a += ys[c] * Z[(size_t)c * n + i];
    x[i] = a;
  }
}

// h_out[c] (c < ncols) = V_c . w
void launch_basis_dots(const double* V, int ncols, const double* w, int n, RedWs ws, double* h_out,
                       hipStream_t s) {
  const int g = kry_grid(n);
  k_basis_dots<<<g, kKryBlock, 0, s>>>(V, ncols, w, n, ws.partials);
  launch_finalize(ws, g, ncols, h_out, s);
}

void launch_basis_update(double* w, const double* V, int ncols, const double* h, int n,
                         int next_dots, RedWs ws, double* out, hipStream_t s) {
  const int g = kry_grid(n);
  k_basis_update<<<g, kKryBlock, 0, s>>>(w, V, ncols, h, n, next_dots, ws.partials);
  launch_finalize(ws, g, next_dots ? ncols : 1, out, s);
}

void launch_scale_inv_sqrt(const double* w, double* v, const double* nrm2, int n, hipStream_t s) {
  k_scale_inv_sqrt<<<kry_grid(n), kKryBlock, 0, s>>>(w, v, nrm2, n);
}

void launch_basis_combine(double* x, const double* Z, int k, const double* y, int n,
                          hipStream_t s) {
  k_basis_combine<<<kry_grid(n), kKryBlock, 0, s>>>(x, Z, k, y, n);
}

int basis_max_cols() { return kKryMaxCols; }
size_t basis_partials(int ncols) { return (size_t)ncols * kKryGrid; }

// ---------------------------------------------------------------------------
// Preconditioned Lanczos probe of M K (the kappa_eff screen of Sec. 4): the
// three vector steps around the K and M applications.

// r = g with fixed DOFs zeroed
__global__ __launch_bounds__(kKryBlock) void k_lanczos_start(const double* __restrict__ g,
                                                            const uint8_t* __restrict__ fixn,
                                                            double* __restrict__ r, int n) {
  const int i = blockIdx.x * kKryBlock + threadIdx.x;
  if (i < n) r[i] = (fixn[i / 3] >> (i % 3)) & 1u ? 0.0 : g[i];
}

// r = s - a w - b w_prev
__global__ __launch_bounds__(kKryBlock) void k_lanczos_resid(const double* __restrict__ sv,
                                                            const double* __restrict__ w,
                                                            const double* __restrict__ wp, double a,
                                                            double b, double* __restrict__ r, int n) {
  const int i = blockIdx.x * kKryBlock + threadIdx.x;
  if (i < n) r[i] = (sv[i] - a * w[i]) - b * wp[i];
}

// w = r / b, v = z / b
__global__ __launch_bounds__(kKryBlock) void k_lanczos_next(const double* __restrict__ r,
                                                           const double* __restrict__ z, double b,
                                                           double* __restrict__ w,
                                                           double* __restrict__ v, int n) {
  const int i = blockIdx.x * kKryBlock + threadIdx.x;
  if (i < n) {
    w[i] = r[i] / b;
    v[i] = z[i] / b;
  }
}

void launch_lanczos_start(const double* g, const uint8_t* fixn, double* r, int n, hipStream_t s) {
  k_lanczos_start<<<div_up(n, kKryBlock), kKryBlock, 0, s>>>(g, fixn, r, n);
}
void launch_lanczos_resid(const double* sv, const double* w, const double* wp, double a, double b,
                          double* r, int n, hipStream_t s) {
  k_lanczos_resid<<<div_up(n, kKryBlock), kKryBlock, 0, s>>>(sv, w, wp, a, b, r, n);
}
void launch_lanczos_next(const double* r, const double* z, double b, double* w, double* v, int n,
                         hipStream_t s) {
  k_lanczos_next<<<div_up(n, kKryBlock), kKryBlock, 0, s>>>(r, z, b, w, v, n);
}

}  // namespace sgmg
