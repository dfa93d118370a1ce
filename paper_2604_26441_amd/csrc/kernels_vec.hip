// Vector kernels: deterministic dot products, PCG updates, casts, power
// iteration helpers.
#include "kernels.hpp"

namespace sgmg {

constexpr int kVecBlock = 256;
constexpr int kVecGrid = 1024;  // grid-stride: fixed grid -> fixed summation order
constexpr int kVecUnroll = 8;   // elements per thread loaded together

// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): output i of the stream with
// seed s is the variant-13 finaliser of s + (i+1) * golden.  Mapped to
// [-1, 1) with 53 bits.  Used only for the power-iteration start vector.
__device__ inline uint64_t splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_power_start(double* __restrict__ x, const uint8_t* __restrict__ fixn, int Nn,
                              uint64_t seed) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * Nn) return;
  const double v = (double)(splitmix64(seed, (uint64_t)i) >> 11) * 0x1.0p-52 - 1.0;
  x[i] = ((fixn[i / 3] >> (i % 3)) & 1u) ? 0.0 : v;
}

void launch_power_start(double* x, const uint8_t* fixn, int Nn, uint64_t seed, hipStream_t s) {
  k_power_start<<<div_up(3L * Nn, 256), 256, 0, s>>>(x, fixn, Nn, seed);
}

__global__ __launch_bounds__(kVecBlock) void k_dot(const double* __restrict__ a,
                                                   const double* __restrict__ b,
                                                   const double* __restrict__ w, int n, RedWs ws,
                                                   double* out) {
  double s = 0.0;
  for (int i = blockIdx.x * kVecBlock + threadIdx.x; i < n; i += gridDim.x * kVecBlock) {
    double t = a[i] * (b ? b[i] : a[i]);
    if (w) t *= w[i];
    s += t;
  }
  const double v[1] = {s};
  grid_sum<1>(v, ws);
}

// Second phase of every reduction: one block adds the block partials of
// each of the nv sums in index order (fixed order: bitwise deterministic).
__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ partials, int nblocks,
                                                  int nv, double* __restrict__ out) {
  __shared__ double lds[16];
  for (int k = 0; k < nv; ++k) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) s += partials[(size_t)k * nblocks + b];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) out[k] = s;
  }
}

void launch_finalize(RedWs ws, int nblocks, int nv, double* out, hipStream_t s) {
  k_finalize<<<1, 256, 0, s>>>(ws.partials, nblocks, nv, out);
}

static unsigned vec_grid(int n) {
  const unsigned g = div_up(n, kVecBlock);
  return g < (unsigned)kVecGrid ? (g ? g : 1u) : (unsigned)kVecGrid;
}

int vec_dot_blocks(int n) { return (int)vec_grid(n); }

void launch_dot(const double* a, const double* b, const double* w, int n, RedWs ws, double* out,
                hipStream_t s) {
  k_dot<<<vec_grid(n), kVecBlock, 0, s>>>(a, b, w, n, ws, out);
  launch_finalize(ws, vec_grid(n), 1, out, s);
}

__global__ __launch_bounds__(kVecBlock) void k_scale_dinv_norm(const double* __restrict__ dinv,
                                                               const double* __restrict__ w,
                                                               double* __restrict__ y, int n,
                                                               RedWs ws, double* out) {
  double s = 0.0;
  for (int i = blockIdx.x * kVecBlock + threadIdx.x; i < n; i += gridDim.x * kVecBlock) {
    const double v = dinv[i] * w[i];
    y[i] = v;
    s += v * v;
  }
  const double v[1] = {s};
  grid_sum<1>(v, ws);
}

void launch_scale_dinv_norm(const double* dinv, const double* w, double* y, int n, RedWs ws,
                            double* out, hipStream_t s) {
  k_scale_dinv_norm<<<vec_grid(n), kVecBlock, 0, s>>>(dinv, w, y, n, ws, out);
  launch_finalize(ws, vec_grid(n), 1, out, s);
}

__global__ void k_normalize(const double* __restrict__ y, const double* __restrict__ nrm2,
                            double* __restrict__ x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = *nrm2 > 0.0 ? 1.0 / sqrt(*nrm2) : 0.0;
  x[i] = y[i] * s;
}

void launch_normalize(const double* y, const double* nrm2, double* x, int n, hipStream_t s) {
  k_normalize<<<div_up(n, 256), 256, 0, s>>>(y, nrm2, x, n);
}

template <typename T>
__global__ void k_vcycle_entry(const double* __restrict__ r, T* __restrict__ b,
                               const T* __restrict__ dinv, double c0, T* __restrict__ x,
                               T* __restrict__ d, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T bv = (T)r[i];
  b[i] = bv;
  const T xv = (T)c0 * dinv[i] * bv;
  x[i] = xv;
  if (d) d[i] = xv;
}

template <typename T>
void launch_vcycle_entry(const double* r, T* b, const T* dinv, double c0, T* x, T* d, int n,
                         hipStream_t s) {
  k_vcycle_entry<T><<<div_up(n, 256), 256, 0, s>>>(r, b, dinv, c0, x, d, n);
}
template void launch_vcycle_entry<float>(const double*, float*, const float*, double, float*,
                                         float*, int, hipStream_t);
template void launch_vcycle_entry<double>(const double*, double*, const double*, double, double*,
                                          double*, int, hipStream_t);

__global__ void k_d2f(const double* __restrict__ in, float* __restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}
__global__ void k_f2d(const float* __restrict__ in, double* __restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (double)in[i];
}
__global__ void k_copy(const double* __restrict__ in, double* __restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i];
}
void launch_d2f(const double* in, float* out, int n, hipStream_t s) {
  k_d2f<<<div_up(n, 256), 256, 0, s>>>(in, out, n);
}
void launch_f2d(const float* in, double* out, int n, hipStream_t s) {
  k_f2d<<<div_up(n, 256), 256, 0, s>>>(in, out, n);
}
void launch_copy(const double* in, double* out, int n, hipStream_t s) {
  k_copy<<<div_up(n, 256), 256, 0, s>>>(in, out, n);
}

// r = f - Ax0 (or f); out = (f.f, r.r)
__global__ __launch_bounds__(kVecBlock) void k_pcg_init(const double* __restrict__ f,
                                                        const double* __restrict__ Ax0,
                                                        int have_x0, double* __restrict__ r,
                                                        int n, RedWs ws, double* out) {
  double ff = 0.0, rr = 0.0;
  for (int i = blockIdx.x * kVecBlock + threadIdx.x; i < n; i += gridDim.x * kVecBlock) {
    const double fv = f[i];
    const double rv = have_x0 ? fv - Ax0[i] : fv;
    r[i] = rv;
    ff += fv * fv;
    rr += rv * rv;
  }
  const double v[2] = {ff, rr};
  grid_sum<2>(v, ws);
}

void launch_pcg_init(const double* f, const double* Ax0, int have_x0, double* r, int n, RedWs ws,
                     double* sc_ff_rr, hipStream_t s) {
  k_pcg_init<<<vec_grid(n), kVecBlock, 0, s>>>(f, Ax0, have_x0, r, n, ws, sc_ff_rr);
  launch_finalize(ws, vec_grid(n), 2, sc_ff_rr, s);
}

// alpha = sc[rz] / sc[pq]; x += alpha p; r -= alpha q; out = r.r
// Optionally also the entry of the V-cycle that follows (the same
// arithmetic as k_vcycle_entry): b = (T) r, x = c0 Dinv b, d = x.
template <typename T>
struct VEntry {
  T* b = nullptr;
  const T* dinv = nullptr;
  double c0 = 0.0;
  T* x = nullptr;
  T* d = nullptr;
};

template <typename T>
__global__ __launch_bounds__(kVecBlock) void k_pcg_update_xr(const double* x_in, double* x,
                                                             double* __restrict__ r,
                                                             double* __restrict__ r_old,
                                                             const double* __restrict__ p,
                                                             const double* __restrict__ q,
                                                             double* __restrict__ sc,
                                                             int slot_rz, int slot_pq,
                                                             const double* __restrict__ pq_part,
                                                             int npq, int n, RedWs ws,
                                                             VEntry<T> e) {
  // A thread's elements are i0 + k stride; their operands are loaded kVecUnroll
  // at a time before any is used (one memory round trip per group instead of
  // one per element), the first group before the p.q partials are summed
  // (that sum is a memory round trip of its own).
  const int i0 = blockIdx.x * kVecBlock + threadIdx.x;
  const int stride = gridDim.x * kVecBlock;
  double rg[kVecUnroll], xg[kVecUnroll], pg[kVecUnroll], qg[kVecUnroll];
  T dg[kVecUnroll];
  auto load = [&](int base) {
#pragma unroll
    for (int k = 0; k < kVecUnroll; ++k) {
      const int i = base + k * stride;
      if (i < n) {
        rg[k] = r[i];
        xg[k] = x_in[i];
        pg[k] = p[i];
        qg[k] = q[i];
        dg[k] = e.b ? e.dinv[i] : (T)0;
      }
    }
  };
  const double rz = sc[slot_rz];
  load(i0);
  // p.q: from sc, or summed here from the K p kernel's block partials by
  // every block in the same order (block 0 also stores it in sc)
  double pq;
  if (pq_part) {
    __shared__ double lds[16];
    __shared__ double tot;
    double a = 0.0;
    // unrolled so that the loads go out together; the adds keep their order
#pragma unroll 8
    for (int i = threadIdx.x; i < npq; i += kVecBlock) a += pq_part[i];
    a = block_sum(a, lds);
    if (threadIdx.x == 0) {
      tot = a;
      if (blockIdx.x == 0) sc[slot_pq] = a;
    }
    __syncthreads();
    pq = tot;
  } else {
    pq = sc[slot_pq];
  }
  const double alpha = rz / pq;
  // a failed step (p.q <= 0 or non-finite) leaves r untouched and x equal
  // to x_in (x_in may be x itself)
  const bool ok = pq > 0.0 && isfinite(alpha);
  double rr = 0.0;
  auto element = [&](int i, double ro, double xi, double pi, double qi, T di) {
    double rv = ro;
    if (!ok && x_in != x) x[i] = xi;
    if (ok) {
      x[i] = xi + alpha * pi;
      if (r_old) r_old[i] = ro;
      rv = ro - alpha * qi;
      r[i] = rv;
    }
    rr += rv * rv;
    if (e.b) {
      const T bv = (T)rv;
      e.b[i] = bv;
      const T xv = (T)e.c0 * di * bv;
      e.x[i] = xv;
      if (e.d) e.d[i] = xv;
    }
  };
  for (int base = i0; base < n; base += kVecUnroll * stride) {
    if (base != i0) load(base);
#pragma unroll
    for (int k = 0; k < kVecUnroll; ++k) {
      const int i = base + k * stride;
      if (i < n) element(i, rg[k], xg[k], pg[k], qg[k], dg[k]);
    }
  }
  const double v[1] = {rr};
  grid_sum<1>(v, ws);
}

template <typename T>
void launch_pcg_update_xr_entry(const double* x_in, double* x, double* r, double* r_old,
                                const double* p, const double* q, double* sc, int slot_rz,
                                int slot_pq, const double* pq_part, int npq, int n, RedWs ws,
                                double* sc_rr, T* b, const T* dinv, double c0, T* xe, T* de,
                                hipStream_t s) {
  VEntry<T> e;
  e.b = b;
  e.dinv = dinv;
  e.c0 = c0;
  e.x = xe;
  e.d = de;
  k_pcg_update_xr<T><<<vec_grid(n), kVecBlock, 0, s>>>(x_in, x, r, r_old, p, q, sc, slot_rz,
                                                       slot_pq, pq_part, npq, n, ws, e);
  if (sc_rr) launch_finalize(ws, vec_grid(n), 1, sc_rr, s);
}
template void launch_pcg_update_xr_entry<float>(const double*, double*, double*, double*,
                                                const double*, const double*, double*, int, int,
                                                const double*, int, int, RedWs, double*, float*,
                                                const float*, double, float*, float*, hipStream_t);
template void launch_pcg_update_xr_entry<double>(const double*, double*, double*, double*,
                                                 const double*, const double*, double*, int, int,
                                                 const double*, int, int, RedWs, double*, double*,
                                                 const double*, double, double*, double*,
                                                 hipStream_t);

// out[0] = r.z ; out[1] = r_old.z (flexible beta numerator r.z - r_old.z)
__global__ __launch_bounds__(kVecBlock) void k_pcg_dot_rz(const double* __restrict__ r,
                                                          const double* __restrict__ z,
                                                          const double* __restrict__ r_old, int n,
                                                          RedWs ws, double* out) {
  double a = 0.0, b = 0.0;
  for (int i = blockIdx.x * kVecBlock + threadIdx.x; i < n; i += gridDim.x * kVecBlock) {
    const double zv = z[i];
    a += r[i] * zv;
    if (r_old) b += r_old[i] * zv;
  }
  const double v[2] = {a, b};
  grid_sum<2>(v, ws);
}

void launch_pcg_dot_rz(const double* r, const double* z, const double* r_old, int n, RedWs ws,
                       double* sc_out2, hipStream_t s) {
  k_pcg_dot_rz<<<vec_grid(n), kVecBlock, 0, s>>>(r, z, r_old, n, ws, sc_out2);
  if (sc_out2) launch_finalize(ws, vec_grid(n), 2, sc_out2, s);
}

int pcg_vec_partials(int n) { return (int)vec_grid(n); }

// p = z + beta p where the block partials of r.z (nrz of them, then as many
// of r_old.z) are added here, by every block in the same order, instead of
// by a separate finalize launch: beta = (rz - [r_old.z]) / sc[slot_den].
// The nb r.r partials are those of the preceding update.
// Block 0 also stores rz (and r_old.z) into sc[slot_num] (sc[slot_num + 1])
// and the sum of the r.r partials of the preceding update into sc[slot_rr].
__global__ __launch_bounds__(kVecBlock) void k_pcg_update_p_red(
    double* __restrict__ p, const double* __restrict__ z, const double* __restrict__ rz_part,
    int nrz, const double* __restrict__ rr_part, int nb, double* __restrict__ sc, int slot_num,
    int flex,
    int slot_den, int slot_rr, int slot_pq, int slot_seq, double* host, double* host_seq, int n) {
  __shared__ double lds[3][16];
  __shared__ double tot[3];
  // the operands of a thread's elements are loaded kVecUnroll at a time, the
  // first group before the partial sums
  const int i0 = blockIdx.x * kVecBlock + threadIdx.x;
  const int stride = gridDim.x * kVecBlock;
  double zg[kVecUnroll], pg[kVecUnroll];
  auto load = [&](int base) {
#pragma unroll
    for (int k = 0; k < kVecUnroll; ++k) {
      const int i = base + k * stride;
      if (i < n) {
        zg[k] = z[i];
        pg[k] = p[i];
      }
    }
  };
  const double den = sc[slot_den];     // written by the previous iteration
  load(i0);
  double a = 0.0, b = 0.0, c = 0.0;
  // unrolled so that the loads go out together; the adds keep their order
#pragma unroll 8
  for (int i = threadIdx.x; i < nrz; i += kVecBlock) {
    a += rz_part[i];
    if (flex) b += rz_part[nrz + i];
  }
  if (blockIdx.x == 0)
#pragma unroll 8
    for (int i = threadIdx.x; i < nb; i += kVecBlock) c += rr_part[i];
  a = block_sum(a, lds[0]);
  b = block_sum(b, lds[1]);
  c = block_sum(c, lds[2]);
  if (threadIdx.x == 0) {
    tot[0] = a;
    tot[1] = b;
    tot[2] = c;
    if (blockIdx.x == 0) {
      sc[slot_num] = a;
      if (flex) sc[slot_num + 1] = b;
      sc[slot_rr] = c;
      if (host) {
        // the iteration's scalars for the host, in sc's slot layout, then
        // the incremented launch counter, which tells the host they are there
        host[slot_num] = a;
        if (flex) host[slot_num + 1] = b;
        host[slot_rr] = c;
        host[slot_pq] = sc[slot_pq];
        const double seq = sc[slot_seq] + 1.0;
        sc[slot_seq] = seq;
        __threadfence_system();
        *(volatile double*)host_seq = seq;
        __threadfence_system();
      }
    }
  }
  __syncthreads();
  const double beta = (tot[0] - (flex ? tot[1] : 0.0)) / den;
  for (int base = i0; base < n; base += kVecUnroll * stride) {
    if (base != i0) load(base);
#pragma unroll
    for (int k = 0; k < kVecUnroll; ++k) {
      const int i = base + k * stride;
      if (i < n) p[i] = zg[k] + beta * pg[k];
    }
  }
}

void launch_pcg_update_p_red(double* p, const double* z, const double* rz_part, int nrz,
                             const double* rr_part, double* sc, int slot_num, int flex,
                             int slot_den, int slot_rr, int slot_pq, int slot_seq, double* host,
                             double* host_seq, int n, hipStream_t s) {
  k_pcg_update_p_red<<<vec_grid(n), kVecBlock, 0, s>>>(p, z, rz_part, nrz, rr_part,
                                                       (int)vec_grid(n), sc, slot_num, flex,
                                                       slot_den, slot_rr, slot_pq, slot_seq, host,
                                                       host_seq, n);
}

// Largest value of a (non-negative entries, or masked by fixn when given).
// Max is order independent, so the atomic on the IEEE bit pattern (monotone
// for non-negative doubles) is deterministic.
__global__ void k_max_nonneg(const double* __restrict__ a, const uint8_t* __restrict__ fixn, int n,
                             unsigned long long* __restrict__ out) {
  double m = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (fixn && ((fixn[i / 3] >> (i % 3)) & 1u)) continue;
    m = fmax(m, a[i]);
  }
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

void launch_max_nonneg(const double* a, const uint8_t* fixn, int n, double* out, hipStream_t s) {
  hipMemsetAsync(out, 0, sizeof(double), s);
  k_max_nonneg<<<vec_grid(n), kVecBlock, 0, s>>>(a, fixn, n, (unsigned long long*)out);
}

// Diagonal floor and inverse (Sec. 3.5: floored away from zero): free DOFs
// D = max(D, 1e-30 max D), Dinv = 1/D; fixed DOFs D = Dinv = 0.
__global__ void k_diag_finalize(double* __restrict__ d, double* __restrict__ dinv64,
                                float* __restrict__ dinv32, const uint8_t* __restrict__ fixn, int n,
                                const double* __restrict__ dmax) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool fixed = (fixn[i / 3] >> (i % 3)) & 1u;
  double v = d[i], iv = 0.0;
  if (fixed) {
    v = 0.0;
  } else {
    v = fmax(v, 1e-30 * *dmax);
    iv = 1.0 / v;
  }
  d[i] = v;
  dinv64[i] = iv;
  dinv32[i] = (float)iv;
}

void launch_diag_finalize(double* d, double* dinv64, float* dinv32, const uint8_t* fixn, int n,
                          const double* dmax, hipStream_t s) {
  k_diag_finalize<<<div_up(n, 256), 256, 0, s>>>(d, dinv64, dinv32, fixn, n, dmax);
}

__global__ void k_apply_dinv(const double* __restrict__ dinv, const double* __restrict__ r,
                             double* __restrict__ z, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = dinv[i] * r[i];
}

void launch_apply_dinv(const double* dinv, const double* r, double* z, int n, hipStream_t s) {
  k_apply_dinv<<<div_up(n, 256), 256, 0, s>>>(dinv, r, z, n);
}

// r = f - Ax ; out = r.r
__global__ __launch_bounds__(kVecBlock) void k_residual(const double* __restrict__ f,
                                                        const double* __restrict__ Ax,
                                                        double* __restrict__ r, int n, RedWs ws,
                                                        double* out) {
  double rr = 0.0;
  for (int i = blockIdx.x * kVecBlock + threadIdx.x; i < n; i += gridDim.x * kVecBlock) {
    const double v = f[i] - Ax[i];
    if (r) r[i] = v;
    rr += v * v;
  }
  const double v[1] = {rr};
  grid_sum<1>(v, ws);
}

void launch_residual(const double* f, const double* Ax, double* r, int n, RedWs ws,
                     double* out_rr, hipStream_t s) {
  k_residual<<<vec_grid(n), kVecBlock, 0, s>>>(f, Ax, r, n, ws, out_rr);
  launch_finalize(ws, vec_grid(n), 1, out_rr, s);
}

}  // namespace sgmg
