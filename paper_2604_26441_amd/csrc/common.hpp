// Internal definitions shared by the HIP translation units of libsimpgmg.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/simpgmg.h"

namespace sgmg {

// ----------------------------------------------------------------------------
// Structured grid of one level: nx*ny*nz elements, (nx+1)(ny+1)(nz+1) nodes.
struct Grid {
  int nx, ny, nz;      // elements
  int Nx, Ny, Nz;      // nodes per axis
  int Nn;              // nodes
  int n;               // DOFs = 3*Nn
  int nel;             // elements
};

inline Grid make_grid(int nx, int ny, int nz) {
  Grid g;
  g.nx = nx; g.ny = ny; g.nz = nz;
  g.Nx = nx + 1; g.Ny = ny + 1; g.Nz = nz + 1;
  g.Nn = g.Nx * g.Ny * g.Nz;
  g.n = 3 * g.Nn;
  g.nel = nx * ny * nz;
  return g;
}

// Per-node fixed flags: bit c set = DOF c of the node is fixed.
// Stencil storage: value of block o (27), row d, column d' at node n is
// S[(o*9 + d*3 + d') * Nn + n]; o = (ox+1) + 3(oy+1) + 9(oz+1).
constexpr int kStencil = 243;

// 1D trilinear weight between fine node i (axis of nf elements) and coarse
// node ic (nc = nf/2): even fine nodes inject, odd interior nodes split 1/2,
// the trailing node of an odd axis takes weight 1 from the last coarse node
// (Sec. 3.3, Eq. trilinear_weights; floor coarsening).
__host__ __device__ inline double w1d(int i, int ic, int nf) {
  const int nc = nf >> 1;
  if ((i & 1) == 0) return (i >> 1) == ic ? 1.0 : 0.0;
  if (i < 2 * nc) return (ic == (i - 1) >> 1 || ic == (i + 1) >> 1) ? 0.5 : 0.0;
  return ic == nc ? 1.0 : 0.0;
}

// ----------------------------------------------------------------------------
// Deterministic reductions: a fixed tree inside each block, then a fixed-order
// sum of the block partials in a second kernel.
struct RedWs {
  double* partials;    // >= NV * (largest grid used with this workspace)
  unsigned* counter;   // unused (kept for layout)
};

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sums v over the block (blockDim.x a multiple of 64, <= 1024).  Result valid
// in thread 0.
__device__ inline double block_sum(double v, double* lds /* >= 16 */) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) t += lds[i];
  }
  __syncthreads();
  return t;
}

// Up to NV simultaneous sums, first phase: each block writes its NV block
// totals to ws.partials[k * gridDim.x + blockIdx.x].  A separate one-block
// kernel (launch_finalize) adds the partials in index order and writes the
// totals.  The kernel boundary makes the partials visible, so no device-scope
// fence is issued per block (on a multi-XCD part such a fence writes back the
// L2 of every block's XCD).
template <int NV>
__device__ inline void grid_sum(const double (&v)[NV], RedWs ws) {
  __shared__ double lds[16 * NV];
  double tot[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) tot[k] = block_sum(v[k], lds + 16 * k);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) ws.partials[(size_t)k * gridDim.x + blockIdx.x] = tot[k];
  }
}

// ----------------------------------------------------------------------------
// Epilogue applied at a node after y = (K x)_node is formed (3 values).
//   EPI_STORE : out = y                         (optional dot x.y)
//   EPI_RESID : out = b - y
//   EPI_SMOOTH: dd = c1*d + c2*Dinv*(b - y); x_out = x + dd; d = dd (if store_d)
// Fixed DOFs are always written as 0.
enum EpiMode { EPI_STORE = 0, EPI_RESID = 1, EPI_SMOOTH = 2 };

template <typename T>
struct Epi {
  int mode;
  T* out;              // STORE/RESID output, SMOOTH: x_out (may be NULL when out64 is set)
  const T* b;
  const T* dinv;
  T* d;                // SMOOTH direction (read if c1 != 0, written if store_d)
  double* out64;       // SMOOTH: optional FP64 copy of x_out
  double c1, c2;
  int store_d;
  int want_dot;        // STORE: accumulate x.y into dot
  RedWs ws;
  double* dot_out;     // finalized by the launcher after the kernel (NULL: the
                       // block partials stay in ws.partials)
  const double* dot64 = nullptr;   // SMOOTH with out64 on the BF16-family MFMA operator:
                                   // block partials of dot64 . out64 into ws.partials
};

template <typename T>
__device__ inline double epilogue3(const Epi<T>& ep, int node, unsigned fx, const T (&x)[3],
                                   const double (&y)[3]) {
  double dot = 0.0;
  const size_t base = 3 * (size_t)node;
  if (ep.mode == EPI_STORE) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double v = (fx >> c) & 1u ? 0.0 : y[c];
      if (ep.out) ep.out[base + c] = (T)v;   // NULL: only the dot is wanted
      dot += (double)x[c] * v;
    }
  } else if (ep.mode == EPI_RESID) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
      ep.out[base + c] = (fx >> c) & 1u ? (T)0 : (T)((double)ep.b[base + c] - y[c]);
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T xo, dd;
      if ((fx >> c) & 1u) {
        xo = (T)0; dd = (T)0;
      } else {
        const T r = (T)((double)ep.b[base + c] - y[c]);
        const T dp = ep.c1 != 0.0 ? ep.d[base + c] : (T)0;
        dd = (T)ep.c1 * dp + (T)ep.c2 * ep.dinv[base + c] * r;
        xo = x[c] + dd;
      }
      if (ep.store_d) ep.d[base + c] = dd;
      if (ep.out) ep.out[base + c] = xo;
      if (ep.out64) ep.out64[base + c] = (double)xo;
    }
  }
  return dot;
}

// Same epilogue with the node's operands already loaded (x, b, dinv, d_prev);
// used by kernels that prefetch them ahead of the contraction.
template <typename T>
__device__ inline double epilogue3_pre(const Epi<T>& ep, int node, unsigned fx, const T (&x)[3],
                                       const double (&y)[3], const T (&b)[3], const T (&dinv)[3],
                                       const T (&dprev)[3]) {
  double dot = 0.0;
  const size_t base = 3 * (size_t)node;
  if (ep.mode == EPI_STORE) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double v = (fx >> c) & 1u ? 0.0 : y[c];
      ep.out[base + c] = (T)v;
      dot += (double)x[c] * v;
    }
  } else if (ep.mode == EPI_RESID) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
      ep.out[base + c] = (fx >> c) & 1u ? (T)0 : (T)((double)b[c] - y[c]);
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T xo, dd;
      if ((fx >> c) & 1u) {
        xo = (T)0; dd = (T)0;
      } else {
        const T r = (T)((double)b[c] - y[c]);
        dd = (T)ep.c1 * dprev[c] + (T)ep.c2 * dinv[c] * r;
        xo = x[c] + dd;
      }
      if (ep.store_d) ep.d[base + c] = dd;
      if (ep.out) ep.out[base + c] = xo;
      if (ep.out64) ep.out64[base + c] = (double)xo;
    }
  }
  return dot;
}

// The same epilogue for one component c of a node (thread per DOF kernels).
// Its vector operands are loaded by epilogue1_load, which a kernel issues
// before it forms the product so that their latency overlaps the product's
// own loads.
template <typename T>
struct Epi1In {
  T b, dinv, d;
};

template <typename T>
__device__ inline Epi1In<T> epilogue1_load(const Epi<T>& ep, size_t dof) {
  Epi1In<T> in{(T)0, (T)0, (T)0};
  if (ep.mode == EPI_RESID || ep.mode == EPI_SMOOTH) in.b = ep.b[dof];
  if (ep.mode == EPI_SMOOTH) {
    in.dinv = ep.dinv[dof];
    if (ep.c1 != 0.0) in.d = ep.d[dof];
  }
  return in;
}

template <typename T>
__device__ inline double epilogue1(const Epi<T>& ep, size_t dof, bool fixed, T x, double y,
                                   const Epi1In<T>& in) {
  if (ep.mode == EPI_STORE) {
    const double v = fixed ? 0.0 : y;
    ep.out[dof] = (T)v;
    return (double)x * v;
  }
  if (ep.mode == EPI_RESID) {
    ep.out[dof] = fixed ? (T)0 : (T)((double)in.b - y);
    return 0.0;
  }
  T xo = (T)0, dd = (T)0;
  if (!fixed) {
    const T r = (T)((double)in.b - y);
    const T dp = ep.c1 != 0.0 ? in.d : (T)0;
    dd = (T)ep.c1 * dp + (T)ep.c2 * in.dinv * r;
    xo = x + dd;
  }
  if (ep.store_d) ep.d[dof] = dd;
  if (ep.out) ep.out[dof] = xo;
  if (ep.out64) ep.out64[dof] = (double)xo;
  return 0.0;
}

// Workgroups of a 1D launch are dispatched round-robin over the 8 XCDs of
// the chip, each with its own L2.  Remapping the block index so that XCD x
// receives one contiguous range of logical blocks keeps neighbouring node
// planes (read by stencil-type kernels) in the same L2.  A bijection of
// [0, nblk) for any nblk.
constexpr int kNumXcd = 8;
__device__ inline int xcd_block(int b, int nblk) {
  const int xcd = b % kNumXcd, idx = b / kNumXcd;
  const int per = nblk / kNumXcd, rem = nblk % kNumXcd;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// ----------------------------------------------------------------------------
// Element stiffness tables computed on the host at setup.
struct KeTables {
  double ke[576];      // K_e, unit cube, E = 1, row-major, local DOF 3a+c
  float ke32[576];
  double kscale;       // s with K_e = kint / s exactly when integral != 0
  int kint[576];
  int integral;        // 1 if s*K_e is an integer matrix with |entries| <= 255
  double lam, mu;      // Lame parameters of K_e (E = 1)
};
void compute_ke(double nu, KeTables* t);

// ----------------------------------------------------------------------------
// Error plumbing.
void set_error(const std::string& msg);
#define SGMG_HIP(call)                                                         \
  do {                                                                         \
    hipError_t _e = (call);                                                    \
    if (_e != hipSuccess) {                                                    \
      ::sgmg::set_error(std::string(#call) + ": " + hipGetErrorString(_e));    \
      return SGMG_EHIP;                                                        \
    }                                                                          \
  } while (0)

inline unsigned div_up(long a, long b) { return (unsigned)((a + b - 1) / b); }

}  // namespace sgmg
