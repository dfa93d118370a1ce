// Persistent batched PCG-GMG: one launch solves many independent systems and
// load cases.  Each workgroup takes (system, load case) work items from a
// device queue and runs the whole solve of the item at block level: FP64
// outer PCG with true-residual acceptance (Sec. 3.6), V-cycle (Eq. vcycle)
// with FP32 Chebyshev smoothing on level 0 and FP64 damped Jacobi on the
// Galerkin levels, dense coarsest solve.  Stages are separated by
// __syncthreads; there is no grid-wide synchronisation and no spin-wait, so
// every workgroup exits once the queue is empty.
#include "batch.hpp"
#include "node_ops.hpp"

namespace sgmg {

// Sum over the block, returned to every thread (fixed order: deterministic).
__device__ inline double block_allsum(double v, double* lds) {
  double t = block_sum(v, lds);
  if (threadIdx.x == 0) lds[15] = t;
  __syncthreads();
  t = lds[15];
  __syncthreads();
  return t;
}

template <int BS>
struct BlockCtx {
  const BSys& S;
  const BItem& I;
  double* lds;

  // y = K^l x with an epilogue, over all nodes of the level (T = level type)
  // float: the FP32 fine operator (level 0); double: the FP64 fine operator
  // (level 0) or the Galerkin stencil (levels >= 1).  Returns this thread's
  // part of x.y for EPI_STORE.
  template <typename T>
  __device__ __attribute__((noinline)) double apply(int l, const T* x, const Epi<T>& ep) const {
    const BLevel& L = S.lev[l];
    double dot = 0.0;
    for (int node = threadIdx.x; node < L.g.Nn; node += BS) {
      T acc[3], xo[3];
      if constexpr (std::is_same<T, float>::value) {
        fine_node_Ku_lowreg<float>(L.g, S.E32, S.ke32, x, node, acc, xo);
      } else {
        if (l == 0) {
          fine_node_Ku_lowreg<double>(L.g, S.E64, S.ke64, x, node, acc, xo);
        } else {
          stencil_node_Ku<double>(L.g, L.S64, x, node, acc);
          const size_t b = 3 * (size_t)node;
          xo[0] = x[b]; xo[1] = x[b + 1]; xo[2] = x[b + 2];
        }
      }
      const double y[3] = {(double)acc[0], (double)acc[1], (double)acc[2]};
      dot += epilogue3(ep, node, L.fixn[node], xo, y);
    }
    __syncthreads();
    return dot;
  }
};

template <typename T>
__device__ inline Epi<T> bepi(int mode, T* out, const T* b, const T* dinv, T* d, double c1,
                              double c2, int store_d, double* out64) {
  Epi<T> e{};
  e.mode = mode;
  e.out = out;
  e.b = b;
  e.dinv = dinv;
  e.d = d;
  e.c1 = c1;
  e.c2 = c2;
  e.store_d = store_d;
  e.out64 = out64;
  return e;
}

// One V-cycle z = V(r) at block level (FP64 in/out).  The operator
// applications and the V-cycle are kept out of line so each gets its own
// register allocation (inlined together they would spill).
template <int BS>
__device__ __attribute__((noinline)) void block_vcycle(const BlockCtx<BS>& C, const double* r, double* z) {
  const BSys& S = C.S;
  const BItem& I = C.I;
  const int L = S.L;
  unsigned cur = 0u;   // bit l: which ping-pong buffer holds level l's iterate
  auto cb = [&](int l) { return (int)((cur >> l) & 1u); };
  auto flip = [&](int l) { cur ^= 1u << l; };
  // level-0 entry: b = (float) r, first smoothing step from zero
  {
    const BLevel& V = S.lev[0];
    const double c0 = V.cheb ? 1.0 / V.theta : V.omega;
    for (int i = threadIdx.x; i < V.g.n; i += BS) {
      const float bv = (float)r[i];
      I.b0[i] = bv;
      const float xv = (float)c0 * V.dinv32[i] * bv;
      I.x0[0][i] = xv;
      I.d0[i] = xv;
    }
    __syncthreads();
  }
  // descend
  for (int l = 0; l < L - 1; ++l) {
    const BLevel& V = S.lev[l];
    double rho = V.cheb ? 1.0 / V.sigma1 : 0.0;
    for (int k = 1; k < V.steps; ++k) {
      double c1 = 0.0, c2 = V.omega;
      if (V.cheb) {
        const double rn = 1.0 / (2.0 * V.sigma1 - rho);
        c1 = rn * rho;
        c2 = 2.0 * rn / V.delta;
        rho = rn;
      }
      const int c = cb(l);
      if (l == 0)
        C.template apply<float>(0, I.x0[c], bepi<float>(EPI_SMOOTH, I.x0[1 - c], I.b0, V.dinv32,
                                                        I.d0, c1, c2, 1, nullptr));
      else
        C.template apply<double>(l, I.lx[l][c], bepi<double>(EPI_SMOOTH, I.lx[l][1 - c], I.lb[l],
                                                             V.dinv64, nullptr, 0.0, c2, 0,
                                                             nullptr));
      flip(l);
    }
    // residual
    if (l == 0)
      C.template apply<float>(0, I.x0[cb(0)], bepi<float>(EPI_RESID, I.r0, I.b0, nullptr, nullptr,
                                                          0.0, 0.0, 0, nullptr));
    else
      C.template apply<double>(l, I.lx[l][cb(l)], bepi<double>(EPI_RESID, I.lr[l], I.lb[l],
                                                               nullptr, nullptr, 0.0, 0.0, 0,
                                                               nullptr));
    // restriction (+ first Jacobi step of the next level unless it is the coarsest)
    const BLevel& W = S.lev[l + 1];
    const bool first = l + 1 < L - 1;
    for (int Ic = threadIdx.x; Ic < W.g.Nn; Ic += BS) {
      double acc[3];
      if (l == 0) restrict_node<float>(V.g, W.g, I.r0, Ic, acc);
      else restrict_node<double>(V.g, W.g, I.lr[l], Ic, acc);
      const unsigned fx = W.fixn[Ic];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const size_t b = 3 * (size_t)Ic + q;
        const double v = (fx >> q) & 1u ? 0.0 : acc[q];
        I.lb[l + 1][b] = v;
        if (first) I.lx[l + 1][0][b] = W.omega * W.dinv64[b] * v;
      }
    }
    cur &= ~(1u << (l + 1));
    __syncthreads();
  }
  // coarsest: dense explicit inverse on the free DOFs
  {
    const double* bc = I.lb[L - 1];
    for (int j = threadIdx.x; j < S.nL; j += BS) I.rc[j] = bc[S.free_idx[j]];
    __syncthreads();
    double* xc = I.lx[L - 1][0];
    for (int i = threadIdx.x; i < S.nL; i += BS) {
      const double* row = S.Ainv + (size_t)i * S.nL;
      double s = 0.0;
      for (int j = 0; j < S.nL; ++j) s += row[j] * I.rc[j];
      xc[S.free_idx[i]] = s;
    }
    cur &= ~(1u << (L - 1));
    __syncthreads();
  }
  // ascend
  for (int l = L - 2; l >= 0; --l) {
    const BLevel& V = S.lev[l];
    const BLevel& W = S.lev[l + 1];
    const double* ec = I.lx[l + 1][cb(l + 1)];
    for (int i = threadIdx.x; i < V.g.Nn; i += BS) {
      double acc[3];
      prolong_node<double>(V.g, W.g, ec, i, acc);
      const unsigned fx = V.fixn[i];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        if ((fx >> q) & 1u) continue;
        const size_t b = 3 * (size_t)i + q;
        if (l == 0) I.x0[cb(0)][b] = (float)((double)I.x0[cb(0)][b] + acc[q]);
        else I.lx[l][cb(l)][b] += acc[q];
      }
    }
    __syncthreads();
    double rho = V.cheb ? 1.0 / V.sigma1 : 0.0;
    for (int k = 0; k < V.steps; ++k) {
      double c1 = 0.0, c2 = V.omega;
      if (V.cheb) {
        if (k == 0) {
          c2 = 1.0 / V.theta;
        } else {
          const double rn = 1.0 / (2.0 * V.sigma1 - rho);
          c1 = rn * rho;
          c2 = 2.0 * rn / V.delta;
          rho = rn;
        }
      }
      const int c = cb(l);
      const bool last = (l == 0 && k == V.steps - 1);
      if (l == 0)
        C.template apply<float>(0, I.x0[c], bepi<float>(EPI_SMOOTH, I.x0[1 - c], I.b0, V.dinv32,
                                                        I.d0, c1, c2, 1, last ? z : nullptr));
      else
        C.template apply<double>(l, I.lx[l][c], bepi<double>(EPI_SMOOTH, I.lx[l][1 - c], I.lb[l],
                                                             V.dinv64, nullptr, 0.0, c2, 0,
                                                             nullptr));
      flip(l);
    }
  }
}

template <int BS>
__device__ void block_pcg(const BSys& S, const BItem& I, BOut& out, double rtol, int maxit,
                          double* lds) {
  BlockCtx<BS> C{S, I, lds};
  const BLevel& V0 = S.lev[0];
  const int n = V0.g.n;
  double* x = I.u;
  auto K64 = [&](const double* in, double* y) -> double {
    return C.template apply<double>(0, in, bepi<double>(EPI_STORE, y, nullptr, nullptr, nullptr,
                                                         0.0, 0.0, 0, nullptr));
  };
  // r = f - K x0
  K64(x, I.q);
  double ff = 0.0, rr = 0.0;
  for (int i = threadIdx.x; i < n; i += BS) {
    const double fv = I.f[i];
    const double rv = fv - I.q[i];
    I.r[i] = rv;
    ff += fv * fv;
    rr += rv * rv;
  }
  ff = block_allsum(ff, lds);
  rr = block_allsum(rr, lds);
  const double nf = sqrt(ff);
  int status = SGMG_MAXIT, iters = 0;
  double rel = 0.0, rel_true = -1.0;
  do {
    if (nf == 0.0) {
      for (int i = threadIdx.x; i < n; i += BS) x[i] = 0.0;
      __syncthreads();
      status = SGMG_CONVERGED;
      rel_true = 0.0;
      break;
    }
    rel = sqrt(rr) / nf;
    if (!isfinite(rel)) { status = SGMG_NONFINITE; break; }
    if (rel < rtol) { status = SGMG_CONVERGED; rel_true = rel; break; }
    if (maxit == 0) break;
    block_vcycle<BS>(C, I.r, I.z);
    double rz = 0.0;
    for (int i = threadIdx.x; i < n; i += BS) {
      I.p[i] = I.z[i];
      rz += I.r[i] * I.z[i];
    }
    rz = block_allsum(rz, lds);
    if (!isfinite(rz)) { status = SGMG_NONFINITE; break; }
    if (rz <= 0.0) { status = SGMG_BREAKDOWN; break; }
    for (int it = 1; it <= maxit; ++it) {
      // q = K p with p.q from the fused epilogue
      const double pq = block_allsum(K64(I.p, I.q), lds);
      double s = 0.0;
      if (!isfinite(pq)) { status = SGMG_NONFINITE; iters = it - 1; break; }
      if (pq <= 0.0) { status = SGMG_BREAKDOWN; iters = it - 1; break; }
      const double alpha = rz / pq;
      s = 0.0;
      for (int i = threadIdx.x; i < n; i += BS) {
        x[i] += alpha * I.p[i];
        const double rv = I.r[i] - alpha * I.q[i];
        I.r[i] = rv;
        s += rv * rv;
      }
      rr = block_allsum(s, lds);
      iters = it;
      rel = sqrt(rr) / nf;
      if (!isfinite(rel)) { status = SGMG_NONFINITE; break; }
      bool restart = false;
      if (rel < rtol) {
        K64(x, I.t);
        s = 0.0;
        for (int i = threadIdx.x; i < n; i += BS) {
          const double v = I.f[i] - I.t[i];
          I.t[i] = v;
          s += v * v;
        }
        const double rt = sqrt(block_allsum(s, lds)) / nf;
        if (rt < rtol) { status = SGMG_CONVERGED; rel_true = rt; break; }
        for (int i = threadIdx.x; i < n; i += BS) I.r[i] = I.t[i];   // residual replacement
        __syncthreads();
        restart = true;
        rel = rt;
      }
      if (it == maxit) { status = SGMG_MAXIT; break; }
      block_vcycle<BS>(C, I.r, I.z);
      s = 0.0;
      for (int i = threadIdx.x; i < n; i += BS) s += I.r[i] * I.z[i];
      const double rzn = block_allsum(s, lds);
      if (!isfinite(rzn)) { status = SGMG_NONFINITE; break; }
      if (rzn <= 0.0) { status = SGMG_BREAKDOWN; break; }
      const double beta = restart ? 0.0 : rzn / rz;
      for (int i = threadIdx.x; i < n; i += BS) I.p[i] = I.z[i] + beta * I.p[i];
      __syncthreads();
      rz = rzn;
    }
  } while (0);
  if (rel_true < 0.0) {
    K64(x, I.t);
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += BS) {
      const double v = I.f[i] - I.t[i];
      s += v * v;
    }
    rel_true = sqrt(block_allsum(s, lds)) / (nf > 0.0 ? nf : 1.0);
  }
  if (threadIdx.x == 0) {
    out.status = status;
    out.iters = iters;
    out.rel_true = rel_true;
    out.rel_recur = rel;
  }
}

template <int BS>
__global__ __launch_bounds__(BS) void k_batch_pcg(const BSys* __restrict__ sys,
                                                  const BItem* __restrict__ items, int nitems,
                                                  int* __restrict__ queue, BOut* __restrict__ out,
                                                  double rtol, int maxit) {
  __shared__ double lds[16];
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it >= nitems) return;     // every workgroup reaches this once the queue is empty
    const BItem& I = items[it];
    block_pcg<BS>(sys[I.sys], I, out[it], rtol, maxit, lds);
    __syncthreads();
  }
}

__global__ void k_zero_int(int* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

void launch_batch_pcg(int bs, int grid, const BSys* sys, const BItem* items, int nitems, int* queue,
                      BOut* out, double rtol, int maxit, hipStream_t s) {
  k_zero_int<<<1, 64, 0, s>>>(queue);       // a kernel, not a memset node, so graphs replay it
  if (bs == 256)
    k_batch_pcg<256><<<grid, 256, 0, s>>>(sys, items, nitems, queue, out, rtol, maxit);
  else
    k_batch_pcg<512><<<grid, 512, 0, s>>>(sys, items, nitems, queue, out, rtol, maxit);
}

}  // namespace sgmg
