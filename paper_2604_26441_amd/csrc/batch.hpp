// Device-side descriptors of the persistent batched solver.
#pragma once
#include <type_traits>

#include "common.hpp"

namespace sgmg {

struct BLevel {
  Grid g;
  const uint8_t* fixn;
  const double* dinv64;
  const float* dinv32;
  const double* S64;        // Galerkin stencil (levels >= 1)
  int cheb;                 // 1: Chebyshev (level 0), 0: damped Jacobi
  int steps;
  double omega, theta, delta, sigma1;
};

struct BSys {               // one system (its hierarchy's operators)
  int L;
  BLevel lev[8];
  const float* E32;
  const float* E32s;        // E / s for the BF16-family MFMA operator
  const uint16_t* atab;     // its A-operand table
  const float* ke32;
  const double* E64;
  const double* atab64;     // A-operand table of the FP64 MFMA operator
  double lam, mu;           // Lame parameters of K_e (E = 1)
  const double* ke64;
  int nL;
  const int* free_idx;
  const double* Ainv;
};

struct BItem {              // one (system, load case) solve and its work vectors
  int sys;
  const double* f;
  double* u;                // in: x0, out: iterate
  double *r, *z, *p, *q, *t;
  float *b0, *d0, *r0;
  float* x0[2];
  double* lb[8];
  double* lx[8][2];
  double* lr[8];
  double* rc;
};

// Chebyshev (Saad 12.1) or damped-Jacobi coefficients of smoothing step k
// (pre: k >= 1, the step from zero being done elsewhere; post: k >= 0).
__device__ inline void smooth_coef(const BLevel& V, bool post, int k, double& c1, double& c2) {
  if (!V.cheb) {
    c1 = 0.0;
    c2 = V.omega;
    return;
  }
  if (post && k == 0) {
    c1 = 0.0;
    c2 = 1.0 / V.theta;
    return;
  }
  double rho = 1.0 / V.sigma1, rn = rho;
  for (int j = 0; j < k; ++j) {
    rn = 1.0 / (2.0 * V.sigma1 - rho);
    c1 = rn * rho;
    rho = rn;
  }
  c2 = 2.0 * rn / V.delta;
}

struct BOut {
  int status, iters;
  double rel_true, rel_recur;
};

void launch_batch_pcg(int bs, int grid, const BSys* sys, const BItem* items, int nitems, int* queue,
                      BOut* out, double rtol, int maxit, hipStream_t s);

}  // namespace sgmg
