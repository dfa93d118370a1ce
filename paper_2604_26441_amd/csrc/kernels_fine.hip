// Level-0 kernels: element stiffness tables, SIMP map, Dirichlet masks,
// diagonal of the fine operator and the node-centric matrix-free K.u.
#include <cmath>

#include "kernels.hpp"
#include "node_ops.hpp"

namespace sgmg {

// ---------------------------------------------------------------------------
// Unit-cube hex8 stiffness (Sec. 3.1): with shape functions N_a = prod_d phi,
// phi_0 = 1 - t, phi_1 = t, every integral int d_i N_a d_j N_b factorises over
// the axes into 1D integrals {int phi phi = 1/3 or 1/6, int phi' phi' = +-1,
// int phi' phi = +-1/2}.  Scaled by 6 per axis they are the integers used
// below, so 216 * int d_i N_a d_j N_b is an integer g(a,b,i,j).
// K[3a+i][3b+j] = lam g_ij + mu g_ji + mu delta_ij sum_k g_kk (all / 216).
static int g216(int a, int b, int i, int j) {
  int v = 1;
  for (int d = 0; d < 3; ++d) {
    const int pa = (a >> d) & 1, pb = (b >> d) & 1;
    const int sa = 2 * pa - 1, sb = 2 * pb - 1;
    int f;
    if (d == i && d == j) f = 6 * sa * sb;
    else if (d == i) f = 3 * sa;
    else if (d == j) f = 3 * sb;
    else f = pa == pb ? 2 : 1;
    v *= f;
  }
  return v;
}

void compute_ke(double nu, KeTables* t) {
  const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double mu = 1.0 / (2.0 * (1.0 + nu));
  const double s = 720.0 * (1.0 + nu) * (1.0 - 2.0 * nu);
  // s*lam = 720 nu, s*mu = 360 (1 - 2 nu): integer coefficients over 216 when
  // 10 nu / 3 and 5 (1 - 2 nu) / 3 make the sums integral (nu = 0.3 does).
  const double cl = 720.0 * nu / 216.0, cm = 360.0 * (1.0 - 2.0 * nu) / 216.0;
  t->kscale = s;
  t->integral = 1;
  t->lam = lam;
  t->mu = mu;
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b) {
      int lap = 0;
      for (int k = 0; k < 3; ++k) lap += g216(a, b, k, k);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          const int gij = g216(a, b, i, j), gji = g216(a, b, j, i);
          const double kval = (lam * gij + mu * gji + (i == j ? mu * lap : 0.0)) / 216.0;
          const double sval = cl * gij + cm * (gji + (i == j ? lap : 0));
          const int idx = (3 * a + i) * 24 + 3 * b + j;
          t->ke[idx] = kval;
          t->ke32[idx] = (float)kval;
          const double r = std::nearbyint(sval);
          t->kint[idx] = (int)r;
          if (std::fabs(sval - r) > 1e-9 || std::fabs(r) > 255.0) t->integral = 0;
        }
    }
}

// ---------------------------------------------------------------------------
__global__ void k_simp(const double* __restrict__ in, double* __restrict__ E64,
                       float* __restrict__ E32, int nel, int is_modulus, double E0, double Emin,
                       double p) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nel) return;
  const double v = in[e];
  const double E = is_modulus ? v : Emin + (E0 - Emin) * pow(v, p);
  E64[e] = E;
  E32[e] = (float)E;
}

void launch_simp(const double* in, double* E64, float* E32, int nel, int is_modulus, double E0,
                 double Emin, double p, hipStream_t s) {
  k_simp<<<div_up(nel, 256), 256, 0, s>>>(in, E64, E32, nel, is_modulus, E0, Emin, p);
}

__global__ void k_mask_from_dofs(const uint8_t* __restrict__ fd, uint8_t* __restrict__ fixn,
                                 int Nn) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= Nn) return;
  fixn[n] = (fd[3 * n] ? 1 : 0) | (fd[3 * n + 1] ? 2 : 0) | (fd[3 * n + 2] ? 4 : 0);
}

void launch_mask_from_dofs(const uint8_t* fixed_dof, uint8_t* fixn, int Nn, hipStream_t s) {
  k_mask_from_dofs<<<div_up(Nn, 256), 256, 0, s>>>(fixed_dof, fixn, Nn);
}

__global__ void k_mask_cantilever(Grid g, uint8_t* __restrict__ fixn) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.Nn) return;
  fixn[n] = (n % g.Nx) == 0 ? 7 : 0;
}

void launch_mask_cantilever(const Grid& g, uint8_t* fixn, hipStream_t s) {
  k_mask_cantilever<<<div_up(g.Nn, 256), 256, 0, s>>>(g, fixn);
}

// Coarse node (i,j,k) inherits the flags of fine node (2i,2j,2k) (Sec. 3.3).
__global__ void k_mask_inject(Grid f, Grid c, const uint8_t* __restrict__ ffix,
                              uint8_t* __restrict__ cfix) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= c.Nn) return;
  const int i = n % c.Nx, t = n / c.Nx, j = t % c.Ny, k = t / c.Ny;
  cfix[n] = ffix[2 * i + f.Nx * (2 * j + f.Ny * 2 * k)];
}

void launch_mask_inject(const Grid& fine, const Grid& coarse, const uint8_t* ffix, uint8_t* cfix,
                        hipStream_t s) {
  k_mask_inject<<<div_up(coarse.Nn, 256), 256, 0, s>>>(fine, coarse, ffix, cfix);
}

// D[node,c] = sum over the elements around the node of E_e K_e[3a+c][3a+c].
__global__ void k_diag_fine(Grid g, const double* __restrict__ E, const double* __restrict__ ke,
                            const uint8_t* __restrict__ fixn, double* __restrict__ d) {
  const int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= g.Nn) return;
  const int i = node % g.Nx, t = node / g.Nx, j = t % g.Ny, k = t / g.Ny;
  double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int kx = q & 1, ky = (q >> 1) & 1, kz = q >> 2;
    const int ex = i - 1 + kx, ey = j - 1 + ky, ez = k - 1 + kz;
    if (ex < 0 || ey < 0 || ez < 0 || ex >= g.nx || ey >= g.ny || ez >= g.nz) continue;
    const double Ee = E[ex + g.nx * (ey + g.ny * ez)];
    const int a = 7 - q;
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] += Ee * ke[(3 * a + c) * 24 + 3 * a + c];
  }
  const unsigned fx = fixn[node];
#pragma unroll
  for (int c = 0; c < 3; ++c) d[3 * node + c] = (fx >> c) & 1u ? 0.0 : acc[c];
}

void launch_diag_fine(const Grid& g, const double* E, const double* ke, const uint8_t* fixn,
                      double* d, hipStream_t s) {
  k_diag_fine<<<div_up(g.Nn, 256), 256, 0, s>>>(g, E, ke, fixn, d);
}

// ---------------------------------------------------------------------------
// Node-centric matrix-free fine operator (Eq. mf_matvec): the thread that owns
// node n gathers the 27-node neighbourhood of u once, and for each of the (up
// to) 8 elements around n adds E_e * (rows of K_e for n's local index) . u_e.
// Every output is written once by its owner: no atomics, bitwise
// deterministic.  Element and neighbour loops are unrolled, so K_e indices
// are compile-time and its entries are read with uniform (scalar) loads.
template <typename T>
__global__ __launch_bounds__(256) void k_apply_fine_node(Grid g, const T* __restrict__ E,
                                                         const T* __restrict__ ke,
                                                         const T* __restrict__ u,
                                                         const uint8_t* __restrict__ fixn,
                                                         Epi<T> ep) {
  const int node = blockIdx.x * 256 + threadIdx.x;
  double dot = 0.0;
  if (node < g.Nn) {
    T acc[3], xo[3];
    fine_node_Ku<T>(g, E, ke, u, node, acc, xo);
    const double y[3] = {(double)acc[0], (double)acc[1], (double)acc[2]};
    dot = epilogue3(ep, node, fixn[node], xo, y);
  }
  if (ep.want_dot) {
    const double v[1] = {dot};
    grid_sum<1>(v, ep.ws);
  }
}

template <typename T>
void launch_apply_fine_node(const Grid& g, const T* E, const T* ke, const T* u,
                            const uint8_t* fixn, const Epi<T>& ep, hipStream_t s) {
  k_apply_fine_node<T><<<div_up(g.Nn, 256), 256, 0, s>>>(g, E, ke, u, fixn, ep);
  if (ep.want_dot && ep.dot_out) launch_finalize(ep.ws, div_up(g.Nn, 256), 1, ep.dot_out, s);
}

template void launch_apply_fine_node<double>(const Grid&, const double*, const double*,
                                             const double*, const uint8_t*, const Epi<double>&,
                                             hipStream_t);
template void launch_apply_fine_node<float>(const Grid&, const float*, const float*, const float*,
                                            const uint8_t*, const Epi<float>&, hipStream_t);

}  // namespace sgmg
