// SIMP outer-loop kernels (Sec. 3.1, Eq. simp_filter): the design ->
// filtered -> physical density chain, compliance sensitivities, and the
// optimality-criteria update with its volume bisection.  Element index
// ex + nx (ey + ny ez); all FP64.
//
// Filter: cone weights w(e, i) = max(0, rmin - |c_e - c_i|) over element
// centres inside the mesh, rho~_e = sum_i w(e, i) rho_i / W_e with W_e the
// row sum; adjoint (F^T g)_i = sum_e w(e, i) g_e / W_e.  The weights are
// recomputed from the integer offsets (r = ceil(rmin) - 1 cells each way), so
// nothing but W is stored.  Projection: H(x) = (tanh(b eta) + tanh(b (x -
// eta))) / (tanh(b eta) + tanh(b (1 - eta))), b = 0 the identity.
#include "kernels.hpp"

namespace sgmg {

constexpr int kSimpBlock = 256;

struct ElemGrid {
  int nx, ny, nz;
  int n;
};

__device__ inline void elem_xyz(const ElemGrid& g, int e, int& x, int& y, int& z) {
  x = e % g.nx;
  const int t = e / g.nx;
  y = t % g.ny;
  z = t / g.ny;
}

__device__ inline double cone_w(double rmin, int dx, int dy, int dz) {
  return rmin - sqrt((double)(dx * dx + dy * dy + dz * dz));
}

// Visits the in-mesh neighbours i of element e with a positive weight:
// f(i, w).
template <typename F>
__device__ inline void for_cone(const ElemGrid& g, double rmin, int r, int e, F&& f) {
  int x, y, z;
  elem_xyz(g, e, x, y, z);
  for (int dz = -r; dz <= r; ++dz) {
    const int jz = z + dz;
    if (jz < 0 || jz >= g.nz) continue;
    for (int dy = -r; dy <= r; ++dy) {
      const int jy = y + dy;
      if (jy < 0 || jy >= g.ny) continue;
      for (int dx = -r; dx <= r; ++dx) {
        const int jx = x + dx;
        if (jx < 0 || jx >= g.nx) continue;
        const double w = cone_w(rmin, dx, dy, dz);
        if (w > 0.0) f(jx + g.nx * (jy + g.ny * jz), w);
      }
    }
  }
}

__device__ inline void heaviside(double x, double beta, double eta, double& h, double& dh) {
  if (beta == 0.0) {
    h = x;
    dh = 1.0;
    return;
  }
  const double den = tanh(beta * eta) + tanh(beta * (1.0 - eta));
  const double t = tanh(beta * (x - eta));
  h = (tanh(beta * eta) + t) / den;
  dh = beta * (1.0 - t * t) / den;
}

__global__ __launch_bounds__(kSimpBlock) void k_filter_wsum(ElemGrid g, double rmin, int r,
                                                           double* __restrict__ W) {
  const int e = blockIdx.x * kSimpBlock + threadIdx.x;
  if (e >= g.n) return;
  double s = 0.0;
  for_cone(g, rmin, r, e, [&](int, double w) { s += w; });
  W[e] = s;
}

// rhohat = H(F rho), dH = H'(F rho)
__global__ __launch_bounds__(kSimpBlock) void k_physical(ElemGrid g, double rmin, int r,
                                                        const double* __restrict__ W,
                                                        const double* __restrict__ rho,
                                                        double beta, double eta,
                                                        double* __restrict__ rhohat,
                                                        double* __restrict__ dH) {
  const int e = blockIdx.x * kSimpBlock + threadIdx.x;
  if (e >= g.n) return;
  double s = 0.0;
  for_cone(g, rmin, r, e, [&](int i, double w) { s += w * rho[i]; });
  double h, dh;
  heaviside(s / W[e], beta, eta, h, dh);
  rhohat[e] = h;
  dH[e] = dh;
}

// Per element: ce = u_e^T K_e u_e (unit modulus), dc_hat = dH * dc/drhohat,
// and block partials of the compliance sum_e E_e ce.
__global__ __launch_bounds__(kSimpBlock) void k_element_energy(Grid g, const double* __restrict__ ke,
                                                              const double* __restrict__ rhohat,
                                                              const double* __restrict__ dH,
                                                              const double* __restrict__ u,
                                                              double p, double E0, double Emin,
                                                              double* __restrict__ gc, RedWs ws) {
  const int e = blockIdx.x * kSimpBlock + threadIdx.x;
  double comp = 0.0;
  if (e < g.nel) {
    const int ex = e % g.nx, t = e / g.nx, ey = t % g.ny, ez = t / g.ny;
    double ue[24];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const size_t nd = (size_t)(ex + (a & 1)) +
                        (size_t)g.Nx * ((ey + ((a >> 1) & 1)) + (size_t)g.Ny * (ez + (a >> 2)));
#pragma unroll
      for (int c = 0; c < 3; ++c) ue[3 * a + c] = u[3 * nd + c];
    }
    double ce = 0.0;
    for (int i = 0; i < 24; ++i) {
      double row = 0.0;
#pragma unroll
      for (int j = 0; j < 24; ++j) row += ke[i * 24 + j] * ue[j];
      ce += ue[i] * row;
    }
    const double rh = rhohat[e];
    comp = (Emin + (E0 - Emin) * pow(rh, p)) * ce;
    gc[e] = dH[e] * (-p * (E0 - Emin) * pow(rh, p - 1.0) * ce);
  }
  const double v[1] = {comp};
  grid_sum<1>(v, ws);
}

// OC ratio from the design sensitivities dc = F^T gc and dv = F^T dH:
// ratio = max(-dc, 0) / max(dv, 1e-300); dc and dv are also written when asked.
__global__ __launch_bounds__(kSimpBlock) void k_oc_ratio(ElemGrid g, double rmin, int r,
                                                        const double* __restrict__ W,
                                                        const double* __restrict__ gc,
                                                        const double* __restrict__ dH,
                                                        double* __restrict__ ratio,
                                                        double* __restrict__ dc_out,
                                                        double* __restrict__ dv_out) {
  const int i = blockIdx.x * kSimpBlock + threadIdx.x;
  if (i >= g.n) return;
  double dc = 0.0, dv = 0.0;
  for_cone(g, rmin, r, i, [&](int e, double w) {
    dc += w * gc[e] / W[e];
    dv += w * dH[e] / W[e];
  });
  ratio[i] = fmax(-dc, 0.0) / fmax(dv, 1e-300);
  if (dc_out) dc_out[i] = dc;
  if (dv_out) dv_out[i] = dv;
}

__device__ inline double oc_candidate(double rho, double ratio, double lam, double move) {
  const double v = rho * sqrt(ratio / lam);
  return fmin(fmax(v, fmax(0.0, rho - move)), fmin(1.0, rho + move));
}

// Block partials of the physical volume of the OC candidate for multiplier
// lam (the candidate of every neighbour formed on the fly).
__global__ __launch_bounds__(kSimpBlock) void k_oc_volume(ElemGrid g, double rmin, int r,
                                                         const double* __restrict__ W,
                                                         const double* __restrict__ rho,
                                                         const double* __restrict__ ratio,
                                                         double lam, double move, double beta,
                                                         double eta, RedWs ws) {
  const int e = blockIdx.x * kSimpBlock + threadIdx.x;
  double vol = 0.0;
  if (e < g.n) {
    double s = 0.0;
    for_cone(g, rmin, r, e, [&](int i, double w) { s += w * oc_candidate(rho[i], ratio[i], lam, move); });
    double h, dh;
    heaviside(s / W[e], beta, eta, h, dh);
    vol = h;
  }
  const double v[1] = {vol};
  grid_sum<1>(v, ws);
}

__global__ __launch_bounds__(kSimpBlock) void k_oc_apply(int n, double* __restrict__ rho,
                                                        const double* __restrict__ ratio,
                                                        double lam, double move,
                                                        RedWs ws) {
  const int i = blockIdx.x * kSimpBlock + threadIdx.x;
  double change = 0.0;
  if (i < n) {
    const double o = rho[i];
    const double v = oc_candidate(o, ratio[i], lam, move);
    rho[i] = v;
    change = fabs(v - o);
  }
  // largest change: a max reduction through the sum machinery is not
  // possible, so the block maxima go to the partials and the host takes
  // their maximum
  __shared__ double lds[kSimpBlock / 64];
  for (int off = 32; off > 0; off >>= 1) change = fmax(change, __shfl_xor(change, off, 64));
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = change;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int w = 0; w < kSimpBlock / 64; ++w) m = fmax(m, lds[w]);
    ws.partials[blockIdx.x] = m;
  }
}

static ElemGrid egrid(int nx, int ny, int nz) { return ElemGrid{nx, ny, nz, nx * ny * nz}; }
static int cone_r(double rmin) { return rmin > 1.0 ? (int)ceil(rmin) - 1 : 0; }

void launch_filter_wsum(int nx, int ny, int nz, double rmin, double* W, hipStream_t s) {
  const ElemGrid g = egrid(nx, ny, nz);
  k_filter_wsum<<<div_up(g.n, kSimpBlock), kSimpBlock, 0, s>>>(g, rmin, cone_r(rmin), W);
}

void launch_physical(int nx, int ny, int nz, double rmin, const double* W, const double* rho,
                     double beta, double eta, double* rhohat, double* dH, hipStream_t s) {
  const ElemGrid g = egrid(nx, ny, nz);
  k_physical<<<div_up(g.n, kSimpBlock), kSimpBlock, 0, s>>>(g, rmin, cone_r(rmin), W, rho, beta,
                                                           eta, rhohat, dH);
}

void launch_element_energy(const Grid& g, const double* ke, const double* rhohat, const double* dH,
                           const double* u, double p, double E0, double Emin, double* gc,
                           RedWs ws, double* comp_out, hipStream_t s) {
  const int nb = div_up(g.nel, kSimpBlock);
  k_element_energy<<<nb, kSimpBlock, 0, s>>>(g, ke, rhohat, dH, u, p, E0, Emin, gc, ws);
  launch_finalize(ws, nb, 1, comp_out, s);
}

void launch_oc_ratio(int nx, int ny, int nz, double rmin, const double* W, const double* gc,
                     const double* dH, double* ratio, double* dc_out, double* dv_out,
                     hipStream_t s) {
  const ElemGrid g = egrid(nx, ny, nz);
  k_oc_ratio<<<div_up(g.n, kSimpBlock), kSimpBlock, 0, s>>>(g, rmin, cone_r(rmin), W, gc, dH,
                                                           ratio, dc_out, dv_out);
}

void launch_oc_volume(int nx, int ny, int nz, double rmin, const double* W, const double* rho,
                      const double* ratio, double lam, double move, double beta, double eta,
                      RedWs ws, double* vol_out, hipStream_t s) {
  const ElemGrid g = egrid(nx, ny, nz);
  const int nb = div_up(g.n, kSimpBlock);
  k_oc_volume<<<nb, kSimpBlock, 0, s>>>(g, rmin, cone_r(rmin), W, rho, ratio, lam, move, beta,
                                        eta, ws);
  launch_finalize(ws, nb, 1, vol_out, s);
}

int oc_apply_blocks(int n) { return div_up(n, kSimpBlock); }

void launch_oc_apply(int n, double* rho, const double* ratio, double lam, double move, RedWs ws,
                     hipStream_t s) {
  k_oc_apply<<<div_up(n, kSimpBlock), kSimpBlock, 0, s>>>(n, rho, ratio, lam, move, ws);
}

}  // namespace sgmg
