// Per-node bodies of the level operators, shared by the grid kernels (one
// thread per node) and the persistent batched solver (block-stride loops), so
// each operator's arithmetic exists once.
#pragma once
#include "common.hpp"

namespace sgmg {

// (K u)_node for the matrix-free fine operator (Eq. mf_matvec): gathers the
// 27-node neighbourhood once and applies, for each of the (up to) 8 elements
// around the node, E_e times the rows of K_e for the node's local index.
// Loops are unrolled so K_e indices are compile-time.  xown = u at the node.
template <typename T>
__device__ inline void fine_node_Ku(const Grid& g, const T* __restrict__ E,
                                    const T* __restrict__ ke, const T* __restrict__ u, int node,
                                    T (&acc)[3], T (&xown)[3]) {
  const int i = node % g.Nx, t = node / g.Nx, j = t % g.Ny, k = t / g.Ny;
  T un[27][3];
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
    const bool ok = (unsigned)(i + ox) < (unsigned)g.Nx && (unsigned)(j + oy) < (unsigned)g.Ny &&
                    (unsigned)(k + oz) < (unsigned)g.Nz;
    const size_t nb = 3 * (size_t)(node + ox + g.Nx * (oy + g.Ny * oz));
#pragma unroll
    for (int c = 0; c < 3; ++c) un[o][c] = ok ? u[nb + c] : (T)0;
  }
  acc[0] = acc[1] = acc[2] = (T)0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int kx = q & 1, ky = (q >> 1) & 1, kz = q >> 2;
    const int ex = i - 1 + kx, ey = j - 1 + ky, ez = k - 1 + kz;
    if (ex < 0 || ey < 0 || ez < 0 || ex >= g.nx || ey >= g.ny || ez >= g.nz) continue;
    const T Ee = E[ex + g.nx * (ey + g.ny * ez)];
    const int a = 7 - q;  // local index of this node in the element
    T s0 = (T)0, s1 = (T)0, s2 = (T)0;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
      const int o = (kx + bx) + 3 * (ky + by) + 9 * (kz + bz);
#pragma unroll
      for (int dd = 0; dd < 3; ++dd) {
        const T uv = un[o][dd];
        s0 += ke[(3 * a + 0) * 24 + 3 * b + dd] * uv;
        s1 += ke[(3 * a + 1) * 24 + 3 * b + dd] * uv;
        s2 += ke[(3 * a + 2) * 24 + 3 * b + dd] * uv;
      }
    }
    acc[0] += Ee * s0;
    acc[1] += Ee * s1;
    acc[2] += Ee * s2;
  }
  xown[0] = un[13][0];
  xown[1] = un[13][1];
  xown[2] = un[13][2];
}

// Same operator with fewer live registers: the element loop gathers each
// element's 24 values in turn instead of the 27-node neighbourhood (more
// loads, for kernels where register pressure matters more than load count).
template <typename T>
__device__ inline void fine_node_Ku_lowreg(const Grid& g, const T* __restrict__ E,
                                           const T* __restrict__ ke, const T* __restrict__ u,
                                           int node, T (&acc)[3], T (&xown)[3]) {
  const int i = node % g.Nx, t = node / g.Nx, j = t % g.Ny, k = t / g.Ny;
  acc[0] = acc[1] = acc[2] = (T)0;
  // element loop kept rolled: its K_e rows are then read with a uniform
  // runtime offset, and only one element's 24 values are live at a time
#pragma unroll 1
  for (int q = 0; q < 8; ++q) {
    const int kx = q & 1, ky = (q >> 1) & 1, kz = q >> 2;
    const int ex = i - 1 + kx, ey = j - 1 + ky, ez = k - 1 + kz;
    if (ex < 0 || ey < 0 || ez < 0 || ex >= g.nx || ey >= g.ny || ez >= g.nz) continue;
    const T Ee = E[ex + g.nx * (ey + g.ny * ez)];
    const int a = 7 - q;
    T s0 = (T)0, s1 = (T)0, s2 = (T)0;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const size_t nb = 3 * (size_t)((ex + (b & 1)) + g.Nx * ((ey + ((b >> 1) & 1)) +
                                                            g.Ny * (ez + (b >> 2))));
#pragma unroll
      for (int dd = 0; dd < 3; ++dd) {
        const T uv = u[nb + dd];
        s0 += ke[(3 * a + 0) * 24 + 3 * b + dd] * uv;
        s1 += ke[(3 * a + 1) * 24 + 3 * b + dd] * uv;
        s2 += ke[(3 * a + 2) * 24 + 3 * b + dd] * uv;
      }
    }
    acc[0] += Ee * s0;
    acc[1] += Ee * s1;
    acc[2] += Ee * s2;
  }
  const size_t b3 = 3 * (size_t)node;
  xown[0] = u[b3];
  xown[1] = u[b3 + 1];
  xown[2] = u[b3 + 2];
}

// (K u)_node on a stored 27-point block stencil, reading only the upper half:
// block o >= 13 of the node and, for lower offsets, the transposed mirrored
// block of the neighbour, A[n, n+o] = (S_{26-o}[n+o])^T.
template <typename T>
__device__ inline void stencil_node_Ku(const Grid& g, const T* __restrict__ S,
                                       const T* __restrict__ u, int node, T (&acc)[3]) {
  const int i = node % g.Nx, t = node / g.Nx, j = t % g.Ny, k = t / g.Ny;
  acc[0] = acc[1] = acc[2] = (T)0;
  const size_t Nn = g.Nn;
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
    const bool ok = (unsigned)(i + ox) < (unsigned)g.Nx && (unsigned)(j + oy) < (unsigned)g.Ny &&
                    (unsigned)(k + oz) < (unsigned)g.Nz;
    if (!ok) continue;
    const int nb = node + ox + g.Nx * (oy + g.Ny * oz);
    const size_t b3 = 3 * (size_t)nb;
    const T u0 = u[b3], u1 = u[b3 + 1], u2 = u[b3 + 2];
    if (o >= 13) {
      const T* Sb = S + (size_t)o * 9 * Nn + node;
#pragma unroll
      for (int d = 0; d < 3; ++d)
        acc[d] += Sb[(3 * d) * Nn] * u0 + Sb[(3 * d + 1) * Nn] * u1 + Sb[(3 * d + 2) * Nn] * u2;
    } else {
      const T* Sb = S + (size_t)(26 - o) * 9 * Nn + nb;
#pragma unroll
      for (int d = 0; d < 3; ++d)
        acc[d] += Sb[d * Nn] * u0 + Sb[(3 + d) * Nn] * u1 + Sb[(6 + d) * Nn] * u2;
    }
  }
}

// (P^T r)_I: coarse node I gathers the <= 27 fine nodes interpolating from it.
template <typename TF>
__device__ inline void restrict_node(const Grid& f, const Grid& c, const TF* __restrict__ rf, int I,
                                     double (&acc)[3]) {
  const int Ix = I % c.Nx, t = I / c.Nx, Iy = t % c.Ny, Iz = t / c.Ny;
  acc[0] = acc[1] = acc[2] = 0.0;
  for (int iz = 2 * Iz - 1; iz <= 2 * Iz + 1; ++iz) {
    if (iz < 0 || iz >= f.Nz) continue;
    const double wz = w1d(iz, Iz, f.nz);
    if (wz == 0.0) continue;
    for (int iy = 2 * Iy - 1; iy <= 2 * Iy + 1; ++iy) {
      if (iy < 0 || iy >= f.Ny) continue;
      const double wy = w1d(iy, Iy, f.ny) * wz;
      if (wy == 0.0) continue;
      for (int ix = 2 * Ix - 1; ix <= 2 * Ix + 1; ++ix) {
        if (ix < 0 || ix >= f.Nx) continue;
        const double w = w1d(ix, Ix, f.nx) * wy;
        if (w == 0.0) continue;
        const size_t b = 3 * (size_t)(ix + f.Nx * (iy + f.Ny * iz));
        acc[0] += w * (double)rf[b];
        acc[1] += w * (double)rf[b + 1];
        acc[2] += w * (double)rf[b + 2];
      }
    }
  }
}

// (P e)_i: fine node i reads the <= 8 coarse nodes it interpolates from.
template <typename TC>
__device__ inline void prolong_node(const Grid& f, const Grid& c, const TC* __restrict__ ec, int i,
                                    double (&acc)[3]) {
  const int ix = i % f.Nx, t = i / f.Nx, iy = t % f.Ny, iz = t / f.Ny;
  int cx[2], cy[2], cz[2];
  double wx[2], wy[2], wz[2];
  auto cand = [](int fi, int nf, int* ci, double* w) {
    const int nc = nf >> 1;
    if ((fi & 1) == 0) { ci[0] = fi >> 1; w[0] = 1.0; ci[1] = 0; w[1] = 0.0; }
    else if (fi < 2 * nc) { ci[0] = (fi - 1) >> 1; ci[1] = (fi + 1) >> 1; w[0] = w[1] = 0.5; }
    else { ci[0] = nc; w[0] = 1.0; ci[1] = 0; w[1] = 0.0; }
  };
  cand(ix, f.nx, cx, wx);
  cand(iy, f.ny, cy, wy);
  cand(iz, f.nz, cz, wz);
  acc[0] = acc[1] = acc[2] = 0.0;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const double w = wx[a & 1] * wy[(a >> 1) & 1] * wz[a >> 2];
    if (w == 0.0) continue;
    const size_t b = 3 * (size_t)(cx[a & 1] + c.Nx * (cy[(a >> 1) & 1] + c.Ny * cz[a >> 2]));
    acc[0] += w * (double)ec[b];
    acc[1] += w * (double)ec[b + 1];
    acc[2] += w * (double)ec[b + 2];
  }
}

}  // namespace sgmg
