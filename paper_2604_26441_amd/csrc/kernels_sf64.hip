// Fine-level FP64 K.u on the vector ALU with the element product written in
// a per-axis sum / difference (Haar) basis (Eq. mf_matvec with the Sec. 3.1
// element stiffness).
//
// With trilinear shape functions on the unit cube, every integral of
// d_i N_a d_j N_b is a product of one 1D integral per axis, and in the basis
// {phi_0 + phi_1, phi_1 - phi_0} of each axis (the constant and the linear
// function) the 1D mass matrix is diagonal and the 1D derivative terms have
// a single non-zero entry.  The tensor-product basis of an element (per
// displacement component: 1, x, y, z, xy, xz, yz, xyz) therefore turns
// K_e into a matrix with 45 non-zero entries in small blocks:
//   constants (rigid translations)            0
//   (x_u, y_v, z_w)                           lam/16 (sum) + mu/8 (own)
//   (x_v, y_u), (x_w, z_u), (y_w, z_v)        mu/16 (sum)
//   (xy_u, yz_w), (xy_v, xz_w), (xz_u, yz_v)  lam/48 (sum) + mu/16 (own)
//   (xy_w, xz_v, yz_u)                        mu/48 (sum) + mu/48 (own)
//   xyz_c                                     (lam + 4 mu)/144
// (coefficients of y = T K_H T^T u with the unnormalised transform T of
// nodal values v0 = s - d, v1 = s + d per axis, the 1/8^2 of T^-1 and the
// 1/216 of the 1D integrals folded in; E = 1, lam, mu the Lame parameters).
// The transforms are butterflies of additions; one element costs about 150
// FP64 operations instead of the 576 multiply-adds of the dense 24 x 24
// product, and the element modulus scales the six coefficients.  Exact in
// exact arithmetic; in FP64 it rounds differently from the dense product
// (relative 1e-16 per entry).
//
// Work decomposition: one wave owns a tile of 16 elements in x (lane & 15)
// by 4 element rows in y (lane >> 4) and marches along z over a chunk of
// node planes, which it stages in its own LDS ring (no barrier, nothing
// shared between waves).  Each lane computes one element per plane and owns
// its (-x, -y, -z) node.  Along z the transform is split: a node face is
// transformed over (x, y) once and carried to the next plane (it is the top
// face of one element and the bottom face of the next), and on the output
// side the top face's contribution is carried in the same (x, y) basis and
// added to the next element's bottom face before one inverse transform per
// plane.  x sums come from lane n - 1 by a DPP row shift, y sums from lane
// - 16 by ds_bpermute.  One halo element on the low side of x and y is
// recomputed, so the tile owns 15 x 3 nodes per plane; every node sums its
// eight element contributions in the same order whatever the chunk length.
#include <algorithm>

#include "batch.hpp"
#include "bstage.hpp"
#include "bufops.hpp"
#include "kernels.hpp"

namespace sgmg {

namespace {

constexpr int kSfWaves = 4;                  // waves per block
constexpr int kSfRow = 17 * 24;              // 17 nodes x 3 doubles
constexpr int kSfPlane = 5 * kSfRow;         // node rows 0 .. 4 of the tile
constexpr int kSfWave = 3 * kSfPlane;        // ring of three node planes

struct SfCoef {
  double a;    // lam / 16: (x_u, y_v, z_w) sum
  double b;    // mu / 8: (x_u, y_v, z_w) own
  double c;    // mu / 16: shear pairs
  double d;    // lam / 48: bilinear pairs, sum
  double e;    // mu / 48: (xy_w, xz_v, yz_u), sum and own
  double f;    // (lam + 4 mu) / 144: xyz
  double g;    // mu / 16: bilinear pairs, own
};

// the coefficients for E = 1 from the Lame parameters
__host__ __device__ inline SfCoef sf_coef(double lam, double mu) {
  return SfCoef{lam / 16.0, mu / 8.0, mu / 16.0, lam / 48.0, mu / 48.0, (lam + 4.0 * mu) / 144.0,
                mu / 16.0};
}

// The same coefficients for the children of a coarse element in the scaled
// representation of the level-1 product (each coefficient with k linear
// axes carried times 2^k on the input side and 2^-k on the output side): a
// block with k linear axes is divided by 4^k.
__host__ __device__ inline SfCoef l1_coef(double lam, double mu) {
  const SfCoef f = sf_coef(lam, mu);
  return SfCoef{f.a / 4.0, f.b / 4.0, f.c / 4.0, f.d / 16.0, f.e / 16.0, f.f / 64.0, f.g / 16.0};
}

// (x, y) transform of one node face: v[dx][dy] -> F[cx][cy] (0 constant,
// 1 linear)
__device__ inline void face_fwd(const double (&v)[2][2], double (&F)[2][2]) {
  const double s0 = v[0][0] + v[1][0], d0 = v[1][0] - v[0][0];
  const double s1 = v[0][1] + v[1][1], d1 = v[1][1] - v[0][1];
  F[0][0] = s0 + s1;
  F[0][1] = s1 - s0;
  F[1][0] = d0 + d1;
  F[1][1] = d1 - d0;
}

// inverse butterflies of a face: P[cx][cy] -> node values w[dx][dy]
__device__ inline void face_bwd(const double (&P)[2][2], double (&w)[2][2]) {
  const double a0 = P[0][0] - P[0][1], a1 = P[0][0] + P[0][1];   // cx = 0, dy = 0 / 1
  const double b0 = P[1][0] - P[1][1], b1 = P[1][0] + P[1][1];   // cx = 1
  w[0][0] = a0 - b0;
  w[0][1] = a1 - b1;
  w[1][0] = a0 + b0;
  w[1][1] = a1 + b1;
}

// The element matrix in the transformed basis: h[c][cx][cy][cz] -> o, the
// coefficients scaled by the element modulus.
__device__ __forceinline__ void haar_op(const double (&h)[3][2][2][2], const SfCoef& k,
                                        double (&o)[3][2][2][2]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) o[c][0][0][0] = 0.0;    // rigid translations
  {  // (x_u, y_v, z_w)
    const double xu = h[0][1][0][0], yv = h[1][0][1][0], zw = h[2][0][0][1];
    const double t = k.a * (xu + yv + zw);
    o[0][1][0][0] = t + k.b * xu;
    o[1][0][1][0] = t + k.b * yv;
    o[2][0][0][1] = t + k.b * zw;
  }
  {  // shear pairs (x_v, y_u), (x_w, z_u), (y_w, z_v)
    const double s0 = k.c * (h[1][1][0][0] + h[0][0][1][0]);
    o[1][1][0][0] = s0;
    o[0][0][1][0] = s0;
    const double s1 = k.c * (h[2][1][0][0] + h[0][0][0][1]);
    o[2][1][0][0] = s1;
    o[0][0][0][1] = s1;
    const double s2 = k.c * (h[2][0][1][0] + h[1][0][0][1]);
    o[2][0][1][0] = s2;
    o[1][0][0][1] = s2;
  }
  {  // bilinear pairs (xy_u, yz_w), (xy_v, xz_w), (xz_u, yz_v)
    double a = h[0][1][1][0], b = h[2][0][1][1], t = k.d * (a + b);
    o[0][1][1][0] = t + k.g * a;
    o[2][0][1][1] = t + k.g * b;
    a = h[1][1][1][0];
    b = h[2][1][0][1];
    t = k.d * (a + b);
    o[1][1][1][0] = t + k.g * a;
    o[2][1][0][1] = t + k.g * b;
    a = h[0][1][0][1];
    b = h[1][0][1][1];
    t = k.d * (a + b);
    o[0][1][0][1] = t + k.g * a;
    o[1][0][1][1] = t + k.g * b;
  }
  {  // (xy_w, xz_v, yz_u)
    const double p = h[2][1][1][0], q = h[1][1][0][1], r = h[0][0][1][1];
    const double t = k.e * (p + q + r);
    o[2][1][1][0] = t + k.e * p;
    o[1][1][0][1] = t + k.e * q;
    o[0][0][1][1] = t + k.e * r;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) o[c][1][1][1] = k.f * h[c][1][1][1];
}

__device__ inline SfCoef scaled(const SfCoef& k, double E) {
  return SfCoef{k.a * E, k.b * E, k.c * E, k.d * E, k.e * E, k.f * E, k.g * E};
}

// z butterflies of the two node faces: h[c][cx][cy][cz]
__device__ inline void z_fwd(const double (&F0)[3][2][2], const double (&F1)[3][2][2],
                             double (&h)[3][2][2][2]) {
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int cx = 0; cx < 2; ++cx)
#pragma unroll
      for (int cy = 0; cy < 2; ++cy) {
        h[c][cx][cy][0] = F0[c][cx][cy] + F1[c][cx][cy];
        h[c][cx][cy][1] = F1[c][cx][cy] - F0[c][cx][cy];
      }
}

// inverse z butterflies: the (x, y) transforms of the bottom and top output faces
__device__ inline void z_bwd(const double (&o)[3][2][2][2], double (&P0)[3][2][2],
                             double (&P1)[3][2][2]) {
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int cx = 0; cx < 2; ++cx)
#pragma unroll
      for (int cy = 0; cy < 2; ++cy) {
        P0[c][cx][cy] = o[c][cx][cy][0] - o[c][cx][cy][1];
        P1[c][cx][cy] = o[c][cx][cy][0] + o[c][cx][cy][1];
      }
}

// One fine element: from the (x, y) transforms of its bottom and top node
// faces (F0, F1; [c][cx][cy]) to those of its bottom and top output faces.
__device__ __forceinline__ void haar_element(const double (&F0)[3][2][2], const double (&F1)[3][2][2],
                                             const SfCoef& k, double (&P0)[3][2][2],
                                             double (&P1)[3][2][2]) {
  double h[3][2][2][2], o[3][2][2][2];
  z_fwd(F0, F1, h);
  haar_op(h, k, o);
  z_bwd(o, P0, P1);
}

// One coarse element of the level-1 Galerkin operator (Eq. galerkin_level1,
// children free of Dirichlet DOFs): sum over its eight children p of
// E_p P_p^T K_e P_p.  Along each axis the trilinear interpolation onto a
// child maps the parent's (sum, difference) pair (S, D) to the child's
// (S -/+ D / 2, D / 2) (- for the lower child), and its transpose maps the
// child's output pair (s, d) to (s, (d -/+ s) / 2).  Carrying every
// difference at twice its value on the input side and at half on the output
// side leaves one multiply-add per pair and folds the factors into the
// coefficients (l1_coef).  E8[p], p = px + 2 py + 4 pz.
__device__ __forceinline__ void l1_element(const double (&F0)[3][2][2], const double (&F1)[3][2][2],
                                           const double (&E8)[8], const SfCoef& k,
                                           double (&P0)[3][2][2], double (&P1)[3][2][2]) {
  double h[3][2][2][2], O[3][2][2][2];
  z_fwd(F0, F1, h);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int i = 0; i < 8; ++i) O[c][i & 1][(i >> 1) & 1][i >> 2] = 0.0;
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    const double sx = (p & 1) ? 0.5 : -0.5, sy = (p & 2) ? 0.5 : -0.5, sz = (p & 4) ? 0.5 : -0.5;
    double ch[3][2][2][2], o[3][2][2][2];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int i = 0; i < 8; ++i) ch[c][i & 1][(i >> 1) & 1][i >> 2] = h[c][i & 1][(i >> 1) & 1][i >> 2];
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int z = 0; z < 2; ++z) ch[c][0][y][z] += sx * ch[c][1][y][z];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int z = 0; z < 2; ++z) ch[c][x][0][z] += sy * ch[c][x][1][z];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) ch[c][x][y][0] += sz * ch[c][x][y][1];
    }
    haar_op(ch, k, o);                 // E_p enters with the accumulation below
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) o[c][x][y][1] += sz * o[c][x][y][0];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int z = 0; z < 2; ++z) o[c][x][1][z] += sy * o[c][x][0][z];
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int z = 0; z < 2; ++z) o[c][1][y][z] += sx * o[c][0][y][z];
#pragma unroll
      for (int i = 0; i < 8; ++i)
        O[c][i & 1][(i >> 1) & 1][i >> 2] += E8[p] * o[c][i & 1][(i >> 1) & 1][i >> 2];
    }
  }
  z_bwd(O, P0, P1);
}

// L1 = false: the fine operator (E: one modulus per element).  L1 = true: the
// level-1 Galerkin operator on the coarse grid g (E: the eight child moduli
// of each coarse element, zero for coarse elements the product does not
// cover; nodes with skip[node] != 0 are left to another kernel).
template <int MODE, bool L1>
__device__ __forceinline__ void fine_sf64_body(Grid g, const double* __restrict__ E, SfCoef cf,
                                               const double* __restrict__ u,
                                               const uint8_t* __restrict__ fixn,
                                               const uint8_t* __restrict__ skip, Epi<double> ep,
                                               int zchunk, int ntx, int nty, int ntiles,
                                               int blk) {
  __shared__ __attribute__((aligned(16))) unsigned char lds_all[kSfWaves * kSfWave];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  unsigned char* const lds = lds_all + wave * kSfWave;
  const int tile = blk * kSfWaves + wave;
  const int tx = tile % ntx, tt = tile / ntx, ty = tt % nty, tz = tt / nty;
  const int gr = lane >> 4, n = lane & 15;
  const int xs = tx * 15, ys = ty * 3, zs = tz * zchunk;
  const int ex = xs - 1 + n, ey = ys - 1 + gr;
  const int zend = tile < ntiles ? min(zs + zchunk, g.Nz) : zs - 1;
  const size_t nvec = (size_t)g.n * sizeof(double);
  const __amdgpu_buffer_rsrc_t ru = make_rsrc(u, nvec);
  constexpr int kEs = L1 ? 64 : 8;                 // modulus bytes per element
  const __amdgpu_buffer_rsrc_t re = make_rsrc(E, (size_t)g.nel * kEs);
  const __amdgpu_buffer_rsrc_t rfix = make_rsrc(fixn, (size_t)g.Nn);
  const __amdgpu_buffer_rsrc_t rskip = make_rsrc(skip, L1 ? (size_t)g.Nn : 0);
  const __amdgpu_buffer_rsrc_t rb = make_rsrc(ep.b, MODE == EPI_RESID || MODE == EPI_SMOOTH ? nvec : 0);
  const __amdgpu_buffer_rsrc_t rdi = make_rsrc(ep.dinv, MODE == EPI_SMOOTH ? nvec : 0);
  const __amdgpu_buffer_rsrc_t rd = make_rsrc(ep.d, MODE == EPI_SMOOTH ? nvec : 0);
  const __amdgpu_buffer_rsrc_t rout = make_rsrc(ep.out, ep.out ? nvec : 0);   // NULL: stores dropped

  // two-part offsets (lane part + plane part); a part that must not be
  // accessed is kPoison, which puts the sum outside every buffer (vectors
  // below 2^30 bytes: sf64_size_ok)
  auto off2 = [](int a, int b) { return (int)((unsigned)a + (unsigned)b); };
  auto part = [](bool ok, int v) { return ok ? v : kPoison; };

  // node planes: load i, lane l < 51 carries node xs - 1 + l % 17 of node
  // row k = 3 i + l / 17 (rows 0 .. 4 of the tile)
  const int um = lane % 17, uk = lane / 17;
  int u_lane[2];
  bool u_on[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int k = 3 * i + uk;
    u_on[i] = lane < 51 && k <= 4;
    u_lane[i] = part(u_on[i] && (unsigned)(xs - 1 + um) < (unsigned)g.Nx &&
                         (unsigned)(ys - 1 + k) < (unsigned)g.Ny,
                     24 * (xs - 1 + um + g.Nx * (ys - 1 + k)));
  }
  double uv[2][3];
  auto load_u = [&](int P, bool need) {
    const int pp = part(need && (unsigned)P < (unsigned)g.Nz, 24 * g.Nx * g.Ny * P);
#pragma unroll
    for (int i = 0; i < 2; ++i) bload3(ru, off2(u_lane[i], pp), uv[i]);
  };
  auto store_u = [&](int P) {
    unsigned char* const slot = lds + ((P + 3) % 3) * kSfPlane + uk * kSfRow + um * 24;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      if (u_on[i]) {
        double* q = (double*)(slot + 3 * i * kSfRow);
        q[0] = uv[i][0];
        q[1] = uv[i][1];
        q[2] = uv[i][2];
      }
    }
  };

  // element modulus (moduli) of this lane, one plane ahead; zero outside the mesh
  const int e_lane = part((unsigned)ex < (unsigned)g.nx && (unsigned)ey < (unsigned)g.ny,
                          kEs * (ex + g.nx * ey));
  constexpr int NEv = L1 ? 8 : 1;
  double ev[NEv];
  auto load_e = [&](int ez, bool need) {
    const int pe = part(need && (unsigned)ez < (unsigned)g.nz, kEs * g.nx * g.ny * ez);
    const int o = off2(e_lane, pe);
    if (L1) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const auto t = __builtin_amdgcn_raw_buffer_load_b128(re, off2(o, 16 * q), 0, 0);
        ev[2 * q] = __hiloint2double((int)t[1], (int)t[0]);
        ev[2 * q + 1] = __hiloint2double((int)t[3], (int)t[2]);
      }
    } else {
      ev[0] = bload1d(re, o);
    }
  };

  // owned node (ex, ey) of each plane: lanes n >= 1, gr >= 1 inside the grid
  const bool own_xy = n >= 1 && gr >= 1 && ex < g.Nx && ey < g.Ny;
  const int o_lane = part(own_xy, 24 * (ex + g.Nx * ey));
  const int f_lane = part(own_xy, ex + g.Nx * ey);
  constexpr int NV = MODE == EPI_SMOOTH ? 3 : MODE == EPI_RESID ? 1 : 0;
  double vv[NV > 0 ? NV : 1][3];
  unsigned fv = 0, sv = 0;
  auto load_v = [&](int ez) {
    const bool own = ez >= zs && ez < zend;
    const int po = part(own, 24 * g.Nx * g.Ny * ez), pf = part(own, g.Nx * g.Ny * ez);
    fv = __builtin_amdgcn_raw_buffer_load_b8(rfix, off2(f_lane, pf), 0, 0);
    if (L1) sv = __builtin_amdgcn_raw_buffer_load_b8(rskip, off2(f_lane, pf), 0, 0);
    const int o = off2(o_lane, po);
    if (MODE == EPI_SMOOTH) {
      bload3(rb, o, vv[0]);
      bload3(rdi, o, vv[1]);
      bload3(rd, ep.c1 != 0.0 ? o : kNoOffset, vv[2]);
    } else if (MODE == EPI_RESID) {
      bload3(rb, o, vv[0]);
    }
  };

  double dot = 0.0;
  const int up = 4 * ((lane + 48) & 63);          // lane - 16 (group gr - 1)
  // node face of this lane's element on plane P: nodes (n + dx, gr + dy)
  double xown[3];                                  // node (n, gr) of the face
  auto read_face = [&](int P, double (&F)[3][2][2]) {
    double v[3][2][2];
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        const double* q = (const double*)(lds + ((P + 3) % 3) * kSfPlane + (gr + dy) * kSfRow +
                                          (n + dx) * 24);
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c][dx][dy] = q[c];
      }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xown[c] = v[c][0][0];
      face_fwd(v[c], F[c]);
    }
  };
  double F0[3][2][2], F1[3][2][2];     // input faces of the element (bottom, top)
  double Pc[3][2][2];                  // output carried from the element below
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int cx = 0; cx < 2; ++cx)
#pragma unroll
      for (int cy = 0; cy < 2; ++cy) Pc[c][cx][cy] = 0.0;
  load_u(zs - 1, true);
  store_u(zs - 1);
  load_u(zs, true);
  store_u(zs);
  load_u(zs + 1, zs + 1 <= zend);
  load_e(zs - 1, true);
  read_face(zs - 1, F0);
  for (int ez = zs - 1; ez < zend; ++ez) {
    store_u(ez + 2);                               // loaded during the previous plane
    double esc[NEv];
#pragma unroll
    for (int q = 0; q < NEv; ++q) esc[q] = ev[q];
    load_u(ez + 3, ez + 3 <= zend);
    load_e(ez + 1, ez + 1 < zend);
    load_v(ez);
    double x[3] = {xown[0], xown[1], xown[2]};     // the owned node's input (plane ez)
    read_face(ez + 1, F1);
    double P0[3][2][2], P1[3][2][2];
    if constexpr (L1)
      l1_element(F0, F1, esc, cf, P0, P1);
    else
      haar_element(F0, F1, scaled(cf, esc[0]), P0, P1);
    // node plane ez: this element's bottom face + the top face of the one
    // below, then the inverse (x, y) butterflies, then x and y sums
    double y[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double P[2][2], w[2][2];
#pragma unroll
      for (int cx = 0; cx < 2; ++cx)
#pragma unroll
        for (int cy = 0; cy < 2; ++cy) {
          P[cx][cy] = P0[c][cx][cy] + Pc[c][cx][cy];
          Pc[c][cx][cy] = P1[c][cx][cy];
          F0[c][cx][cy] = F1[c][cx][cy];
        }
      face_bwd(P, w);
      const double x0 = w[0][0] + dpp_shr1(w[1][0]);   // dx = 1 of lane n - 1
      const double x1 = w[0][1] + dpp_shr1(w[1][1]);
      y[c] = x0 + bpermute(up, x1);                    // dy = 1 of lane - 16
    }
    const int o = off2(o_lane, part(ez >= zs && ez < zend && sv == 0, 24 * g.Nx * g.Ny * ez));
    const bool mine = (unsigned)o < (unsigned)kPoison;
    double out[3], dd[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const bool fixed = (fv >> c) & 1u;
      const double xo = x[c];
      if (MODE == EPI_STORE || MODE == kStoreDot) {
        out[c] = fixed ? 0.0 : y[c];
        if (MODE == kStoreDot && mine) dot += xo * out[c];
      } else if (MODE == EPI_RESID) {
        out[c] = fixed ? 0.0 : vv[0][c] - y[c];
      } else {
        const double r = vv[0][c] - y[c];
        dd[c] = fixed ? 0.0 : ep.c1 * vv[2][c] + ep.c2 * vv[1][c] * r;
        out[c] = fixed ? 0.0 : xo + dd[c];
      }
    }
    bstore3(rout, o, out[0], out[1], out[2]);
    if (MODE == EPI_SMOOTH) {
      if (ep.store_d) bstore3(rd, o, dd[0], dd[1], dd[2]);
      if (ep.out64 && mine) {                      // the cycle's result (ep.out may be NULL)
        double* q = ep.out64 + (o >> 3);
        q[0] = out[0];
        q[1] = out[1];
        q[2] = out[2];
      }
    }
  }
  if (MODE == kStoreDot) {
    const double vd[1] = {dot};
    grid_sum<1>(vd, ep.ws);
  }
}

template <int MODE>
__global__ __launch_bounds__(64 * kSfWaves) void k_apply_fine_sf64(
    Grid g, const double* __restrict__ E, SfCoef cf, const double* __restrict__ u,
    const uint8_t* __restrict__ fixn, Epi<double> ep, int zchunk, int ntx, int nty, int ntiles) {
  fine_sf64_body<MODE, false>(g, E, cf, u, fixn, nullptr, ep, zchunk, ntx, nty, ntiles,
                              xcd_block(blockIdx.x, gridDim.x));
}

// Thread t = (listed node i, component d): the gathered stencil row
// (Sd[(o * 9 + 3 d + e) * nlist + i]) times the 27 neighbour values, then
// the epilogue.
__device__ inline void l1_list_row(const Grid& g, const double* __restrict__ Sd,
                                   const double* __restrict__ u, const uint8_t* __restrict__ fixn,
                                   const Epi<double>& ep, const int* __restrict__ list, int nlist,
                                   int t) {
  if (t >= 3 * nlist) return;
  const int i = t / 3, d = t - 3 * i;
  const int node = list[i];
  const size_t dof = 3 * (size_t)node + d;
  const Epi1In<double> ein = epilogue1_load(ep, dof);
  const unsigned fx = fixn[node];
  const int x = node % g.Nx, tt = node / g.Nx, y = tt % g.Ny, z = tt / g.Ny;
  double acc = 0.0;
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
    const bool ok = (unsigned)(x + ox) < (unsigned)g.Nx && (unsigned)(y + oy) < (unsigned)g.Ny &&
                    (unsigned)(z + oz) < (unsigned)g.Nz;
    const double* un = u + 3 * (size_t)(ok ? node + ox + g.Nx * (oy + g.Ny * oz) : node);
    const double* Sb = Sd + ((size_t)o * 9 + 3 * d) * nlist + i;
    acc += Sb[0] * un[0] + Sb[nlist] * un[1] + Sb[2 * (size_t)nlist] * un[2];
  }
  epilogue1(ep, dof, (fx >> d) & 1u, u[dof], acc, ein);
}

// Blocks [0, nlb): the listed rows; the rest: the element-product tiles.
template <int MODE>
__global__ __launch_bounds__(64 * kSfWaves) void k_apply_l1_haar(
    Grid g, const double* __restrict__ E8, SfCoef cf, const double* __restrict__ u,
    const uint8_t* __restrict__ fixn, const uint8_t* __restrict__ skip, Epi<double> ep, int zchunk,
    int ntx, int nty, int ntiles, const double* __restrict__ Sd, const int* __restrict__ list,
    int nlist, int nlb) {
  if ((int)blockIdx.x < nlb) {                 // uniform over the block
    l1_list_row(g, Sd, u, fixn, ep, list, nlist, blockIdx.x * 64 * kSfWaves + threadIdx.x);
    return;
  }
  const int nt = gridDim.x - nlb;
  fine_sf64_body<MODE, true>(g, E8, cf, u, fixn, skip, ep, zchunk, ntx, nty, ntiles,
                             xcd_block(blockIdx.x - nlb, nt));
}

// Stage-batched outer q = K p with the p.q block partials: block b is entry
// tab[b] = (item, block of the item's tile grid); geo[item] holds that grid
// (ntx, nty, ntiles) for zchunk planes (the tiles of the MFMA operator with 4
// rows).
__global__ __launch_bounds__(64 * kSfWaves) void k_bs_fine_sf64(
    const BSys* __restrict__ sys, const BItem* __restrict__ items, const int2* __restrict__ tab,
    const int4* __restrict__ geo, const int* __restrict__ flags, double* __restrict__ part,
    int zchunk) {
  const int2 e = tab[blockIdx.x];
  if (!flags[e.x]) return;                     // uniform over the block
  const BItem& I = items[e.x];
  const BSys& S = sys[I.sys];
  const BLevel& V = S.lev[0];
  const int4 gm = geo[e.x];
  Epi<double> ep{};
  ep.mode = EPI_STORE;
  ep.out = I.q;
  ep.want_dot = 1;
  ep.ws.partials = part;
  fine_sf64_body<kStoreDot, false>(V.g, S.E64, sf_coef(S.lam, S.mu), I.p, V.fixn, nullptr, ep,
                                   zchunk, gm.x, gm.y, gm.z, e.y);
}

struct SfLaunch { int ntx, nty, ntiles, blocks; };
SfLaunch sf_launch(const Grid& g, int zchunk) {
  SfLaunch m;
  m.ntx = div_up(g.Nx, 15);
  m.nty = div_up(g.Ny, 3);
  m.ntiles = m.ntx * m.nty * div_up(g.Nz, zchunk);
  m.blocks = div_up(m.ntiles, kSfWaves);
  return m;
}

}  // namespace

// Child moduli of each coarse element (p = px + 2 py + 4 pz) and whether the
// element is left out: a Dirichlet DOF on one of its 27 fine nodes, or the
// last element along an odd fine axis (three children there).
__global__ void k_l1_child_moduli(Grid f, Grid c, const double* __restrict__ E,
                                  const uint8_t* __restrict__ ffix, double* __restrict__ E8,
                                  uint8_t* __restrict__ el_out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= c.nel) return;
  const int cx = e % c.nx, t = e / c.nx, cy = t % c.ny, cz = t / c.ny;
  bool out = (2 * cx + 2 < f.nx && cx == c.nx - 1) || (2 * cy + 2 < f.ny && cy == c.ny - 1) ||
             (2 * cz + 2 < f.nz && cz == c.nz - 1);
  for (int a = 0; a < 27 && !out; ++a) {
    const int x = 2 * cx + a % 3, y = 2 * cy + (a / 3) % 3, z = 2 * cz + a / 9;
    out = ffix[x + f.Nx * (y + f.Ny * z)] != 0;
  }
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    const int x = 2 * cx + (p & 1), y = 2 * cy + ((p >> 1) & 1), z = 2 * cz + (p >> 2);
    E8[8 * (size_t)e + p] = out ? 0.0 : E[x + f.nx * (y + f.ny * z)];
  }
  el_out[e] = out ? 1 : 0;
}

// Coarse nodes whose row the matrix-free product does not complete: next to
// a left-out element, or with a Dirichlet DOF.
__global__ void k_l1_skip_nodes(Grid c, const uint8_t* __restrict__ el_out,
                                const uint8_t* __restrict__ cfix, uint8_t* __restrict__ skip) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= c.Nn) return;
  const int i = n % c.Nx, t = n / c.Nx, j = t % c.Ny, k = t / c.Ny;
  bool sk = cfix[n] != 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int ex = i - 1 + (q & 1), ey = j - 1 + ((q >> 1) & 1), ez = k - 1 + (q >> 2);
    if ((unsigned)ex < (unsigned)c.nx && (unsigned)ey < (unsigned)c.ny && (unsigned)ez < (unsigned)c.nz)
      sk = sk || el_out[ex + c.nx * (ey + c.ny * ez)] != 0;
  }
  skip[n] = sk ? 1 : 0;
}

void launch_l1_child_moduli(const Grid& fine, const Grid& coarse, const double* E,
                            const uint8_t* ffix, double* E8, uint8_t* el_out, hipStream_t s) {
  k_l1_child_moduli<<<div_up(coarse.nel, 256), 256, 0, s>>>(fine, coarse, E, ffix, E8, el_out);
}

void launch_l1_skip_nodes(const Grid& coarse, const uint8_t* el_out, const uint8_t* cfix,
                          uint8_t* skip, hipStream_t s) {
  k_l1_skip_nodes<<<div_up(coarse.Nn, 256), 256, 0, s>>>(coarse, el_out, cfix, skip);
}

bool l1_haar_size_ok(const Grid& c) {
  return (size_t)c.nel * 64 < ((size_t)1 << 30) - 64 && (size_t)c.n * sizeof(double) < ((size_t)1 << 30) - 64;
}

void launch_apply_l1_haar(const Grid& c, int zchunk, const double* E8, double lam, double mu,
                          const double* u, const uint8_t* fixn, const uint8_t* skip,
                          const double* Sd, const int* list, int nlist, const Epi<double>& ep,
                          hipStream_t s) {
  if (zchunk < 1) zchunk = 1;
  const SfLaunch m = sf_launch(c, zchunk);
  const SfCoef cf = l1_coef(lam, mu);
  const int nlb = div_up(3 * std::max(nlist, 0), 64 * kSfWaves);
  const dim3 grid(nlb + m.blocks), block(64 * kSfWaves);
#define SGMG_L1(M)                                                                          \
  k_apply_l1_haar<M><<<grid, block, 0, s>>>(c, E8, cf, u, fixn, skip, ep, zchunk, m.ntx, m.nty, \
                                            m.ntiles, Sd, list, nlist, nlb)
  if (ep.mode == EPI_STORE) SGMG_L1(EPI_STORE);
  else if (ep.mode == EPI_RESID) SGMG_L1(EPI_RESID);
  else SGMG_L1(EPI_SMOOTH);
#undef SGMG_L1
}

bool sf64_size_ok(const Grid& g) {
  return (size_t)g.n * sizeof(double) < ((size_t)1 << 30) - 64;
}

void bs_fine_sf64_store_dot(const BsArgs& a, const BsTable& t, const int4* geo, const int* flags,
                            int zchunk, double* part, hipStream_t s) {
  if (t.n == 0) return;
  k_bs_fine_sf64<<<t.n, 64 * kSfWaves, 0, s>>>(a.sys, a.items, t.blk, geo, flags, part, zchunk);
}

size_t apply_fine_sf64_blocks(const Grid& g, int zchunk) {
  return (size_t)sf_launch(g, zchunk < 1 ? 1 : zchunk).blocks;
}

void launch_apply_fine_sf64(const Grid& g, int zchunk, const double* E, double lam, double mu,
                            const double* u, const uint8_t* fixn, const Epi<double>& ep,
                            hipStream_t s) {
  if (zchunk < 1) zchunk = 1;
  const SfLaunch m = sf_launch(g, zchunk);
  const SfCoef cf = sf_coef(lam, mu);
  const dim3 grid(m.blocks), block(64 * kSfWaves);
  if (ep.mode == EPI_STORE && ep.want_dot)
    k_apply_fine_sf64<kStoreDot><<<grid, block, 0, s>>>(g, E, cf, u, fixn, ep, zchunk, m.ntx,
                                                        m.nty, m.ntiles);
  else if (ep.mode == EPI_STORE)
    k_apply_fine_sf64<EPI_STORE><<<grid, block, 0, s>>>(g, E, cf, u, fixn, ep, zchunk, m.ntx,
                                                        m.nty, m.ntiles);
  else if (ep.mode == EPI_RESID)
    k_apply_fine_sf64<EPI_RESID><<<grid, block, 0, s>>>(g, E, cf, u, fixn, ep, zchunk, m.ntx,
                                                        m.nty, m.ntiles);
  else
    k_apply_fine_sf64<EPI_SMOOTH><<<grid, block, 0, s>>>(g, E, cf, u, fixn, ep, zchunk, m.ntx,
                                                         m.nty, m.ntiles);
  if (ep.mode == EPI_STORE && ep.want_dot && ep.dot_out)
    launch_finalize(ep.ws, m.blocks, 1, ep.dot_out, s);
}

}  // namespace sgmg
