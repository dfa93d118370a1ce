// Galerkin levels (l >= 1): assembly into a structured 27-point block
// stencil, its application, and the trilinear transfer kernels.
#include "batch.hpp"
#include "bstage.hpp"
#include "kernels.hpp"
#include "node_ops.hpp"

namespace sgmg {

// 1D local pattern of a fine element inside its coarse element (Sec. 3.3):
// pattern p = fine index - 2 * coarse index in {0, 1, 2}; entry [dx][cx] is
// the weight of coarse local node cx at fine local node dx.  Pattern 2 is the
// last fine element of an odd axis, whose two nodes both map onto the last
// coarse node (trailing-node weight 1).
__device__ __constant__ double c_pat[3][2][2] = {
    {{1.0, 0.0}, {0.5, 0.5}}, {{0.5, 0.5}, {0.0, 1.0}}, {{0.0, 1.0}, {0.0, 1.0}}};

__device__ inline bool elem_has_fixed(const Grid& f, const uint8_t* ffix, int ex, int ey, int ez) {
  unsigned any = 0;
#pragma unroll
  for (int a = 0; a < 8; ++a)
    any |= ffix[(ex + (a & 1)) + f.Nx * ((ey + ((a >> 1) & 1)) + f.Ny * (ez + (a >> 2)))];
  return any != 0;
}

// Level-1 Galerkin aggregation (Eq. galerkin_level1).  Thread (I, o) owns the
// 3x3 block K^1[I, I+o]: it visits the coarse elements that contain both
// nodes and their fine children, adding E_child * G_p[rows of I, cols of J]
// where G_p = P_p^T K_e P_p is the precomputed local triple product of the
// child's pattern.  Children touching a fixed fine DOF use M_e K_e M_e,
// formed on the fly.  Finally rows/columns of fixed coarse DOFs are zeroed.
__global__ __launch_bounds__(256) void k_galerkin_l1(Grid f, Grid c, const double* __restrict__ E,
                                                     const double* __restrict__ gtab,
                                                     const double* __restrict__ ke,
                                                     const uint8_t* __restrict__ ffix,
                                                     const uint8_t* __restrict__ cfix,
                                                     double* __restrict__ S) {
  const int I = blockIdx.x * 256 + threadIdx.x;
  const int o = blockIdx.y;
  if (I >= c.Nn) return;
  const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
  const int Ix = I % c.Nx, t = I / c.Nx, Iy = t % c.Ny, Iz = t / c.Ny;
  const int Jx = Ix + ox, Jy = Iy + oy, Jz = Iz + oz;
  double acc[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) acc[q] = 0.0;
  const bool jok = (unsigned)Jx < (unsigned)c.Nx && (unsigned)Jy < (unsigned)c.Ny &&
                   (unsigned)Jz < (unsigned)c.Nz;
  if (jok) {
    // coarse elements containing both I and J, per axis
    const int cx0 = max(max(Ix, Jx) - 1, 0), cx1 = min(min(Ix, Jx), c.nx - 1);
    const int cy0 = max(max(Iy, Jy) - 1, 0), cy1 = min(min(Iy, Jy), c.ny - 1);
    const int cz0 = max(max(Iz, Jz) - 1, 0), cz1 = min(min(Iz, Jz), c.nz - 1);
    for (int cz = cz0; cz <= cz1; ++cz)
      for (int cy = cy0; cy <= cy1; ++cy)
        for (int cx = cx0; cx <= cx1; ++cx) {
          const int aI = (Ix - cx) + 2 * (Iy - cy) + 4 * (Iz - cz);
          const int aJ = (Jx - cx) + 2 * (Jy - cy) + 4 * (Jz - cz);
          const int npx = (cx == c.nx - 1 && (f.nx & 1)) ? 3 : 2;
          const int npy = (cy == c.ny - 1 && (f.ny & 1)) ? 3 : 2;
          const int npz = (cz == c.nz - 1 && (f.nz & 1)) ? 3 : 2;
          for (int pz = 0; pz < npz; ++pz)
            for (int py = 0; py < npy; ++py)
              for (int px = 0; px < npx; ++px) {
                const int ex = 2 * cx + px, ey = 2 * cy + py, ez = 2 * cz + pz;
                const double Ee = E[ex + f.nx * (ey + f.ny * ez)];
                const int p = px + 3 * py + 9 * pz;
                if (!elem_has_fixed(f, ffix, ex, ey, ez)) {
                  const double* G = gtab + (size_t)p * 576;
#pragma unroll
                  for (int d = 0; d < 3; ++d)
#pragma unroll
                    for (int e = 0; e < 3; ++e)
                      acc[3 * d + e] += Ee * G[(3 * aI + d) * 24 + 3 * aJ + e];
                } else {
                  // masked child: sum_{alpha,beta} W(alpha,aI) W(beta,aJ) m K_e m
                  for (int al = 0; al < 8; ++al) {
                    const double wa = c_pat[px][al & 1][aI & 1] *
                                      c_pat[py][(al >> 1) & 1][(aI >> 1) & 1] *
                                      c_pat[pz][al >> 2][aI >> 2];
                    if (wa == 0.0) continue;
                    const unsigned fa = ffix[(ex + (al & 1)) + f.Nx * ((ey + ((al >> 1) & 1)) +
                                                                        f.Ny * (ez + (al >> 2)))];
                    for (int be = 0; be < 8; ++be) {
                      const double wb = c_pat[px][be & 1][aJ & 1] *
                                        c_pat[py][(be >> 1) & 1][(aJ >> 1) & 1] *
                                        c_pat[pz][be >> 2][aJ >> 2];
                      if (wb == 0.0) continue;
                      const unsigned fb =
                          ffix[(ex + (be & 1)) +
                               f.Nx * ((ey + ((be >> 1) & 1)) + f.Ny * (ez + (be >> 2)))];
                      for (int d = 0; d < 3; ++d) {
                        if ((fa >> d) & 1u) continue;
                        for (int e = 0; e < 3; ++e) {
                          if ((fb >> e) & 1u) continue;
                          acc[3 * d + e] += Ee * wa * wb * ke[(3 * al + d) * 24 + 3 * be + e];
                        }
                      }
                    }
                  }
                }
              }
        }
  }
  const unsigned fI = cfix[I];
  const unsigned fJ = jok ? cfix[Jx + c.Nx * (Jy + c.Ny * Jz)] : 7u;
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const bool z = ((fI >> d) & 1u) || ((fJ >> e) & 1u);
      S[(size_t)(o * 9 + 3 * d + e) * c.Nn + I] = z ? 0.0 : acc[3 * d + e];
    }
}

void launch_galerkin_l1(const Grid& fine, const Grid& coarse, const double* E, const double* gtab,
                        const double* ke, const uint8_t* ffix, const uint8_t* cfix, double* S,
                        hipStream_t s) {
  dim3 grid(div_up(coarse.Nn, 256), 27);
  k_galerkin_l1<<<grid, 256, 0, s>>>(fine, coarse, E, gtab, ke, ffix, cfix, S);
}

// Deeper Galerkin product K^{l+1} = M P^T K^l P M on stencils (Sec. 3.3).
// Thread (I, o) sums w(i,I) w(j,J) K^l[i, j] over the fine nodes i that
// interpolate from I and their stencil neighbours j.  The weights factor over
// the axes, so each axis contributes a 3 x 3 table of pair weights
// w1d(i,I) w1d(j,J) for i = 2I + a - 1, j = i + b - 1 (zero where a node is
// outside the grid or outside the support).  The loops over the z and y pairs
// skip zero weights before any load.  K^l is stored masked, so only the coarse mask is applied here.
__device__ inline double axis_pair_weight(int I, int J, int nf, int k) {
  const int i = 2 * I + k / 3 - 1, j = i + k % 3 - 1;
  return ((unsigned)i <= (unsigned)nf && (unsigned)j <= (unsigned)nf) ? w1d(i, I, nf) * w1d(j, J, nf)
                                                                      : 0.0;
}

// Sum over the pairs of one thread.  Of the nine x pairs, only those with
// i and j both in the supports of I and J = I + OX can carry weight (the
// support of a coarse node J is fine nodes 2J-1 .. 2J+1): pairs {0, 1, 3} for
// OX = -1, {1, .., 7} for OX = 0 and {5, 7, 8} for OX = +1.  Those are loaded
// without branches so that their loads are in flight together; a pair whose
// weight is zero at the grid's edge reads an entry inside the grid and adds
// 0 times it (every stencil entry is written, and finite).
template <int OX>
__device__ inline void galerkin_pairs(const Grid& f, const double* __restrict__ Sf, int Ix,
                                      int Iy, int Iz, int Jy, int Jz, double (&acc)[9]) {
  constexpr unsigned kMask = OX < 0 ? 0x00Bu : (OX == 0 ? 0x0FEu : 0x1A0u);
  double wx[9];
#pragma unroll
  for (int k = 0; k < 9; ++k)
    wx[k] = (kMask >> k) & 1u ? axis_pair_weight(Ix, Ix + OX, f.nx, k) : 0.0;
  // fine x index of each pair, clamped into the grid: where the clamp moves
  // it the pair's weight is zero, and the load only has to stay in bounds
  int ix[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) ix[k] = min(max(2 * Ix + k / 3 - 1, 0), f.nx);
  const size_t blk = (size_t)9 * f.Nn;       // distance between stencil blocks q, q+1
  for (int kz = 0; kz < 9; ++kz) {
    const double wz = axis_pair_weight(Iz, Jz, f.nz, kz);
    if (wz == 0.0) continue;
    const int iz = 2 * Iz + kz / 3 - 1;
    for (int ky = 0; ky < 9; ++ky) {
      const double wyz = axis_pair_weight(Iy, Jy, f.ny, ky) * wz;
      if (wyz == 0.0) continue;
      const int iy = 2 * Iy + ky / 3 - 1;
      // block of (qx = -1, qy, qz) at fine node (0, iy, iz)
      const int q0 = 3 * (ky % 3) + 9 * (kz % 3);
      const double* row = Sf + (size_t)q0 * blk + f.Nx * (iy + f.Ny * iz);
#pragma unroll
      for (int kx = 0; kx < 9; ++kx) {
        if (!((kMask >> kx) & 1u)) continue;
        const double w = wx[kx] * wyz;
        const double* src = row + (size_t)(kx % 3) * blk + ix[kx];
#pragma unroll
        for (int de = 0; de < 9; ++de) acc[de] += w * src[(size_t)de * f.Nn];
      }
    }
  }
}

// Two waves per SIMD: the register budget lets the scheduler keep a whole
// y pair's loads in flight (the kernel is bound by their latency).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void
k_galerkin_stencil(Grid f, Grid c, const double* __restrict__ Sf, const uint8_t* __restrict__ cfix,
                   double* __restrict__ Sc) {
  const int I = blockIdx.x * 256 + threadIdx.x;
  const int o = blockIdx.y;
  if (I >= c.Nn) return;
  const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
  const int Ix = I % c.Nx, t = I / c.Nx, Iy = t % c.Ny, Iz = t / c.Ny;
  const int Jx = Ix + ox, Jy = Iy + oy, Jz = Iz + oz;
  double acc[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) acc[q] = 0.0;
  const bool jok = (unsigned)Jx < (unsigned)c.Nx && (unsigned)Jy < (unsigned)c.Ny &&
                   (unsigned)Jz < (unsigned)c.Nz;
  if (jok) {
    if (ox < 0)
      galerkin_pairs<-1>(f, Sf, Ix, Iy, Iz, Jy, Jz, acc);
    else if (ox == 0)
      galerkin_pairs<0>(f, Sf, Ix, Iy, Iz, Jy, Jz, acc);
    else
      galerkin_pairs<1>(f, Sf, Ix, Iy, Iz, Jy, Jz, acc);
  }
  const unsigned fI = cfix[I];
  const unsigned fJ = jok ? cfix[Jx + c.Nx * (Jy + c.Ny * Jz)] : 7u;
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const bool z = ((fI >> d) & 1u) || ((fJ >> e) & 1u);
      Sc[(size_t)(o * 9 + 3 * d + e) * c.Nn + I] = z ? 0.0 : acc[3 * d + e];
    }
}

void launch_galerkin_stencil(const Grid& fine, const Grid& coarse, const double* Sf,
                             const uint8_t* cfix, double* Sc, hipStream_t s) {
  dim3 grid(div_up(coarse.Nn, 256), 27);
  k_galerkin_stencil<<<grid, 256, 0, s>>>(fine, coarse, Sf, cfix, Sc);
}

__global__ void k_stencil_diag(Grid g, const double* __restrict__ S, double* __restrict__ d) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.Nn) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) d[3 * n + c] = S[(size_t)(13 * 9 + 4 * c) * g.Nn + n];
}

void launch_stencil_diag(const Grid& g, const double* S, double* d, hipStream_t s) {
  k_stencil_diag<<<div_up(g.Nn, 256), 256, 0, s>>>(g, S, d);
}

__global__ void k_stencil_to_f32(const double* __restrict__ S, float* __restrict__ S32, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) S32[i] = (float)S[i];
}

void launch_stencil_to_f32(const double* S, float* S32, size_t n, hipStream_t s) {
  k_stencil_to_f32<<<div_up((long)n, 256), 256, 0, s>>>(S, S32, n);
}

// y = K^l u on the stored stencil with a fused epilogue.
// Only the upper half of the stencil is read: block o >= 13 (offsets that are
// lexicographically >= 0) of node n, and for the lower offsets the transpose
// of the mirrored block of the neighbour, A[n, n+o] = A[n+o, n]^T =
// (S_{26-o}[n+o])^T.  The neighbour's block is that neighbour's own upper
// block, so the second read is served from cache: about half the HBM bytes of
// the full stencil, and the applied operator is exactly symmetric.
// Two kernel forms, both with a block of 64 consecutive nodes (every stencil
// load of a wave is 64 consecutive values of one slot) and the block index
// remapped per XCD so each L2 sees a contiguous node range.
//
// Row-split form, for small levels (level 2 of an 80^3 mesh has 9,261
// nodes) that need many waves to cover memory latency: one thread per (node,
// output component, stencil row (oy, oz)).  A block of nine waves is one
// component d of 64 nodes, wave = row, so the grid has three blocks per node
// tile (enough to reach every CU on such levels) and each thread has only
// the three offsets of its row in flight; the offsets are read
// unconditionally (offsets outside the grid read the node itself, a valid
// address, and add zero) and the nine row partials are added in LDS in a
// fixed order.
// The body takes the block's index lb (component lb % 3 of node tile
// lb / 3), so one mesh (lb from the launch grid) and the stage-batched
// solver (lb from its table of (item, block) entries) share it.
constexpr int kRowSplitThreads = 9 * 64;

template <typename T>
__device__ __forceinline__ void stencil_c_body(Grid g, const T* __restrict__ S,
                                               const T* __restrict__ u,
                                               const uint8_t* __restrict__ fixn, Epi<T> ep,
                                               int lb) {
  __shared__ double part[9][64];
  const int lane = threadIdx.x & 63, pr = threadIdx.x >> 6;
  const int d = lb % 3;
  const int node0 = (lb / 3) * 64 + lane;
  const bool in = node0 < g.Nn;
  // lanes past the grid work on the last node and store nothing
  const int node = in ? node0 : g.Nn - 1;
  // the epilogue's operands are loaded first (one memory round trip less)
  const size_t dof = 3 * (size_t)node + d;
  const bool epi = in && pr == 4;
  Epi1In<T> ein{(T)0, (T)0, (T)0};
  unsigned fx = 0;
  T xown = (T)0;
  if (epi) {
    ein = epilogue1_load(ep, dof);
    fx = fixn[node];
    xown = u[dof];
  }
  {
    const int i = node % g.Nx, t = node / g.Nx, j = t % g.Ny, k = t / g.Ny;
    const size_t Nn = g.Nn;
    T acc = (T)0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int o = 3 * pr + q;
      const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
      const bool ok = (unsigned)(i + ox) < (unsigned)g.Nx && (unsigned)(j + oy) < (unsigned)g.Ny &&
                      (unsigned)(k + oz) < (unsigned)g.Nz;
      const int nb = ok ? node + ox + g.Nx * (oy + g.Ny * oz) : node;
      const size_t b3 = 3 * (size_t)nb;
      const T u0 = u[b3], u1 = u[b3 + 1], u2 = u[b3 + 2];
      T v;
      if (o >= 13) {
        const T* Sb = S + ((size_t)o * 9 + 3 * d) * Nn + node;
        v = Sb[0] * u0 + Sb[Nn] * u1 + Sb[2 * Nn] * u2;
      } else {
        const T* Sb = S + ((size_t)(26 - o) * 9 + d) * Nn + nb;
        v = Sb[0] * u0 + Sb[3 * Nn] * u1 + Sb[6 * Nn] * u2;
      }
      acc += ok ? v : (T)0;
    }
    part[pr][lane] = (double)acc;
  }
  __syncthreads();
  double dot = 0.0;
  if (epi) {
    double y = 0.0;
#pragma unroll
    for (int r = 0; r < 9; ++r) y += part[r][lane];
    dot = epilogue1(ep, dof, (fx >> d) & 1u, xown, y, ein);
  }
  if (ep.want_dot) {
    const double v[1] = {dot};
    grid_sum<1>(v, ep.ws);
  }
}

template <typename T>
__global__ __launch_bounds__(kRowSplitThreads) void k_stencil_apply_c(Grid g,
                                                                      const T* __restrict__ S,
                                                                      const T* __restrict__ u,
                                                                      const uint8_t* __restrict__ fixn,
                                                                      Epi<T> ep) {
  stencil_c_body<T>(g, S, u, fixn, ep, xcd_block(blockIdx.x, gridDim.x));
}

// Stage-batched form on Galerkin level l: the damped-Jacobi step (MODE
// EPI_SMOOTH) or the residual (EPI_RESID) of every active item, block b being
// entry tab[b] = (item, block of the item's level-l grid); the vectors and
// the damping are the item's (damped Jacobi with the level's omega).
template <int MODE>
__global__ __launch_bounds__(kRowSplitThreads) void k_bs_stencil(const BSys* __restrict__ sys,
                                                                 const BItem* __restrict__ items,
                                                                 const int2* __restrict__ tab,
                                                                 const int* __restrict__ flags,
                                                                 int l, int cin) {
  const int2 e = tab[blockIdx.x];
  if (!flags[e.x]) return;                     // uniform over the block
  const BItem& I = items[e.x];
  const BSys& Sy = sys[I.sys];
  const BLevel& V = Sy.lev[l];
  Epi<double> ep{};
  ep.mode = MODE;
  ep.b = I.lb[l];
  if (MODE == EPI_RESID) {
    ep.out = I.lr[l];
  } else {
    ep.out = I.lx[l][1 - cin];
    ep.dinv = V.dinv64;
    ep.c2 = V.omega;
  }
  stencil_c_body<double>(V.g, V.S64, I.lx[l][cin], V.fixn, ep, e.y);
}

int bs_stencil_blocks(const Grid& g) { return 3 * (int)div_up(g.Nn, 64); }

void bs_stencil(const BsArgs& a, const BsTable& t, const int* flags, int l, int mode, int cin,
                hipStream_t s) {
  if (t.n == 0) return;
  if (mode == EPI_RESID)
    k_bs_stencil<EPI_RESID><<<t.n, kRowSplitThreads, 0, s>>>(a.sys, a.items, t.blk, flags, l, cin);
  else
    k_bs_stencil<EPI_SMOOTH><<<t.n, kRowSplitThreads, 0, s>>>(a.sys, a.items, t.blk, flags, l, cin);
}

// LDS-staged form, for large levels (from kStencilSplitNodes nodes on): one
// thread per (node, output component), all 27 offsets, neighbour values from
// LDS.  Each block stages the u entries its 64 nodes touch once:
// for each of the 9 (oy, oz) rows, the 66 nodes node0 - 1 + oy Nx + oz Nx Ny
// ... node0 + 64 + oy Nx + oz Nx Ny (all three components, contiguous in
// memory, so the staging loads are coalesced; entries outside the vector
// are zero).  The three waves (one per output component) then read only
// their stencil entries from memory: 3 coalesced loads per offset, no branch
// (offsets outside the grid read valid stencil slots and are masked), so
// the loads of many offsets are in flight together, while the
// stride-3 neighbour reads that would otherwise triple the vector-memory
// instructions go to LDS.
template <typename T>
__device__ __forceinline__ void stencil_s_body(Grid g, const T* __restrict__ S,
                                               const T* __restrict__ u,
                                               const uint8_t* __restrict__ fixn, Epi<T> ep,
                                               int lb) {
  constexpr int kRow = 66 * 3;
  __shared__ T us[9][kRow];
  const int lane = threadIdx.x & 63, d = threadIdx.x >> 6;
  const long node0 = (long)lb * 64;
  const bool in = node0 + lane < g.Nn;
  const int node = in ? (int)node0 + lane : g.Nn - 1;
  // the epilogue's operands are loaded first (one memory round trip less)
  const size_t dof = 3 * (size_t)node + d;
  const Epi1In<T> ein = epilogue1_load(ep, dof);
  const unsigned fx = fixn[node];
  {
    // thread t stages entry t of each row (and entry 192 + t for t < 6);
    // the loads read clamped indices unconditionally so that all of them
    // are in flight together, and the value is zeroed outside the vector
    static_assert(kRow > 192 && kRow - 192 <= 64, "row staging covers 192 + a wave");
    const long n3 = 3L * g.Nn, plane = (long)g.Nx * g.Ny;
    const int t = threadIdx.x;
    long base[9];
    T v[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      base[r] = 3 * (node0 - 1 + (r % 3 - 1) * (long)g.Nx + (r / 3 - 1) * plane);
      const long i0 = base[r] + t;
      v[r] = u[i0 < 0 ? 0 : i0 >= n3 ? n3 - 1 : i0];
    }
    if (t < kRow - 192) {
      T w[9];
#pragma unroll
      for (int r = 0; r < 9; ++r) {
        const long i1 = base[r] + 192 + t;
        w[r] = u[i1 < 0 ? 0 : i1 >= n3 ? n3 - 1 : i1];
      }
#pragma unroll
      for (int r = 0; r < 9; ++r) {
        const long i1 = base[r] + 192 + t;
        us[r][192 + t] = (i1 >= 0 && i1 < n3) ? w[r] : (T)0;
      }
    }
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      const long i0 = base[r] + t;
      us[r][t] = (i0 >= 0 && i0 < n3) ? v[r] : (T)0;
    }
  }
  __syncthreads();
  const int i = node % g.Nx, tt = node / g.Nx, j = tt % g.Ny, k = tt / g.Ny;
  const size_t Nn = g.Nn;
  T acc = (T)0;
  // offsets in the order 13, 12, 14, 11, 15, ..., 0, 26: the entries of a
  // lower offset 13 - p are the neighbour's entries of the upper offset
  // 13 + p, the same array this block reads for its own nodes at the next
  // step and the neighbouring blocks read at about the same time, so the
  // second read of each line finds it in L2
#pragma unroll
  for (int q = 0; q < 27; ++q) {
    const int o = (q & 1) ? 13 - ((q + 1) >> 1) : 13 + (q >> 1);
    const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
    const bool ok = (unsigned)(i + ox) < (unsigned)g.Nx && (unsigned)(j + oy) < (unsigned)g.Ny &&
                    (unsigned)(k + oz) < (unsigned)g.Nz;
    const T* ur = &us[(oy + 1) + 3 * (oz + 1)][3 * (lane + 1 + ox)];
    const T u0 = ur[0], u1 = ur[1], u2 = ur[2];
    T v;
    if (o >= 13) {
      const T* Sb = S + ((size_t)o * 9 + 3 * d) * Nn + node;
      v = Sb[0] * u0 + Sb[Nn] * u1 + Sb[2 * Nn] * u2;
    } else {
      const int nb = ok ? node + ox + g.Nx * (oy + g.Ny * oz) : node;
      const T* Sb = S + ((size_t)(26 - o) * 9 + d) * Nn + nb;
      v = Sb[0] * u0 + Sb[3 * Nn] * u1 + Sb[6 * Nn] * u2;
    }
    acc += ok ? v : (T)0;
  }
  double dot = 0.0;
  if (in) dot = epilogue1(ep, dof, (fx >> d) & 1u, us[4][3 * (lane + 1) + d], (double)acc, ein);
  if (ep.want_dot) {
    const double v[1] = {dot};
    grid_sum<1>(v, ep.ws);
  }
}

template <typename T>
__global__ __launch_bounds__(192) void k_stencil_apply_s(
    Grid g, const T* __restrict__ S, const T* __restrict__ u, const uint8_t* __restrict__ fixn,
    Epi<T> ep) {
  stencil_s_body<T>(g, S, u, fixn, ep, xcd_block(blockIdx.x, gridDim.x));
}

// Stage-batched LDS-staged form (one block per 64-node tile of an item's
// level l, three waves for the output components): the same stages as
// k_bs_stencil.
template <int MODE>
__global__ __launch_bounds__(192) void k_bs_stencil_s(const BSys* __restrict__ sys,
                                                      const BItem* __restrict__ items,
                                                      const int2* __restrict__ tab,
                                                      const int* __restrict__ flags, int l,
                                                      int cin) {
  const int2 e = tab[blockIdx.x];
  if (!flags[e.x]) return;                     // uniform over the block
  const BItem& I = items[e.x];
  const BSys& Sy = sys[I.sys];
  const BLevel& V = Sy.lev[l];
  Epi<double> ep{};
  ep.mode = MODE;
  ep.b = I.lb[l];
  if (MODE == EPI_RESID) {
    ep.out = I.lr[l];
  } else {
    ep.out = I.lx[l][1 - cin];
    ep.dinv = V.dinv64;
    ep.c2 = V.omega;
  }
  stencil_s_body<double>(V.g, V.S64, I.lx[l][cin], V.fixn, ep, e.y);
}

int bs_stencil_s_blocks(const Grid& g) { return (int)div_up(g.Nn, 64); }

void bs_stencil_s(const BsArgs& a, const BsTable& t, const int* flags, int l, int mode, int cin,
                  hipStream_t s) {
  if (t.n == 0) return;
  if (mode == EPI_RESID)
    k_bs_stencil_s<EPI_RESID><<<t.n, 192, 0, s>>>(a.sys, a.items, t.blk, flags, l, cin);
  else
    k_bs_stencil_s<EPI_SMOOTH><<<t.n, 192, 0, s>>>(a.sys, a.items, t.blk, flags, l, cin);
}

// Listed nodes only (the rows a matrix-free product leaves out).  Their
// rows are first gathered, entry-major, into Sd[(o * 9 + 3 d + e) * nlist +
// i] (the upper blocks from the node, the lower blocks transposed from the
// neighbour, zero outside the grid), so that the product reads them with
// consecutive lanes on consecutive listed nodes.
template <typename T>
__global__ __launch_bounds__(256) void k_stencil_gather_rows(Grid g, const T* __restrict__ S,
                                                             const int* __restrict__ list, int nlist,
                                                             T* __restrict__ Sd) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int q = blockIdx.y;                    // entry (o, d, e) = q
  if (i >= nlist) return;
  const int o = q / 9, d = (q / 3) % 3, e = q % 3;
  const int node = list[i];
  const int x = node % g.Nx, t = node / g.Nx, y = t % g.Ny, z = t / g.Ny;
  const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
  const bool ok = (unsigned)(x + ox) < (unsigned)g.Nx && (unsigned)(y + oy) < (unsigned)g.Ny &&
                  (unsigned)(z + oz) < (unsigned)g.Nz;
  T v = (T)0;
  if (ok) {
    const size_t Nn = g.Nn;
    const int nb = node + ox + g.Nx * (oy + g.Ny * oz);
    v = o >= 13 ? S[((size_t)o * 9 + 3 * d + e) * Nn + node]
                : S[((size_t)(26 - o) * 9 + 3 * e + d) * Nn + nb];
  }
  Sd[(size_t)q * nlist + i] = v;
}

template <typename T>
void launch_stencil_gather_rows(const Grid& g, const T* S, const int* list, int nlist, T* Sd,
                                hipStream_t s) {
  if (nlist <= 0) return;
  k_stencil_gather_rows<T><<<dim3(div_up(nlist, 256), kStencil), 256, 0, s>>>(g, S, list, nlist, Sd);
}
template void launch_stencil_gather_rows<double>(const Grid&, const double*, const int*, int,
                                                 double*, hipStream_t);

// levels with fewer nodes use the plane-split form
constexpr int kStencilSplitNodes = 40000;

// the larger of the two forms' grids (the plane-split form runs three blocks
// per 64-node tile)
size_t stencil_apply_blocks(const Grid& g) { return 3 * div_up(g.Nn, 64); }

template <typename T>
void launch_stencil_apply(const Grid& g, const T* S, const T* u, const uint8_t* fixn,
                          const Epi<T>& ep, int form, hipStream_t s) {
  const int tiles = (int)div_up(g.Nn, 64);
  const bool staged = form == 1 || (form == 0 && g.Nn >= kStencilSplitNodes);
  const int nb = staged ? tiles : 3 * tiles;
  if (staged)
    k_stencil_apply_s<T><<<nb, 192, 0, s>>>(g, S, u, fixn, ep);
  else
    k_stencil_apply_c<T><<<nb, kRowSplitThreads, 0, s>>>(g, S, u, fixn, ep);
  if (ep.want_dot && ep.dot_out) launch_finalize(ep.ws, nb, 1, ep.dot_out, s);
}
template void launch_stencil_apply<double>(const Grid&, const double*, const double*,
                                           const uint8_t*, const Epi<double>&, int, hipStream_t);
template void launch_stencil_apply<float>(const Grid&, const float*, const float*, const uint8_t*,
                                          const Epi<float>&, int, hipStream_t);

// Restriction launch: one thread per coarse DOF.  A block covers (part of)
// one x-row of coarse nodes, 3 Nx consecutive DOFs, so a wave's stores are
// contiguous, the row's y and z indices are uniform over the block (no
// per-thread division by the grid sizes), and each thread sums one component
// in the same order as the node-level definition.
struct RowLaunch {
  int threads;    // per block: 3 Nx rounded up to a whole number of waves, <= 256
  int chunks;     // blocks per row
  int blocks;     // chunks x rows
};
static RowLaunch row_launch(const Grid& g) {
  RowLaunch r;
  const int dofs = 3 * g.Nx;
  r.threads = div_up(dofs, 64) * 64;
  if (r.threads > 256) r.threads = 256;
  r.chunks = div_up(dofs, r.threads);
  r.blocks = r.chunks * g.Ny * g.Nz;
  return r;
}

// Restriction (R = P^T, Eq. vector_prolongation): coarse node I gathers the
// <= 27 fine nodes that interpolate from it.  Optional fused first smoothing
// step from a zero iterate: x_c = c0 * Dinv_c * b_c, d_c = x_c.
// 1D weights of fine nodes 2I - 1, 2I, 2I + 1 towards coarse node I on an
// axis of nf fine elements (the closed form of w1d for those three nodes).
__device__ inline void restrict_w1d(int I, int nf, double (&w)[3]) {
  const int nc = nf >> 1;
  w[0] = I >= 1 ? 0.5 : 0.0;
  w[1] = 1.0;
  w[2] = 2 * I + 1 < 2 * nc ? 0.5 : (2 * I + 1 == nf ? 1.0 : 0.0);
}

// Thread per coarse DOF.  The 27 fine nodes are read unconditionally at
// clamped indices and weighted (zero weights for nodes outside the grid).
template <typename TF, typename TC>
__global__ __launch_bounds__(256) void k_restrict(Grid f, Grid c, int chunks,
                                                  const TF* __restrict__ rf,
                                                  const uint8_t* __restrict__ cfix,
                                                  TC* __restrict__ bc,
                                                  const TC* __restrict__ dinv_c, double c0,
                                                  TC* __restrict__ xc, TC* __restrict__ dc) {
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int row = blk / chunks, q = (blk - row * chunks) * blockDim.x + threadIdx.x;
  if (q >= 3 * c.Nx) return;
  const int Iy = row % c.Ny, Iz = row / c.Ny;
  const int Ix = q / 3, k = q - 3 * Ix;
  // the output's mask and diagonal are loaded with the fine values
  const size_t I = Ix + (size_t)c.Nx * row;
  const size_t dof = 3 * I + k;
  const unsigned fx = cfix[I];
  const TC dv = xc ? dinv_c[dof] : (TC)0;
  double wx[3], wy[3], wz[3];
  restrict_w1d(Ix, f.nx, wx);
  restrict_w1d(Iy, f.ny, wy);
  restrict_w1d(Iz, f.nz, wz);
  double acc = 0.0;
#pragma unroll
  for (int cz = 0; cz < 3; ++cz) {
    const int iz = min(max(2 * Iz - 1 + cz, 0), f.Nz - 1);
#pragma unroll
    for (int cy = 0; cy < 3; ++cy) {
      const int iy = min(max(2 * Iy - 1 + cy, 0), f.Ny - 1);
      const double wyz = wy[cy] * wz[cz];
      const size_t frow = (size_t)f.Nx * (iy + (size_t)f.Ny * iz);
#pragma unroll
      for (int cx = 0; cx < 3; ++cx) {
        const int ix = min(max(2 * Ix - 1 + cx, 0), f.Nx - 1);
        acc += wx[cx] * wyz * (double)rf[3 * (frow + ix) + k];
      }
    }
  }
  const TC v = (fx >> k) & 1u ? (TC)0 : (TC)acc;
  bc[dof] = v;
  if (xc) {
    const TC x = (TC)c0 * dv * v;
    xc[dof] = x;
    if (dc) dc[dof] = x;
  }
}

template <typename TF, typename TC>
void launch_restrict(const Grid& fine, const Grid& coarse, const TF* rf, const uint8_t* cfix,
                     TC* bc, const TC* dinv_c, double c0, TC* xc, TC* dc, hipStream_t s) {
  const RowLaunch r = row_launch(coarse);
  k_restrict<TF, TC><<<r.blocks, r.threads, 0, s>>>(fine, coarse, r.chunks, rf, cfix, bc, dinv_c,
                                                    c0, xc, dc);
}
template void launch_restrict<float, double>(const Grid&, const Grid&, const float*,
                                             const uint8_t*, double*, const double*, double,
                                             double*, double*, hipStream_t);
template void launch_restrict<float, float>(const Grid&, const Grid&, const float*,
                                            const uint8_t*, float*, const float*, double, float*,
                                            float*, hipStream_t);
template void launch_restrict<double, double>(const Grid&, const Grid&, const double*,
                                              const uint8_t*, double*, const double*, double,
                                              double*, double*, hipStream_t);
template void launch_restrict<double, float>(const Grid&, const Grid&, const double*,
                                             const uint8_t*, float*, const float*, double,
                                             float*, float*, hipStream_t);

// Prolongation and correction x_f += M_f P e_c: fine node i reads the <= 8
// coarse nodes it interpolates from.  Per axis the two candidates and their
// weights are in closed form (even node: its coarse node, weight 1; odd
// interior node: both neighbours, 1/2 each; trailing odd node: the last
// coarse node, weight 1); the 8 corners are read unconditionally at valid
// indices with zero weights where a candidate does not exist.
__device__ inline void prolong_w1d(int i, int nf, int (&ci)[2], double (&w)[2]) {
  const int nc = nf >> 1;
  if ((i & 1) == 0) { ci[0] = ci[1] = i >> 1; w[0] = 1.0; w[1] = 0.0; }
  else if (i < 2 * nc) { ci[0] = (i - 1) >> 1; ci[1] = (i + 1) >> 1; w[0] = w[1] = 0.5; }
  else { ci[0] = ci[1] = nc; w[0] = 1.0; w[1] = 0.0; }
}

// Row form: a block owns (a chunk of up to 256 nodes of) one fine x-row.
// The row's y and z candidates are uniform over the block, so the <= 4
// coarse rows it reads are first combined with their y-z weights into one
// coarse row segment in LDS (coalesced loads, zero weights skipped); each
// thread then interpolates its node from two segment entries and updates
// the node's three components (a free component gets its correction, a
// masked one is stored back unchanged).
constexpr int kProlongChunk = 256;                 // fine nodes per block (at most)
constexpr int kProlongSeg = kProlongChunk / 2 + 1;  // coarse nodes per chunk (at most)

template <typename TF, typename TC>
__global__ __launch_bounds__(kProlongChunk) void k_prolong_add(Grid f, Grid c, int chunks,
                                                               const TC* __restrict__ ec,
                                                               const uint8_t* __restrict__ ffix,
                                                               TF* __restrict__ xf) {
  __shared__ double seg[3 * kProlongSeg];
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int row = blk / chunks, x0 = (blk - row * chunks) * kProlongChunk;
  const int iy = row % f.Ny, iz = row / f.Ny;
  int cy[2], cz[2];
  double wy[2], wz[2];
  prolong_w1d(iy, f.ny, cy, wy);
  prolong_w1d(iz, f.nz, cz, wz);
  const int cx0 = x0 >> 1;
  const int nseg = min(kProlongSeg, c.Nx - cx0);
  // the node's values and mask are loaded first, so their latency overlaps
  // the segment's loads
  const int ix = x0 + threadIdx.x;
  const bool act = ix < f.Nx;
  const size_t node = (size_t)(act ? ix : f.Nx - 1) + (size_t)f.Nx * row;
  TF* xn = xf + 3 * node;
  TF xv[3] = {xn[0], xn[1], xn[2]};
  const unsigned fx = ffix[node];
  for (int q = threadIdx.x; q < 3 * nseg; q += blockDim.x) {
    double v = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const double w = wy[a & 1] * wz[a >> 1];
      if (w != 0.0)
        v += w * (double)ec[3 * ((size_t)cx0 + (size_t)c.Nx * (cy[a & 1] + (size_t)c.Ny * cz[a >> 1])) + q];
    }
    seg[q] = v;
  }
  __syncthreads();
  if (!act) return;
  int cx[2];
  double wx[2];
  prolong_w1d(ix, f.nx, cx, wx);
  const int s0 = 3 * (cx[0] - cx0), s1 = 3 * (cx[1] - cx0);
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (!((fx >> k) & 1u)) xv[k] = (TF)((double)xv[k] + (wx[0] * seg[s0 + k] + wx[1] * seg[s1 + k]));
  xn[0] = xv[0];
  xn[1] = xv[1];
  xn[2] = xv[2];
}

template <typename TF, typename TC>
void launch_prolong_add(const Grid& fine, const Grid& coarse, const TC* ec, const uint8_t* ffix,
                        TF* xf, hipStream_t s) {
  const int chunks = div_up(fine.Nx, kProlongChunk);
  const int threads = fine.Nx >= kProlongChunk ? kProlongChunk : div_up(fine.Nx, 64) * 64;
  k_prolong_add<TF, TC><<<chunks * fine.Ny * fine.Nz, threads, 0, s>>>(fine, coarse, chunks, ec,
                                                                       ffix, xf);
}
template void launch_prolong_add<float, double>(const Grid&, const Grid&, const double*,
                                                const uint8_t*, float*, hipStream_t);
template void launch_prolong_add<float, float>(const Grid&, const Grid&, const float*,
                                               const uint8_t*, float*, hipStream_t);
template void launch_prolong_add<double, double>(const Grid&, const Grid&, const double*,
                                                 const uint8_t*, double*, hipStream_t);
template void launch_prolong_add<double, float>(const Grid&, const Grid&, const float*,
                                                const uint8_t*, double*, hipStream_t);

// ---------------------------------------------------------------------------
// Iterative coarsest solve (Sec. 3.2; Table repro_defaults: above the dense
// cutoff, a fixed number of PCG steps): Jacobi-preconditioned CG on the
// coarsest stencil from x = 0, `iters` steps, stopping early only when
// p.Kp <= 0 or r.z = 0.
//
// Each step is two launches over the whole chip (a single workgroup would
// stream the coarsest stencil through one CU).  Every reduction is written
// as per-block partials into a slot of its own step, and every block of the
// next launch re-sums those partials in one fixed order, so all blocks see
// bit-identical scalars and take the same early-stop decision without any
// grid-wide synchronisation or host round trip:
//   prz[k][b]  block partials of r_k . z_k, z_k = D^-1 r_k   (k = 0..iters)
//   ppq[k][b]  block partials of p_k . K p_k                  (k = 0..iters-1)
//   done[k]    1 when an earlier step stopped; later steps change nothing.
// The apply launch forms p_k = z_k + beta_k p_{k-1} (beta_k = rz_k / rz_{k-1};
// p_0 = z_0) on the fly for its node and the 26 neighbours, writes p_k into
// the other half of a ping-pong pair and q = K p_k; the update launch forms
// x += a p_k, r -= a q, z = D^-1 r with a = rz_k / pq_k.  Both kernels issue
// their vector and stencil loads before they read the flag and the partials,
// so the chain of dependent memory round trips per launch stays short.

// Sum of n values in a fixed order: lane-strided partial sums, then the
// butterfly (every lane of every wave ends with the same bits).
__device__ inline double wave_total(const double* __restrict__ v, int n) {
  double t = 0.0;
  for (int i = threadIdx.x & 63; i < n; i += 64) t += v[i];
  return wave_sum(t);
}

__global__ __launch_bounds__(256) void k_cpcg_init(int n, const double* __restrict__ b,
                                                   const double* __restrict__ dinv,
                                                   double* __restrict__ x, double* __restrict__ r,
                                                   double* __restrict__ z,
                                                   double* __restrict__ prz, int* __restrict__ done) {
  __shared__ double lds[16];
  const int i = blockIdx.x * 256 + threadIdx.x;
  double part = 0.0;
  if (i < n) {
    const double ri = b[i], zi = dinv[i] * ri;
    x[i] = 0.0;
    r[i] = ri;
    z[i] = zi;
    part = ri * zi;
  }
  const double t = block_sum(part, lds);
  if (threadIdx.x == 0) {
    prz[blockIdx.x] = t;
    if (blockIdx.x == 0) done[0] = 0;
  }
}

// 576 threads: 64 nodes x 3 rows x 3 groups of 9 stencil offsets.  Offsets
// outside the grid read the node itself (a valid address) and add nothing.
// K p_k is accumulated as K z_k + beta_k (K p_{k-1}) (the same product up
// to rounding), so the stencil and vector loads need no beta and are all in
// flight before the partials that give beta arrive.  Step 0 passes pold = z
// and beta = 0: fma(0, z, z) = z exactly.
__global__ __launch_bounds__(576) void k_cpcg_apply(Grid g, const double* __restrict__ S,
                                                    const uint8_t* __restrict__ fixn,
                                                    const double* __restrict__ z,
                                                    const double* __restrict__ pold,
                                                    double* __restrict__ pnew, double* __restrict__ q,
                                                    const double* __restrict__ prz,
                                                    double* __restrict__ ppq,
                                                    const int* __restrict__ done, int k, int nbu) {
  __shared__ double part[2][3][3][64];
  __shared__ double lds[16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int d = w % 3, pz = w / 3;
  const int node0 = blockIdx.x * 64 + lane;
  const bool in = node0 < g.Nn;
  const int node = in ? node0 : g.Nn - 1;
  const int i = node % g.Nx, t = node / g.Nx, j = t % g.Ny, kk = t / g.Ny;
  const size_t Nn = g.Nn;
  double az = 0.0, ap = 0.0;
#pragma unroll
  for (int qq = 0; qq < 9; ++qq) {
    const int o = 9 * pz + qq;
    const int ox = qq % 3 - 1, oy = qq / 3 - 1, oz = pz - 1;
    const bool ok = (unsigned)(i + ox) < (unsigned)g.Nx && (unsigned)(j + oy) < (unsigned)g.Ny &&
                    (unsigned)(kk + oz) < (unsigned)g.Nz;
    const int nb = ok ? node + ox + g.Nx * (oy + g.Ny * oz) : node;
    const size_t b3 = 3 * (size_t)nb;
    // upper blocks from the node, lower blocks mirrored from the neighbour
    const double* Sb = o >= 13 ? S + ((size_t)o * 9 + 3 * d) * Nn + node
                               : S + ((size_t)(26 - o) * 9 + d) * Nn + nb;
    const size_t st = o >= 13 ? Nn : 3 * Nn;
    double vz = 0.0, vp = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double cf = Sb[c * st];
      vz += cf * z[b3 + c];
      vp += cf * pold[b3 + c];
    }
    az += ok ? vz : 0.0;
    ap += ok ? vp : 0.0;
  }
  part[0][pz][d][lane] = az;
  part[1][pz][d][lane] = ap;
  const size_t dof = 3 * (size_t)node + d;
  const double zown = z[dof], pold_own = pold[dof];
  const unsigned fx = fixn[node];
  const bool stop = done[k] != 0;
  const double beta = k > 0 ? wave_total(prz + (size_t)k * nbu, nbu) /
                                  wave_total(prz + (size_t)(k - 1) * nbu, nbu)
                            : 0.0;
  if (stop) return;                                   // uniform over the grid
  __syncthreads();
  double dot = 0.0;
  if (in && pz == 1) {
    const double kz = (part[0][0][d][lane] + part[0][1][d][lane]) + part[0][2][d][lane];
    const double kp = (part[1][0][d][lane] + part[1][1][d][lane]) + part[1][2][d][lane];
    const double pown = __builtin_fma(beta, pold_own, zown);
    const double y = (fx >> d) & 1u ? 0.0 : __builtin_fma(beta, kp, kz);
    pnew[dof] = pown;
    q[dof] = y;
    dot = pown * y;
  }
  const double tot = block_sum(dot, lds);
  if (threadIdx.x == 0) ppq[(size_t)k * gridDim.x + blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_cpcg_update(int n, const double* __restrict__ dinv,
                                                     double* __restrict__ x, double* __restrict__ r,
                                                     double* __restrict__ z,
                                                     const double* __restrict__ p,
                                                     const double* __restrict__ q,
                                                     double* __restrict__ prz,
                                                     const double* __restrict__ ppq,
                                                     int* __restrict__ done, int k, int nba) {
  __shared__ double lds[16];
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  const int i0 = blockIdx.x * 256 + threadIdx.x;
  const bool in = i0 < n;
  const int i = in ? i0 : n - 1;
  const double xi = x[i], pi = p[i], qi = q[i], ri = r[i], di = dinv[i];
  const bool was_done = done[k] != 0;
  const double pq = wave_total(ppq + (size_t)k * nba, nba);
  const double rz = wave_total(prz + (size_t)k * gridDim.x, gridDim.x);
  if (was_done || !(pq > 0.0) || rz == 0.0) {         // uniform over the grid
    if (lead) done[k + 1] = 1;
    return;
  }
  const double a = rz / pq;
  double part = 0.0;
  if (in) {
    const double rn = ri - a * qi, zn = di * rn;
    x[i] = xi + a * pi;
    r[i] = rn;
    z[i] = zn;
    part = rn * zn;
  }
  const double t = block_sum(part, lds);
  if (threadIdx.x == 0) prz[(size_t)(k + 1) * gridDim.x + blockIdx.x] = t;
  if (lead) done[k + 1] = 0;
}

size_t coarse_pcg_scratch(const Grid& g, int iters) {
  const size_t nbu = div_up(g.n, 256), nba = div_up(g.Nn, 64);
  return (size_t)(iters + 1) * nbu + (size_t)iters * nba;
}

void launch_coarse_pcg(const Grid& g, const double* S, const double* dinv, const uint8_t* fixn,
                       const double* b, double* x, double* r, double* z, double* p0, double* p1,
                       double* q, double* scratch, int* done, int iters, hipStream_t s) {
  const int nbu = (int)div_up(g.n, 256), nba = (int)div_up(g.Nn, 64);
  double* prz = scratch;
  double* ppq = scratch + (size_t)(iters + 1) * nbu;
  k_cpcg_init<<<nbu, 256, 0, s>>>(g.n, b, dinv, x, r, z, prz, done);
  double* pp[2] = {p0, p1};
  for (int k = 0; k < iters; ++k) {
    const double* pold = k == 0 ? z : pp[(k + 1) & 1];
    k_cpcg_apply<<<nba, 576, 0, s>>>(g, S, fixn, z, pold, pp[k & 1], q, prz, ppq, done, k, nbu);
    k_cpcg_update<<<nbu, 256, 0, s>>>(g.n, dinv, x, r, z, pp[k & 1], q, prz, ppq, done, k, nba);
  }
}

}  // namespace sgmg
