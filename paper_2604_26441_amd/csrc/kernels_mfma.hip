// Fine-level K.u on the gfx950 matrix cores (Eq. mf_matvec; Sec. 3.5 BF16
// semantics).  The element matrix s*K_e is an integer matrix with entries of
// magnitude <= 88, hence exact in BF16; each input value is rounded to BF16
// (NSPLIT = 1) or split into two or three BF16 terms (NSPLIT = 3 carries the
// whole FP32 significand).  Products are exact and accumulate in FP32 on
// v_mfma_f32_16x16x32_bf16; E_e / s is applied in FP32 afterwards.  The FP64
// form runs the same tiles on v_mfma_f64_16x16x4_f64.
//
// Work decomposition: one wave owns a tile of 16 elements in x (the MFMA's
// N dimension, one element per lane column) by YC element rows in y, and
// marches along z over a chunk of node planes.  Nothing is shared between
// waves and there is no barrier.  MFMA h = 0 produces the element's dy = 0
// nodes, h = 1 its dy = 1 nodes.  Node sums:
//   * y: the dy = 1 rows of element row ey and the dy = 0 rows of row ey + 1
//     sit in the same lanes: an in-register carry from row to row.
//   * x: dx = 1 of element n - 1 meets dx = 0 of element n through a DPP row
//     shift by one lane fused into an add.
//   * z: dz = 1 of plane ez meets dz = 0 of plane ez + 1 through a per-row
//     carry across planes.
// A wave recomputes one halo element on the low side of each axis so that
// every node it writes is complete (15 owned nodes in x, YC - 1 node rows,
// all planes of its chunk).  Every node sums its 8 element contributions in
// the same order whatever the tile shape: results are bitwise independent of
// the launch shape.
//
// BF16 family: each wave stages its node planes in LDS, split into BF16 terms
// once per value, and output row m = 4 c + (dx + 2 dz) puts component c of
// all four (dx, dz) nodes in lane group c.  FP64: element inputs are loaded
// per element, and lane group dx + 2 dz holds the three components of node
// (dx, dy, dz), so the x and z sums first move lane groups together with
// v_permlane16_swap / v_permlane32_swap.
#include <climits>
#include <cstring>
#include <type_traits>

#include "batch.hpp"
#include "bstage.hpp"
#include "bufops.hpp"
#include "kernels.hpp"

namespace sgmg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int kMfmaWavesPerBlock = 4;

// Per-wave LDS of the BF16-family kernel:
//   U: NSPLIT terms x a ring of 3 node planes x (YC + 1) node rows x 17 nodes
//      x 4 BF16 (components 0, 1, 2 and a zero), so the two nodes of a lane's
//      pair are 16 contiguous bytes;
//   O: (YC - 1) owned node rows x 16 columns x 4 floats: the node sums of a
//      plane, written in the matrix-core lane layout, read back per node.
template <int NSPLIT, int YC>
struct FineLds {
  static constexpr int kRow = 17 * 8;
  static constexpr int kPlane = (YC + 1) * kRow;
  static constexpr int kTerm = 3 * kPlane;
  static constexpr int kU = (NSPLIT * kTerm + 15) / 16 * 16;
  static constexpr int kORow = 16 * 16;
  static constexpr int kWave = kU + (YC - 1) * kORow;
};


// BF16-family fine operator.
//   * Node values are read once per wave with 12-byte loads (one node per
//     lane), split into NSPLIT BF16 terms once and written to the wave's LDS
//     ring of node planes; the B operand of every element is then two 8-byte
//     LDS reads per term.
//   * MFMA output rows are m = 4 c + (dx + 2 dz) (build_mfma_atab): lane
//     group c holds component c of the four nodes (dx, dz) of its column's
//     element, so the x-combination is one DPP-shifted add per dz, the
//     z-combination a register carry across planes and the y-combination a
//     carry across rows.  Lane group c < 3 of column n >= 1 then holds
//     component c of node (ex, ey, ez), which goes to the wave's LDS O rows.
//   * At the end of each plane the epilogue runs in node layout: one lane per
//     owned node reads its three sums from O and applies the epilogue with
//     operands loaded by 12-byte loads at the start of the plane, then
//     stores 12 bytes.  Element moduli come with one 4-byte load per lane per
//     four rows and reach their columns by ds_bpermute.
//   Every vector-memory instruction thus moves 12 bytes per lane (4 for the
//   moduli and 1 for the Dirichlet flags): the address unit processes a
//   wave-wide memory instruction at a fixed rate, which per-step 4-byte
//   accesses had made the limit.
//   All loads for plane ez are issued at its start (node plane ez + 3,
//   moduli of plane ez + 1, epilogue operands of plane ez) and consumed by
//   its end or the start of the next plane, unconditionally (an unneeded
//   load reads zeros), so the compiler's load-counter waits stay exact.
//   The body takes the block's index in the mesh's tile grid (blk), so the
//   same code serves one mesh (blk from the launch grid) and the stage-
//   batched solver (blk from its table of (item, block) entries).
template <int NSPLIT, int YC, int MODE>
__device__ __forceinline__ void fine_mfma_body(Grid g, const float* __restrict__ Es,
                                               const uint16_t* __restrict__ atab,
                                               const float* __restrict__ u,
                                               const uint8_t* __restrict__ fixn,
                                               Epi<float> ep, int zchunk, int ntx, int nty,
                                               int ntiles, int blk) {
  using LD = FineLds<NSPLIT, YC>;
  static_assert(YC == 4 || YC == 8, "tile rows");
  __shared__ __attribute__((aligned(16))) unsigned char lds_all[kMfmaWavesPerBlock * LD::kWave];
  const int lane = threadIdx.x & 63;
  // wave index made wave-uniform, so all tile arithmetic stays scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  unsigned char* const lds = lds_all + wave * LD::kWave;
  const int tile = blk * kMfmaWavesPerBlock + wave;
  const int tx = tile % ntx, tt = tile / ntx, ty = tt % nty, tz = tt / nty;
  const int grp = lane >> 4, n = lane & 15;
  const int xs = tx * 15, ys = ty * (YC - 1), zs = tz * zchunk;
  const int ex = xs - 1 + n;
  const int dy_in = grp & 1, dz_in = grp >> 1;

  bf16x8 a0, a1;
  {
    const uint16_t* t0 = atab + lane * 8;
    const uint16_t* t1 = atab + 512 + lane * 8;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      a0[j] = __builtin_bit_cast(__bf16, t0[j]);
      a1[j] = __builtin_bit_cast(__bf16, t1[j]);
    }
  }

  const int zend = tile < ntiles ? min(zs + zchunk, g.Nz) : zs - 1;
  const size_t nvec = (size_t)g.n * sizeof(float);
  const __amdgpu_buffer_rsrc_t ru = make_rsrc(u, nvec);
  const __amdgpu_buffer_rsrc_t re = make_rsrc(Es, (size_t)g.nel * sizeof(float));
  const __amdgpu_buffer_rsrc_t rfix = make_rsrc(fixn, (size_t)g.Nn);
  constexpr bool kSm = MODE == EPI_SMOOTH || MODE == kSmoothDot;
  const __amdgpu_buffer_rsrc_t rb = make_rsrc(ep.b, MODE == EPI_RESID || kSm ? nvec : 0);
  const __amdgpu_buffer_rsrc_t rdi = make_rsrc(ep.dinv, kSm ? nvec : 0);
  const __amdgpu_buffer_rsrc_t rd = make_rsrc(ep.d, kSm ? nvec : 0);
  const __amdgpu_buffer_rsrc_t rout = make_rsrc(ep.out, ep.out ? nvec : 0);   // NULL: stores dropped
  const __amdgpu_buffer_rsrc_t rr = make_rsrc(ep.dot64, MODE == kSmoothDot ? 2 * nvec : 0);

  // Offsets are the sum of a per-lane part fixed for the whole wave and a
  // plane part; a part that must not be accessed is kPoison.  Vectors are
  // below 2^30 bytes (mfma_size_ok) and valid parts are non-negative with a
  // sum below that, so a sum holding one or two kPoison parts lies in
  // [2^30, 2^31]: outside every buffer as an unsigned offset.
  auto off2 = [](int a, int b) { return (int)((unsigned)a + (unsigned)b); };
  auto part = [](bool ok, int v) { return ok ? v : kPoison; };

  // node planes: load i, lane l < 51 carries node xs - 1 + l % 17 of node
  // row k = 3 i + l / 17 (rows 0 .. YC of the tile)
  constexpr int NU = (YC + 3) / 3;
  const int um = lane % 17, uk = lane / 17;
  int u_lane[NU];
  bool u_on[NU];
#pragma unroll
  for (int i = 0; i < NU; ++i) {
    const int k = 3 * i + uk;
    u_on[i] = lane < 51 && k <= YC;
    u_lane[i] = part(u_on[i] && (unsigned)(xs - 1 + um) < (unsigned)g.Nx &&
                         (unsigned)(ys - 1 + k) < (unsigned)g.Ny,
                     12 * (xs - 1 + um + g.Nx * (ys - 1 + k)));
  }
  // register buffers of raw node planes: in the store modes (HBM-bound on
  // large meshes) a plane's loads are issued two planes before it is split
  // into LDS, so each wave keeps two planes of loads in flight; the smoothing
  // and residual modes (more live registers) keep one
  constexpr int kAhead = (MODE == EPI_STORE || MODE == kStoreDot) ? 2 : 1;
  float uvA[NU][3], uvB[NU][3];
  auto load_u = [&](float (&uv)[NU][3], int P, bool need) {
    const int pp = part(need && (unsigned)P < (unsigned)g.Nz, 12 * g.Nx * g.Ny * P);
#pragma unroll
    for (int i = 0; i < NU; ++i) bload3(ru, off2(u_lane[i], pp), uv[i]);
  };
  // exact NSPLIT-term BF16 split (round to nearest even; each residual is
  // exact in FP32) of the loaded node plane P into its ring slot
  auto split_u = [&](const float (&uv)[NU][3], int P) {
    unsigned char* const slot = lds + ((P + 3) % 3) * LD::kPlane + uk * LD::kRow + um * 8;
#pragma unroll
    for (int i = 0; i < NU; ++i) {
      if (u_on[i]) {
        float v0 = uv[i][0], v1 = uv[i][1], v2 = uv[i][2];
#pragma unroll
        for (int sp = 0; sp < NSPLIT; ++sp) {
          const unsigned w0 = __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{v0, v1}, bf16x2));
          const unsigned w1 = __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{v2, 0.f}, bf16x2));
          *(uint2*)(slot + 3 * i * LD::kRow + sp * LD::kTerm) = uint2{w0, w1};
          if (sp + 1 < NSPLIT) {
            v0 -= __uint_as_float(w0 << 16);
            v1 -= __uint_as_float(w0 & 0xffff0000u);
            v2 -= __uint_as_float(w1 << 16);
          }
        }
      }
    }
  };
  // B operand of element row r: lane group (dy, dz) reads nodes (n, n + 1)
  // of node row r + dy in the slot of plane ez + dz
  auto read_b = [&](int base, int r, u32x4 (&b)[NSPLIT]) {
#pragma unroll
    for (int sp = 0; sp < NSPLIT; ++sp) {
      const unsigned char* q = lds + base + r * LD::kRow + sp * LD::kTerm;
      const uint2 lo = *(const uint2*)q;
      const uint2 hi = *(const uint2*)(q + 8);
      b[sp] = u32x4{lo.x, lo.y, hi.x, hi.y};
    }
  };
  auto contract = [&](const u32x4 (&b)[NSPLIT], f32x4& c0, f32x4& c1) {
    c0 = f32x4{0.f, 0.f, 0.f, 0.f};
    c1 = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int sp = NSPLIT - 1; sp >= 0; --sp) {    // smallest terms first
      const bf16x8 bb = __builtin_bit_cast(bf16x8, b[sp]);
      c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bb, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bb, c1, 0, 0, 0);
    }
  };

  // element moduli E / s: load i, lane l holds column l & 15 of element row
  // 4 i + l / 16; zero outside the mesh, which also cancels the products of
  // elements that do not exist
  constexpr int NE = YC / 4;
  int e_lane[NE];
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    const int ey = ys - 1 + 4 * i + grp;
    e_lane[i] = part((unsigned)ex < (unsigned)g.nx && (unsigned)ey < (unsigned)g.ny,
                     4 * (ex + g.nx * ey));
  }
  float ev[NE], esc[NE];
  auto load_e = [&](int ez, bool need) {
    const int pe = part(need && (unsigned)ez < (unsigned)g.nz, 4 * g.nx * g.ny * ez);
#pragma unroll
    for (int i = 0; i < NE; ++i) ev[i] = bload(re, off2(e_lane[i], pe));
  };

  // node-layout epilogue: group i, lane l < 60 owns node xs + l % 15 of node
  // row 1 + 4 i + l / 15 (rows 1 .. YC - 1 of the tile)
  constexpr int NG = (YC + 2) / 4;
  constexpr int NV = kSm ? 4 : (MODE == EPI_RESID || MODE == kStoreDot) ? 1 : 0;
  const int oj = lane % 15, orr = lane / 15;
  int o_lane[NG], f_lane[NG], o_lds[NG];
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    const int rr = 1 + 4 * i + orr;
    const bool on = lane < 60 && rr <= YC - 1 && xs + oj < g.Nx && ys - 1 + rr < g.Ny;
    o_lane[i] = part(on, 12 * (xs + oj + g.Nx * (ys - 1 + rr)));
    f_lane[i] = part(on, xs + oj + g.Nx * (ys - 1 + rr));
    o_lds[i] = LD::kU + (min(rr, YC - 1) - 1) * LD::kORow + (oj + 1) * 16;
  }
  float vv[NG][NV > 0 ? NV : 1][3];
  double rv[MODE == kSmoothDot ? NG : 1][3];    // the FP64 dot partner of owned nodes
  unsigned fv[NG];
  auto load_v = [&](int ez) {
    const bool own = ez >= zs && ez < zend;
    const int po = part(own, 12 * g.Nx * g.Ny * ez), pf = part(own, g.Nx * g.Ny * ez);
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      fv[i] = __builtin_amdgcn_raw_buffer_load_b8(rfix, off2(f_lane[i], pf), 0, 0);
      const int o = off2(o_lane[i], po);
      if (kSm) {
        bload3(ru, o, vv[i][0]);
        bload3(rb, o, vv[i][1]);
        bload3(rdi, o, vv[i][2]);
        bload3(rd, ep.c1 != 0.0 ? o : kNoOffset, vv[i][3]);
        // 24 B per node at twice the float offset (below 2^31 for owned nodes)
        if (MODE == kSmoothDot)
          bload3(rr, (unsigned)o < (unsigned)kPoison ? 2 * o : kNoOffset, rv[i]);
      } else if (MODE == EPI_RESID) {
        bload3(rb, o, vv[i][0]);
      } else if (MODE == kStoreDot) {
        bload3(ru, o, vv[i][0]);
      }
    }
  };
  double dot = 0.0;
  auto finish_plane = [&](int ez) {
    const int po = part(ez >= zs && ez < zend, 12 * g.Nx * g.Ny * ez);
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      const f32x4 yq = *(const f32x4*)(lds + o_lds[i]);
      const int o = off2(o_lane[i], po);
      const bool mine = (unsigned)o < (unsigned)kPoison;
      float out[3], dd[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const bool fixed = (fv[i] >> c) & 1u;
        const float y = yq[c];
        if (MODE == EPI_STORE || MODE == kStoreDot) {
          out[c] = fixed ? 0.f : y;
          if (MODE == kStoreDot && mine) dot += (double)vv[i][0][c] * (double)out[c];
        } else if (MODE == EPI_RESID) {
          out[c] = fixed ? 0.f : vv[i][0][c] - y;
        } else {
          const float r = vv[i][1][c] - y;
          dd[c] = fixed ? 0.f : (float)ep.c1 * vv[i][3][c] + (float)ep.c2 * vv[i][2][c] * r;
          out[c] = fixed ? 0.f : vv[i][0][c] + dd[c];
        }
      }
      bstore3(rout, o, out[0], out[1], out[2]);
      if (kSm) {
        if (ep.store_d) bstore3(rd, o, dd[0], dd[1], dd[2]);
        if (ep.out64 && mine) {
          double* q = ep.out64 + (o >> 2);
          q[0] = (double)out[0];
          q[1] = (double)out[1];
          q[2] = (double)out[2];
        }
        if (MODE == kSmoothDot && mine)
          dot += rv[i][0] * (double)out[0] + rv[i][1] * (double)out[1] + rv[i][2] * (double)out[2];
      }
    }
  };

  // lane (c, n) of the matrix-core layout writes its node sum to O column n
  const int o_w = LD::kU + n * 16 + grp * 4;
  float zc[YC];
#pragma unroll
  for (int r = 0; r < YC; ++r) zc[r] = 0.f;

  load_u(uvA, zs - 1, true);
  split_u(uvA, zs - 1);
  load_u(uvA, zs, true);
  split_u(uvA, zs);
  load_u(uvA, zs + 1, zs + 1 <= zend);
  if (kAhead == 2) load_u(uvB, zs + 2, zs + 2 <= zend);
  load_e(zs - 1, true);
  // plane ez: its node plane ez + 2 (loaded kAhead planes earlier, in uv)
  // goes to LDS and uv takes the loads of plane ez + 2 + kAhead
  auto plane = [&](int ez, float (&uv)[NU][3]) {
    split_u(uv, ez + 2);
#pragma unroll
    for (int i = 0; i < NE; ++i) esc[i] = ev[i];
    load_u(uv, ez + 2 + kAhead, ez + 2 + kAhead <= zend);
    load_e(ez + 1, ez + 1 < zend);
    load_v(ez);
    const int base = ((ez + dz_in + 3) % 3) * LD::kPlane + dy_in * LD::kRow + n * 8;
    u32x4 bc[NSPLIT], bn[NSPLIT];
    read_b(base, 0, bc);
    float yc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int r = 0; r < YC; ++r) {
      if (r + 1 < YC) read_b(base, r + 1, bn);
      const float sc = __int_as_float(
          __builtin_amdgcn_ds_bpermute(4 * (n + 16 * (r & 3)), __float_as_int(esc[r >> 2])));
      f32x4 c0, c1;
      contract(bc, c0, c1);
      float t[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        t[k] = c0[k] * sc + yc[k];    // y: dy = 0 of this row + dy = 1 of the row below
        yc[k] = c1[k] * sc;
      }
      // x: dx = 0 of element n + dx = 1 of element n - 1; z: plane ez + plane ez - 1
      const float w0 = t[0] + dpp_shr1(t[1]);
      const float w1 = t[2] + dpp_shr1(t[3]);
      const float fin = w0 + zc[r];
      zc[r] = w1;
      if (r >= 1) *(float*)(lds + o_w + (r - 1) * LD::kORow) = fin;
      if (r + 1 < YC) {
#pragma unroll
        for (int sp = 0; sp < NSPLIT; ++sp) bc[sp] = bn[sp];
      }
    }
    finish_plane(ez);
  };
  if (kAhead == 2) {
    for (int ez = zs - 1; ez < zend; ez += 2) {
      plane(ez, uvA);
      if (ez + 1 < zend) plane(ez + 1, uvB);
    }
  } else {
    for (int ez = zs - 1; ez < zend; ++ez) plane(ez, uvA);
  }
  if (MODE == kStoreDot || MODE == kSmoothDot) {
    const double vd[1] = {dot};
    grid_sum<1>(vd, ep.ws);
  }
}

template <int NSPLIT, int YC, int MODE>
__global__ __launch_bounds__(64 * kMfmaWavesPerBlock) void k_apply_fine_mfma(
    Grid g, const float* __restrict__ Es, const uint16_t* __restrict__ atab,
    const float* __restrict__ u, const uint8_t* __restrict__ fixn, Epi<float> ep, int zchunk,
    int ntx, int nty, int ntiles) {
  fine_mfma_body<NSPLIT, YC, MODE>(g, Es, atab, u, fixn, ep, zchunk, ntx, nty, ntiles,
                                   xcd_block(blockIdx.x, gridDim.x));
}

// Stage-batched form: one launch applies the level-0 smoothing step or
// residual of every active item.  Block b is entry tab[b] = (item, block of
// the item's tile grid); geo[item] holds that grid (ntx, nty, ntiles) for
// the launch shape (YC rows, zchunk planes).  The epilogue's vectors and
// smoothing coefficients are the item's (those of k_bs_apply0).
template <int YC, int MODE>
__global__ __launch_bounds__(64 * kMfmaWavesPerBlock) void k_bs_fine_mfma(
    const BSys* __restrict__ sys, const BItem* __restrict__ items, const int2* __restrict__ tab,
    const int4* __restrict__ geo, const int* __restrict__ flags, int post, int k, int cin,
    int last, int zchunk) {
  const int2 e = tab[blockIdx.x];
  if (!flags[e.x]) return;                     // uniform over the block
  const BItem& I = items[e.x];
  const BSys& S = sys[I.sys];
  const BLevel& V = S.lev[0];
  const int4 gm = geo[e.x];
  Epi<float> ep{};
  ep.mode = MODE;
  ep.b = I.b0;
  if (MODE == EPI_RESID) {
    ep.out = I.r0;
  } else {
    double c1 = 0.0, c2 = 0.0;
    smooth_coef(V, post != 0, k, c1, c2);
    ep.out = I.x0[1 - cin];
    ep.dinv = V.dinv32;
    ep.d = I.d0;
    ep.c1 = c1;
    ep.c2 = c2;
    ep.store_d = 1;
    ep.out64 = last ? I.z : nullptr;
  }
  fine_mfma_body<3, YC, MODE>(V.g, S.E32s, S.atab, I.x0[cin], V.fixn, ep, zchunk, gm.x, gm.y,
                              gm.z, e.y);
}

// ---------------------------------------------------------------------------
// FP64 fine operator on v_mfma_f64_16x16x4_f64 (outer PCG products, FP64
// smoothing, power iteration): the tiles, carries and plane-level pipeline of
// the BF16-family kernel with FP64 node records in LDS and no split.  K = 24
// inputs take six k-steps of 4: at step st lane group q (node pair (dy, dz))
// supplies value st of its pair, so A holds K_e[row m][input (q, st)] per
// (h, st).  This MFMA returns row m in lane group m mod 4, register m / 4
// (measured on gfx950), so the A-table rows m = 4 (dx + 2 dz) + c put
// component c in lane group c and node (dx, dz) in register dx + 2 dz, as in
// the BF16 kernel.  Exact products, FP64 accumulation.
template <int YC>
struct FineLds64 {
  static constexpr int kRow = 17 * 24;               // 17 nodes x 3 doubles
  static constexpr int kPlane = (YC + 1) * kRow;
  static constexpr int kU = (3 * kPlane + 15) / 16 * 16;
  static constexpr int kORow = 16 * 32;              // 16 columns x 4 doubles
  static constexpr int kWave = kU + (YC - 1) * kORow;
};

template <int YC, int MODE>
__device__ __forceinline__ void fine_mfma64_body(Grid g, const double* __restrict__ E,
                                                 const double* __restrict__ atab,
                                                 const double* __restrict__ u,
                                                 const uint8_t* __restrict__ fixn,
                                                 Epi<double> ep, int zchunk, int ntx, int nty,
                                                 int ntiles, int blk) {
  typedef double f64x4 __attribute__((ext_vector_type(4)));
  using LD = FineLds64<YC>;
  static_assert(YC == 4 || YC == 8, "tile rows");
  __shared__ __attribute__((aligned(16))) unsigned char lds_all[kMfmaWavesPerBlock * LD::kWave];
  const int lane = threadIdx.x & 63;
  // wave index made wave-uniform, so all tile arithmetic stays scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  unsigned char* const lds = lds_all + wave * LD::kWave;
  const int tile = blk * kMfmaWavesPerBlock + wave;
  const int tx = tile % ntx, tt = tile / ntx, ty = tt % nty, tz = tt / nty;
  const int grp = lane >> 4, n = lane & 15;
  const int xs = tx * 15, ys = ty * (YC - 1), zs = tz * zchunk;
  const int ex = xs - 1 + n;
  const int dy_in = grp & 1, dz_in = grp >> 1;

  double a0[6], a1[6];
#pragma unroll
  for (int st = 0; st < 6; ++st) {
    a0[st] = atab[st * 64 + lane];
    a1[st] = atab[(6 + st) * 64 + lane];
  }

  const int zend = tile < ntiles ? min(zs + zchunk, g.Nz) : zs - 1;
  const size_t nvec = (size_t)g.n * sizeof(double);
  const __amdgpu_buffer_rsrc_t ru = make_rsrc(u, nvec);
  const __amdgpu_buffer_rsrc_t re = make_rsrc(E, (size_t)g.nel * sizeof(double));
  const __amdgpu_buffer_rsrc_t rfix = make_rsrc(fixn, (size_t)g.Nn);
  const __amdgpu_buffer_rsrc_t rb = make_rsrc(ep.b, MODE == EPI_RESID || MODE == EPI_SMOOTH ? nvec : 0);
  const __amdgpu_buffer_rsrc_t rdi = make_rsrc(ep.dinv, MODE == EPI_SMOOTH ? nvec : 0);
  const __amdgpu_buffer_rsrc_t rd = make_rsrc(ep.d, MODE == EPI_SMOOTH ? nvec : 0);
  const __amdgpu_buffer_rsrc_t rout = make_rsrc(ep.out, ep.out ? nvec : 0);   // NULL: stores dropped

  // two-part offsets with kPoison parts, as in the BF16-family kernel
  // (vectors below 2^30 bytes: mfma64_size_ok)
  auto off2 = [](int a, int b) { return (int)((unsigned)a + (unsigned)b); };
  auto part = [](bool ok, int v) { return ok ? v : kPoison; };

  // node planes: load i, lane l < 51 carries node xs - 1 + l % 17 of node
  // row k = 3 i + l / 17 (rows 0 .. YC of the tile)
  constexpr int NU = (YC + 3) / 3;
  const int um = lane % 17, uk = lane / 17;
  int u_lane[NU];
  bool u_on[NU];
#pragma unroll
  for (int i = 0; i < NU; ++i) {
    const int k = 3 * i + uk;
    u_on[i] = lane < 51 && k <= YC;
    u_lane[i] = part(u_on[i] && (unsigned)(xs - 1 + um) < (unsigned)g.Nx &&
                         (unsigned)(ys - 1 + k) < (unsigned)g.Ny,
                     24 * (xs - 1 + um + g.Nx * (ys - 1 + k)));
  }
  double uv[NU][3];
  auto load_u = [&](int P, bool need) {
    const int pp = part(need && (unsigned)P < (unsigned)g.Nz, 24 * g.Nx * g.Ny * P);
#pragma unroll
    for (int i = 0; i < NU; ++i) bload3(ru, off2(u_lane[i], pp), uv[i]);
  };
  auto store_u = [&](int P) {
    unsigned char* const slot = lds + ((P + 3) % 3) * LD::kPlane + uk * LD::kRow + um * 24;
#pragma unroll
    for (int i = 0; i < NU; ++i) {
      if (u_on[i]) {
        double* q = (double*)(slot + 3 * i * LD::kRow);
        q[0] = uv[i][0];
        q[1] = uv[i][1];
        q[2] = uv[i][2];
      }
    }
  };
  // B operands of element row r: lane group (dy, dz) reads the six values of
  // nodes (n, n + 1) of node row r + dy in the slot of plane ez + dz
  auto read_b = [&](int base, int r, double (&b)[6]) {
    const double* q = (const double*)(lds + base + r * LD::kRow);
#pragma unroll
    for (int st = 0; st < 6; ++st) b[st] = q[st];
  };
  auto contract = [&](const double (&b)[6], f64x4& c0, f64x4& c1) {
    c0 = f64x4{0.0, 0.0, 0.0, 0.0};
    c1 = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int st = 0; st < 6; ++st) {
      c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[st], b[st], c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[st], b[st], c1, 0, 0, 0);
    }
  };

  // element moduli: load i, lane l holds column l & 15 of element row
  // 4 i + l / 16; zero outside the mesh
  constexpr int NE = YC / 4;
  int e_lane[NE];
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    const int ey = ys - 1 + 4 * i + grp;
    e_lane[i] = part((unsigned)ex < (unsigned)g.nx && (unsigned)ey < (unsigned)g.ny,
                     8 * (ex + g.nx * ey));
  }
  double ev[NE], esc[NE];
  auto load_e = [&](int ez, bool need) {
    const int pe = part(need && (unsigned)ez < (unsigned)g.nz, 8 * g.nx * g.ny * ez);
#pragma unroll
    for (int i = 0; i < NE; ++i) ev[i] = bload1d(re, off2(e_lane[i], pe));
  };

  // node-layout epilogue: group i, lane l < 60 owns node xs + l % 15 of node
  // row 1 + 4 i + l / 15
  constexpr int NG = (YC + 2) / 4;
  constexpr int NV = MODE == EPI_SMOOTH ? 4 : (MODE == EPI_RESID || MODE == kStoreDot) ? 1 : 0;
  const int oj = lane % 15, orr = lane / 15;
  int o_lane[NG], f_lane[NG], o_lds[NG];
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    const int rr = 1 + 4 * i + orr;
    const bool on = lane < 60 && rr <= YC - 1 && xs + oj < g.Nx && ys - 1 + rr < g.Ny;
    o_lane[i] = part(on, 24 * (xs + oj + g.Nx * (ys - 1 + rr)));
    f_lane[i] = part(on, xs + oj + g.Nx * (ys - 1 + rr));
    o_lds[i] = LD::kU + (min(rr, YC - 1) - 1) * LD::kORow + (oj + 1) * 32;
  }
  double vv[NG][NV > 0 ? NV : 1][3];
  unsigned fv[NG];
  auto load_v = [&](int ez) {
    const bool own = ez >= zs && ez < zend;
    const int po = part(own, 24 * g.Nx * g.Ny * ez), pf = part(own, g.Nx * g.Ny * ez);
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      fv[i] = __builtin_amdgcn_raw_buffer_load_b8(rfix, off2(f_lane[i], pf), 0, 0);
      const int o = off2(o_lane[i], po);
      if (MODE == EPI_SMOOTH) {
        bload3(ru, o, vv[i][0]);
        bload3(rb, o, vv[i][1]);
        bload3(rdi, o, vv[i][2]);
        bload3(rd, ep.c1 != 0.0 ? o : kNoOffset, vv[i][3]);
      } else if (MODE == EPI_RESID) {
        bload3(rb, o, vv[i][0]);
      } else if (MODE == kStoreDot) {
        bload3(ru, o, vv[i][0]);
      }
    }
  };
  double dot = 0.0;
  auto finish_plane = [&](int ez) {
    const int po = part(ez >= zs && ez < zend, 24 * g.Nx * g.Ny * ez);
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      const double* yq = (const double*)(lds + o_lds[i]);
      const double yv[3] = {yq[0], yq[1], yq[2]};
      const int o = off2(o_lane[i], po);
      const bool mine = (unsigned)o < (unsigned)kPoison;
      double out[3], dd[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const bool fixed = (fv[i] >> c) & 1u;
        if (MODE == EPI_STORE || MODE == kStoreDot) {
          out[c] = fixed ? 0.0 : yv[c];
          if (MODE == kStoreDot && mine) dot += vv[i][0][c] * out[c];
        } else if (MODE == EPI_RESID) {
          out[c] = fixed ? 0.0 : vv[i][0][c] - yv[c];
        } else {
          const double r = vv[i][1][c] - yv[c];
          dd[c] = fixed ? 0.0 : ep.c1 * vv[i][3][c] + ep.c2 * vv[i][2][c] * r;
          out[c] = fixed ? 0.0 : vv[i][0][c] + dd[c];
        }
      }
      bstore3(rout, o, out[0], out[1], out[2]);
      if (MODE == EPI_SMOOTH) {
        if (ep.store_d) bstore3(rd, o, dd[0], dd[1], dd[2]);
        if (ep.out64 && mine) {
          double* q = ep.out64 + (o >> 3);
          q[0] = out[0];
          q[1] = out[1];
          q[2] = out[2];
        }
      }
    }
  };

  // lane (c, n) of the matrix-core layout writes its node sum to O column n
  const int o_w = LD::kU + n * 32 + grp * 8;
  double zc[YC];
#pragma unroll
  for (int r = 0; r < YC; ++r) zc[r] = 0.0;

  load_u(zs - 1, true);
  store_u(zs - 1);
  load_u(zs, true);
  store_u(zs);
  load_u(zs + 1, zs + 1 <= zend);
  load_e(zs - 1, true);
  for (int ez = zs - 1; ez < zend; ++ez) {
    store_u(ez + 2);                              // loaded during the previous plane
#pragma unroll
    for (int i = 0; i < NE; ++i) esc[i] = ev[i];
    load_u(ez + 3, ez + 3 <= zend);
    load_e(ez + 1, ez + 1 < zend);
    load_v(ez);
    const int base = ((ez + dz_in + 3) % 3) * LD::kPlane + dy_in * LD::kRow + n * 24;
    double bc[6], bn[6];
    read_b(base, 0, bc);
    double yc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < YC; ++r) {
      if (r + 1 < YC) read_b(base, r + 1, bn);
      const double sc = bpermute(4 * (n + 16 * (r & 3)), esc[r >> 2]);
      f64x4 c0, c1;
      contract(bc, c0, c1);
      double t[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        t[k] = c0[k] * sc + yc[k];    // y: dy = 0 of this row + dy = 1 of the row below
        yc[k] = c1[k] * sc;
      }
      // x: dx = 0 of element n + dx = 1 of element n - 1; z: plane ez + plane ez - 1
      const double w0 = t[0] + dpp_shr1(t[1]);
      const double w1 = t[2] + dpp_shr1(t[3]);
      const double fin = w0 + zc[r];
      zc[r] = w1;
      if (r >= 1) *(double*)(lds + o_w + (r - 1) * LD::kORow) = fin;
      if (r + 1 < YC) {
#pragma unroll
        for (int st = 0; st < 6; ++st) bc[st] = bn[st];
      }
    }
    finish_plane(ez);
  }
  if (MODE == kStoreDot) {
    const double vd[1] = {dot};
    grid_sum<1>(vd, ep.ws);
  }
}

template <int YC, int MODE>
__global__ __launch_bounds__(64 * kMfmaWavesPerBlock) void k_apply_fine_mfma64(
    Grid g, const double* __restrict__ E, const double* __restrict__ atab,
    const double* __restrict__ u, const uint8_t* __restrict__ fixn, Epi<double> ep, int zchunk,
    int ntx, int nty, int ntiles) {
  fine_mfma64_body<YC, MODE>(g, E, atab, u, fixn, ep, zchunk, ntx, nty, ntiles,
                             xcd_block(blockIdx.x, gridDim.x));
}

// Stage-batched FP64 q = K p of every active item with the block partials of
// p.q (part[b] for table entry b = (item, block of the item's tile grid),
// geo[item] the grid for the launch shape).
template <int YC>
__global__ __launch_bounds__(64 * kMfmaWavesPerBlock) void k_bs_fine_mfma64(
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
  fine_mfma64_body<YC, kStoreDot>(V.g, S.E64, S.atab64, I.p, V.fixn, ep, zchunk, gm.x, gm.y, gm.z,
                                  e.y);
}

namespace {
struct MfmaLaunch { int ntx, nty, ntz, ntiles, blocks; };
MfmaLaunch mfma_launch(const Grid& g, int rows, int zchunk) {
  MfmaLaunch m;
  m.ntx = div_up(g.Nx, 15);
  m.nty = div_up(g.Ny, rows - 1);
  m.ntz = div_up(g.Nz, zchunk);
  m.ntiles = m.ntx * m.nty * m.ntz;
  m.blocks = div_up(m.ntiles, kMfmaWavesPerBlock);
  return m;
}
}  // namespace

bool mfma_size_ok(const Grid& g) {
  return (size_t)g.n * sizeof(float) < ((size_t)1 << 30) - 64;
}

bool mfma_shape_valid(int rows, int zchunk) {
  return (rows == 4 || rows == 8) && zchunk >= 1;
}

size_t apply_fine_mfma_blocks(const Grid& g, int rows, int zchunk) {
  return (size_t)mfma_launch(g, rows, zchunk).blocks;
}

template <int NSPLIT, int YC>
static void launch_shape(const Grid& g, const MfmaLaunch& m, int zchunk, const float* Es,
                         const uint16_t* at, const float* u, const uint8_t* fixn,
                         const Epi<float>& ep, hipStream_t s) {
  const dim3 grid(m.blocks), block(64 * kMfmaWavesPerBlock);
  if (ep.mode == EPI_STORE && ep.want_dot)
    k_apply_fine_mfma<NSPLIT, YC, kStoreDot><<<grid, block, 0, s>>>(g, Es, at, u, fixn, ep, zchunk,
                                                                   m.ntx, m.nty, m.ntiles);
  else if (ep.mode == EPI_STORE)
    k_apply_fine_mfma<NSPLIT, YC, EPI_STORE><<<grid, block, 0, s>>>(g, Es, at, u, fixn, ep, zchunk,
                                                                   m.ntx, m.nty, m.ntiles);
  else if (ep.mode == EPI_RESID)
    k_apply_fine_mfma<NSPLIT, YC, EPI_RESID><<<grid, block, 0, s>>>(g, Es, at, u, fixn, ep, zchunk,
                                                                   m.ntx, m.nty, m.ntiles);
  else if (ep.dot64)
    k_apply_fine_mfma<NSPLIT, YC, kSmoothDot><<<grid, block, 0, s>>>(
        g, Es, at, u, fixn, ep, zchunk, m.ntx, m.nty, m.ntiles);
  else
    k_apply_fine_mfma<NSPLIT, YC, EPI_SMOOTH><<<grid, block, 0, s>>>(
        g, Es, at, u, fixn, ep, zchunk, m.ntx, m.nty, m.ntiles);
}

void launch_apply_fine_mfma(const Grid& g, int nsplit, int rows, int zchunk, const float* Escaled,
                            const void* atab, const float* u, const uint8_t* fixn,
                            const Epi<float>& ep, hipStream_t s) {
  if (zchunk < 1) zchunk = 1;
  if (rows != 4) rows = 8;
  const MfmaLaunch m = mfma_launch(g, rows, zchunk);
  const uint16_t* at = (const uint16_t*)atab;
  if (nsplit == 3) {
    if (rows == 4) launch_shape<3, 4>(g, m, zchunk, Escaled, at, u, fixn, ep, s);
    else launch_shape<3, 8>(g, m, zchunk, Escaled, at, u, fixn, ep, s);
  } else if (nsplit == 2) {
    if (rows == 4) launch_shape<2, 4>(g, m, zchunk, Escaled, at, u, fixn, ep, s);
    else launch_shape<2, 8>(g, m, zchunk, Escaled, at, u, fixn, ep, s);
  } else {
    if (rows == 4) launch_shape<1, 4>(g, m, zchunk, Escaled, at, u, fixn, ep, s);
    else launch_shape<1, 8>(g, m, zchunk, Escaled, at, u, fixn, ep, s);
  }
  if (ep.mode == EPI_STORE && ep.want_dot && ep.dot_out)
    launch_finalize(ep.ws, m.blocks, 1, ep.dot_out, s);
}

template <int YC>
static void launch_shape64(const Grid& g, const MfmaLaunch& m, int zchunk, const double* E,
                           const double* at, const double* u, const uint8_t* fixn,
                           const Epi<double>& ep, hipStream_t s) {
  const dim3 grid(m.blocks), block(64 * kMfmaWavesPerBlock);
  if (ep.mode == EPI_STORE && ep.want_dot)
    k_apply_fine_mfma64<YC, kStoreDot><<<grid, block, 0, s>>>(g, E, at, u, fixn, ep, zchunk, m.ntx,
                                                              m.nty, m.ntiles);
  else if (ep.mode == EPI_STORE)
    k_apply_fine_mfma64<YC, EPI_STORE><<<grid, block, 0, s>>>(g, E, at, u, fixn, ep, zchunk, m.ntx,
                                                              m.nty, m.ntiles);
  else if (ep.mode == EPI_RESID)
    k_apply_fine_mfma64<YC, EPI_RESID><<<grid, block, 0, s>>>(g, E, at, u, fixn, ep, zchunk, m.ntx,
                                                              m.nty, m.ntiles);
  else
    k_apply_fine_mfma64<YC, EPI_SMOOTH><<<grid, block, 0, s>>>(g, E, at, u, fixn, ep, zchunk, m.ntx,
                                                               m.nty, m.ntiles);
}

void launch_apply_fine_mfma64(const Grid& g, int rows, int zchunk, const double* E,
                              const double* atab64, const double* u, const uint8_t* fixn,
                              const Epi<double>& ep, hipStream_t s) {
  if (zchunk < 1) zchunk = 1;
  if (rows != 4) rows = 8;
  const MfmaLaunch m = mfma_launch(g, rows, zchunk);
  if (rows == 4) launch_shape64<4>(g, m, zchunk, E, atab64, u, fixn, ep, s);
  else launch_shape64<8>(g, m, zchunk, E, atab64, u, fixn, ep, s);
  if (ep.mode == EPI_STORE && ep.want_dot && ep.dot_out)
    launch_finalize(ep.ws, m.blocks, 1, ep.dot_out, s);
}

bool mfma64_size_ok(const Grid& g) {
  return (size_t)g.n * sizeof(double) < ((size_t)1 << 30) - 64;
}

// Host: FP64 A operand, [h][step][lane]: row m = lane % 16 of half h, input
// (q = lane / 16, step) = node (step / 3, q & 1, q >> 1) component step % 3.
// The FP64 MFMA returns row m in lane group m % 4, register m / 4 (measured
// on gfx950; the FP32 16x16 layout is group m / 4, register m % 4), so row
// m = 4 (dx + 2 dz) + c carries component c of node (dx, h, dz): lane group c
// then holds component c and register dx + 2 dz the node, as in the BF16
// kernel (c = 3: zero row).
void build_mfma_atab64(const KeTables& kt, double* out /* 2*6*64 */) {
  for (int h = 0; h < 2; ++h)
    for (int st = 0; st < 6; ++st)
      for (int lane = 0; lane < 64; ++lane) {
        const int m = lane & 15, q = lane >> 4;
        const int c = m & 3, k = m >> 2;
        const int dx = k & 1, dz = k >> 1;
        const int aout = dx + 2 * h + 4 * dz;
        const int bin = (st / 3) + 2 * (q & 1) + 4 * (q >> 1);
        out[(h * 6 + st) * 64 + lane] =
            c < 3 ? kt.ke[(3 * aout + c) * 24 + 3 * bin + (st % 3)] : 0.0;
      }
}

// E / s in FP32 for the MFMA kernel.
__global__ void k_scale_E(const double* __restrict__ E, float* __restrict__ Es, int nel,
                          double inv_s) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nel) Es[e] = (float)(E[e] * inv_s);
}

void launch_scale_E(const double* E, float* Es, int nel, double inv_s, hipStream_t s) {
  k_scale_E<<<div_up(nel, 256), 256, 0, s>>>(E, Es, nel, inv_s);
}

// Host: A-operand table in BF16 bit patterns (integers <= 255 are exact),
// [h][lane][8]: row m = lane % 16 = 4 c + (dx + 2 dz) is component c (c = 3:
// zero row) of output node (dx, h, dz); slot j of lane group q = lane / 16 is
// component j % 4 (3: zero) of input node (j / 4, q & 1, q >> 1).
void build_mfma_atab(const KeTables& kt, uint16_t* out /* 2*64*8 */) {
  for (int h = 0; h < 2; ++h)
    for (int lane = 0; lane < 64; ++lane) {
      const int m = lane & 15, q = lane >> 4;
      const int c = m >> 2, k = m & 3;
      const int dx = k & 1, dz = k >> 1;
      const int aout = dx + 2 * h + 4 * dz;
      for (int j = 0; j < 8; ++j) {
        float v = 0.f;
        const int cin = j & 3;
        if (c < 3 && cin < 3) {
          const int bin = (j >> 2) + 2 * (q & 1) + 4 * (q >> 1);
          v = (float)kt.kint[(3 * aout + c) * 24 + 3 * bin + cin];
        }
        uint32_t bits;
        std::memcpy(&bits, &v, 4);
        out[(h * 64 + lane) * 8 + j] = (uint16_t)(bits >> 16);
      }
    }
}

int4 bs_mfma_geometry(const Grid& g, int rows, int zchunk) {
  const MfmaLaunch m = mfma_launch(g, rows, zchunk);
  return int4{m.ntx, m.nty, m.ntiles, m.blocks};
}

void bs_fine_mfma(const BsArgs& a, const BsTable& t, const int4* geo, const int* flags, int rows,
                  int zchunk, int mode, int post, int k, int cin, int last, hipStream_t s) {
  if (t.n == 0) return;
  const dim3 grid(t.n), block(64 * kMfmaWavesPerBlock);
#define SGMG_BSF(YC, M)                                                                       \
  k_bs_fine_mfma<YC, M><<<grid, block, 0, s>>>(a.sys, a.items, t.blk, geo, flags, post, k, cin, \
                                               last, zchunk)
  if (rows == 4) {
    if (mode == EPI_RESID) SGMG_BSF(4, EPI_RESID);
    else SGMG_BSF(4, EPI_SMOOTH);
  } else {
    if (mode == EPI_RESID) SGMG_BSF(8, EPI_RESID);
    else SGMG_BSF(8, EPI_SMOOTH);
  }
#undef SGMG_BSF
}

void bs_fine_mfma64_store_dot(const BsArgs& a, const BsTable& t, const int4* geo, const int* flags,
                              int rows, int zchunk, double* part, hipStream_t s) {
  if (t.n == 0) return;
  if (rows == 1) {
    bs_fine_sf64_store_dot(a, t, geo, flags, zchunk, part, s);
    return;
  }
  const dim3 grid(t.n), block(64 * kMfmaWavesPerBlock);
  if (rows == 4)
    k_bs_fine_mfma64<4><<<grid, block, 0, s>>>(a.sys, a.items, t.blk, geo, flags, part, zchunk);
  else
    k_bs_fine_mfma64<8><<<grid, block, 0, s>>>(a.sys, a.items, t.blk, geo, flags, part, zchunk);
}

}  // namespace sgmg
