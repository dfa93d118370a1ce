// Fine-level K.u on the gfx950 matrix cores (Eq. mf_matvec; Sec. 3.5 BF16
// semantics).  The element matrix s*K_e is an integer matrix with entries of
// magnitude <= 88, hence exact in BF16; the element input tile is rounded to
// BF16 (NSPLIT = 1) or split into three BF16 terms that together carry the
// FP32 significand (NSPLIT = 3).  Products are exact and accumulate in FP32 on
// v_mfma_f32_16x16x32_bf16; E_e / s is applied in FP32 afterwards.
//
// Work decomposition (one workgroup = WAVES waves):
//   * a wave owns one element row (fixed ey) of a 16-element x-batch and
//     marches along z; the MFMA output rows are laid out as
//     [dz (M half)] x [dx + 2 dy (lane group)] x [component], so the dz = 1
//     half of plane ez and the dz = 0 half of plane ez+1 meet in the same
//     lane: z-neighbour sums are a register carry;
//   * x-neighbours (dx = 1 of element n, dx = 0 of element n+1) are combined
//     with one ds_bpermute;
//   * y-neighbours (dy = 1 of row ey, dy = 0 of row ey+1) are combined in LDS
//     in two fixed-order sub-steps (first every wave's dy = 0 writes, then the
//     dy = 1 adds): a colored, atomic-free, deterministic scatter.
//   The workgroup recomputes one halo element on the low side in x and y so
//   that every node it writes is complete: 15 owned nodes per 16-element
//   batch in x, WAVES-1 owned node rows in y.
#include <cstring>

#include "kernels.hpp"

namespace sgmg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMfmaWaves = 4;   // waves per workgroup (owned node rows + 1)

// A operand table: [h][lane][8] BF16 bit patterns, built on the host.
// Row m = lane % 16 = 4 * (dx + 2 dy) + c of output node (dx, dy, dz = h);
// slot j of lane group g = lane / 16 is input node (j / 3, g & 1, g >> 1),
// component j % 3 (slots 6, 7 and c = 3 are zero padding).

template <int NSPLIT, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_apply_fine_mfma(
    Grid g, const float* __restrict__ Es, const uint16_t* __restrict__ atab,
    const float* __restrict__ u, const uint8_t* __restrict__ fixn, Epi<float> ep, int zchunk) {
  __shared__ float plane[WAVES + 1][16][3];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int grp = lane >> 4;          // input edge (dy_in, dz_in) / output (dx, dy)
  const int n = lane & 15;            // element position in the x-batch
  const int xs = blockIdx.x * 15;     // first owned node in x
  const int ys = blockIdx.y * (WAVES - 1);
  const int zs = blockIdx.z * zchunk;
  const int ex = xs - 1 + n;
  const int ey = ys - 1 + w;
  const bool exy_ok = ex >= 0 && ex < g.nx && ey >= 0 && ey < g.ny;
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

  // raw operands of element plane ez (6 input values, E / s)
  struct In { float v[6]; float es; };
  auto load_in = [&](int ez, In& in) {
    const bool ok = exy_ok && ez >= 0 && ez < g.nz;
#pragma unroll
    for (int j = 0; j < 6; ++j) in.v[j] = 0.f;
    in.es = 0.f;
    if (ok) {
      const size_t base = 3 * (size_t)(ex + g.Nx * ((ey + dy_in) + g.Ny * (ez + dz_in)));
#pragma unroll
      for (int j = 0; j < 6; ++j) in.v[j] = u[base + j];
      in.es = Es[ex + g.nx * (ey + g.ny * ez)];
    }
  };
  // contraction: acc for node plane ez (c0) and ez+1 (c1), scaled by E / s
  auto contract = [&](const In& in, f32x4& c0, f32x4& c1) {
    c0 = f32x4{0.f, 0.f, 0.f, 0.f};
    c1 = f32x4{0.f, 0.f, 0.f, 0.f};
    bf16x8 b[NSPLIT];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      float r = in.v[j];
#pragma unroll
      for (int sp = 0; sp < NSPLIT; ++sp) {
        const __bf16 t = (__bf16)r;
        b[sp][j] = t;
        r -= (float)t;
      }
    }
#pragma unroll
    for (int sp = 0; sp < NSPLIT; ++sp) {
      b[sp][6] = (__bf16)0.f;
      b[sp][7] = (__bf16)0.f;
    }
#pragma unroll
    for (int sp = NSPLIT - 1; sp >= 0; --sp) {    // smallest terms first
      c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b[sp], c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b[sp], c1, 0, 0, 0);
    }
    // column n of the result (lane % 16) is element n, whose E / s every lane
    // of that column loaded itself
    c0 *= in.es;
    c1 *= in.es;
  };

  // the epilogue node of this thread (rows 1..WAVES-1, positions 1..15)
  const int t = threadIdx.x;
  const int er = 1 + t / 15, eq = 1 + t % 15;
  const int enx = xs - 1 + eq, eny = ys - 1 + er;
  const bool e_own = t < 15 * (WAVES - 1) && enx < g.Nx && eny < g.Ny;
  const bool need_b = ep.mode != EPI_STORE;
  const bool need_sm = ep.mode == EPI_SMOOTH;
  const bool need_d = need_sm && ep.c1 != 0.0;

  In cur, nxt;
  f32x4 carry, dummy;
  load_in(zs - 1, cur);
  load_in(zs, nxt);
  contract(cur, dummy, carry);   // prologue: dz = 1 half of the plane below
  double dot = 0.0;
  const int dx = grp & 1, dyo = grp >> 1;
  const int src = ((grp | 1) << 4) + ((n + 15) & 15);   // lane of (dx = 1, same dy, n - 1)
  const int zend = min(zs + zchunk, g.Nz);
  for (int ez = zs; ez < zend; ++ez) {
    cur = nxt;
    if (ez + 1 < zend) load_in(ez + 1, nxt);           // prefetch the next plane
    // prefetch the epilogue operands of this plane
    float ex_[3] = {0.f, 0.f, 0.f}, eb[3] = {0.f, 0.f, 0.f}, edi[3] = {0.f, 0.f, 0.f},
          edp[3] = {0.f, 0.f, 0.f};
    unsigned efx = 7u;
    int node = 0;
    if (e_own) {
      node = enx + g.Nx * (eny + g.Ny * ez);
      const size_t b3 = 3 * (size_t)node;
      efx = fixn[node];
#pragma unroll
      for (int c = 0; c < 3; ++c) ex_[c] = u[b3 + c];
      if (need_b) {
#pragma unroll
        for (int c = 0; c < 3; ++c) eb[c] = ep.b[b3 + c];
      }
      if (need_sm) {
#pragma unroll
        for (int c = 0; c < 3; ++c) edi[c] = ep.dinv[b3 + c];
      }
      if (need_d) {
#pragma unroll
        for (int c = 0; c < 3; ++c) edp[c] = ep.d[b3 + c];
      }
    }
    f32x4 c0, c1;
    contract(cur, c0, c1);
    const float v0 = c0[0] + carry[0], v1 = c0[1] + carry[1], v2 = c0[2] + carry[2];
    carry = c1;
    // x: node (xs - 1 + n) gets dx = 0 of element n and dx = 1 of element n - 1
    const float p0 = __int_as_float(__builtin_amdgcn_ds_bpermute(src * 4, __float_as_int(v0)));
    const float p1 = __int_as_float(__builtin_amdgcn_ds_bpermute(src * 4, __float_as_int(v1)));
    const float p2 = __int_as_float(__builtin_amdgcn_ds_bpermute(src * 4, __float_as_int(v2)));
    // y: two colored sub-steps in LDS (rows are ey + dy - (ys - 1))
    if (dx == 0 && dyo == 0) {
      plane[w][n][0] = v0 + p0;
      plane[w][n][1] = v1 + p1;
      plane[w][n][2] = v2 + p2;
    }
    __syncthreads();
    if (dx == 0 && dyo == 1) {
      plane[w + 1][n][0] += v0 + p0;
      plane[w + 1][n][1] += v1 + p1;
      plane[w + 1][n][2] += v2 + p2;
    }
    __syncthreads();
    if (e_own) {
      const double y[3] = {(double)plane[er][eq][0], (double)plane[er][eq][1],
                           (double)plane[er][eq][2]};
      dot += epilogue3_pre(ep, node, efx, ex_, y, eb, edi, edp);
    }
    __syncthreads();
  }
  if (ep.want_dot) {
    const double vv[1] = {dot};
    grid_sum<1>(vv, ep.ws);
  }
}

static dim3 mfma_grid(const Grid& g, int zchunk) {
  return dim3(div_up(g.Nx, 15), div_up(g.Ny, kMfmaWaves - 1), div_up(g.Nz, zchunk));
}

size_t apply_fine_mfma_blocks(const Grid& g, int zchunk) {
  const dim3 d = mfma_grid(g, zchunk);
  return (size_t)d.x * d.y * d.z;
}

void launch_apply_fine_mfma(const Grid& g, int nsplit, int zchunk, const float* Escaled,
                            const void* atab, const float* u, const uint8_t* fixn,
                            const Epi<float>& ep, hipStream_t s) {
  if (zchunk < 1) zchunk = 1;
  const int g_zchunk = zchunk;
  const dim3 grid = mfma_grid(g, zchunk);
  const dim3 block(64 * kMfmaWaves);
  const uint16_t* at = (const uint16_t*)atab;
  if (nsplit == 3)
    k_apply_fine_mfma<3, kMfmaWaves><<<grid, block, 0, s>>>(g, Escaled, at, u, fixn, ep, g_zchunk);
  else
    k_apply_fine_mfma<1, kMfmaWaves><<<grid, block, 0, s>>>(g, Escaled, at, u, fixn, ep, g_zchunk);
  if (ep.want_dot)
    launch_finalize(ep.ws, (int)(grid.x * grid.y * grid.z), 1, ep.dot_out, s);
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

// Host: A-operand table in BF16 bit patterns (integers <= 255 are exact).
void build_mfma_atab(const KeTables& kt, uint16_t* out /* 2*64*8 */) {
  for (int h = 0; h < 2; ++h)
    for (int lane = 0; lane < 64; ++lane) {
      const int m = lane & 15, gq = lane >> 4;
      const int go = m >> 2, c = m & 3;
      const int dx = go & 1, dy = go >> 1;
      const int aout = dx + 2 * dy + 4 * h;
      for (int j = 0; j < 8; ++j) {
        float v = 0.f;
        if (c < 3 && j < 6) {
          const int bin = (j / 3) + 2 * (gq & 1) + 4 * (gq >> 1);
          v = (float)kt.kint[(3 * aout + c) * 24 + 3 * bin + (j % 3)];
        }
        uint32_t bits;
        std::memcpy(&bits, &v, 4);
        out[(h * 64 + lane) * 8 + j] = (uint16_t)(bits >> 16);
      }
    }
}

}  // namespace sgmg
