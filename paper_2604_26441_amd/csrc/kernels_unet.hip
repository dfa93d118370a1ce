// Training and inference kernels of the warm-start 3D U-Net (extension, not
// a passage of the paper).  Tensors are (N, C, D, H, W) in FP32; weights are
// held in BF16 precision (values rounded to BF16, stored as FP32 so the
// arithmetic is FP32 accumulation of BF16-exact weights) in the layout
// w[(ci * K^3 + tap) * Cop + co], Cop = output channels padded to 16, so the
// 16 weights of one (ci, tap) are contiguous and read with uniform loads.
#include "kernels.hpp"
#include "node_ops.hpp"
#include "unet.hpp"

namespace sgmg {

constexpr int kCOB = 16;   // output channels per thread

// y[n, co] = epi(b[co] + sum_{ci, tap} w * x[n, ci, v + tap - r]) for co in a
// block of 16; epi: optional ReLU, optional stored pre-add value r, optional
// skip add.  Zero padding outside the volume.
template <int K>
__global__ __launch_bounds__(256) void k_conv_fwd(const float* __restrict__ x, int Ci, int Co,
                                                  int Cop, int D, int H, int W,
                                                  const float* __restrict__ w,
                                                  const float* __restrict__ bias, int relu,
                                                  float* __restrict__ rpre,
                                                  const float* __restrict__ add,
                                                  float* __restrict__ y) {
  constexpr int R = K / 2;
  constexpr int K3 = K * K * K;
  const int HW = H * W, DHW = D * HW;
  const int v = blockIdx.x * 256 + threadIdx.x;
  const int co0 = blockIdx.y * kCOB;
  const int n = blockIdx.z;
  if (v >= DHW) return;
  const int d = v / HW, hh = (v / W) % H, ww = v % W;
  float acc[kCOB];
#pragma unroll
  for (int c = 0; c < kCOB; ++c) acc[c] = 0.f;
  const float* xn = x + (size_t)n * Ci * DHW;
  for (int ci = 0; ci < Ci; ++ci) {
    const float* xc = xn + (size_t)ci * DHW;
    const float* wc = w + (size_t)ci * K3 * Cop + co0;
#pragma unroll
    for (int t = 0; t < K3; ++t) {
      const int dz = t / (K * K) - R, dy = (t / K) % K - R, dx = t % K - R;
      const int zz = d + dz, yy = hh + dy, xx = ww + dx;
      const bool ok = (unsigned)zz < (unsigned)D && (unsigned)yy < (unsigned)H &&
                      (unsigned)xx < (unsigned)W;
      const float xv = ok ? xc[(size_t)zz * HW + yy * W + xx] : 0.f;
      const float* wt = wc + (size_t)t * Cop;
#pragma unroll
      for (int c = 0; c < kCOB; ++c) acc[c] += wt[c] * xv;
    }
  }
#pragma unroll
  for (int c = 0; c < kCOB; ++c) {
    const int co = co0 + c;
    if (co >= Co) break;
    float val = acc[c] + (bias ? bias[co] : 0.f);
    if (relu) val = fmaxf(val, 0.f);
    const size_t o = ((size_t)n * Co + co) * DHW + v;
    if (rpre) rpre[o] = val;
    if (add) val += add[o];
    y[o] = val;
  }
}

void launch_conv_fwd(int K, const float* x, int N, int Ci, int Co, int D, int H, int W,
                     const float* w, const float* b, int relu, float* rpre, const float* add,
                     float* y, hipStream_t s) {
  const int Cop = (Co + kCOB - 1) / kCOB * kCOB;
  dim3 grid(div_up((long)D * H * W, 256), Cop / kCOB, N);
  if (K == 3)
    k_conv_fwd<3><<<grid, 256, 0, s>>>(x, Ci, Co, Cop, D, H, W, w, b, relu, rpre, add, y);
  else
    k_conv_fwd<1><<<grid, 256, 0, s>>>(x, Ci, Co, Cop, D, H, W, w, b, relu, rpre, add, y);
}

// ---------------------------------------------------------------------------
// 3x3x3 convolution as an implicit GEMM on the matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation).  Per MFMA the A operand is
// 16 output channels x 32 reduction slots and the B operand 32 reduction
// slots x 16 output voxels (one x-run of a tile row); the 32 slots are 4 taps
// x 8 input channels: lane group q = lane / 16 takes tap 4 s + q of k-step s
// (7 steps cover the 27 taps, tap 27 has zero weights) and channels
// 8 ch .. 8 ch + 7 of channel chunk ch.  The activations are FP32: each value
// is split exactly into three BF16 terms (truncation: hi, then the
// remainder's hi, then what is left, 8 + 8 + 8 significand bits), and the
// three products with the BF16 weight are exact in FP32, so the result is an
// FP32 sum of the exact products (the accuracy of the FP32 vector-ALU form).
//
// Block: an output tile of 16 (x) x 4 (y) x 4 (z) voxels of one sample and
// COT tiles of 16 output channels; wave w owns the 4 tile rows of z = w.
// Per channel chunk the 18 x 6 x 6 input halo is staged once in LDS as the
// three term planes, 8 channels (16 B) per voxel, so one ds_read_b128 is a
// lane's B operand; zero outside the volume (the padding).
constexpr int kCTX = 16, kCTY = 4, kCTZ = 4;
constexpr int kCHX = kCTX + 2, kCHY = kCTY + 2, kCHZ = kCTZ + 2;
constexpr int kCHV = kCHX * kCHY * kCHZ;       // 648 staged voxels
constexpr int kCSteps = 7;                     // k-steps of 4 taps

typedef __bf16 cbf16x8 __attribute__((ext_vector_type(8)));
typedef float cf32x4 __attribute__((ext_vector_type(4)));

// exact three-term BF16 split of v; returns the terms' bit patterns
__device__ inline void split3(float v, unsigned& t0, unsigned& t1, unsigned& t2) {
  const unsigned b = __float_as_uint(v);
  const unsigned h = b & 0xffff0000u;
  const float r1 = v - __uint_as_float(h);
  const unsigned m = __float_as_uint(r1) & 0xffff0000u;
  const float r2 = r1 - __uint_as_float(m);
  t0 = h >> 16;
  t1 = m >> 16;
  t2 = __float_as_uint(r2) >> 16;
}

template <int COT>
__global__ __launch_bounds__(256) void k_conv3_mfma(const float* __restrict__ x, int up, int Ci,
                                                    int Co, int Cop, int D, int H, int W, int tx,
                                                    int ty, const uint4* __restrict__ wp,
                                                    const float* __restrict__ bias, int relu,
                                                    float* __restrict__ rpre,
                                                    const float* __restrict__ add,
                                                    float* __restrict__ y) {
  __shared__ uint4 lds[3][kCHV];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int col = lane & 15, q = lane >> 4;
  const int tile = xcd_block(blockIdx.x, gridDim.x);
  const int n = blockIdx.y, ct0 = blockIdx.z * COT;
  const int bx = tile % tx, by = (tile / tx) % ty, bz = tile / (tx * ty);
  const int x0 = bx * kCTX, y0 = by * kCTY, z0 = bz * kCTZ;
  const long HW = (long)H * W, DHW = (long)D * HW;
  // with up = 1 the input is stored at half resolution and read as its
  // nearest-neighbour upsampling (voxel v of the output grid reads v / 2)
  const int Wi = W >> up, Hi = H >> up;
  const long HWi = (long)Hi * Wi, DHWi = (long)(D >> up) * HWi;
  const float* xn = x + (size_t)n * Ci * DHWi;
  const int nchunk = (Ci + 7) >> 3;
  cf32x4 acc[kCTY][COT];
#pragma unroll
  for (int r = 0; r < kCTY; ++r)
#pragma unroll
    for (int c = 0; c < COT; ++c) acc[r][c] = cf32x4{0.f, 0.f, 0.f, 0.f};

  for (int ch = 0; ch < nchunk; ++ch) {
    __syncthreads();                       // the previous chunk's reads are done
    for (int v = threadIdx.x; v < kCHV; v += 256) {
      const int hx = v % kCHX, hy = (v / kCHX) % kCHY, hz = v / (kCHX * kCHY);
      const int gx = x0 - 1 + hx, gy = y0 - 1 + hy, gz = z0 - 1 + hz;
      const bool in = (unsigned)gx < (unsigned)W && (unsigned)gy < (unsigned)H &&
                      (unsigned)gz < (unsigned)D;
      const size_t off = in ? (size_t)(gz >> up) * HWi + (size_t)(gy >> up) * Wi + (gx >> up) : 0;
      unsigned p0[4], p1[4], p2[4];
#pragma unroll
      for (int j = 0; j < 8; j += 2) {
        const int c = 8 * ch + j;
        const float a = in && c < Ci ? xn[(size_t)c * DHWi + off] : 0.f;
        const float b = in && c + 1 < Ci ? xn[(size_t)(c + 1) * DHWi + off] : 0.f;
        unsigned a0, a1, a2, b0, b1, b2;
        split3(a, a0, a1, a2);
        split3(b, b0, b1, b2);
        p0[j >> 1] = a0 | (b0 << 16);
        p1[j >> 1] = a1 | (b1 << 16);
        p2[j >> 1] = a2 | (b2 << 16);
      }
      lds[0][v] = uint4{p0[0], p0[1], p0[2], p0[3]};
      lds[1][v] = uint4{p1[0], p1[1], p1[2], p1[3]};
      lds[2][v] = uint4{p2[0], p2[1], p2[2], p2[3]};
    }
    __syncthreads();
    const uint4* wc = wp + (size_t)ch * kCSteps * Cop * 4;
#pragma unroll 1
    for (int s = 0; s < kCSteps; ++s) {
      uint4 a[COT];
#pragma unroll
      for (int c = 0; c < COT; ++c) a[c] = wc[((size_t)s * Cop + (ct0 + c) * 16 + col) * 4 + q];
      // tap 27 (weights zero) reads tap 26's voxel, a staged finite value
      const int t = 4 * s + q < 27 ? 4 * s + q : 26;
      const int dx = t % 3, dy = (t / 3) % 3, dz = t / 9;
#pragma unroll
      for (int r = 0; r < kCTY; ++r) {
        const int v = ((w + dz) * kCHY + (r + dy)) * kCHX + col + dx;
        const cbf16x8 b2 = __builtin_bit_cast(cbf16x8, lds[2][v]);
        const cbf16x8 b1 = __builtin_bit_cast(cbf16x8, lds[1][v]);
        const cbf16x8 b0 = __builtin_bit_cast(cbf16x8, lds[0][v]);
#pragma unroll
        for (int c = 0; c < COT; ++c) {       // smallest terms first
          const cbf16x8 av = __builtin_bit_cast(cbf16x8, a[c]);
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b2, acc[r][c], 0, 0, 0);
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b1, acc[r][c], 0, 0, 0);
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b0, acc[r][c], 0, 0, 0);
        }
      }
    }
  }
  // epilogue: lane holds output channels 16 c + 4 q + i of voxel column col
  const int gx = x0 + col, gz = z0 + w;
  if (gx >= W || gz >= D) return;
#pragma unroll
  for (int r = 0; r < kCTY; ++r) {
    const int gy = y0 + r;
    if (gy >= H) break;
    const size_t vox = (size_t)gz * HW + (size_t)gy * W + gx;
#pragma unroll
    for (int c = 0; c < COT; ++c)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int co = (ct0 + c) * 16 + 4 * q + i;
        if (co >= Co) continue;
        float val = acc[r][c][i] + (bias ? bias[co] : 0.f);
        if (relu) val = fmaxf(val, 0.f);
        const size_t o = ((size_t)n * Co + co) * DHW + vox;
        if (rpre) rpre[o] = val;
        if (add) val += add[o];
        y[o] = val;
      }
  }
}

// Packed A operands: wp[((ch * 7 + s) * Cop + co) * 4 + q] holds the BF16
// weights of input channels 8 ch .. 8 ch + 7 at tap 4 s + q for output
// channel co (zero past Ci and for tap 27), from the BF16-exact FP32 layout
// w[(ci * 27 + tap) * Cop + co].
__global__ void k_pack_conv3(const float* __restrict__ w, int Ci, int Cop, int total,
                             uint4* __restrict__ wp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int q = i & 3, co = (i >> 2) % Cop, s = (i / (4 * Cop)) % kCSteps,
            ch = i / (4 * Cop * kCSteps);
  const int t = 4 * s + q;
  unsigned p[4];
#pragma unroll
  for (int j = 0; j < 8; j += 2) {
    const int c = 8 * ch + j;
    const float a = t < 27 && c < Ci ? w[((size_t)c * 27 + t) * Cop + co] : 0.f;
    const float b = t < 27 && c + 1 < Ci ? w[((size_t)(c + 1) * 27 + t) * Cop + co] : 0.f;
    p[j >> 1] = (__float_as_uint(a) >> 16) | (__float_as_uint(b) & 0xffff0000u);
  }
  wp[i] = uint4{p[0], p[1], p[2], p[3]};
}

size_t conv3_packed_words(int Ci, int Co) {
  const int Cop = (Co + kCOB - 1) / kCOB * kCOB;
  return (size_t)((Ci + 7) / 8) * kCSteps * Cop * 4;
}

void launch_pack_conv3(const float* w, int Ci, int Co, uint4* wp, hipStream_t s) {
  const int Cop = (Co + kCOB - 1) / kCOB * kCOB;
  const int total = (int)conv3_packed_words(Ci, Co);
  k_pack_conv3<<<div_up(total, 256), 256, 0, s>>>(w, Ci, Cop, total, wp);
}

void launch_conv3_mfma(const float* x, int up, int N, int Ci, int Co, int D, int H, int W,
                       const uint4* wp, const float* b, int relu, float* rpre, const float* add,
                       float* y, hipStream_t s) {
  const int Cop = (Co + kCOB - 1) / kCOB * kCOB, ntile = Cop / 16;
  const int tx = div_up(W, kCTX), ty = div_up(H, kCTY), tz = div_up(D, kCTZ);
  const long tiles = (long)tx * ty * tz;
  // channel tiles per block: the largest power of two dividing ntile (<= 8),
  // halved while the grid has fewer than 1024 blocks
  int cot = 1;
  while (cot < 8 && ntile % (2 * cot) == 0) cot *= 2;
  while (cot > 1 && tiles * N * (ntile / cot) < 1024) cot /= 2;
  dim3 grid((unsigned)tiles, N, ntile / cot);
#define SGMG_CONV3(C)                                                                      \
  k_conv3_mfma<C><<<grid, 256, 0, s>>>(x, up, Ci, Co, Cop, D, H, W, tx, ty, wp, b, relu, rpre, \
                                       add, y)
  switch (cot) {
    case 8: SGMG_CONV3(8); break;
    case 4: SGMG_CONV3(4); break;
    case 2: SGMG_CONV3(2); break;
    default: SGMG_CONV3(1); break;
  }
#undef SGMG_CONV3
}

// Weights for the data gradient: wt[(co * K3 + (K3 - 1 - t)) * Cip + ci] =
// w[(ci * K3 + t) * Cop + co]  (channels swapped, taps flipped).
__global__ void k_weight_transpose(const float* __restrict__ w, int Ci, int Co, int Cop, int K3,
                                   int Cip, float* __restrict__ wt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Co * K3 * Cip) return;
  const int ci = i % Cip, t = (i / Cip) % K3, co = i / (Cip * K3);
  wt[i] = ci < Ci ? w[((size_t)ci * K3 + (K3 - 1 - t)) * Cop + co] : 0.f;
}

void launch_weight_transpose(const float* w, int Ci, int Co, int K, float* wt, hipStream_t s) {
  const int Cop = (Co + kCOB - 1) / kCOB * kCOB;
  const int Cip = (Ci + kCOB - 1) / kCOB * kCOB;
  const int K3 = K * K * K;
  k_weight_transpose<<<div_up((long)Co * K3 * Cip, 256), 256, 0, s>>>(w, Ci, Co, Cop, K3, Cip, wt);
}

// Weight and bias gradients, first stage: block (ci, co-quad, chunk) sums
// dy[n, co, v] * x[n, ci, v + tap - r] over its voxel chunk for 4 output
// channels and all taps; the block totals go to part[chunk][...] and a
// second kernel adds the chunks in order (deterministic).
constexpr int kWGChunk = 4096;

template <int K>
__global__ __launch_bounds__(256) void k_conv_wgrad(const float* __restrict__ x, int up,
                                                    const float* __restrict__ dy, int N, int Ci,
                                                    int Co, int D, int H, int W,
                                                    float* __restrict__ part) {
  constexpr int R = K / 2;
  constexpr int K3 = K * K * K;
  __shared__ float red[4][4 * K3 + 4];
  const int HW = H * W, DHW = D * HW;
  const long total = (long)N * DHW;
  const int ci = blockIdx.x;
  const int co0 = blockIdx.y * 4;
  const int chunk = blockIdx.z;
  float acc[4][K3];
  float accb[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    accb[c] = 0.f;
#pragma unroll
    for (int t = 0; t < K3; ++t) acc[c][t] = 0.f;
  }
  const long beg = (long)chunk * kWGChunk;
  const long end = beg + kWGChunk < total ? beg + kWGChunk : total;
  for (long g = beg + threadIdx.x; g < end; g += 256) {
    const int n = (int)(g / DHW), v = (int)(g % DHW);
    const int d = v / HW, hh = (v / W) % H, ww = v % W;
    float gy[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
      gy[c] = co0 + c < Co ? dy[((size_t)n * Co + co0 + c) * DHW + v] : 0.f;
    // up = 1: x is stored at half resolution and read as its upsampling
    const int Wi = W >> up, HWi = (H >> up) * Wi;
    const float* xc = x + ((size_t)n * Ci + ci) * (size_t)((D >> up) * HWi);
#pragma unroll
    for (int t = 0; t < K3; ++t) {
      const int dz = t / (K * K) - R, dyy = (t / K) % K - R, dx = t % K - R;
      const int zz = d + dz, yy = hh + dyy, xx = ww + dx;
      const bool ok = (unsigned)zz < (unsigned)D && (unsigned)yy < (unsigned)H &&
                      (unsigned)xx < (unsigned)W;
      const float xv = ok ? xc[(size_t)(zz >> up) * HWi + (yy >> up) * Wi + (xx >> up)] : 0.f;
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c][t] += gy[c] * xv;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) accb[c] += gy[c];
  }
  // fixed-order block reduction: wave sums, then the 4 wave totals in order
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int t = 0; t < K3; ++t) {
      float s = acc[c][t];
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      if (lane == 0) red[wv][c * K3 + t] = s;
    }
    float sb = accb[c];
    for (int off = 32; off > 0; off >>= 1) sb += __shfl_xor(sb, off, 64);
    if (lane == 0) red[wv][4 * K3 + c] = sb;
  }
  __syncthreads();
  const int nv = 4 * K3 + 4;
  // layout of part: [chunk][ci][co-quad][4 * K3 + 4]
  const int nq = (Co + 3) / 4;
  float* dst = part + (((size_t)chunk * Ci + ci) * nq + blockIdx.y) * nv;
  for (int i = threadIdx.x; i < nv; i += 256) dst[i] = red[0][i] + red[1][i] + red[2][i] + red[3][i];
}

// Second stage: dw[(ci * K3 + t) * Cop + co] and db[co] (db taken from ci = 0).
__global__ void k_conv_wgrad_sum(const float* __restrict__ part, int nchunks, int Ci, int Co,
                                 int Cop, int K3, float* __restrict__ dw, float* __restrict__ db) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nq = (Co + 3) / 4;
  const int nv = 4 * K3 + 4;
  if (i >= Ci * nq * nv) return;
  const int j = i % nv, q = (i / nv) % nq, ci = i / (nv * nq);
  float s = 0.f;
  for (int c = 0; c < nchunks; ++c) s += part[(((size_t)c * Ci + ci) * nq + q) * nv + j];
  if (j < 4 * K3) {
    const int c = j / K3, t = j % K3, co = q * 4 + c;
    if (co < Co) dw[((size_t)ci * K3 + t) * Cop + co] = s;
  } else if (ci == 0) {
    const int co = q * 4 + (j - 4 * K3);
    if (co < Co) db[co] = s;
  }
}

size_t conv_wgrad_part_floats(int N, int Ci, int Co, int D, int H, int W, int K) {
  const long total = (long)N * D * H * W;
  const long nchunks = (total + kWGChunk - 1) / kWGChunk;
  return (size_t)nchunks * Ci * ((Co + 3) / 4) * (4 * K * K * K + 4);
}

void launch_conv_wgrad(int K, const float* x, int up, const float* dy, int N, int Ci, int Co, int D,
                       int H, int W, float* part, float* dw, float* db, hipStream_t s) {
  const long total = (long)N * D * H * W;
  const int nchunks = (int)((total + kWGChunk - 1) / kWGChunk);
  const int nq = (Co + 3) / 4;
  dim3 grid(Ci, nq, nchunks);
  if (K == 3) k_conv_wgrad<3><<<grid, 256, 0, s>>>(x, up, dy, N, Ci, Co, D, H, W, part);
  else k_conv_wgrad<1><<<grid, 256, 0, s>>>(x, up, dy, N, Ci, Co, D, H, W, part);
  const int Cop = (Co + kCOB - 1) / kCOB * kCOB;
  const int K3 = K * K * K;
  k_conv_wgrad_sum<<<div_up((long)Ci * nq * (4 * K3 + 4), 256), 256, 0, s>>>(part, nchunks, Ci, Co,
                                                                             Cop, K3, dw, db);
}

// 2x2x2 mean pooling and its adjoint; nearest x2 upsampling and its adjoint.
// Grid: x over (volume nc, output plane d), y over the voxels of the plane;
// the plane and volume indices are uniform over a block.
__global__ void k_pool(const float* __restrict__ x, int D, int H, int W, float* __restrict__ y) {
  const int Do = D >> 1, Ho = H >> 1, Wo = W >> 1;
  const int j = blockIdx.y * blockDim.x + threadIdx.x;
  if (j >= Ho * Wo) return;
  const int dd = blockIdx.x % Do, nc = blockIdx.x / Do;
  const int ho = j / Wo, wo = j - ho * Wo;
  const float* b = x + ((size_t)nc * D + 2 * dd) * H * W + (size_t)(2 * ho) * W + 2 * wo;
  float s = 0.f;
  for (int a = 0; a < 8; ++a) s += b[(size_t)(a >> 2) * H * W + ((a >> 1) & 1) * W + (a & 1)];
  y[((size_t)nc * Do + dd) * Ho * Wo + j] = s * 0.125f;
}

// pool adjoint (scale 1/8) or upsampling (scale 1): y(fine) = scale * x(coarse)
__global__ void k_expand(const float* __restrict__ x, int D, int H, int W, float scale,
                         float* __restrict__ y) {
  const int j = blockIdx.y * blockDim.x + threadIdx.x;
  if (j >= H * W) return;
  const int d = blockIdx.x % D, nc = blockIdx.x / D;
  const int h = j / W, w = j - h * W;
  const int Hc = H >> 1, Wc = W >> 1;
  y[((size_t)nc * D + d) * H * W + j] =
      scale * x[(((size_t)nc * (D >> 1) + (d >> 1)) * Hc + (h >> 1)) * Wc + (w >> 1)];
}

// upsampling adjoint: y(coarse) = sum of the 8 children
__global__ void k_sum8(const float* __restrict__ x, int D, int H, int W, float* __restrict__ y) {
  const int Do = D >> 1, Ho = H >> 1, Wo = W >> 1;
  const int j = blockIdx.y * blockDim.x + threadIdx.x;
  if (j >= Ho * Wo) return;
  const int dd = blockIdx.x % Do, nc = blockIdx.x / Do;
  const int ho = j / Wo, wo = j - ho * Wo;
  const float* b = x + ((size_t)nc * D + 2 * dd) * H * W + (size_t)(2 * ho) * W + 2 * wo;
  float s = 0.f;
  for (int a = 0; a < 8; ++a) s += b[(size_t)(a >> 2) * H * W + ((a >> 1) & 1) * W + (a & 1)];
  y[((size_t)nc * Do + dd) * Ho * Wo + j] = s;
}

void launch_pool(const float* x, int NC, int D, int H, int W, float* y, hipStream_t s) {
  k_pool<<<dim3(NC * (D / 2), div_up((H / 2) * (W / 2), 256)), 256, 0, s>>>(x, D, H, W, y);
}
void launch_expand(const float* x, int NC, int D, int H, int W, float scale, float* y, hipStream_t s) {
  k_expand<<<dim3(NC * D, div_up(H * W, 256)), 256, 0, s>>>(x, D, H, W, scale, y);
}
void launch_sum8(const float* x, int NC, int D, int H, int W, float* y, hipStream_t s) {
  k_sum8<<<dim3(NC * (D / 2), div_up((H / 2) * (W / 2), 256)), 256, 0, s>>>(x, D, H, W, y);
}

// dr = dy * (r > 0) [+ extra]; extra may be NULL
__global__ void k_relu_bwd(const float* __restrict__ dy, const float* __restrict__ r,
                           const float* __restrict__ extra, long n, float* __restrict__ dr) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = (extra ? extra[i] : 0.f) + dy[i];
  dr[i] = r[i] > 0.f ? g : 0.f;
}

void launch_relu_bwd(const float* dy, const float* r, const float* extra, long n, float* dr,
                     hipStream_t s) {
  k_relu_bwd<<<div_up(n, 256), 256, 0, s>>>(dy, r, extra, n, dr);
}

__global__ void k_add(const float* __restrict__ a, const float* __restrict__ b, long n,
                      float* __restrict__ y) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a[i] + b[i];
}

void launch_add(const float* a, const float* b, long n, float* y, hipStream_t s) {
  k_add<<<div_up(n, 256), 256, 0, s>>>(a, b, n, y);
}

// Masked MSE: loss = sum m (y - t)^2 / sum m over (N, 3, DHW), m = mask[n, v]
// broadcast over the channels; dy = 2 m (y - t) / sum m.  Deterministic:
// block partials + launch_finalize.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ y, const float* __restrict__ t,
                                             const float* __restrict__ mask, int N, int C, int DHW,
                                             float* __restrict__ dy, RedWs ws) {
  const long total = (long)N * C * DHW;
  double se = 0.0, sm = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < total; i += (long)gridDim.x * 256) {
    const int v = (int)(i % DHW);
    const int n = (int)(i / ((long)C * DHW));
    const float m = mask ? mask[(size_t)n * DHW + v] : 1.f;
    const float e = y[i] - t[i];
    se += (double)m * e * e;
    sm += m;
    dy[i] = m * e;            // scaled in k_mse_scale once sum m is known
  }
  const double vv[2] = {se, sm};
  grid_sum<2>(vv, ws);
}

__global__ void k_mse_scale(float* __restrict__ dy, long n, const double* __restrict__ sums) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dy[i] = (float)(2.0 / sums[1]) * dy[i];
}

void launch_mse(const float* y, const float* t, const float* mask, int N, int C, int DHW, float* dy,
                RedWs ws, double* sums, hipStream_t s) {
  const long total = (long)N * C * DHW;
  const unsigned grid = (unsigned)std::min<long>(div_up(total, 256), 1024);
  k_mse<<<grid, 256, 0, s>>>(y, t, mask, N, C, DHW, dy, ws);
  launch_finalize(ws, grid, 2, sums, s);
  k_mse_scale<<<div_up(total, 256), 256, 0, s>>>(dy, total, sums);
}

// Adam on FP32 master weights; the compute copy is the master value rounded
// to BF16 (round to nearest even), stored as FP32.
__device__ inline float round_bf16(float v) {
  return (float)(__bf16)v;
}

__global__ void k_adam(float* __restrict__ p, float* __restrict__ pq, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, long n, float lr, float b1,
                       float b2, float eps, float c1, float c2, int quantize) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float upd = lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  const float np = p[i] - upd;
  p[i] = np;
  if (pq) pq[i] = quantize ? round_bf16(np) : np;
}

void launch_adam(float* p, float* pq, const float* g, float* m, float* v, long n, float lr, float b1,
                 float b2, float eps, int step, int quantize, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  k_adam<<<div_up(n, 256), 256, 0, s>>>(p, pq, g, m, v, n, lr, b1, b2, eps, c1, c2, quantize);
}

__global__ void k_round_bf16(const float* __restrict__ p, float* __restrict__ q, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) q[i] = round_bf16(p[i]);
}

void launch_round_bf16(const float* p, float* q, long n, hipStream_t s) {
  k_round_bf16<<<div_up(n, 256), 256, 0, s>>>(p, q, n);
}

// Network input on the padded node grid (Dp, Hp, Wp >= Nz, Ny, Nx):
// channel 0 = mean density of the elements around the node, 1..3 = load
// divided by max |f|, 4 = 1 where any DOF of the node is clamped.
__global__ void k_unet_input(Grid g, const double* __restrict__ rho, const double* __restrict__ f,
                             const uint8_t* __restrict__ fixn, const double* __restrict__ fmax,
                             int Dp, int Hp, int Wp, float* __restrict__ in) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long vol = (long)Dp * Hp * Wp;
  if (i >= vol) return;
  const int x = i % Wp, y = (i / Wp) % Hp, z = i / ((long)Wp * Hp);
  float ch[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  if (x < g.Nx && y < g.Ny && z < g.Nz) {
    double s = 0.0;
    int c = 0;
    for (int q = 0; q < 8; ++q) {
      const int ex = x - 1 + (q & 1), ey = y - 1 + ((q >> 1) & 1), ez = z - 1 + (q >> 2);
      if (ex < 0 || ey < 0 || ez < 0 || ex >= g.nx || ey >= g.ny || ez >= g.nz) continue;
      s += rho[ex + g.nx * (ey + g.ny * ez)];
      ++c;
    }
    ch[0] = (float)(c ? s / c : 0.0);
    const int node = x + g.Nx * (y + g.Ny * z);
    const double sc = *fmax > 0.0 ? 1.0 / *fmax : 0.0;
    for (int k = 0; k < 3; ++k) ch[1 + k] = (float)(f[3 * (size_t)node + k] * sc);
    ch[4] = fixn[node] ? 1.f : 0.f;
  }
  for (int k = 0; k < 5; ++k) in[k * vol + i] = ch[k];
}

__global__ void k_absmax(const double* __restrict__ a, int n, unsigned long long* __restrict__ out) {
  double m = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    m = fmax(m, fabs(a[i]));
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

__global__ void k_zero_u64(unsigned long long* p) { *p = 0ull; }

void launch_unet_input(const Grid& g, const double* rho, const double* f, const uint8_t* fixn,
                       double* fmax_scratch, int Dp, int Hp, int Wp, float* in, hipStream_t s) {
  k_zero_u64<<<1, 1, 0, s>>>((unsigned long long*)fmax_scratch);
  k_absmax<<<256, 256, 0, s>>>(f, g.n, (unsigned long long*)fmax_scratch);
  k_unet_input<<<div_up((long)Dp * Hp * Wp, 256), 256, 0, s>>>(g, rho, f, fixn, fmax_scratch, Dp,
                                                               Hp, Wp, in);
}

// Network output (3 channels on the padded grid) -> FP64 DOF vector, zero on
// clamped DOFs.
__global__ void k_unet_output(Grid g, const float* __restrict__ out, const uint8_t* __restrict__ fixn,
                              int Dp, int Hp, int Wp, double* __restrict__ u) {
  const int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= g.Nn) return;
  const int x = node % g.Nx, y = (node / g.Nx) % g.Ny, z = node / (g.Nx * g.Ny);
  const long vol = (long)Dp * Hp * Wp;
  const long v = ((long)z * Hp + y) * Wp + x;
  const unsigned fx = fixn[node];
  for (int k = 0; k < 3; ++k)
    u[3 * (size_t)node + k] = (fx >> k) & 1u ? 0.0 : (double)out[k * vol + v];
}

void launch_unet_output(const Grid& g, const float* out, const uint8_t* fixn, int Dp, int Hp, int Wp,
                        double* u, hipStream_t s) {
  k_unet_output<<<div_up(g.Nn, 256), 256, 0, s>>>(g, out, fixn, Dp, Hp, Wp, u);
}

// Training target: u / max|u| on the padded grid (3 channels) and a mask that
// is 1 on the nodes of the mesh.
__global__ void k_unet_target(Grid g, const double* __restrict__ u, const double* __restrict__ umax,
                              int Dp, int Hp, int Wp, float* __restrict__ t, float* __restrict__ m) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long vol = (long)Dp * Hp * Wp;
  if (i >= vol) return;
  const int x = i % Wp, y = (i / Wp) % Hp, z = i / ((long)Wp * Hp);
  const bool in = x < g.Nx && y < g.Ny && z < g.Nz;
  const double sc = *umax > 0.0 ? 1.0 / *umax : 0.0;
  const size_t node = in ? (size_t)(x + g.Nx * (y + g.Ny * z)) : 0;
  for (int k = 0; k < 3; ++k) t[k * vol + i] = in ? (float)(u[3 * node + k] * sc) : 0.f;
  if (m) m[i] = in ? 1.f : 0.f;
}

void launch_unet_target(const Grid& g, const double* u, double* umax_scratch, int Dp, int Hp, int Wp,
                        float* t, float* m, hipStream_t s) {
  k_zero_u64<<<1, 1, 0, s>>>((unsigned long long*)umax_scratch);
  k_absmax<<<256, 256, 0, s>>>(u, g.n, (unsigned long long*)umax_scratch);
  k_unet_target<<<div_up((long)Dp * Hp * Wp, 256), 256, 0, s>>>(g, u, umax_scratch, Dp, Hp, Wp, t, m);
}

// ---------------------------------------------------------------------------
// Energy-norm training score of the network's displacement shapes.  Sample
// n's output channels on the node voxels give u (zero on clamped DOFs); with
// a = f.u, b = u.K u and the compliance c = f.u* the best multiple (a / b) u
// leaves the squared energy-norm error c - a^2 / b, so the score
// 1 - a^2 / (b c) is 0 for the exact shape and 1 for u = 0.  The batch loss is
// the mean score; its output gradient is -(2 a / (b c N)) (f - (a / b) K u) on
// free DOFs.
__global__ void k_energy_u(EnergyBatch e, const float* __restrict__ y) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const Grid& g = e.g;
  if (i >= (long)e.N * g.Nn) return;
  const int n = (int)(i / g.Nn), node = (int)(i % g.Nn);
  const int x = node % g.Nx, yy = (node / g.Nx) % g.Ny, z = node / (g.Nx * g.Ny);
  const long vol = (long)e.Dp * e.Hp * e.Wp;
  const long v = ((long)z * e.Hp + yy) * e.Wp + x;
  const unsigned fx = e.fixn[node];
  double* u = e.u + (size_t)n * g.n + 3 * (size_t)node;
#pragma unroll
  for (int c = 0; c < 3; ++c)
    u[c] = (fx >> c) & 1u ? 0.0 : (double)y[((size_t)n * 3 + c) * vol + v];
}

__global__ __launch_bounds__(256) void k_energy_Ku(EnergyBatch e) {
  __shared__ double lds[32];
  const Grid& g = e.g;
  const int n = blockIdx.y;
  const int node = blockIdx.x * 256 + threadIdx.x;
  double a = 0.0, b = 0.0;
  if (node < g.Nn) {
    const size_t off = (size_t)n * g.n, base = off + 3 * (size_t)node;
    double acc[3], xo[3];
    fine_node_Ku<double>(g, e.E + (size_t)n * g.nel, e.ke, e.u + off, node, acc, xo);
    const unsigned fx = e.fixn[node];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double kv = (fx >> c) & 1u ? 0.0 : acc[c];
      e.Ku[base + c] = kv;
      a += e.f[base + c] * xo[c];
      b += xo[c] * kv;
    }
  }
  a = block_sum(a, lds);
  b = block_sum(b, lds + 16);
  if (threadIdx.x == 0) {
    double* p = e.part + ((size_t)n * e.nb + blockIdx.x) * 2;
    p[0] = a;
    p[1] = b;
  }
}

// one block per sample: the block partials in a fixed order, then the score
// and the gradient factors (score 1 and the gradient -f / (c N) when u.K u is
// not positive)
__global__ __launch_bounds__(256) void k_energy_final(EnergyBatch e) {
  __shared__ double lds[32];
  const int n = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < e.nb; i += 256) {
    a += e.part[((size_t)n * e.nb + i) * 2];
    b += e.part[((size_t)n * e.nb + i) * 2 + 1];
  }
  a = block_sum(a, lds);
  b = block_sum(b, lds + 16);
  if (threadIdx.x != 0) return;
  const double c = e.cstar[n];
  double* sc = e.scal + 4 * (size_t)n;
  if (b > 0.0 && c > 0.0 && isfinite(a) && isfinite(b)) {
    sc[0] = 1.0 - a * a / (b * c);
    sc[1] = -2.0 * a / (b * c * e.N);
    sc[2] = a / b;
  } else {
    sc[0] = 1.0;
    sc[1] = c > 0.0 ? -1.0 / (c * e.N) : 0.0;
    sc[2] = 0.0;
  }
  sc[3] = 0.0;
}

__global__ void k_energy_grad(EnergyBatch e, float* __restrict__ gy) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long vol = (long)e.Dp * e.Hp * e.Wp;
  if (i >= (long)e.N * 3 * vol) return;
  const Grid& g = e.g;
  const int n = (int)(i / (3 * vol)), c = (int)((i / vol) % 3);
  const long v = i % vol;
  const int x = (int)(v % e.Wp), yy = (int)((v / e.Wp) % e.Hp), z = (int)(v / ((long)e.Wp * e.Hp));
  double val = 0.0;
  if (x < g.Nx && yy < g.Ny && z < g.Nz) {
    const int node = x + g.Nx * (yy + g.Ny * z);
    if (!((e.fixn[node] >> c) & 1u)) {
      const size_t d = (size_t)n * g.n + 3 * (size_t)node + c;
      const double* sc = e.scal + 4 * (size_t)n;
      val = sc[1] * (e.f[d] - sc[2] * e.Ku[d]);
    }
  }
  gy[i] = (float)val;
}

void launch_energy_loss(const EnergyBatch& e, const float* y, float* gy, hipStream_t s) {
  k_energy_u<<<div_up((long)e.N * e.g.Nn, 256), 256, 0, s>>>(e, y);
  k_energy_Ku<<<dim3(e.nb, e.N), 256, 0, s>>>(e);
  k_energy_final<<<e.N, 256, 0, s>>>(e);
  k_energy_grad<<<div_up((long)e.N * 3 * e.Dp * e.Hp * e.Wp, 256), 256, 0, s>>>(e, gy);
}

// x0 = alpha u0 with alpha = (f . u0) / (u0 . K u0) (sums[0], sums[1]).
__global__ void k_scale_by_ratio(double* __restrict__ u, int n, const double* __restrict__ num,
                                 const double* __restrict__ den, double* __restrict__ alpha_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const double a = *den > 0.0 ? *num / *den : 0.0;
  if (i == 0 && alpha_out) *alpha_out = a;
  if (i < n) u[i] *= a;
}

void launch_scale_by_ratio(double* u, int n, const double* num, const double* den, double* alpha,
                           hipStream_t s) {
  k_scale_by_ratio<<<div_up(n, 256), 256, 0, s>>>(u, n, num, den, alpha);
}

}  // namespace sgmg
