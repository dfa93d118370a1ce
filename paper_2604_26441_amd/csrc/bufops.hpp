// Device helpers shared by the fine-level kernels: raw buffer loads and
// stores with out-of-range offsets reading zeros, and lane moves.
#pragma once
#include <climits>

#include "common.hpp"

namespace sgmg {

// Raw buffer loads: an offset past the buffer's byte size returns zeros, so
// halo and out-of-mesh operands need no branch (straight-line code keeps the
// compiler's load-counter waits exact across the software pipeline).  Offsets
// are 32-bit: the launcher rejects vectors of 2^31 bytes or more, and
// kNoOffset (2^31) is past every buffer.
constexpr int kNoOffset = INT_MIN;
// Poison part of a two-part offset (the kernels that use it take vectors
// below 2^30 bytes).
constexpr int kPoison = 1 << 30;
__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* p, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ inline float bload(__amdgpu_buffer_rsrc_t r, int off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ inline void bload3(__amdgpu_buffer_rsrc_t r, int off, float* v) {
  const auto t = __builtin_amdgcn_raw_buffer_load_b96(r, off, 0, 0);
  // (__builtin_bit_cast on an element of the returned vector loses elements)
  v[0] = __uint_as_float(t[0]);
  v[1] = __uint_as_float(t[1]);
  v[2] = __uint_as_float(t[2]);
}

__device__ inline void bload3(__amdgpu_buffer_rsrc_t r, int off, double* v) {
  const auto t = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
  const auto w = __builtin_amdgcn_raw_buffer_load_b64(r, off == kNoOffset ? kNoOffset : off + 16, 0, 0);
  v[0] = __hiloint2double((int)t[1], (int)t[0]);
  v[1] = __hiloint2double((int)t[3], (int)t[2]);
  v[2] = __hiloint2double((int)w[1], (int)w[0]);
}

// Kernel-internal epilogue variants: EPI_STORE plus the x.y dot product;
// EPI_SMOOTH with the FP64 copy of x_out plus the dot of that copy with the
// FP64 vector ep.dot64 (the cycle's last step and the PCG's r.z in one pass).
constexpr int kStoreDot = 3;
constexpr int kSmoothDot = 4;

__device__ inline void bstore3(__amdgpu_buffer_rsrc_t r, int off, float a, float b, float c) {
  typedef unsigned u32x3 __attribute__((ext_vector_type(3)));
  const u32x3 v = {__float_as_uint(a), __float_as_uint(b), __float_as_uint(c)};
  __builtin_amdgcn_raw_buffer_store_b96(v, r, off, 0, 0);
}

__device__ inline void bstore3(__amdgpu_buffer_rsrc_t r, int off, double a, double b, double c) {
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
  const u32x4 v = {(unsigned)__double2loint(a), (unsigned)__double2hiint(a),
                   (unsigned)__double2loint(b), (unsigned)__double2hiint(b)};
  const u32x2 w = {(unsigned)__double2loint(c), (unsigned)__double2hiint(c)};
  __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, 0);
  __builtin_amdgcn_raw_buffer_store_b64(w, r, off == kNoOffset ? kNoOffset : off + 16, 0, 0);
}

__device__ inline float dpp_shr1(float v) {   // lane n-1 of the same 16-lane row (0 for n = 0)
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x111, 0xf, 0xf, true));
}

__device__ inline double dpp_shr1(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x111, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x111, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

__device__ inline double bpermute(int addr, double v) {
  const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

__device__ inline double bload1d(__amdgpu_buffer_rsrc_t r, int off) {
  const auto t = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
  return __hiloint2double((int)t[1], (int)t[0]);
}

}  // namespace sgmg
