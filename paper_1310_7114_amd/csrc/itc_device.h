// Device helpers for the lattice ITC kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "itc_internal.h"

namespace itc {

// A lattice position (u = row, v = column).
template <typename T>
struct V2 {
  T u, v;
};

// Scalar-register copy of a wave-uniform value.
__device__ __forceinline__ float to_sgpr(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}
__device__ __forceinline__ double to_sgpr(double x) {
  int2 v = __builtin_bit_cast(int2, x);
  v.x = __builtin_amdgcn_readfirstlane(v.x);
  v.y = __builtin_amdgcn_readfirstlane(v.y);
  return __builtin_bit_cast(double, v);
}
// Value of lane `l` (compile-time after unrolling) of a per-lane value, as a scalar.
__device__ __forceinline__ float lane_value(float x, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
}
__device__ __forceinline__ double lane_value(double x, int l) {
  int2 v = __builtin_bit_cast(int2, x);
  v.x = __builtin_amdgcn_readlane(v.x, l);
  v.y = __builtin_amdgcn_readlane(v.y, l);
  return __builtin_bit_cast(double, v);
}

// f(integral_constant<int, I>) for I = 0, 1, ... in order (compile-time indices
// for register arrays in unrolled loops)
template <typename F, int... I>
__device__ __forceinline__ void for_each_index(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Cross-lane moves through DPP (data-parallel primitives of the VALU): no LDS
// round trip, so a whole-wave reduction costs a few VALU latencies. Lanes of
// rows that ROWS leaves out are not written and hold undefined values: the
// reductions below read their result from lanes that every step writes.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ double dpp_f64(double x) {
  int2 v = __builtin_bit_cast(int2, x);
  v.x = __builtin_amdgcn_mov_dpp(v.x, CTRL, ROWS, 0xf, false);
  v.y = __builtin_amdgcn_mov_dpp(v.y, CTRL, ROWS, 0xf, false);
  return __builtin_bit_cast(double, v);
}
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ float dpp_f32(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, ROWS, 0xf, false));
}
// DPP controls: quad_perm [1,0,3,2] and [2,3,0,1], row_half_mirror,
// row_mirror, row_bcast:15 (into rows 1 and 3), row_bcast:31 (into rows 2, 3).
constexpr int DPP_QP_1032 = 0xb1, DPP_QP_2301 = 0x4e, DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140,
              DPP_BCAST15 = 0x142, DPP_BCAST31 = 0x143;

// Sum over the 64 lanes of a wave in a fixed order; every lane gets it.
__device__ __forceinline__ double wave_sum(double x) {
  x += dpp_f64<DPP_QP_1032>(x);
  x += dpp_f64<DPP_QP_2301>(x);
  x += dpp_f64<DPP_HALF_MIRROR>(x);
  x += dpp_f64<DPP_MIRROR>(x);
  x += dpp_f64<DPP_BCAST15, 0xa>(x);
  x += dpp_f64<DPP_BCAST31, 0xc>(x);
  return lane_value(x, 63);
}
// Two independent wave sums in the same order as wave_sum, interleaved so
// that each step's cross-lane moves of one overlap the other's addition.
__device__ __forceinline__ void wave_sum2(double& a, double& b) {
  a += dpp_f64<DPP_QP_1032>(a);
  b += dpp_f64<DPP_QP_1032>(b);
  a += dpp_f64<DPP_QP_2301>(a);
  b += dpp_f64<DPP_QP_2301>(b);
  a += dpp_f64<DPP_HALF_MIRROR>(a);
  b += dpp_f64<DPP_HALF_MIRROR>(b);
  a += dpp_f64<DPP_MIRROR>(a);
  b += dpp_f64<DPP_MIRROR>(b);
  a += dpp_f64<DPP_BCAST15, 0xa>(a);
  b += dpp_f64<DPP_BCAST15, 0xa>(b);
  a += dpp_f64<DPP_BCAST31, 0xc>(a);
  b += dpp_f64<DPP_BCAST31, 0xc>(b);
  a = lane_value(a, 63);
  b = lane_value(b, 63);
}
// Sum over aligned groups of P lanes (P a power of two); every lane of a group
// gets the same value (each step adds a commutative pair).
template <int P>
__device__ __forceinline__ float group_sum(float x) {
  if constexpr (P >= 2) x += dpp_f32<DPP_QP_1032>(x);
  if constexpr (P >= 4) x += dpp_f32<DPP_QP_2301>(x);
  if constexpr (P >= 8) x += dpp_f32<DPP_HALF_MIRROR>(x);
  if constexpr (P >= 16) x += dpp_f32<DPP_MIRROR>(x);
  if constexpr (P >= 32) x += __shfl_xor(x, 16, 64);
  if constexpr (P >= 64) x += __shfl_xor(x, 32, 64);
  return x;
}
template <int P>
__device__ __forceinline__ double group_sum(double x) {
  if constexpr (P >= 2) x += dpp_f64<DPP_QP_1032>(x);
  if constexpr (P >= 4) x += dpp_f64<DPP_QP_2301>(x);
  if constexpr (P >= 8) x += dpp_f64<DPP_HALF_MIRROR>(x);
  if constexpr (P >= 16) x += dpp_f64<DPP_MIRROR>(x);
  if constexpr (P >= 32) x += __shfl_xor(x, 16, 64);
  if constexpr (P >= 64) x += __shfl_xor(x, 32, 64);
  return x;
}

// Min over the 64 lanes of a wave (NaN lanes are ignored unless all are NaN);
// every lane gets it.
__device__ __forceinline__ double wave_min(double x) {
  x = fmin(x, dpp_f64<DPP_QP_1032>(x));
  x = fmin(x, dpp_f64<DPP_QP_2301>(x));
  x = fmin(x, dpp_f64<DPP_HALF_MIRROR>(x));
  x = fmin(x, dpp_f64<DPP_MIRROR>(x));
  x = fmin(x, dpp_f64<DPP_BCAST15, 0xa>(x));
  x = fmin(x, dpp_f64<DPP_BCAST31, 0xc>(x));
  return lane_value(x, 63);
}

// Max over the 64 lanes of a wave of non-negative values; every lane gets it.
__device__ __forceinline__ float wave_max_nonneg(float x) {
  x = fmaxf(x, dpp_f32<DPP_QP_1032>(x));
  x = fmaxf(x, dpp_f32<DPP_QP_2301>(x));
  x = fmaxf(x, dpp_f32<DPP_HALF_MIRROR>(x));
  x = fmaxf(x, dpp_f32<DPP_MIRROR>(x));
  x = fmaxf(x, dpp_f32<DPP_BCAST15, 0xa>(x));
  x = fmaxf(x, dpp_f32<DPP_BCAST31, 0xc>(x));
  return lane_value(x, 63);
}

// ---------------------------------------------------------------------------
// Buffer access: a uniform base in a resource descriptor, a per-lane 32-bit
// byte offset and a uniform 32-bit byte offset (scalar register). The
// descriptor holds the buffer's size: a load at a per-lane offset of BUF_OOB
// (past any buffer this library addresses, and the scalar offsets added to it
// stay below 2^31) returns 0 without a memory request, and a store there is
// dropped. Kernels use such offsets for the lanes that must not access memory,
// instead of branches, so that loads stay in flight across the code that
// follows; every other access stays inside the buffer.
// ---------------------------------------------------------------------------
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr uint32_t BUF_OOB = 0x80000000u;

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

template <typename WT>
__device__ __forceinline__ WT buf_load(rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(WT) == 1) {
    return (WT)__builtin_amdgcn_raw_buffer_load_b8(r, voff, soff, 0);
  } else if constexpr (sizeof(WT) == 4) {
    return __builtin_bit_cast(WT, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  } else {
    return __builtin_bit_cast(WT, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  }
}

template <typename T>
__device__ __forceinline__ void buf_store(T v, rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) uint32_t, v),
                                          r, voff, soff, 0);
}

// Deterministic FP64 sum of n values by one workgroup of nt threads (nt a
// multiple of 64): thread t adds t, t+nt, ...; then each wave by a fixed xor
// tree; then the waves in order. `red` is shared scratch of nt/64 doubles.
// Every thread gets the total.
// The workgroup total of one FP64 value per thread: each wave by a fixed xor
// tree, then the waves in order. Every thread gets the total.
__device__ inline double block_reduce_fixed(double s, double* red) {
  const int nt = blockDim.x, tid = threadIdx.x;
  s = wave_sum(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < nt / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}

template <typename P>
__device__ inline double block_sum_fixed(const P* p, int64_t n, double* red) {
  const int nt = blockDim.x, tid = threadIdx.x;
  double s = 0.0;
  for (int64_t i = tid; i < n; i += nt) s += (double)p[i];
  return block_reduce_fixed(s, red);
}

}  // namespace itc
