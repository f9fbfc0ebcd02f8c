// Device helpers for the lattice ITC kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "itc_internal.h"

namespace itc {

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

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Sum over the 64 lanes of a wave by a fixed xor tree (same order every call).
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
  return x;
}
__device__ __forceinline__ float wave_max(float x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x = fmaxf(x, __shfl_xor(x, m, 64));
  return x;
}

// ---------------------------------------------------------------------------
// Buffer access: a uniform base in a resource descriptor, a per-lane 32-bit
// byte offset and a uniform 32-bit byte offset (scalar register). Callers keep
// every access inside [base, base + bytes); the hardware range check is not
// relied on.
// ---------------------------------------------------------------------------
using rsrc_t = __amdgpu_buffer_rsrc_t;

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
template <typename P>
__device__ inline double block_sum_fixed(const P* p, int64_t n, double* red) {
  const int nt = blockDim.x, tid = threadIdx.x;
  double s = 0.0;
  for (int64_t i = tid; i < n; i += nt) s += (double)p[i];
  s = wave_sum(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < nt / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}

}  // namespace itc
