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

// Stored weight of pixel (y, x) times the scale, in double; 0 off the lattice.
__device__ __forceinline__ double load_weight(const char* base, int wdtype, int64_t pitch, int H,
                                              int W, int y, int x, double scale) {
  if (y < 0 || y >= H || x < 0 || x >= W) return 0.0;
  const int64_t i = (int64_t)y * pitch + x;
  double v;
  if (wdtype == 0)
    v = (double)((const uint8_t*)base)[i];
  else if (wdtype == 1)
    v = (double)((const float*)base)[i];
  else
    v = ((const double*)base)[i];
  return v * scale;
}

// Deterministic sum of n doubles by one workgroup of nt threads (nt a
// multiple of 64): thread t adds t, t+nt, ...; then waves, then wave 0.
// `red` is shared scratch of nt/64 doubles. Every thread gets the total.
__device__ inline double block_sum_fixed(const double* p, int n, double* red) {
  const int nt = blockDim.x, tid = threadIdx.x;
  double s = 0.0;
  for (int i = tid; i < n; i += nt) s += p[i];
  s = wave_sum(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < nt / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}

}  // namespace itc
