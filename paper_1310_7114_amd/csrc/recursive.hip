// Maps for large kernel widths by recursive filtering (Section 3.1: for large
// widths the finite masks give way to recursive filters; the paper cites
// Deriche and van Vliet). The filter is Young and van Vliet's third-order
// recursive Gaussian: along a line, a causal pass
//   w[n] = B x[n] + a1 w[n-1] + a2 w[n-2] + a3 w[n-3]
// then an anticausal pass y[n] = B w[n] + a1 y[n+1] + a2 y[n+2] + a3 y[n+3],
// with B, a1..a3 from sigma (host side) and unit DC gain; the output is
// scaled by sqrt(2 pi) sigma to the mass of the sampled unnormalised Gaussian.
// Its cost per pixel does not depend on sigma. Every line is the lattice line
// grown by one zero pixel at each end plus m = ceil(6 sigma) zeros after it,
// so the causal response has decayed before the anticausal pass starts.
// A is filtered along v, then along u, on the lattice grown by a one-pixel
// ring; M = -sigma^2 grad A by central differences (exact for a Gaussian
// kernel: sum_y h(y) (x - y) g(x - y) = -sigma^2 d/dx sum_y h(y) g(x - y)).
//
// Both passes run down columns (one lane per column, coalesced rows), so the
// image is first transposed into an FP64 buffer E1 (rows = v), filtered,
// transposed into E2 (rows = u), filtered, and the maps and S_X partials are
// read off E2. The recursions run in FP64.
#include "itc_device.h"

namespace itc {

namespace {

constexpr int RT = 32;  // transpose tile

// E1[r][c] = h(u = c - 1, v = r - 1) on the grown lattice, zero elsewhere.
template <typename WT>
__global__ void __launch_bounds__(RT * 8) rec_load_kernel(const WT* __restrict__ x, int64_t pitch, double scale,
                                                          int H, int W, double* __restrict__ E1, int64_t p1,
                                                          int rows1) {
  __shared__ double tile[RT][RT + 1];
  const int r0 = blockIdx.y * RT, c0 = blockIdx.x * RT;  // E1 tile: rows r0.., cols c0..
  const int tx = threadIdx.x & (RT - 1), ty = threadIdx.x / RT;
  // read along v (E1 rows) for fixed u (E1 column): contiguous in x
  for (int k = ty; k < RT; k += 8) {
    const int u = c0 + k - 1, v = r0 + tx - 1;
    double val = 0.0;
    if (u >= 0 && u < H && v >= 0 && v < W) val = scale * (double)x[(int64_t)u * pitch + v];
    tile[k][tx] = val;  // tile[u][v]
  }
  __syncthreads();
  for (int k = ty; k < RT; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    if (r < rows1 && c < H + 2) E1[(int64_t)r * p1 + c] = tile[tx][k];
  }
}

// E2[r][c] = E1[c][r] for r < H + 2 (rows = u, cols = v), zero in the margin rows.
__global__ void __launch_bounds__(RT * 8) rec_transpose_kernel(const double* __restrict__ E1, int64_t p1, int H,
                                                               int W, double* __restrict__ E2, int64_t p2,
                                                               int rows2) {
  __shared__ double tile[RT][RT + 1];
  const int r0 = blockIdx.y * RT, c0 = blockIdx.x * RT;  // E2 tile
  const int tx = threadIdx.x & (RT - 1), ty = threadIdx.x / RT;
  for (int k = ty; k < RT; k += 8) {
    const int v = c0 + k, u = r0 + tx;  // E1 row v, column u
    tile[k][tx] = (v < W + 2 && u < H + 2) ? E1[(int64_t)v * p1 + u] : 0.0;
  }
  __syncthreads();
  for (int k = ty; k < RT; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    if (r < rows2 && c < W + 2) E2[(int64_t)r * p2 + c] = tile[tx][k];
  }
}

// Causal then anticausal pass down every column of E (rows x cols), in place.
constexpr int RB = 8;

__global__ void __launch_bounds__(64) rec_filter_kernel(double* __restrict__ E, int64_t p, int rows, int cols,
                                                        double B, double a1, double a2, double a3, double gain) {
  const int c = blockIdx.x * 64 + threadIdx.x;
  if (c >= cols) return;
  double* col = E + c;
  double w1 = 0.0, w2 = 0.0, w3 = 0.0;
  for (int r0 = 0; r0 < rows; r0 += RB) {
    double v[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) v[k] = r0 + k < rows ? col[(int64_t)(r0 + k) * p] : 0.0;
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      const double w = B * v[k] + a1 * w1 + a2 * w2 + a3 * w3;
      w3 = w2;
      w2 = w1;
      w1 = w;
      v[k] = w;
    }
#pragma unroll
    for (int k = 0; k < RB; ++k)
      if (r0 + k < rows) col[(int64_t)(r0 + k) * p] = v[k];
  }
  double y1 = 0.0, y2 = 0.0, y3 = 0.0;
  for (int r1 = rows - 1; r1 >= 0; r1 -= RB) {
    double v[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) v[k] = r1 - k >= 0 ? col[(int64_t)(r1 - k) * p] : 0.0;
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      const double y = B * v[k] + a1 * y1 + a2 * y2 + a3 * y3;
      y3 = y2;
      y2 = y1;
      y1 = y;
      v[k] = y * gain;
    }
#pragma unroll
    for (int k = 0; k < RB; ++k)
      if (r1 - k >= 0) col[(int64_t)(r1 - k) * p] = v[k];
  }
}

// Maps (FP32 planes, map pitch) and S_X partials from the filtered E2:
// thread = (8-row group, map column).
template <typename WT>
__global__ void __launch_bounds__(64) rec_maps_kernel(const double* __restrict__ E2, int64_t p2, const WT* x,
                                                      int64_t pitch, double scale, double sigma, ImageDesc im,
                                                      char* maps) {
  const int v = blockIdx.x * 64 + threadIdx.x;  // map column (< map_pitch)
  const int grp = blockIdx.y;
  const int64_t plane = (int64_t)im.H * im.map_pitch;
  float* A = reinterpret_cast<float*>(maps);
  float* Mu = A + plane;
  float* Mv = Mu + plane;
  const double k = -0.5 * sigma * sigma;
  double sx = 0.0;
  for (int i = 0; i < CONV_GROUP; ++i) {
    const int u = grp * CONV_GROUP + i;
    if (u >= im.H) break;
    float a = 0.f, mu = 0.f, mv = 0.f;
    if (v < im.W) {
      const double* e = E2 + (int64_t)(u + 1) * p2 + (v + 1);
      const double ac = e[0];
      a = (float)ac;
      mu = (float)(k * (e[p2] - e[-p2]));
      mv = (float)(k * (e[1] - e[-1]));
      sx = fma(scale * (double)x[(int64_t)u * pitch + v], (double)a, sx);
    }
    const int64_t o = (int64_t)u * im.map_pitch + v;
    A[o] = a;
    Mu[o] = mu;
    Mv[o] = mv;
  }
  float* part = reinterpret_cast<float*>(maps + im.part_off);
  part[((int64_t)(v / CONV_TW) * im.ngroups + grp) * CONV_TW + (v % CONV_TW)] = (float)sx;
}

template <typename WT>
hipError_t launch_recursive_t(const ImageDesc& im, const void* x, double scale, double sigma, const RecCoeffs& rc,
                              double* E1, double* E2, void* maps, hipStream_t s) {
  const int H = im.H, W = im.W;
  const int rows1 = W + 2 + rc.m, cols1 = H + 2;
  const int rows2 = H + 2 + rc.m, cols2 = W + 2;
  const int64_t p1 = cols1, p2 = cols2;
  hipLaunchKernelGGL(rec_load_kernel<WT>, dim3((cols1 + RT - 1) / RT, (rows1 + RT - 1) / RT), dim3(RT * 8), 0, s,
                     (const WT*)x, im.pitch, scale, H, W, E1, p1, rows1);
  hipLaunchKernelGGL(rec_filter_kernel, dim3((cols1 + 63) / 64), dim3(64), 0, s, E1, p1, rows1, cols1, rc.B, rc.a1,
                     rc.a2, rc.a3, rc.gain);
  hipLaunchKernelGGL(rec_transpose_kernel, dim3((cols2 + RT - 1) / RT, (rows2 + RT - 1) / RT), dim3(RT * 8), 0, s,
                     (const double*)E1, p1, H, W, E2, p2, rows2);
  hipLaunchKernelGGL(rec_filter_kernel, dim3((cols2 + 63) / 64), dim3(64), 0, s, E2, p2, rows2, cols2, rc.B, rc.a1,
                     rc.a2, rc.a3, rc.gain);
  hipLaunchKernelGGL(rec_maps_kernel<WT>, dim3((unsigned)(im.map_pitch / 64), (unsigned)im.ngroups), dim3(64), 0,
                     s, (const double*)E2, p2, (const WT*)x, im.pitch, scale, sigma, im, (char*)maps);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_recursive(const ImageDesc& im, const void* x, double scale, double sigma, const RecCoeffs& rc,
                            double* E1, double* E2, void* maps, hipStream_t s) {
  switch (im.wdtype) {
    case 0: return launch_recursive_t<uint8_t>(im, x, scale, sigma, rc, E1, E2, maps, s);
    case 1: return launch_recursive_t<float>(im, x, scale, sigma, rc, E1, E2, maps, s);
    default: return launch_recursive_t<double>(im, x, scale, sigma, rc, E1, E2, maps, s);
  }
}

}  // namespace itc
