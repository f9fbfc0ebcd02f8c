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
// Both passes run down columns (lanes along columns, coalesced rows), so the
// image is first transposed into an FP64 buffer E1 (rows = v), filtered,
// transposed into E2 (rows = u), filtered, and the maps and S_X partials are
// read off E2. The recursions run in FP64, segment-parallel along the lines.
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

// The recursions run down columns of E (rows x cols, one lane per column),
// split into segments of REC_SEG rows so that every segment of every column
// has a lane. With the state z = (w[n-1], w[n-2], w[n-3]) the recursion is
// linear, z' = A z + B x e1 with the companion matrix A of (a1, a2, a3), so
// the state after a segment is A^REC_SEG z_start plus the state the segment
// reaches from zero. Per direction: every segment's zero-state end, a scan
// over the segments of each column for the true start states, and a rerun of
// every segment from its start state that writes the values.
constexpr int RB = 8;

// Recursion over rows [lo, hi) of one column, ascending (dir > 0) or
// descending, from and into (z1, z2, z3); with OUT the values times `gain`
// replace the inputs.
template <bool OUT>
__device__ __forceinline__ void rec_run(double* col, int64_t p, int lo, int hi, int dir, const RecCoeffs& rc,
                                        double gain, double& z1, double& z2, double& z3) {
  const int n = hi - lo;
  for (int k0 = 0; k0 < n; k0 += RB) {
    double v[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      const int r = dir > 0 ? lo + k0 + k : hi - 1 - k0 - k;
      v[k] = k0 + k < n ? col[(int64_t)r * p] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      if (k0 + k < n) {  // uniform: every lane runs the same segment
        const double w = fma(rc.a1, z1, fma(rc.a2, z2, fma(rc.a3, z3, rc.B * v[k])));
        z3 = z2;
        z2 = z1;
        z1 = w;
        v[k] = w * gain;
      }
    }
    if (OUT) {
#pragma unroll
      for (int k = 0; k < RB; ++k) {
        const int r = dir > 0 ? lo + k0 + k : hi - 1 - k0 - k;
        if (k0 + k < n) col[(int64_t)r * p] = v[k];
      }
    }
  }
}

// Z layout: [segment][3][cols].
__device__ __forceinline__ double* zat(double* Z, int sg, int q, int cols, int c) {
  return Z + ((int64_t)sg * 3 + q) * cols + c;
}

// Zero-state end of every segment along dir (blockIdx.y = segment).
__global__ void __launch_bounds__(64) rec_seg_end_kernel(double* __restrict__ E, int64_t p, int rows, int cols,
                                                         RecCoeffs rc, int dir, double* __restrict__ Z) {
  const int c = blockIdx.x * 64 + threadIdx.x, sg = blockIdx.y;
  if (c >= cols) return;
  const int lo = sg * REC_SEG, hi = min(lo + REC_SEG, rows);
  double z1 = 0.0, z2 = 0.0, z3 = 0.0;
  rec_run<false>(E + c, p, lo, hi, dir, rc, 1.0, z1, z2, z3);
  *zat(Z, sg, 0, cols, c) = z1;
  *zat(Z, sg, 1, cols, c) = z2;
  *zat(Z, sg, 2, cols, c) = z3;
}

// Start states from the zero-state ends, in place: segments in the order of
// dir, z_start(first) = 0, z_start(next) = A^REC_SEG z_start + z_end0. Only
// the segment last in that order can be shorter, and its end is not carried.
__global__ void __launch_bounds__(64) rec_seg_scan_kernel(double* __restrict__ Z, int nseg, int cols, RecCoeffs rc,
                                                          int dir) {
  const int c = blockIdx.x * 64 + threadIdx.x;
  if (c >= cols) return;
  const double* P = rc.P;
  double z1 = 0.0, z2 = 0.0, z3 = 0.0;
  constexpr int SB = 8;  // segments whose ends are loaded together
  for (int i0 = 0; i0 < nseg; i0 += SB) {
    double f[SB][3];
#pragma unroll
    for (int q = 0; q < SB; ++q) {
      const int i = i0 + q;
      const int sg = dir > 0 ? i : nseg - 1 - i;
      f[q][0] = f[q][1] = f[q][2] = 0.0;
      if (i < nseg) {
        f[q][0] = *zat(Z, sg, 0, cols, c);
        f[q][1] = *zat(Z, sg, 1, cols, c);
        f[q][2] = *zat(Z, sg, 2, cols, c);
      }
    }
#pragma unroll
    for (int q = 0; q < SB; ++q) {
      const int i = i0 + q;
      if (i >= nseg) break;
      const int sg = dir > 0 ? i : nseg - 1 - i;
      *zat(Z, sg, 0, cols, c) = z1;
      *zat(Z, sg, 1, cols, c) = z2;
      *zat(Z, sg, 2, cols, c) = z3;
      const double n1 = fma(P[0], z1, fma(P[1], z2, fma(P[2], z3, f[q][0])));
      const double n2 = fma(P[3], z1, fma(P[4], z2, fma(P[5], z3, f[q][1])));
      const double n3 = fma(P[6], z1, fma(P[7], z2, fma(P[8], z3, f[q][2])));
      z1 = n1;
      z2 = n2;
      z3 = n3;
    }
  }
}

// Rerun of every segment from its start state. Causal (dir > 0): writes w,
// then leaves in Z the zero-state end of the anticausal pass over the same
// rows (this lane's own values, just written). Anticausal: writes y * gain.
__global__ void __launch_bounds__(64) rec_seg_apply_kernel(double* __restrict__ E, int64_t p, int rows, int cols,
                                                           RecCoeffs rc, int dir, double* __restrict__ Z) {
  const int c = blockIdx.x * 64 + threadIdx.x, sg = blockIdx.y;
  if (c >= cols) return;
  const int lo = sg * REC_SEG, hi = min(lo + REC_SEG, rows);
  double z1 = *zat(Z, sg, 0, cols, c), z2 = *zat(Z, sg, 1, cols, c), z3 = *zat(Z, sg, 2, cols, c);
  if (dir > 0) {
    rec_run<true>(E + c, p, lo, hi, 1, rc, 1.0, z1, z2, z3);
    z1 = z2 = z3 = 0.0;
    rec_run<false>(E + c, p, lo, hi, -1, rc, 1.0, z1, z2, z3);
    *zat(Z, sg, 0, cols, c) = z1;
    *zat(Z, sg, 1, cols, c) = z2;
    *zat(Z, sg, 2, cols, c) = z3;
  } else {
    rec_run<true>(E + c, p, lo, hi, -1, rc, rc.gain, z1, z2, z3);
  }
}

// Causal then anticausal pass down every column of E, in place.
void rec_filter(double* E, int64_t p, int rows, int cols, const RecCoeffs& rc, double* Z, hipStream_t s) {
  const dim3 g((cols + 63) / 64, (rows + REC_SEG - 1) / REC_SEG), b(64);
  const int nseg = (int)g.y;
  hipLaunchKernelGGL(rec_seg_end_kernel, g, b, 0, s, E, p, rows, cols, rc, 1, Z);
  hipLaunchKernelGGL(rec_seg_scan_kernel, dim3(g.x), b, 0, s, Z, nseg, cols, rc, 1);
  hipLaunchKernelGGL(rec_seg_apply_kernel, g, b, 0, s, E, p, rows, cols, rc, 1, Z);
  hipLaunchKernelGGL(rec_seg_scan_kernel, dim3(g.x), b, 0, s, Z, nseg, cols, rc, -1);
  hipLaunchKernelGGL(rec_seg_apply_kernel, g, b, 0, s, E, p, rows, cols, rc, -1, Z);
}

// Maps (FP32 planes, panel layout) and the FP64 S_X partials from the
// filtered E2: a block of 64 threads takes one panel (16 columns) of one
// S_X row group, lane (c, r) = (lane mod 16, lane / 16) columns c and rows
// r, r + 4, ... of it. Panels past the width (the last strip's) only clear
// their partial slot; columns past the width inside the last panel are 0.
template <typename WT>
__global__ void __launch_bounds__(64) rec_maps_kernel(const double* __restrict__ E2, int64_t p2, const WT* x,
                                                      int64_t pitch, double scale, double sigma, ImageDesc im,
                                                      char* maps) {
  const int panel = blockIdx.x, grp = blockIdx.y;
  const int lane = threadIdx.x, c = lane & 15, r = lane >> 4;
  const int v = panel * MAP_PANEL + c;
  float* A = reinterpret_cast<float*>(maps);
  float* Mu = A + im.plane;
  float* Mv = Mu + im.plane;
  const double k = -0.5 * sigma * sigma;
  double sx = 0.0;
  if (panel < im.npanels) {
    for (int i = 0; i < SX_ROWS / 4; ++i) {
      const int u = grp * SX_ROWS + r + 4 * i;
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
      const int64_t o = map_index(im.H, u, v);
      A[o] = a;
      Mu[o] = mu;
      Mv[o] = mv;
    }
  }
  sx = wave_sum(sx);
  if (lane == 0) {
    double* part = reinterpret_cast<double*>(maps + im.part_off);
    part[((int64_t)(panel / 4) * im.nsxg + grp) * SX_SLOTS + panel % 4] = sx;
  }
}

template <typename WT>
hipError_t launch_recursive_t(const ImageDesc& im, const void* x, double scale, double sigma, const RecCoeffs& rc,
                              double* E1, double* E2, double* Z, void* maps, hipStream_t s) {
  const int H = im.H, W = im.W;
  const int rows1 = W + 2 + rc.m, cols1 = H + 2;
  const int rows2 = H + 2 + rc.m, cols2 = W + 2;
  const int64_t p1 = cols1, p2 = cols2;
  hipLaunchKernelGGL(rec_load_kernel<WT>, dim3((cols1 + RT - 1) / RT, (rows1 + RT - 1) / RT), dim3(RT * 8), 0, s,
                     (const WT*)x, im.pitch, scale, H, W, E1, p1, rows1);
  rec_filter(E1, p1, rows1, cols1, rc, Z, s);
  hipLaunchKernelGGL(rec_transpose_kernel, dim3((cols2 + RT - 1) / RT, (rows2 + RT - 1) / RT), dim3(RT * 8), 0, s,
                     (const double*)E1, p1, H, W, E2, p2, rows2);
  rec_filter(E2, p2, rows2, cols2, rc, Z, s);
  static_assert(SX_SLOTS * MAP_PANEL == CONV_TW, "four panels per strip");
  hipLaunchKernelGGL(rec_maps_kernel<WT>, dim3((unsigned)(im.nstrips * SX_SLOTS), (unsigned)im.nsxg), dim3(64), 0,
                     s, (const double*)E2, p2, (const WT*)x, im.pitch, scale, sigma, im, (char*)maps);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_recursive(const ImageDesc& im, const void* x, double scale, double sigma, const RecCoeffs& rc,
                            double* E1, double* E2, double* Z, void* maps, hipStream_t s) {
  switch (im.wdtype) {
    case 0: return launch_recursive_t<uint8_t>(im, x, scale, sigma, rc, E1, E2, Z, maps, s);
    case 1: return launch_recursive_t<float>(im, x, scale, sigma, rc, E1, E2, Z, maps, s);
    default: return launch_recursive_t<double>(im, x, scale, sigma, rc, E1, E2, Z, maps, s);
  }
}

}  // namespace itc
