// Lattice ITC on 3-D lattices (volumes): the maps of Section 3.1 with a
// third separable pass and the update eq. (4) in three dimensions (the paper
// develops the method on 2-D lattices and notes it carries over to higher
// dimensions). Coordinates x = (s, u, v): slice, row, column.
//
// Maps: A = h * g(s) g(u) g(v) and the moments M_a = sum_y h(y) (x_a - y_a)
// g(x - y) for a = s, u, v, each a chain of 1-D correlations:
//   v pass:  P0 = h *_v g,   P1 = h *_v tg
//   u pass:  Q00 = P0 *_u g, Q01 = P0 *_u tg, Q10 = P1 *_u g
//   s pass:  A = Q00 *_s g,  M_s = Q00 *_s tg, M_u = Q01 *_s g, M_v = Q10 *_s g
// (tg[t] = t g[t], t = x_a - y_a). Two kernels:
//   * in-plane: a workgroup stages a 64-column x 32-row tile of one slice
//     with its R halo in LDS, runs the v pass in place (each row becomes its
//     P0 | P1) and the u pass out to the three FP32 Q volumes in the caller's
//     work buffer;
//   * depth: each thread walks 8 consecutive outputs along s for one (u, v),
//     reading every Q value of its window once, writes A, M_s, M_u, M_v and
//     adds h A into a per-workgroup FP64 partial of S_X.
// The column passes are register-blocked: input k of the window feeds the 8
// outputs through a zero-padded tap table, so every input is loaded once and
// no tap index leaves the table. Taps are kernel arguments (scalar loads).
// S_X is summed in two fixed-order levels (workgroups, then their partials).
//
// Fit: one workgroup; P lanes share a codevector (P the largest power of two
// <= 64 with M P <= 256) or each thread owns up to four codevectors (FP64
// positions); per sweep trilinear reads of the four maps at w_k (eight
// corners, off-lattice corners 0; the corner values are kept while w_k stays
// in its cell), the M x M Gaussian terms over an FP32 copy of the codebook in
// LDS (scaled by sqrt(log2 e / 2 sigma^2) and centred on the volume, so each
// pair is one exp2), FP64 reductions of S_XW and S_W in a fixed order, and the
// Jacobi update.
#include <algorithm>
#include <climits>
#include <cmath>

#include "itc_device.h"

namespace itc {

namespace {

constexpr int VOL_NT = 256;
constexpr int VOL_TR = 32;   // rows of an in-plane tile (4 waves x VOL_RUN)
constexpr int VOL_RUN = 8;   // outputs per thread of a column pass
constexpr int VOL_UR = 4;    // rows of a depth-pass workgroup (one per wave)
constexpr int VOL_MAXR = 32;
constexpr int VOL_TAPS = 2 * VOL_MAXR + 1 + 2 * (VOL_RUN - 1);
constexpr int VOL_MAXPASS = 4;

// Taps with VOL_RUN - 1 zeros on each side: f[t + R + VOL_RUN - 1] = f(t) for
// |t| <= R, zero elsewhere in the table.
struct VolTaps {
  float g[VOL_TAPS];
  float tg[VOL_TAPS];
};

template <typename WT>
__device__ __forceinline__ double weight_at(const WT* x, const VolumeGeom& vg, int s, int u, int v) {
  return vg.scale * (double)x[(int64_t)s * vg.slice_pitch + (int64_t)u * vg.row_pitch + v];
}

// In-plane passes of one tile: Q00, Q01, Q10 for rows [u0, u0 + 32) and
// columns [v0, v0 + 64) of slice s (blockIdx = (column tile, row tile, s)).
// SROWS >= (32 + 2R) / 4 rows of the staged tile per wave (12, 16 or 24).
template <typename WT, int SROWS>
__global__ void __launch_bounds__(VOL_NT) vol_plane_kernel(const WT* __restrict__ x, VolumeGeom vg, VolTaps tp,
                                                           float* __restrict__ q00, float* __restrict__ q01,
                                                           float* __restrict__ q10) {
  extern __shared__ float X[];  // [4 SROWS][RP]: weights of rows u0 - R.., columns v0 - R.., then P0 | P1
  const int R = vg.R, XW = 64 + 2 * R, RP = XW > 128 ? XW : 128;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int v0 = blockIdx.x * 64, u0 = blockIdx.y * VOL_TR, s = blockIdx.z;
  // staging: wave wv takes rows wv, wv + 4, ... (SROWS of them, at most 2
  // columns per lane) and issues all their loads before the first is used;
  // positions off the lattice load a clamped position and store 0
  const WT* xs = x + (int64_t)s * vg.slice_pitch;
  WT raw[SROWS][2];
#pragma unroll
  for (int q = 0; q < SROWS; ++q) {
    const int u = min(max(u0 - R + wv + q * (VOL_NT / 64), 0), vg.H - 1);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int v = min(max(v0 - R + lane + 64 * h, 0), vg.W - 1);
      raw[q][h] = xs[(int64_t)u * vg.row_pitch + v];
    }
  }
#pragma unroll
  for (int q = 0; q < SROWS; ++q) {
    const int j = wv + q * (VOL_NT / 64), u = u0 - R + j;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = lane + 64 * h, v = v0 - R + c;
      const bool on = u >= 0 && u < vg.H && v >= 0 && v < vg.W;
      if (c < XW) X[j * RP + c] = on ? (float)(vg.scale * (double)raw[q][h]) : 0.f;
    }
  }
  // v pass, taps outermost (each tap is fetched once per wave): output column
  // lane of each of the wave's rows reads columns lane + R - t of that row,
  // which no other wave touches, so P0 | P1 overwrite the rows in place
  {
    float a0[SROWS], a1[SROWS];
#pragma unroll
    for (int q = 0; q < SROWS; ++q) a0[q] = a1[q] = 0.f;
    const float* xr = X + wv * RP + lane + R;
    for (int t = -R; t <= R; ++t) {
      const float g = tp.g[t + R + VOL_RUN - 1], tg = tp.tg[t + R + VOL_RUN - 1];
#pragma unroll
      for (int q = 0; q < SROWS; ++q) {
        const float h = xr[q * (VOL_NT / 64) * RP - t];
        a0[q] = fmaf(g, h, a0[q]);
        a1[q] = fmaf(tg, h, a1[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < SROWS; ++q) {
      X[(wv + q * (VOL_NT / 64)) * RP + lane] = a0[q];
      X[(wv + q * (VOL_NT / 64)) * RP + 64 + lane] = a1[q];
    }
  }
  __syncthreads();
  // u pass: wave wv makes tile rows r0 .. r0 + 7; input k of the window is
  // P row r0 + k (image row u0 - R + r0 + k) and reaches output o with
  // t = o + R - k, |t| <= R. For R >= 3 the window splits into a ramp-up
  // (k < 7: outputs 0..k), a middle (all outputs) and a ramp-down (k = 2R + d:
  // outputs d..7), so no zero tap is multiplied.
  const int r0 = wv * VOL_RUN;
  float c00[VOL_RUN], c01[VOL_RUN], c10[VOL_RUN];
#pragma unroll
  for (int o = 0; o < VOL_RUN; ++o) c00[o] = c01[o] = c10[o] = 0.f;
  auto feed = [&](int k, int olo, int ohi) __attribute__((always_inline)) {
    const float p0 = X[(r0 + k) * RP + lane], p1 = X[(r0 + k) * RP + 64 + lane];
    const int b = 2 * R - k + VOL_RUN - 1;
#pragma unroll
    for (int o = olo; o <= ohi; ++o) {
      const float g = tp.g[b + o], tg = tp.tg[b + o];
      c00[o] = fmaf(g, p0, c00[o]);
      c01[o] = fmaf(tg, p0, c01[o]);
      c10[o] = fmaf(g, p1, c10[o]);
    }
  };
  if (R >= 3) {
#pragma unroll
    for (int k = 0; k < VOL_RUN - 1; ++k) feed(k, 0, k);
#pragma unroll 2
    for (int k = VOL_RUN - 1; k <= 2 * R; ++k) feed(k, 0, VOL_RUN - 1);
#pragma unroll
    for (int d = 1; d < VOL_RUN; ++d) feed(2 * R + d, d, VOL_RUN - 1);
  } else {
    for (int k = 0; k < 2 * R + VOL_RUN; ++k) feed(k, 0, VOL_RUN - 1);
  }
  const int v = v0 + lane;
  if (v >= vg.W) return;
#pragma unroll
  for (int o = 0; o < VOL_RUN; ++o) {
    const int u = u0 + r0 + o;
    if (u < vg.H) {
      const int64_t i = ((int64_t)s * vg.H + u) * vg.W + v;
      q00[i] = c00[o];
      q01[i] = c01[o];
      q10[i] = c10[o];
    }
  }
}

// Depth pass and S_X partials: blockIdx = (column tile, 4-row group, 8-slice
// group); thread (wave wv, lane) owns (u, v) and slices s0 .. s0 + 7.
template <typename WT>
__global__ void __launch_bounds__(VOL_NT) vol_depth_kernel(const WT* __restrict__ x, VolumeGeom vg, VolTaps tp,
                                                           const float* __restrict__ q00,
                                                           const float* __restrict__ q01,
                                                           const float* __restrict__ q10, float* __restrict__ maps,
                                                           double* __restrict__ blk) {
  __shared__ double red[VOL_NT / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int v = blockIdx.x * 64 + lane, u = blockIdx.y * VOL_UR + wv, s0 = blockIdx.z * VOL_RUN;
  const bool in = u < vg.H && v < vg.W;
  const int R = vg.R;
  const int64_t plane = (int64_t)vg.H * vg.W, n = plane * vg.D, col = (int64_t)u * vg.W + v;
  float a[VOL_RUN], ms[VOL_RUN], mu[VOL_RUN], mv[VOL_RUN];
#pragma unroll
  for (int o = 0; o < VOL_RUN; ++o) a[o] = ms[o] = mu[o] = mv[o] = 0.f;
  // input k is slice s0 - R + k; only slices inside the lattice contribute
  const int k0 = R - s0 > 0 ? R - s0 : 0;
  const int k1 = min(2 * R + VOL_RUN, vg.D - s0 + R);
  // four window inputs per step, their loads issued together
  for (int k = k0; k < k1; k += 4) {
    float f[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      f[q][0] = f[q][1] = f[q][2] = 0.f;
      if (in && k + q < k1) {
        const int64_t i = (int64_t)(s0 - R + k + q) * plane + col;
        f[q][0] = q00[i];
        f[q][1] = q01[i];
        f[q][2] = q10[i];
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (k + q >= k1) break;
      const int b = 2 * R - (k + q) + VOL_RUN - 1;
#pragma unroll
      for (int o = 0; o < VOL_RUN; ++o) {
        const float g = tp.g[b + o], tg = tp.tg[b + o];
        a[o] = fmaf(g, f[q][0], a[o]);
        ms[o] = fmaf(tg, f[q][0], ms[o]);
        mu[o] = fmaf(g, f[q][1], mu[o]);
        mv[o] = fmaf(g, f[q][2], mv[o]);
      }
    }
  }
  double sx = 0.0;
#pragma unroll
  for (int o = 0; o < VOL_RUN; ++o) {
    const int s = s0 + o;
    if (in && s < vg.D) {
      const int64_t i = (int64_t)s * plane + col;
      maps[i] = a[o];
      maps[n + i] = ms[o];
      maps[2 * n + i] = mu[o];
      maps[3 * n + i] = mv[o];
      sx = fma(weight_at(x, vg, s, u, v), (double)a[o], sx);
    }
  }
  sx = block_reduce_fixed(sx, red);
  if (threadIdx.x == 0) blk[((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = sx;
}

__global__ void __launch_bounds__(VOL_NT) vol_sx_total_kernel(const double* __restrict__ blk, int nb, double* s_x) {
  __shared__ double red[VOL_NT / 64];
  const double s = block_sum_fixed(blk, (int64_t)nb, red);
  if (threadIdx.x == 0) *s_x = s;
}

// The workgroup totals of two FP64 values per thread (each wave by a fixed
// DPP tree, then the waves in order); every thread gets both.
__device__ __forceinline__ void block_reduce2(double& x, double& y, double (*red)[VOL_NT / 64]) {
  const int tid = threadIdx.x;
  x = wave_sum(x);
  y = wave_sum(y);
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = x;
    red[1][tid >> 6] = y;
  }
  __syncthreads();
  x = y = 0.0;
#pragma unroll
  for (int w = 0; w < VOL_NT / 64; ++w) {
    x += red[0][w];
    y += red[1][w];
  }
}

// The eight corners of a lattice cell for the four maps, kept in registers
// while a codevector stays in the cell.
struct Cell {
  int s0, u0, v0;
  float a[8], ms[8], mu[8], mv[8];
};

__device__ __forceinline__ void cell_load(Cell& c, rsrc_t rs, uint32_t plane_bytes, const VolumeGeom& vg, int s0,
                                          int u0, int v0) {
  c.s0 = s0;
  c.u0 = u0;
  c.v0 = v0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int s = s0 + (q >> 2), u = u0 + ((q >> 1) & 1), v = v0 + (q & 1);
    const bool on = s >= 0 && s < vg.D && u >= 0 && u < vg.H && v >= 0 && v < vg.W;
    // off-lattice corners take an offset past the buffer: the load returns 0
    const uint32_t off = on ? (uint32_t)((((int64_t)s * vg.H + u) * vg.W + v) * 4) : 0x80000000u;
    c.a[q] = buf_load<float>(rs, off, 0);
    c.ms[q] = buf_load<float>(rs, off, plane_bytes);
    c.mu[q] = buf_load<float>(rs, off, 2 * plane_bytes);
    c.mv[q] = buf_load<float>(rs, off, 3 * plane_bytes);
  }
}

// Trilinear read at fractional offsets fr: A and g = sum_c b_c ((c - w) A(c) - M(c)).
__device__ __forceinline__ void cell_read(const Cell& c, const float fr[3], float& A, float g[3]) {
  A = 0.f;
  g[0] = g[1] = g[2] = 0.f;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int ds = q >> 2, du = (q >> 1) & 1, dv = q & 1;
    const float bs = ds ? fr[0] : 1.f - fr[0], bu = du ? fr[1] : 1.f - fr[1], bv = dv ? fr[2] : 1.f - fr[2];
    const float b = bs * bu * bv;
    A = fmaf(b, c.a[q], A);
    g[0] = fmaf(b, fmaf((float)ds - fr[0], c.a[q], -c.ms[q]), g[0]);
    g[1] = fmaf(b, fmaf((float)du - fr[1], c.a[q], -c.mu[q]), g[1]);
    g[2] = fmaf(b, fmaf((float)dv - fr[2], c.a[q], -c.mv[q]), g[2]);
  }
}

// P lanes per codevector (NPASS = 1), or NPASS codevectors per thread (P = 1).
template <int P, int NPASS>
__global__ void __launch_bounds__(VOL_NT) vol_fit_kernel(const float* __restrict__ maps, VolumeGeom vg,
                                                         const double* __restrict__ s_x_in, int M,
                                                         const float* __restrict__ w_init, int iters, double theta,
                                                         float* w_out, double* d_trace, int32_t* iters_done) {
  static_assert(P == 1 || NPASS == 1, "lanes per codevector need one pass");
  constexpr int SLOTS = VOL_NT / P;
  extern __shared__ float4 cb[];  // [M] scaled centred codebook
  __shared__ double red[2][VOL_NT / 64];
  __shared__ float redf[VOL_NT / 64];
  const int tid = threadIdx.x, part = tid % P, slot = tid / P;
  const int64_t n = (int64_t)vg.D * vg.H * vg.W;
  const uint32_t plane_bytes = (uint32_t)(n * 4);
  const rsrc_t rs = make_rsrc(maps, 4 * plane_bytes);
  const double s_x = *s_x_in;
  const double sc = sqrt(1.4426950408889634 / (2.0 * vg.sigma * vg.sigma)), isc = 1.0 / sc;
  const double cs0 = 0.5 * vg.D, cu0 = 0.5 * vg.H, cv0 = 0.5 * vg.W;
  double ws[NPASS], wu[NPASS], wv[NPASS];
  Cell cell[NPASS];
#pragma unroll
  for (int p = 0; p < NPASS; ++p) {
    const int k = p * SLOTS + slot;
    ws[p] = wu[p] = wv[p] = 0.0;
    cell[p].s0 = INT_MIN;
    if (k < M) {
      ws[p] = w_init[3 * k];
      wu[p] = w_init[3 * k + 1];
      wv[p] = w_init[3 * k + 2];
      if (part == 0)
        cb[k] = make_float4((float)(sc * (ws[p] - cs0)), (float)(sc * (wu[p] - cu0)), (float)(sc * (wv[p] - cv0)),
                            0.f);
    }
  }
  __syncthreads();
  bool stop = false;
  int t = 0;
  for (;; ++t) {
    const bool last = t == iters || stop;
    float Ak[NPASS], gk[NPASS][3], Ek[NPASS][3];
    double sxw = 0.0, sw = 0.0;
#pragma unroll
    for (int p = 0; p < NPASS; ++p) {
      const int k = p * SLOTS + slot;
      Ak[p] = 0.f;
      gk[p][0] = gk[p][1] = gk[p][2] = Ek[p][0] = Ek[p][1] = Ek[p][2] = 0.f;
      if (k < M) {
        const double fs = floor(ws[p]), fu = floor(wu[p]), fv = floor(wv[p]);
        const int s0 = (int)fs, u0 = (int)fu, v0 = (int)fv;
        // with several passes the cells are reloaded every sweep (registers)
        if (NPASS > 1 || s0 != cell[p].s0 || u0 != cell[p].u0 || v0 != cell[p].v0)
          cell_load(cell[p], rs, plane_bytes, vg, s0, u0, v0);
        const float fr[3] = {(float)(ws[p] - fs), (float)(wu[p] - fu), (float)(wv[p] - fv)};
        cell_read(cell[p], fr, Ak[p], gk[p]);
        const float4 hk = cb[k];
        float C = 0.f, E0 = 0.f, E1 = 0.f, E2 = 0.f;
        for (int j = part; j < M; j += P) {
          const float4 hj = cb[j];
          const float d0 = hj.x - hk.x, d1 = hj.y - hk.y, d2 = hj.z - hk.z;
          const float e = __builtin_amdgcn_exp2f(-fmaf(d0, d0, fmaf(d1, d1, d2 * d2)));
          C += e;
          E0 = fmaf(e, d0, E0);
          E1 = fmaf(e, d1, E1);
          E2 = fmaf(e, d2, E2);
        }
        C = group_sum<P>(C);
        Ek[p][0] = group_sum<P>(E0);
        Ek[p][1] = group_sum<P>(E1);
        Ek[p][2] = group_sum<P>(E2);
        if (part == 0) {
          sxw += (double)Ak[p];
          sw += (double)C;
        }
      }
    }
    block_reduce2(sxw, sw, red);
    const double S_XW = sxw, S_W = sw;
    // D = log(S_W S_X / S_XW^2): the argument now, the logarithms after the
    // last sweep by all threads at once
    if (tid == 0 && d_trace) d_trace[t] = S_W * s_x / (S_XW * S_XW);
    if (last) break;
    const double c = S_XW / S_W * isc;  // E = E' / sc
    float step = 0.f;
#pragma unroll
    for (int p = 0; p < NPASS; ++p) {
      const int k = p * SLOTS + slot;
      if (k < M && Ak[p] != 0.f) {
        const double inv = 1.0 / (double)Ak[p];
        const double d0 = ((double)gk[p][0] - c * (double)Ek[p][0]) * inv;
        const double d1 = ((double)gk[p][1] - c * (double)Ek[p][1]) * inv;
        const double d2 = ((double)gk[p][2] - c * (double)Ek[p][2]) * inv;
        ws[p] += d0;
        wu[p] += d1;
        wv[p] += d2;
        if (theta >= 0.0) step = fmaxf(step, (float)sqrt(d0 * d0 + d1 * d1 + d2 * d2));
      }
    }
    __syncthreads();  // every thread has read the codebook and the sums of this sweep
#pragma unroll
    for (int p = 0; p < NPASS; ++p) {
      const int k = p * SLOTS + slot;
      if (k < M && part == 0)
        cb[k] = make_float4((float)(sc * (ws[p] - cs0)), (float)(sc * (wu[p] - cu0)), (float)(sc * (wv[p] - cv0)),
                            0.f);
    }
    if (theta >= 0.0) {
      step = wave_max_nonneg(step);
      if ((tid & 63) == 0) redf[tid >> 6] = step;
      __syncthreads();
      float smax = 0.f;
      for (int q = 0; q < VOL_NT / 64; ++q) smax = fmaxf(smax, redf[q]);
      stop = (double)smax <= theta;
    }
    __syncthreads();  // the new codebook is visible; redf is read before it is written again
  }
#pragma unroll
  for (int p = 0; p < NPASS; ++p) {
    const int k = p * SLOTS + slot;
    if (k < M && part == 0) {
      w_out[3 * k] = (float)ws[p];
      w_out[3 * k + 1] = (float)wu[p];
      w_out[3 * k + 2] = (float)wv[p];
    }
  }
  if (tid == 0 && iters_done) *iters_done = t;
  if (d_trace) {
    __threadfence_block();
    __syncthreads();
    for (int i = tid; i <= t; i += VOL_NT) d_trace[i] = log(d_trace[i]);
  }
}

VolTaps make_taps(const VolumeGeom& vg) {
  VolTaps tp;
  for (int i = 0; i < VOL_TAPS; ++i) tp.g[i] = tp.tg[i] = 0.f;
  for (int t = -vg.R; t <= vg.R; ++t) {
    const double g = std::exp(-(double)(t * t) / (2.0 * vg.sigma * vg.sigma));
    tp.g[t + vg.R + VOL_RUN - 1] = (float)g;
    tp.tg[t + vg.R + VOL_RUN - 1] = (float)((double)t * g);
  }
  return tp;
}

dim3 depth_grid(const VolumeGeom& vg) {
  return dim3((vg.W + 63) / 64, (vg.H + VOL_UR - 1) / VOL_UR, (vg.D + VOL_RUN - 1) / VOL_RUN);
}

template <typename WT>
hipError_t launch_volume_maps_t(const VolumeGeom& vg, const void* x, float* work, float* maps, double* sx_blk,
                                double* s_x, hipStream_t s) {
  const int64_t n = (int64_t)vg.D * vg.H * vg.W;
  float *Q00 = work, *Q01 = work + n, *Q10 = work + 2 * n;
  const VolTaps tp = make_taps(vg);
  // the staged tile has 32 + 2R <= 4 SROWS rows of max(64 + 2R, 128) floats: at most 48 KiB
  const size_t rp = (size_t)std::max(64 + 2 * vg.R, 128) * sizeof(float);
  const dim3 pg((vg.W + 63) / 64, (vg.H + VOL_TR - 1) / VOL_TR, vg.D);
  if (vg.R <= 8)
    hipLaunchKernelGGL((vol_plane_kernel<WT, 12>), pg, dim3(VOL_NT), 48 * rp, s, (const WT*)x, vg, tp, Q00, Q01, Q10);
  else if (vg.R <= 16)
    hipLaunchKernelGGL((vol_plane_kernel<WT, 16>), pg, dim3(VOL_NT), 64 * rp, s, (const WT*)x, vg, tp, Q00, Q01, Q10);
  else
    hipLaunchKernelGGL((vol_plane_kernel<WT, 24>), pg, dim3(VOL_NT), 96 * rp, s, (const WT*)x, vg, tp, Q00, Q01, Q10);
  const dim3 dg = depth_grid(vg);
  hipLaunchKernelGGL(vol_depth_kernel<WT>, dg, dim3(VOL_NT), 0, s, (const WT*)x, vg, tp, (const float*)Q00,
                     (const float*)Q01, (const float*)Q10, maps, sx_blk);
  hipLaunchKernelGGL(vol_sx_total_kernel, dim3(1), dim3(VOL_NT), 0, s, (const double*)sx_blk,
                     (int)(dg.x * dg.y * dg.z), s_x);
  return hipGetLastError();
}

template <int P, int NPASS>
void launch_fit_t(const VolumeGeom& vg, const float* maps, const double* s_x, int M, const float* w_init, int iters,
                  double theta, float* w_out, double* d_trace, int32_t* iters_done, hipStream_t s) {
  hipLaunchKernelGGL((vol_fit_kernel<P, NPASS>), dim3(1), dim3(VOL_NT), (size_t)M * sizeof(float4), s, maps, vg,
                     s_x, M, w_init, iters, theta, w_out, d_trace, iters_done);
}

}  // namespace

int volume_sx_blocks(const VolumeGeom& vg) {
  const dim3 dg = depth_grid(vg);
  return (int)(dg.x * dg.y * dg.z);
}

hipError_t launch_volume_maps(const VolumeGeom& vg, int wdtype, const void* x, float* work, float* maps,
                              double* sx_blk, double* s_x, hipStream_t s) {
  if (vg.R < 1 || vg.R > VOL_MAXR) return hipErrorInvalidValue;
  switch (wdtype) {
    case 0: return launch_volume_maps_t<uint8_t>(vg, x, work, maps, sx_blk, s_x, s);
    case 1: return launch_volume_maps_t<float>(vg, x, work, maps, sx_blk, s_x, s);
    default: return launch_volume_maps_t<double>(vg, x, work, maps, sx_blk, s_x, s);
  }
}

hipError_t launch_volume_fit(const VolumeGeom& vg, const float* maps, const double* s_x, int M, const float* w_init,
                             int iters, double theta, float* w_out, double* d_trace, int32_t* iters_done,
                             hipStream_t s) {
  const int npass = (M + VOL_NT - 1) / VOL_NT;
  if (npass > VOL_MAXPASS) return hipErrorInvalidValue;
  if (npass > 2) {
    launch_fit_t<1, 4>(vg, maps, s_x, M, w_init, iters, theta, w_out, d_trace, iters_done, s);
  } else if (npass == 2) {
    launch_fit_t<1, 2>(vg, maps, s_x, M, w_init, iters, theta, w_out, d_trace, iters_done, s);
  } else {
    int P = 1;
    while (P < 64 && M * 2 * P <= VOL_NT) P *= 2;
    switch (P) {
      case 64: launch_fit_t<64, 1>(vg, maps, s_x, M, w_init, iters, theta, w_out, d_trace, iters_done, s); break;
      case 32: launch_fit_t<32, 1>(vg, maps, s_x, M, w_init, iters, theta, w_out, d_trace, iters_done, s); break;
      case 16: launch_fit_t<16, 1>(vg, maps, s_x, M, w_init, iters, theta, w_out, d_trace, iters_done, s); break;
      case 8: launch_fit_t<8, 1>(vg, maps, s_x, M, w_init, iters, theta, w_out, d_trace, iters_done, s); break;
      case 4: launch_fit_t<4, 1>(vg, maps, s_x, M, w_init, iters, theta, w_out, d_trace, iters_done, s); break;
      case 2: launch_fit_t<2, 1>(vg, maps, s_x, M, w_init, iters, theta, w_out, d_trace, iters_done, s); break;
      default: launch_fit_t<1, 1>(vg, maps, s_x, M, w_init, iters, theta, w_out, d_trace, iters_done, s); break;
    }
  }
  return hipGetLastError();
}

}  // namespace itc
