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
// (tg[t] = t g[t], t = x_a - y_a). One thread per output voxel and axis pass;
// intermediates are FP32 volumes in the caller's work buffer. S_X = sum h A
// is summed in two fixed-order levels (4,096-voxel blocks, then the blocks).
//
// Fit: one workgroup; each thread owns up to four codevectors (FP64
// positions); per sweep trilinear reads of the four maps at w_k (eight
// corners, off-lattice corners 0), the M x M Gaussian terms over an FP32
// copy of the codebook in LDS (scaled by sqrt(log2 e / 2 sigma^2) and centred
// on the volume, so each pair is one exp2), FP64 reductions of S_XW and S_W
// in a fixed order, and the Jacobi update.
#include "itc_device.h"

namespace itc {

namespace {

constexpr int VOL_NT = 256;
constexpr int VOL_SXB = 4096;  // voxels per S_X block
constexpr int VOL_MAXPASS = 4;

__device__ __forceinline__ void taps_of(int t, double k2, double& g, double& tg) {
  g = exp(k2 * (double)(t * t));
  tg = (double)t * g;
}

template <typename WT>
__device__ __forceinline__ float weight_at(const WT* x, const VolumeGeom& vg, int s, int u, int v) {
  return (float)(vg.scale * (double)x[(int64_t)s * vg.slice_pitch + (int64_t)u * vg.row_pitch + v]);
}

// v pass from the stored weights: P0 = h *_v g, P1 = h *_v tg.
template <typename WT>
__global__ void __launch_bounds__(VOL_NT) vol_pass_v_kernel(const WT* __restrict__ x, VolumeGeom vg,
                                                            float* __restrict__ P0, float* __restrict__ P1) {
  extern __shared__ float tap[];  // [2R + 1] g, then [2R + 1] tg
  const int R = vg.R;
  const double k2 = -0.5 / (vg.sigma * vg.sigma);
  for (int t = threadIdx.x; t <= 2 * R; t += blockDim.x) {
    double g, tg;
    taps_of(t - R, k2, g, tg);
    tap[t] = (float)g;
    tap[2 * R + 1 + t] = (float)tg;
  }
  __syncthreads();
  const int64_t n = (int64_t)vg.D * vg.H * vg.W;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int v = (int)(i % vg.W);
    const int64_t r = i / vg.W;
    const int u = (int)(r % vg.H), s = (int)(r / vg.H);
    float a0 = 0.f, a1 = 0.f;
    for (int t = -R; t <= R; ++t) {
      const int y = v - t;
      if (y < 0 || y >= vg.W) continue;
      const float h = weight_at(x, vg, s, u, y);
      a0 = fmaf(tap[t + R], h, a0);
      a1 = fmaf(tap[2 * R + 1 + t + R], h, a1);
    }
    P0[i] = a0;
    P1[i] = a1;
  }
}

// A pass along the u (stride W) or s (stride H W) axis of a contiguous
// volume: o0 = in *_a g and, when o1 is set, o1 = in *_a tg.
__global__ void __launch_bounds__(VOL_NT) vol_pass_kernel(const float* __restrict__ in, VolumeGeom vg, int axis,
                                                          float* __restrict__ o0, float* __restrict__ o1) {
  extern __shared__ float tap[];
  const int R = vg.R;
  const double k2 = -0.5 / (vg.sigma * vg.sigma);
  for (int t = threadIdx.x; t <= 2 * R; t += blockDim.x) {
    double g, tg;
    taps_of(t - R, k2, g, tg);
    tap[t] = (float)g;
    tap[2 * R + 1 + t] = (float)tg;
  }
  __syncthreads();
  const int64_t n = (int64_t)vg.D * vg.H * vg.W;
  const int64_t stride = axis == 1 ? (int64_t)vg.W : (int64_t)vg.H * vg.W;
  const int len = axis == 1 ? vg.H : vg.D;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int pos = (int)((i / stride) % len);
    float a0 = 0.f, a1 = 0.f;
    for (int t = -R; t <= R; ++t) {
      const int y = pos - t;
      if (y < 0 || y >= len) continue;
      const float f = in[i - (int64_t)t * stride];
      a0 = fmaf(tap[t + R], f, a0);
      a1 = fmaf(tap[2 * R + 1 + t + R], f, a1);
    }
    o0[i] = a0;
    if (o1) o1[i] = a1;
  }
}

// S_X block sums: block b sums h A over voxels [4096 b, 4096 (b + 1)).
template <typename WT>
__global__ void __launch_bounds__(VOL_NT) vol_sx_blocks_kernel(const WT* __restrict__ x, VolumeGeom vg,
                                                               const float* __restrict__ A, double* __restrict__ blk) {
  __shared__ double red[VOL_NT / 64];
  const int64_t n = (int64_t)vg.D * vg.H * vg.W;
  const int64_t i0 = (int64_t)blockIdx.x * VOL_SXB;
  double s = 0.0;
  for (int k = threadIdx.x; k < VOL_SXB; k += blockDim.x) {
    const int64_t i = i0 + k;
    if (i >= n) break;
    const int v = (int)(i % vg.W);
    const int64_t r = i / vg.W;
    const int u = (int)(r % vg.H), sl = (int)(r / vg.H);
    s = fma((double)weight_at(x, vg, sl, u, v), (double)A[i], s);
  }
  s = block_reduce_fixed(s, red);
  if (threadIdx.x == 0) blk[blockIdx.x] = s;
}

__global__ void __launch_bounds__(VOL_NT) vol_sx_total_kernel(const double* __restrict__ blk, int nb, double* s_x) {
  __shared__ double red[VOL_NT / 64];
  const double s = block_sum_fixed(blk, (int64_t)nb, red);
  if (threadIdx.x == 0) *s_x = s;
}

// Trilinear read of the four maps at w: A, and g = sum_c b_c ((c - w) A(c) - M(c)).
__device__ __forceinline__ void vol_read(const float* maps, const VolumeGeom& vg, double ws, double wu, double wv,
                                         float& A, float g[3], float dA[3]) {
  const int64_t vol = (int64_t)vg.D * vg.H * vg.W;
  const double fs0 = floor(ws), fu0 = floor(wu), fv0 = floor(wv);
  const int s0 = (int)fs0, u0 = (int)fu0, v0 = (int)fv0;
  const float fr[3] = {(float)(ws - fs0), (float)(wu - fu0), (float)(wv - fv0)};
  A = 0.f;
  g[0] = g[1] = g[2] = 0.f;
  dA[0] = dA[1] = dA[2] = 0.f;
  for (int c = 0; c < 8; ++c) {
    const int ds = c >> 2, du = (c >> 1) & 1, dv = c & 1;
    const int s = s0 + ds, u = u0 + du, v = v0 + dv;
    if (s < 0 || s >= vg.D || u < 0 || u >= vg.H || v < 0 || v >= vg.W) continue;
    const int64_t o = ((int64_t)s * vg.H + u) * vg.W + v;
    const float a = maps[o], ms = maps[vol + o], mu = maps[2 * vol + o], mv = maps[3 * vol + o];
    const float bs = ds ? fr[0] : 1.f - fr[0], bu = du ? fr[1] : 1.f - fr[1], bv = dv ? fr[2] : 1.f - fr[2];
    const float b = bs * bu * bv;
    A = fmaf(b, a, A);
    g[0] = fmaf(b, fmaf((float)ds - fr[0], a, -ms), g[0]);
    g[1] = fmaf(b, fmaf((float)du - fr[1], a, -mu), g[1]);
    g[2] = fmaf(b, fmaf((float)dv - fr[2], a, -mv), g[2]);
  }
}

__global__ void __launch_bounds__(VOL_NT) vol_fit_kernel(const float* __restrict__ maps, VolumeGeom vg,
                                                         const double* __restrict__ s_x_in, int M, const float* __restrict__ w_init, int iters,
                                                         double theta, float* w_out, double* d_trace,
                                                         int32_t* iters_done) {
  extern __shared__ float4 cb[];  // [Mpad] scaled centred codebook
  __shared__ double red[VOL_NT / 64];
  __shared__ float redf[VOL_NT / 64];
  const int tid = threadIdx.x;
  const double s_x = *s_x_in;
  const int npass = (M + VOL_NT - 1) / VOL_NT;
  const double sc = sqrt(1.4426950408889634 / (2.0 * vg.sigma * vg.sigma));
  const double cs0 = 0.5 * vg.D, cu0 = 0.5 * vg.H, cv0 = 0.5 * vg.W;
  double ws[VOL_MAXPASS], wu[VOL_MAXPASS], wv[VOL_MAXPASS];
#pragma unroll
  for (int p = 0; p < VOL_MAXPASS; ++p) {
    const int k = p * VOL_NT + tid;
    ws[p] = wu[p] = wv[p] = 0.0;
    if (p < npass && k < M) {
      ws[p] = w_init[3 * k];
      wu[p] = w_init[3 * k + 1];
      wv[p] = w_init[3 * k + 2];
      cb[k] = make_float4((float)(sc * (ws[p] - cs0)), (float)(sc * (wu[p] - cu0)), (float)(sc * (wv[p] - cv0)), 0.f);
    }
  }
  __syncthreads();
  bool stop = false;
  int t = 0;
  for (;; ++t) {
    const bool last = t == iters || stop;
    float Ak[VOL_MAXPASS], gk[VOL_MAXPASS][3], Ek[VOL_MAXPASS][3];
    double sxw = 0.0, sw = 0.0;
#pragma unroll
    for (int p = 0; p < VOL_MAXPASS; ++p) {
      const int k = p * VOL_NT + tid;
      Ak[p] = 0.f;
      gk[p][0] = gk[p][1] = gk[p][2] = Ek[p][0] = Ek[p][1] = Ek[p][2] = 0.f;
      if (p < npass && k < M) {
        float dA[3];
        vol_read(maps, vg, ws[p], wu[p], wv[p], Ak[p], gk[p], dA);
        const float4 hk = cb[k];
        float C = 0.f, E0 = 0.f, E1 = 0.f, E2 = 0.f;
        for (int j = 0; j < M; ++j) {
          const float4 hj = cb[j];
          const float d0 = hj.x - hk.x, d1 = hj.y - hk.y, d2 = hj.z - hk.z;
          const float e = __builtin_amdgcn_exp2f(-fmaf(d0, d0, fmaf(d1, d1, d2 * d2)));
          C += e;
          E0 = fmaf(e, d0, E0);
          E1 = fmaf(e, d1, E1);
          E2 = fmaf(e, d2, E2);
        }
        Ek[p][0] = E0;
        Ek[p][1] = E1;
        Ek[p][2] = E2;
        sxw += (double)Ak[p];
        sw += (double)C;
      }
    }
    const double S_XW = block_reduce_fixed(sxw, red);
    const double S_W = block_reduce_fixed(sw, red);
    if (tid == 0 && d_trace) d_trace[t] = log(S_W) + log(s_x) - 2.0 * log(S_XW);
    if (last) break;
    const double c = S_XW / S_W / sc;  // E = E' / sc
    float step = 0.f;
#pragma unroll
    for (int p = 0; p < VOL_MAXPASS; ++p) {
      const int k = p * VOL_NT + tid;
      if (p < npass && k < M && Ak[p] != 0.f) {
        const double inv = 1.0 / (double)Ak[p];
        const double d0 = ((double)gk[p][0] - c * (double)Ek[p][0]) * inv;
        const double d1 = ((double)gk[p][1] - c * (double)Ek[p][1]) * inv;
        const double d2 = ((double)gk[p][2] - c * (double)Ek[p][2]) * inv;
        ws[p] += d0;
        wu[p] += d1;
        wv[p] += d2;
        step = fmaxf(step, (float)sqrt(d0 * d0 + d1 * d1 + d2 * d2));
      }
    }
    __syncthreads();  // every thread has read the codebook of this sweep
#pragma unroll
    for (int p = 0; p < VOL_MAXPASS; ++p) {
      const int k = p * VOL_NT + tid;
      if (p < npass && k < M)
        cb[k] = make_float4((float)(sc * (ws[p] - cs0)), (float)(sc * (wu[p] - cu0)), (float)(sc * (wv[p] - cv0)), 0.f);
    }
    step = wave_max_nonneg(step);
    if ((tid & 63) == 0) redf[tid >> 6] = step;
    __syncthreads();
    if (theta >= 0.0) {
      float smax = 0.f;
      for (int q = 0; q < VOL_NT / 64; ++q) smax = fmaxf(smax, redf[q]);
      stop = (double)smax <= theta;
    }
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < VOL_MAXPASS; ++p) {
    const int k = p * VOL_NT + tid;
    if (p < npass && k < M) {
      w_out[3 * k] = (float)ws[p];
      w_out[3 * k + 1] = (float)wu[p];
      w_out[3 * k + 2] = (float)wv[p];
    }
  }
  if (tid == 0 && iters_done) *iters_done = t;
}

template <typename WT>
hipError_t launch_volume_maps_t(const VolumeGeom& vg, const void* x, float* work, float* maps, double* sx_blk,
                                double* s_x, hipStream_t s) {
  const int64_t n = (int64_t)vg.D * vg.H * vg.W;
  float *P0 = work, *P1 = work + n, *Q00 = work + 2 * n, *Q01 = work + 3 * n, *Q10 = work + 4 * n;
  const int grid = (int)std::min<int64_t>((n + VOL_NT - 1) / VOL_NT, 8192);
  const size_t tapb = (size_t)(2 * (2 * vg.R + 1)) * sizeof(float);
  hipLaunchKernelGGL(vol_pass_v_kernel<WT>, dim3(grid), dim3(VOL_NT), tapb, s, (const WT*)x, vg, P0, P1);
  hipLaunchKernelGGL(vol_pass_kernel, dim3(grid), dim3(VOL_NT), tapb, s, (const float*)P0, vg, 1, Q00, Q01);
  hipLaunchKernelGGL(vol_pass_kernel, dim3(grid), dim3(VOL_NT), tapb, s, (const float*)P1, vg, 1, Q10,
                     (float*)nullptr);
  hipLaunchKernelGGL(vol_pass_kernel, dim3(grid), dim3(VOL_NT), tapb, s, (const float*)Q00, vg, 0, maps, maps + n);
  hipLaunchKernelGGL(vol_pass_kernel, dim3(grid), dim3(VOL_NT), tapb, s, (const float*)Q01, vg, 0, maps + 2 * n,
                     (float*)nullptr);
  hipLaunchKernelGGL(vol_pass_kernel, dim3(grid), dim3(VOL_NT), tapb, s, (const float*)Q10, vg, 0, maps + 3 * n,
                     (float*)nullptr);
  const int nb = (int)((n + VOL_SXB - 1) / VOL_SXB);
  hipLaunchKernelGGL(vol_sx_blocks_kernel<WT>, dim3(nb), dim3(VOL_NT), 0, s, (const WT*)x, vg, (const float*)maps,
                     sx_blk);
  hipLaunchKernelGGL(vol_sx_total_kernel, dim3(1), dim3(VOL_NT), 0, s, (const double*)sx_blk, nb, s_x);
  return hipGetLastError();
}

}  // namespace

int volume_sx_blocks(int64_t n) { return (int)((n + VOL_SXB - 1) / VOL_SXB); }

hipError_t launch_volume_maps(const VolumeGeom& vg, int wdtype, const void* x, float* work, float* maps,
                              double* sx_blk, double* s_x, hipStream_t s) {
  switch (wdtype) {
    case 0: return launch_volume_maps_t<uint8_t>(vg, x, work, maps, sx_blk, s_x, s);
    case 1: return launch_volume_maps_t<float>(vg, x, work, maps, sx_blk, s_x, s);
    default: return launch_volume_maps_t<double>(vg, x, work, maps, sx_blk, s_x, s);
  }
}

hipError_t launch_volume_fit(const VolumeGeom& vg, const float* maps, const double* s_x, int M, const float* w_init,
                             int iters, double theta, float* w_out, double* d_trace, int32_t* iters_done,
                             hipStream_t s) {
  hipLaunchKernelGGL(vol_fit_kernel, dim3(1), dim3(VOL_NT), (size_t)M * sizeof(float4), s, maps, vg, s_x, M, w_init,
                     iters, theta, w_out, d_trace, iters_done);
  return hipGetLastError();
}

}  // namespace itc
