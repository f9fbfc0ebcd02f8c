// Separable Gaussian convolution maps of a lattice weight image (Section 3.1:
// the Parzen sum of delta impulses is the image convolved with a Gaussian; for
// small widths the 2-D mask factorises into 1-D masks). One pass produces
//   A   = (I *_v g) *_u g,   M_u = (I *_v g) *_u tg,   M_v = (I *_v tg) *_u g
// with g[t] = exp(-t^2/(2 sigma^2)), tg[t] = t g[t], |t| <= R, and per 4-row
// group FP64 partial sums of S_X = sum I A.
//
// Work decomposition (gfx950): a 256-thread workgroup owns a strip of 64
// columns and a segment of rows and streams down it in chunks of 16 rows.
// Per chunk:
//   1. the chunk's input rows (with an R-column halo on both sides) are staged
//      in LDS as the real type (prefetched into registers one chunk ahead);
//   2. row pass (along v): each thread makes 4 adjacent columns of R0 = I*g and
//      R1 = I*tg for one row and writes them into an LDS ring of the last
//      2R+16 rows. Every row is written twice (slot q and q + RING) so that any
//      window of 2R+4 consecutive rows is contiguous: the column pass then
//      addresses all its reads with compile-time offsets from one base;
//   3. column pass (along u, lags the row pass by R rows): each thread makes 4
//      consecutive rows of one column of A, M_u, M_v, stores them coalesced
//      (lanes = columns) and adds h*A to the wave's S_X partial.
// Taps are computed once per workgroup in FP64 (one per lane) and held in
// scalar registers; the tap loops are fully unrolled for the radius class.
#include "itc_device.h"

namespace itc {

template <typename T, int R>
struct ConvGeom {
  static constexpr int J0 = (2 * R + CONV_CH - 1) / CONV_CH;  // chunks before the first column pass
  static constexpr int RING = (J0 + 1) * CONV_CH;             // ring rows, >= 2R + CH
  static constexpr int NXL = 2 * R + 4;                       // row-pass inputs per thread
  static constexpr int XP = 60 + 4 * ((NXL + 3) / 4);         // staging row pitch (elements)
  static constexpr int XW = CONV_TW + 2 * R;                  // staged columns per row
  static constexpr int NSTAGE = (CONV_CH * XW + CONV_NT - 1) / CONV_NT;  // staged elements per thread
  static constexpr size_t RING_ELEMS = (size_t)2 * RING * CONV_TW;        // one plane, doubled
  static constexpr size_t SMEM = (2 * RING_ELEMS + (size_t)CONV_CH * XP) * sizeof(T);
};

template <typename T, int R>
__device__ __forceinline__ void conv_segment(const ImageDesc& im, int strip, int s0, int S,
                                             const char* __restrict__ wbase, char* __restrict__ mbase,
                                             char* __restrict__ smem) {
  using G = ConvGeom<T, R>;
  T* ring0 = reinterpret_cast<T*>(smem);
  T* ring1 = ring0 + G::RING_ELEMS;
  T* xin = ring1 + G::RING_ELEMS;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int H = im.H, W = im.W;
  const int v0 = strip * CONV_TW;
  const int seg_end = min(s0 + S, H);
  const int n_out = (seg_end - s0 + CONV_CH - 1) / CONV_CH;
  const int nchunks = G::J0 + n_out;
  const int origin = s0 - R;                 // absolute row of ring row 0
  const int need_end = min(H, seg_end + R);  // row-pass rows at or past this are never read

  const char* wimg = wbase + im.weight_off;
  const int wdtype = im.wdtype;
  const int64_t pitch = im.pitch;
  const double scale = im.scale;

  // ---- taps: g[t], tg[t] for t = 0..R (zero beyond the true radius) ----
  T g[R + 1], tg[R + 1];
  {
    const double k = -0.5 / (im.sigma * im.sigma);
    const double gl = (lane <= im.R) ? exp(k * (double)(lane * lane)) : 0.0;
    const T gT = (T)gl, tgT = (T)((double)lane * gl);
#pragma unroll
    for (int t = 0; t <= R; ++t) {
      g[t] = lane_value(gT, t);
      tg[t] = lane_value(tgT, t);
    }
  }

  // ---- staging of chunk j's input rows into registers ----
  T pre[G::NSTAGE];
  auto fetch = [&](int j) {
#pragma unroll
    for (int e = 0; e < G::NSTAGE; ++e) {
      const int idx = tid + e * CONV_NT;
      T v = (T)0;
      if (idx < CONV_CH * G::XW) {
        const int r = idx / G::XW, c = idx - r * G::XW;
        v = (T)load_weight(wimg, wdtype, pitch, H, W, origin + j * CONV_CH + r, v0 - R + c, scale);
      }
      pre[e] = v;
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int e = 0; e < G::NSTAGE; ++e) {
      const int idx = tid + e * CONV_NT;
      if (idx < CONV_CH * G::XW) {
        const int r = idx / G::XW, c = idx - r * G::XW;
        xin[r * G::XP + c] = pre[e];
      }
    }
  };

  T* Aout = reinterpret_cast<T*>(mbase + im.map_off);
  T* Muout = Aout + (size_t)H * im.map_pitch;
  T* Mvout = Muout + (size_t)H * im.map_pitch;
  double* part = reinterpret_cast<double*>(mbase + im.map_off + im.part_off);

  const int rr = tid >> 4, cg = tid & 15;  // row pass: chunk row, column group of 4

  fetch(0);
  for (int j = 0; j < nchunks; ++j) {
    stage();
    __syncthreads();
    if (j + 1 < nchunks) fetch(j + 1);

    // ---------------- row pass: ring rows of chunk j ----------------
    {
      const int first = origin + j * CONV_CH;
      const int q = (j * CONV_CH) % G::RING + rr;
      T r0[4], r1[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) r0[k] = r1[k] = (T)0;
      if (first + CONV_CH > 0 && first < need_end) {
        const T* xr = xin + rr * G::XP + 4 * cg;
        T x[G::NXL];
#pragma unroll
        for (int i = 0; i < G::NXL; ++i) x[i] = xr[i];
#pragma unroll
        for (int i = 0; i < G::NXL; ++i) {
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int s = k + R - i;  // tap index t = x_out - x_in
            if (s >= -R && s <= R) {
              r0[k] = fma_t(g[s < 0 ? -s : s], x[i], r0[k]);
              if (s > 0) r1[k] = fma_t(tg[s], x[i], r1[k]);
              if (s < 0) r1[k] = fma_t(-tg[-s], x[i], r1[k]);
            }
          }
        }
      }
      T* d0 = ring0 + q * CONV_TW + 4 * cg;
      T* d1 = ring1 + q * CONV_TW + 4 * cg;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        d0[k] = r0[k];
        d0[k + G::RING * CONV_TW] = r0[k];
        d1[k] = r1[k];
        d1[k + G::RING * CONV_TW] = r1[k];
      }
    }
    __syncthreads();

    // ---------------- column pass: output rows of chunk j - J0 ----------------
    if (j >= G::J0) {
      const int ob = (j - G::J0) * CONV_CH;
      const int ofirst = s0 + ob + 4 * wave;
      if (ofirst < seg_end) {
        const int sb = ob % G::RING + 4 * wave;
        const T* p0 = ring0 + sb * CONV_TW + lane;
        const T* p1 = ring1 + sb * CONV_TW + lane;
        T a[4], mu[4], mv[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) a[k] = mu[k] = mv[k] = (T)0;
#pragma unroll
        for (int i = 0; i < G::NXL; ++i) {
          const T y = p0[i * CONV_TW];
          const T z = p1[i * CONV_TW];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int s = k + R - i;
            if (s >= -R && s <= R) {
              const T gs = g[s < 0 ? -s : s];
              a[k] = fma_t(gs, y, a[k]);
              mv[k] = fma_t(gs, z, mv[k]);
              if (s > 0) mu[k] = fma_t(tg[s], y, mu[k]);
              if (s < 0) mu[k] = fma_t(-tg[-s], y, mu[k]);
            }
          }
        }
        const int col = v0 + lane;
        double sx = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int o = ofirst + k;
          if (o < seg_end && col < W) {
            const size_t off = (size_t)o * im.map_pitch + col;
            Aout[off] = a[k];
            Muout[off] = mu[k];
            Mvout[off] = mv[k];
            sx += load_weight(wimg, wdtype, pitch, H, W, o, col, scale) * (double)a[k];
          }
        }
        sx = wave_sum(sx);
        if (lane == 0) part[(size_t)strip * im.ngroups + ofirst / CONV_GROUP] = sx;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// single image: one workgroup per (strip, segment); exact LDS for the class
// ---------------------------------------------------------------------------
template <typename T, int R>
__global__ void __launch_bounds__(CONV_NT) conv_image_kernel(ImageDesc im, int S, const char* wbase,
                                                             char* mbase) {
  __shared__ __align__(16) char smem[ConvGeom<T, R>::SMEM];
  const int strip = blockIdx.x % im.nstrips;
  const int seg = blockIdx.x / im.nstrips;
  conv_segment<T, R>(im, strip, seg * S, S, wbase, mbase, smem);
}

// ---------------------------------------------------------------------------
// batched: persistent workgroups of one radius class walk its tile list
// (cost-sorted by the planner)
// ---------------------------------------------------------------------------
template <typename T, int R>
__global__ void __launch_bounds__(CONV_NT) conv_tiles_kernel(const ImageDesc* __restrict__ images,
                                                             const ConvTile* __restrict__ tiles,
                                                             int ntiles, const char* wbase, char* mbase) {
  __shared__ __align__(16) char smem[ConvGeom<T, R>::SMEM];
  for (int i = blockIdx.x; i < ntiles; i += gridDim.x) {
    const ConvTile t = tiles[i];
    const ImageDesc im = images[t.img];
    conv_segment<T, R>(im, t.strip, t.s0, t.S, wbase, mbase, smem);
    __syncthreads();  // the next tile reuses the shared memory
  }
}

// S_X of one image from its partials (fixed summation order).
template <typename T>
__global__ void __launch_bounds__(256) sx_finalize_kernel(ImageDesc im, const char* mbase, double* s_x) {
  __shared__ double red[4];
  const double* part = reinterpret_cast<const double*>(mbase + im.map_off + im.part_off);
  const double s = block_sum_fixed(part, im.nstrips * im.ngroups, red);
  if (threadIdx.x == 0) *s_x = s;
}

// ---------------------------------------------------------------------------
// host-side launch helpers
// ---------------------------------------------------------------------------
#define ITC_FOR_CLASSES_F32(X) X(2) X(3) X(4) X(6) X(8) X(10) X(12) X(14) X(16) X(18) X(20) X(24) X(28) X(32)
#define ITC_FOR_CLASSES_F64(X) X(2) X(3) X(4) X(6) X(8) X(12) X(16)

// Segment length for a single image: enough workgroups to fill the chip,
// but long enough that the 2R-row warm-up of each segment stays small.
int conv_segment_rows(const ImageDesc& im) {
  const int target = 1024;  // ~4 workgroups per compute unit
  int segs = (target + im.nstrips - 1) / im.nstrips;
  int S = (im.H + segs - 1) / segs;
  const int smin = 4 * im.rclass > 64 ? 4 * im.rclass : 64;
  if (S < smin) S = smin;
  S = (S + CONV_CH - 1) / CONV_CH * CONV_CH;
  return S;
}

hipError_t launch_conv_image(bool f64, const ImageDesc& im, const void* w, void* m, hipStream_t s) {
  const int S = conv_segment_rows(im);
  const dim3 grid(im.nstrips * ((im.H + S - 1) / S));
#define ITC_CASE_F(RR)                                                                           \
  case RR:                                                                                      \
    hipLaunchKernelGGL((conv_image_kernel<float, RR>), grid, dim3(CONV_NT), 0, s, im, S,         \
                       (const char*)w, (char*)m);                                                \
    return hipGetLastError();
#define ITC_CASE_D(RR)                                                                           \
  case RR:                                                                                      \
    hipLaunchKernelGGL((conv_image_kernel<double, RR>), grid, dim3(CONV_NT), 0, s, im, S,        \
                       (const char*)w, (char*)m);                                                \
    return hipGetLastError();
  if (f64) {
    switch (im.rclass) { ITC_FOR_CLASSES_F64(ITC_CASE_D) default: return hipErrorInvalidValue; }
  }
  switch (im.rclass) { ITC_FOR_CLASSES_F32(ITC_CASE_F) default: return hipErrorInvalidValue; }
#undef ITC_CASE_F
#undef ITC_CASE_D
}

hipError_t launch_conv_tiles(bool f64, int rclass, const ImageDesc* d_images, const ConvTile* d_tiles,
                             int ntiles, const void* w, void* m, int grid, hipStream_t s) {
#define ITC_CASE_F(RR)                                                                              \
  case RR:                                                                                         \
    hipLaunchKernelGGL((conv_tiles_kernel<float, RR>), dim3(grid), dim3(CONV_NT), 0, s, d_images,    \
                       d_tiles, ntiles, (const char*)w, (char*)m);                                  \
    return hipGetLastError();
#define ITC_CASE_D(RR)                                                                              \
  case RR:                                                                                         \
    hipLaunchKernelGGL((conv_tiles_kernel<double, RR>), dim3(grid), dim3(CONV_NT), 0, s, d_images,   \
                       d_tiles, ntiles, (const char*)w, (char*)m);                                  \
    return hipGetLastError();
  if (f64) {
    switch (rclass) { ITC_FOR_CLASSES_F64(ITC_CASE_D) default: return hipErrorInvalidValue; }
  }
  switch (rclass) { ITC_FOR_CLASSES_F32(ITC_CASE_F) default: return hipErrorInvalidValue; }
#undef ITC_CASE_F
#undef ITC_CASE_D
}

int conv_tiles_blocks_per_cu(bool f64, int rclass) {
  int nb = 0;
#define ITC_CASE_F(RR)                                                                               \
  case RR:                                                                                          \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, conv_tiles_kernel<float, RR>, CONV_NT, 0) != \
        hipSuccess)                                                                                 \
      return 0;                                                                                     \
    return nb;
#define ITC_CASE_D(RR)                                                                                \
  case RR:                                                                                           \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, conv_tiles_kernel<double, RR>, CONV_NT, 0) != \
        hipSuccess)                                                                                  \
      return 0;                                                                                      \
    return nb;
  if (f64) {
    switch (rclass) { ITC_FOR_CLASSES_F64(ITC_CASE_D) default: return 0; }
  }
  switch (rclass) { ITC_FOR_CLASSES_F32(ITC_CASE_F) default: return 0; }
#undef ITC_CASE_F
#undef ITC_CASE_D
}

hipError_t launch_sx_finalize(bool f64, const ImageDesc& img, const void* maps, double* s_x,
                              hipStream_t s) {
  if (f64)
    hipLaunchKernelGGL(sx_finalize_kernel<double>, dim3(1), dim3(256), 0, s, img, (const char*)maps, s_x);
  else
    hipLaunchKernelGGL(sx_finalize_kernel<float>, dim3(1), dim3(256), 0, s, img, (const char*)maps, s_x);
  return hipGetLastError();
}

}  // namespace itc
