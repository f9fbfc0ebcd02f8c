// Pixel-to-codevector labelling: every pixel of weight > 0 gets the index of
// the nearest codevector (Euclidean; the smaller index on ties), every other
// pixel -1 (the shape segments that a codebook induces, Section 4). The
// squared distance is (u - w_u)^2 + (v - w_v)^2 in FP64 with two rounded
// products and a rounded sum (no fused multiply-add), so the decisions are
// reproducible bit for bit by any IEEE evaluation in the same order.
//
// A workgroup labels tiles of LB_ROWS x LB_COLS pixels, one pixel per thread.
// Per tile it scans only the codevectors that can be nearest to one of its
// pixels: with L_k and U_k the least and the greatest squared distance from
// w_k to the box of the tile's pixel centres, every pixel's nearest distance
// is at most U* = min_k U_k, so a codevector with L_k > U* (1 + 1e-9) is
// farther than the nearest one from every pixel of the tile, by more than any
// rounding of the FP64 distances (a few 2^-53 relative). The others are
// listed in increasing index and scanned with the same arithmetic and the
// same strict comparison as a scan over all codevectors, so the labels,
// ties included, are those of the full scan. Tiles without a pixel of weight
// > 0 skip the list.
#include "itc_device.h"

namespace itc {

namespace {

constexpr int LB_NT = 256;
constexpr int LB_ROWS = 8;
constexpr int LB_COLS = LB_NT / LB_ROWS;  // 32
constexpr double LB_MARGIN = 1.0 + 1e-9;

// Codebook of one image into LDS as FP64 (u, v).
template <typename T>
__device__ __forceinline__ void stage_codebook(const T* w, int M, double2* sw) {
  for (int k = threadIdx.x; k < M; k += blockDim.x) sw[k] = make_double2((double)w[2 * k], (double)w[2 * k + 1]);
}

__device__ __forceinline__ double sq_dist(double u, double v, double2 c) {
  const double du = u - c.x, dv = v - c.y;
  return __dadd_rn(__dmul_rn(du, du), __dmul_rn(dv, dv));
}

// Nearest of the listed codevectors (increasing index; the first on ties).
__device__ __forceinline__ int nearest(double u, double v, const double2* sw, const int32_t* cand, int nc) {
  int bk = cand[0];
  double best = sq_dist(u, v, sw[bk]);
  for (int c = 1; c < nc; ++c) {
    const int k = cand[c];
    const double d = sq_dist(u, v, sw[k]);
    if (d < best) {
      best = d;
      bk = k;
    }
  }
  return bk;
}

struct LabelSmem {
  int32_t* cand;  // [M] candidate list of the current tile
  double* red;    // [LB_NT / 64] per-wave minima
  int32_t* cnt;   // [LB_NT / 64] per-wave candidate counts
};

// Rows r0 .. r0 + n - 1 (n <= LB_ROWS) of one image, tile by tile along the
// row group; each thread's weight of the next tile is loaded while the
// current tile is labelled (pixels outside the image load at an out-of-range
// offset, which reads 0).
template <typename WT>
__device__ __forceinline__ void label_rows_t(const char* x, double scale, int64_t pitch, int H, int W, int r0,
                                             int n, const double2* sw, int M, int32_t* lab, const LabelSmem& sm) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tr = tid / LB_COLS, tc = tid - tr * LB_COLS;
  const rsrc_t xr = make_rsrc(x, (uint32_t)((uint64_t)H * (uint64_t)pitch * sizeof(WT)));
  const int r = r0 + tr;
  const uint32_t rowoff = (uint32_t)((int64_t)r * pitch * (int64_t)sizeof(WT));
  auto fetch = [&](int c0) {
    const int v = c0 + tc;
    const uint32_t bad = (uint32_t)!(tr < n && v < W) << 31;
    return buf_load<WT>(xr, (rowoff + (uint32_t)v * (uint32_t)sizeof(WT)) | bad, 0);
  };
  WT wnext = fetch(0);
  for (int c0 = 0; c0 < W; c0 += LB_COLS) {
    const int v = c0 + tc;
    const bool in = tr < n && v < W;
    const int64_t e = (int64_t)r * pitch + v;
    const WT wcur = wnext;
    wnext = fetch(c0 + LB_COLS);  // past the width: reads 0, unused
    const bool fg = in && (double)wcur * scale > 0.0;
    if (!__syncthreads_or(fg)) {  // uniform: no pixel of the tile is labelled
      if (in) lab[e] = -1;
      continue;
    }
    // box of the tile's pixel centres
    const double ulo = (double)r0, uhi = (double)(r0 + n - 1);
    const double vlo = (double)c0, vhi = (double)(min(c0 + LB_COLS, W) - 1);
    // U* = min_k of the greatest squared distance from w_k to the box
    double umin = 1e300;
    for (int k = tid; k < M; k += LB_NT) {
      const double2 w = sw[k];
      const double du = fmax(fabs(w.x - ulo), fabs(w.x - uhi)), dv = fmax(fabs(w.y - vlo), fabs(w.y - vhi));
      umin = fmin(umin, __dadd_rn(__dmul_rn(du, du), __dmul_rn(dv, dv)));
    }
    umin = wave_min(umin);
    if (lane == 0) sm.red[wave] = umin;
    __syncthreads();
    double ustar = sm.red[0];
#pragma unroll
    for (int w2 = 1; w2 < LB_NT / 64; ++w2) ustar = fmin(ustar, sm.red[w2]);
    const double thr = ustar * LB_MARGIN;
    // candidates in increasing index: L_k <= thr
    int nc = 0;
    for (int k0 = 0; k0 < M; k0 += LB_NT) {  // uniform
      const int k = k0 + tid;
      bool keep = false;
      if (k < M) {
        const double2 w = sw[k];
        const double du = fmax(fmax(ulo - w.x, w.x - uhi), 0.0), dv = fmax(fmax(vlo - w.y, w.y - vhi), 0.0);
        const double lk = __dadd_rn(__dmul_rn(du, du), __dmul_rn(dv, dv));
        // a non-finite codevector 0 starts the full scan's comparisons with a
        // NaN and so wins every pixel there: keep it; other NaNs never win
        keep = lk <= thr || (k == 0 && isnan(lk));
      }
      const uint64_t m = __ballot(keep);
      if (lane == 0) sm.cnt[wave] = (int)__popcll(m);
      __syncthreads();
      int off = nc;
      for (int w2 = 0; w2 < wave; ++w2) off += sm.cnt[w2];
      int tot = nc;
#pragma unroll
      for (int w2 = 0; w2 < LB_NT / 64; ++w2) tot += sm.cnt[w2];
      if (keep) sm.cand[off + (int)__popcll(m & ((1ull << lane) - 1ull))] = k;
      nc = tot;
      __syncthreads();  // cnt is rewritten by the next pass; the list is complete
    }
    if (in) lab[e] = fg ? nearest((double)r, (double)v, sw, sm.cand, nc) : -1;
    __syncthreads();  // the list is rebuilt for the next tile
  }
}

__device__ __forceinline__ void label_rows(const char* x, int wdtype, double scale, int64_t pitch, int H, int W, int r0,
                                           int n, const double2* sw, int M, int32_t* lab, const LabelSmem& sm) {
  if (wdtype == 0)
    label_rows_t<uint8_t>(x, scale, pitch, H, W, r0, n, sw, M, lab, sm);
  else if (wdtype == 1)
    label_rows_t<float>(x, scale, pitch, H, W, r0, n, sw, M, lab, sm);
  else
    label_rows_t<double>(x, scale, pitch, H, W, r0, n, sw, M, lab, sm);
}

template <typename T>
__global__ void __launch_bounds__(LB_NT) label_kernel(const char* x, int wdtype, double scale, int64_t pitch, int H,
                                                      int W, const T* w, int M, int32_t* lab) {
  extern __shared__ double2 sw[];
  __shared__ double red[LB_NT / 64];
  __shared__ int32_t cnt[LB_NT / 64];
  const LabelSmem sm{reinterpret_cast<int32_t*>(sw + M), red, cnt};
  stage_codebook(w, M, sw);
  __syncthreads();
  const int r0 = blockIdx.x * LB_ROWS;
  label_rows(x, wdtype, scale, pitch, H, W, r0, min(LB_ROWS, H - r0), sw, M, lab, sm);
}

__global__ void __launch_bounds__(LB_NT) label_batched_kernel(const ImageDesc* __restrict__ images,
                                                              const ChamferTask* __restrict__ tasks, int ntasks,
                                                              int m_max, const char* x, const float* w,
                                                              int32_t* lab) {
  extern __shared__ double2 sw[];
  __shared__ double red[LB_NT / 64];
  __shared__ int32_t cnt[LB_NT / 64];
  const LabelSmem sm{reinterpret_cast<int32_t*>(sw + m_max), red, cnt};
  int last = -1;
  for (int k = blockIdx.x; k < ntasks; k += gridDim.x) {
    const ChamferTask t = tasks[k];
    const ImageDesc im = images[t.img];
    if (t.img != last) {  // tasks of one image are consecutive: restage only on a change
      __syncthreads();
      stage_codebook(w + 2 * im.w_off, im.M, sw);
      __syncthreads();
      last = t.img;
    }
    const int64_t esz = im.wdtype == 0 ? 1 : (im.wdtype == 1 ? 4 : 8);
    label_rows(x + im.weight_off, im.wdtype, im.scale, im.pitch, im.H, im.W, t.pos, min(LB_ROWS, im.H - t.pos), sw,
               im.M, lab + im.weight_off / esz, sm);
  }
}

}  // namespace

int label_rows_per_task() { return LB_ROWS; }

hipError_t launch_label(bool f64, const ImageDesc& im, const void* x, const void* w, int M, int32_t* lab,
                        hipStream_t s) {
  const dim3 grid((im.H + LB_ROWS - 1) / LB_ROWS);
  const size_t smem = (size_t)M * (sizeof(double2) + sizeof(int32_t));
  if (f64)
    hipLaunchKernelGGL(label_kernel<double>, grid, dim3(LB_NT), smem, s, (const char*)x, im.wdtype, im.scale,
                       im.pitch, im.H, im.W, (const double*)w, M, lab);
  else
    hipLaunchKernelGGL(label_kernel<float>, grid, dim3(LB_NT), smem, s, (const char*)x, im.wdtype, im.scale,
                       im.pitch, im.H, im.W, (const float*)w, M, lab);
  return hipGetLastError();
}

hipError_t launch_label_batched(const ImageDesc* d_images, const ChamferTask* d_tasks, int ntasks, int m_max,
                                const void* x, const void* w, int32_t* lab, int grid, hipStream_t s) {
  hipLaunchKernelGGL(label_batched_kernel, dim3(grid), dim3(LB_NT), (size_t)m_max * (sizeof(double2) + sizeof(int32_t)),
                     s, d_images, d_tasks, ntasks, m_max, (const char*)x, (const float*)w, lab);
  return hipGetLastError();
}

}  // namespace itc
