// Pixel-to-codevector labelling: every pixel of weight > 0 gets the index of
// the nearest codevector (Euclidean; the smaller index on ties), every other
// pixel -1 (the shape segments that a codebook induces, Section 4). The
// squared distance is (u - w_u)^2 + (v - w_v)^2 in FP64 with two rounded
// products and a rounded sum (no fused multiply-add), so the decisions are
// reproducible bit for bit by any IEEE evaluation in the same order.
#include "itc_device.h"

namespace itc {

namespace {

constexpr int LB_NT = 256;
constexpr int LB_ROWS = 8;

template <typename WT>
__device__ __forceinline__ double stored_weight(const char* p, int64_t i) {
  return (double)reinterpret_cast<const WT*>(p)[i];
}

__device__ __forceinline__ double stored_at(const char* p, int wdtype, int64_t i) {
  return wdtype == 0 ? stored_weight<uint8_t>(p, i)
                     : (wdtype == 1 ? stored_weight<float>(p, i) : stored_weight<double>(p, i));
}

// Codebook of one image into LDS as FP64 (u, v).
template <typename T>
__device__ __forceinline__ void stage_codebook(const T* w, int M, double2* sw) {
  for (int k = threadIdx.x; k < M; k += blockDim.x) sw[k] = make_double2((double)w[2 * k], (double)w[2 * k + 1]);
}

__device__ __forceinline__ int nearest(double u, double v, const double2* sw, int M) {
  double best = __dadd_rn(__dmul_rn(u - sw[0].x, u - sw[0].x), __dmul_rn(v - sw[0].y, v - sw[0].y));
  int bk = 0;
  for (int k = 1; k < M; ++k) {
    const double du = u - sw[k].x, dv = v - sw[k].y;
    const double d = __dadd_rn(__dmul_rn(du, du), __dmul_rn(dv, dv));
    if (d < best) {
      best = d;
      bk = k;
    }
  }
  return bk;
}

__device__ __forceinline__ void label_rows(const char* x, int wdtype, double scale, int64_t pitch, int W, int r0,
                                           int n, const double2* sw, int M, int32_t* lab) {
  const int64_t base = (int64_t)r0 * pitch;
  const int cnt = n * W;
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    const int r = i / W, v = i - r * W;
    const int64_t e = base + (int64_t)r * pitch + v;
    const bool fg = stored_at(x, wdtype, e) * scale > 0.0;
    lab[e] = fg ? nearest((double)(r0 + r), (double)v, sw, M) : -1;
  }
}

template <typename T>
__global__ void __launch_bounds__(LB_NT) label_kernel(const char* x, int wdtype, double scale, int64_t pitch, int H,
                                                      int W, const T* w, int M, int32_t* lab) {
  extern __shared__ double2 sw[];
  stage_codebook(w, M, sw);
  __syncthreads();
  const int r0 = blockIdx.x * LB_ROWS;
  label_rows(x, wdtype, scale, pitch, W, r0, min(LB_ROWS, H - r0), sw, M, lab);
}

__global__ void __launch_bounds__(LB_NT) label_batched_kernel(const ImageDesc* __restrict__ images,
                                                              const ChamferTask* __restrict__ tasks, int ntasks,
                                                              const char* x, const float* w, int32_t* lab) {
  extern __shared__ double2 sw[];
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
    label_rows(x + im.weight_off, im.wdtype, im.scale, im.pitch, im.W, t.pos, min(LB_ROWS, im.H - t.pos), sw,
               im.M, lab + im.weight_off / esz);
  }
}

}  // namespace

int label_rows_per_task() { return LB_ROWS; }

hipError_t launch_label(bool f64, const ImageDesc& im, const void* x, const void* w, int M, int32_t* lab,
                        hipStream_t s) {
  const dim3 grid((im.H + LB_ROWS - 1) / LB_ROWS);
  const size_t smem = (size_t)M * sizeof(double2);
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
  hipLaunchKernelGGL(label_batched_kernel, dim3(grid), dim3(LB_NT), (size_t)m_max * sizeof(double2), s, d_images,
                     d_tasks, ntasks, (const char*)x, (const float*)w, lab);
  return hipGetLastError();
}

}  // namespace itc
