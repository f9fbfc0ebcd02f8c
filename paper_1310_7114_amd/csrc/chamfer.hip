// Chamfer distance transform T(X) of a binary lattice image (Section 5: the
// foreground pixels are weighted by a distance transform so that interior
// pixels count more, P = T(X) * G_xi; the paper names Borgefors' chamfer
// transforms). T(p) is the least cost of a path from p to the background on
// the 8-connected lattice, orthogonal steps costing a and diagonal steps b;
// everything outside the H x W lattice is background. Borgefors computes it
// with two sequential raster passes. Here the same values come from two
// data-parallel passes:
//
// * For 1 <= a <= b <= 2a the least path cost to a pixel q is
//     phi(|du|, |dv|) = a max(|du|, |dv|) + (b - a) min(|du|, |dv|)
//   (diagonal steps for the shorter extent, orthogonal for the rest), so
//   T(i, j) = min over background q of phi(|i - q_u|, |j - q_v|).
// * phi is non-decreasing in |du| for a fixed |dv|, so the best background
//   pixel of column l is the one nearest to row i in that column:
//     T(i, j) = min over l of phi(|j - l|, g(i, l)),
//   g(i, l) = rows from (i, l) to the nearest background pixel of column l
//   (rows -1 and H and columns -1 and W are background).
//
// Pass 1 (columns): one thread per column walks down and up the column and
// writes g (columns of up to 1,024 rows are first packed into a bit mask, so
// the image is read once and g written once). Pass 2 (rows): a workgroup stages one row of g in LDS and every
// thread searches outward from its column, stopping once a |j - l| reaches
// the best cost found (phi >= a |j - l|). Values are exact integers, stored
// as FP32 so that T can feed the convolution as a weight image.
#include "itc_device.h"

namespace itc {

namespace {

constexpr int CH_ROWS_NT = 256;
constexpr int CH_ROWS_PER_TASK = 8;

__device__ __forceinline__ int phi(int a, int b, int x, int y) {
  const int mx = x > y ? x : y, mn = x > y ? y : x;
  return a * mx + (b - a) * mn;
}

// Pass 1 for the 64 columns of one strip: lane = column.
__device__ __forceinline__ void chamfer_cols(const uint8_t* __restrict__ x, int64_t pitch, float* __restrict__ t,
                                             int H, int W, int v0) {
  const int j = v0 + (int)(threadIdx.x & 63);
  if (j >= W) return;
  const uint8_t* xc = x + j;
  float* tc = t + j;
  int run = 0;  // rows to the nearest background pixel above (row -1 is background)
#pragma unroll 8
  for (int i = 0; i < H; ++i) {
    run = xc[(int64_t)i * pitch] ? run + 1 : 0;
    tc[(int64_t)i * pitch] = (float)run;
  }
  run = 0;  // and below (row H is background)
#pragma unroll 8
  for (int i = H - 1; i >= 0; --i) {
    run = xc[(int64_t)i * pitch] ? run + 1 : 0;
    const float up = tc[(int64_t)i * pitch];
    tc[(int64_t)i * pitch] = fminf(up, (float)run);
  }
}

// Pass 1 for columns of at most 32 * CH_WORDS rows: the column is read once
// into a bit mask (bit k of word w: row 32w + k is foreground) and the first
// background row at or after each word is found walking the words upwards;
// then one walk down the rows writes g, each row needing only its own word.
// Every LDS word belongs to one lane, so no synchronisation is needed.
constexpr int CH_WORDS = 32;

__device__ __forceinline__ void chamfer_cols_bits(const uint8_t* __restrict__ x, int64_t pitch,
                                                  float* __restrict__ t, int H, int W, int v0,
                                                  uint32_t* __restrict__ sbits, int32_t* __restrict__ snext) {
  const int lane = (int)(threadIdx.x & 63);
  const int j = v0 + lane;
  const bool col = j < W;
  const uint8_t* xc = x + (col ? j : 0);
  const int nw = (H + 31) / 32;
  for (int w = 0; w < nw; ++w) {
    uint32_t m = 0u;
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      const int i = 32 * w + k;
      const bool fg = col && i < H && xc[(int64_t)i * pitch] != 0;
      m |= fg ? 1u << k : 0u;
    }
    sbits[w * 64 + lane] = m;  // rows >= H stay background
  }
  int nxt = H;  // row H is background
  for (int w = nw - 1; w >= 0; --w) {
    const uint32_t inv = ~sbits[w * 64 + lane];
    if (inv) nxt = 32 * w + __builtin_ctz(inv);
    snext[w * 64 + lane] = nxt;
  }
  if (!col) return;
  float* tc = t + j;
  int last = -1;  // row -1 is background
  for (int w = 0; w < nw; ++w) {
    const uint32_t m = sbits[w * 64 + lane];
    const int after = w + 1 < nw ? snext[(w + 1) * 64 + lane] : H;
    const int kn = min(32, H - 32 * w);
    for (int k = 0; k < kn; ++k) {
      const int i = 32 * w + k;
      int g = 0;
      if ((m >> k) & 1u) {
        const uint32_t inv = ~m >> k;  // background rows at or after i within the word
        const int down = inv ? i + __builtin_ctz(inv) : after;
        g = min(i - last, down - i);
      } else {
        last = i;
      }
      tc[(int64_t)i * pitch] = (float)g;
    }
  }
}

// Pass 2 for rows r0 .. r0 + n - 1 (in place: a row of g is staged in LDS
// before any of its T values is written).
__device__ __forceinline__ void chamfer_rows(float* __restrict__ t, int64_t pitch, int W, int r0, int n, int a,
                                             int b, float* __restrict__ gs) {
  for (int i = r0; i < r0 + n; ++i) {
    float* tr = t + (int64_t)i * pitch;
    for (int j = threadIdx.x; j < W; j += blockDim.x) gs[j] = tr[j];
    __syncthreads();
    for (int j = threadIdx.x; j < W; j += blockDim.x) {
      const int gj = (int)gs[j];
      int best = a * min(j + 1, W - j);  // columns -1 and W are background
      best = min(best, a * gj);          // this column
      for (int r = 1; a * r < best; ++r) {
        if (j - r >= 0) best = min(best, phi(a, b, r, (int)gs[j - r]));
        if (j + r < W) best = min(best, phi(a, b, r, (int)gs[j + r]));
      }
      tr[j] = (float)best;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(64) chamfer_cols_kernel(const uint8_t* x, int64_t pitch, float* t, int H, int W) {
  __shared__ uint32_t sbits[CH_WORDS * 64];
  __shared__ int32_t snext[CH_WORDS * 64];
  if (H <= 32 * CH_WORDS)
    chamfer_cols_bits(x, pitch, t, H, W, blockIdx.x * 64, sbits, snext);
  else
    chamfer_cols(x, pitch, t, H, W, blockIdx.x * 64);
}

__global__ void __launch_bounds__(CH_ROWS_NT) chamfer_rows_kernel(float* t, int64_t pitch, int H, int W, int a,
                                                                  int b) {
  extern __shared__ float gs[];
  const int r0 = blockIdx.x * CH_ROWS_PER_TASK;
  chamfer_rows(t, pitch, W, r0, min(CH_ROWS_PER_TASK, H - r0), a, b, gs);
}

__global__ void __launch_bounds__(64) chamfer_cols_batched_kernel(const ImageDesc* __restrict__ images,
                                                                  const ChamferTask* __restrict__ tasks, int ntasks,
                                                                  const uint8_t* x, float* t) {
  __shared__ uint32_t sbits[CH_WORDS * 64];
  __shared__ int32_t snext[CH_WORDS * 64];
  for (int k = blockIdx.x; k < ntasks; k += gridDim.x) {
    const ChamferTask c = tasks[k];
    const ImageDesc im = images[c.img];
    if (im.H <= 32 * CH_WORDS)
      chamfer_cols_bits(x + im.weight_off, im.pitch, t + im.weight_off, im.H, im.W, c.pos * 64, sbits, snext);
    else
      chamfer_cols(x + im.weight_off, im.pitch, t + im.weight_off, im.H, im.W, c.pos * 64);
  }
}

__global__ void __launch_bounds__(CH_ROWS_NT) chamfer_rows_batched_kernel(const ImageDesc* __restrict__ images,
                                                                          const ChamferTask* __restrict__ tasks,
                                                                          int ntasks, float* t, int a, int b) {
  extern __shared__ float gs[];
  for (int k = blockIdx.x; k < ntasks; k += gridDim.x) {
    const ChamferTask c = tasks[k];
    const ImageDesc im = images[c.img];
    chamfer_rows(t + im.weight_off, im.pitch, im.W, c.pos, min(CH_ROWS_PER_TASK, im.H - c.pos), a, b, gs);
  }
}

}  // namespace

int chamfer_rows_per_task() { return CH_ROWS_PER_TASK; }

hipError_t launch_chamfer(const ImageDesc& im, const void* x, float* t, int a, int b, hipStream_t s) {
  hipLaunchKernelGGL(chamfer_cols_kernel, dim3((im.W + 63) / 64), dim3(64), 0, s, (const uint8_t*)x, im.pitch, t,
                     im.H, im.W);
  hipLaunchKernelGGL(chamfer_rows_kernel, dim3((im.H + CH_ROWS_PER_TASK - 1) / CH_ROWS_PER_TASK),
                     dim3(CH_ROWS_NT), (size_t)im.W * sizeof(float), s, t, im.pitch, im.H, im.W, a, b);
  return hipGetLastError();
}

hipError_t launch_chamfer_batched(const ImageDesc* d_images, const ChamferTask* d_cols, int ncols,
                                  const ChamferTask* d_rows, int nrows, int w_max, const void* x, float* t, int a,
                                  int b, int grid_cols, int grid_rows, hipStream_t s) {
  hipLaunchKernelGGL(chamfer_cols_batched_kernel, dim3(grid_cols), dim3(64), 0, s, d_images, d_cols, ncols,
                     (const uint8_t*)x, t);
  hipLaunchKernelGGL(chamfer_rows_batched_kernel, dim3(grid_rows), dim3(CH_ROWS_NT), (size_t)w_max * sizeof(float),
                     s, d_images, d_rows, nrows, t, a, b);
  return hipGetLastError();
}

}  // namespace itc
