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
// Pass 1 (columns): a workgroup of four waves takes a strip of 64 columns,
// one lane per column. Columns of up to 1,024 rows are packed into a bit mask
// in LDS (the waves share the rows), then for every word the first background
// row at or after it and the last at or before it are found, and the four
// waves walk their quarters of the rows writing g. So the image is read once
// and g written once, as 16-bit integers at the start of each row of the
// output (the FP32 row has room for two). Pass 2 (rows): a workgroup stages
// one row of g in LDS and every thread searches outward from its column on
// both sides at once, stopping once a |j - l| reaches the best cost found
// (phi >= a |j - l|). The row of g is in LDS before any T of the row is
// written over it; T values are exact integers, stored as FP32 so that T can
// feed the convolution as a weight image. When every cost fits 16 bits the
// two sides of the search share packed 16-bit registers (one multiply-add per
// term for both), three steps per trip with their LDS reads issued together
// (2.92 -> 2.51 ms for the batch of 1,400 silhouettes; one step per trip 2.78,
// two 2.57, four 3.09: the steps past the stop grow with the trip).
#include "itc_device.h"

namespace itc {

namespace {

constexpr int CH_ROWS_NT = 256;
constexpr int CH_ROWS_PER_TASK = 8;
constexpr int CH_COLS_NT = 256;  // four waves share one strip of 64 columns
constexpr int CH_COLS_WAVES = CH_COLS_NT / 64;
constexpr int CH_WORDS = 32;     // columns of up to 32 CH_WORDS rows take the bit-mask pass
constexpr int CH_GUARD = 4;      // zero columns on each side of the row of g in LDS
#ifndef ITC_CH_STEP
#define ITC_CH_STEP 3
#endif
constexpr int CH_STEP = ITC_CH_STEP;  // search steps per trip of the packed row search
static_assert(CH_STEP >= 1 && CH_STEP <= CH_GUARD, "the steps past the stop stay within the guards");

// Every cost of the row search fits 16 bits: a g + c r and c g + a r with
// g <= H and r <= W + CH_GUARD (the guard columns), and the least found so
// far below a (W + 1).
__device__ __forceinline__ bool chamfer_packed(int H, int W, int a, int b) {
  return (int64_t)(a + b) * (int64_t)(H + W + 2 * CH_GUARD) < 65536;
}

// g of row i (16-bit, at the start of row i of the output)
__device__ __forceinline__ uint16_t* g_row(float* t, int64_t pitch, int i) {
  return reinterpret_cast<uint16_t*>(t + (int64_t)i * pitch);
}

// Pass 1, two walks down and up the column (columns taller than the bit-mask
// pass takes), by the first wave: lane = column.
__device__ __forceinline__ void chamfer_cols_walk(const uint8_t* __restrict__ x, int64_t pitch,
                                                  float* __restrict__ t, int H, int W, int v0) {
  const int j = v0 + (int)(threadIdx.x & 63);
  if (threadIdx.x >= 64 || j >= W) return;
  const uint8_t* xc = x + j;
  int run = 0;  // rows to the nearest background pixel above (row -1 is background)
#pragma unroll 8
  for (int i = 0; i < H; ++i) {
    run = xc[(int64_t)i * pitch] ? run + 1 : 0;
    g_row(t, pitch, i)[j] = (uint16_t)run;
  }
  run = 0;  // and below (row H is background)
#pragma unroll 8
  for (int i = H - 1; i >= 0; --i) {
    run = xc[(int64_t)i * pitch] ? run + 1 : 0;
    uint16_t* gp = g_row(t, pitch, i) + j;
    const int up = *gp;
    *gp = (uint16_t)(up < run ? up : run);
  }
}

// Pass 1 with the bit mask: bit k of word w is row 32 w + k (rows >= H and
// columns >= W are background). LDS: sbits, snext (first background row at or
// after word w, H if none), slast (last background row at or before the end
// of word w, -1 if none), each [CH_WORDS][64].
__device__ __forceinline__ void chamfer_cols_bits(const uint8_t* __restrict__ x, int64_t pitch,
                                                  float* __restrict__ t, int H, int W, int v0,
                                                  uint32_t* __restrict__ sbits, int32_t* __restrict__ snext,
                                                  int32_t* __restrict__ slast) {
  const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
  const int j = v0 + lane;
  const bool col = j < W;
  // byte offsets below 2^31 (the image is smaller than 2 GiB)
  const rsrc_t xr = make_rsrc(x, (uint32_t)((int64_t)H * pitch));
  const int nw = (H + 31) / 32;
  // a word's 32 loads are issued together: rows past the image and columns
  // past the width load at an offset with bit 31 set (beyond the buffer),
  // which reads 0, so no branch makes the compiler wait for each load
  const uint32_t cbad = (uint32_t)!col << 31;
  for (int w = wave; w < nw; w += CH_COLS_WAVES) {
    uint32_t v[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      const int i = 32 * w + k;
      const uint32_t rbad = (uint32_t)(i >= H) << 31;  // uniform
      v[k] = buf_load<uint8_t>(xr, ((uint32_t)i * (uint32_t)pitch + (uint32_t)j) | rbad | cbad, 0);
    }
    uint32_t m = 0u;
#pragma unroll
    for (int k = 0; k < 32; ++k) m |= (v[k] != 0u ? 1u : 0u) << k;
    sbits[w * 64 + lane] = m;
  }
  __syncthreads();
  if (wave == 0) {
    int nxt = H;  // row H is background
    for (int w = nw - 1; w >= 0; --w) {
      const uint32_t inv = ~sbits[w * 64 + lane];
      if (inv) nxt = 32 * w + __builtin_ctz(inv);
      snext[w * 64 + lane] = nxt;
    }
  } else if (wave == 1) {
    int lst = -1;  // row -1 is background
    for (int w = 0; w < nw; ++w) {
      const uint32_t inv = ~sbits[w * 64 + lane];
      if (inv) lst = 32 * w + 31 - __builtin_clz(inv);
      slast[w * 64 + lane] = lst;
    }
  }
  __syncthreads();
  const int w0 = nw * wave / CH_COLS_WAVES, w1 = nw * (wave + 1) / CH_COLS_WAVES;
  if (col) {
    int last = w0 > 0 ? slast[(w0 - 1) * 64 + lane] : -1;
    for (int w = w0; w < w1; ++w) {
      const uint32_t m = sbits[w * 64 + lane];
      const int after = w + 1 < nw ? snext[(w + 1) * 64 + lane] : H;
      const int kn = min(32, H - 32 * w);
      for (int k = 0; k < kn; ++k) {
        const int i = 32 * w + k;
        const uint32_t inv = ~m >> k;  // background rows at or after i within the word
        const int down = inv ? i + __builtin_ctz(inv) : after;
        const int g = min(i - last, down - i);  // 0 on a background row (down == i)
        last = (m >> k) & 1u ? last : i;
        g_row(t, pitch, i)[j] = (uint16_t)g;
      }
    }
  }
  __syncthreads();  // LDS is reused by the next strip
}

typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));

// Pass 2 for rows r0 .. r0 + n - 1, in place; gs: one row of g (LDS). With
// packed set ((a + b)(H + W) < 2^16, so every cost below fits 16 bits) the
// two sides of the search run in the two halves of packed 16-bit registers:
// one multiply-add per term for both sides.
__device__ __forceinline__ void chamfer_rows(float* __restrict__ t, int64_t pitch, int W, int r0, int n, int a,
                                             int b, bool packed, uint16_t* __restrict__ gs) {
  const int c = b - a;
  for (int i = r0; i < r0 + n; ++i) {
    float* tr = t + (int64_t)i * pitch;
    const uint16_t* gr = g_row(t, pitch, i);
    // gs[-CH_GUARD .. -1] and gs[W .. W + CH_GUARD - 1] hold 0: columns
    // outside the image are background
    for (int j = threadIdx.x - CH_GUARD; j < W + CH_GUARD; j += blockDim.x)
      gs[j] = j >= 0 && j < W ? gr[j] : (uint16_t)0;
    __syncthreads();
    if (packed) {  // uniform
      const u16x2 A2 = {(uint16_t)a, (uint16_t)a}, C2 = {(uint16_t)c, (uint16_t)c};
      for (int j = threadIdx.x; j < W; j += blockDim.x) {
        const int b0 = a * min(min(j + 1, W - j), (int)gs[j]);
        u16x2 best = {(uint16_t)b0, (uint16_t)b0};  // least cost found left and right of j
        u16x2 ar = A2, cr = C2;                      // a r and c r at the next r
        int lim = b0;
        // CH_STEP steps per trip, their reads issued together; the steps past
        // the stop cost at least a r >= lim and change nothing, and their reads
        // stay within the guards (r < min(j + 1, W - j) + CH_STEP)
        for (int r = 1; a * r < lim; r += CH_STEP) {
          u16x2 g2[CH_STEP];
#pragma unroll
          for (int q = 0; q < CH_STEP; ++q) g2[q] = u16x2{gs[j - r - q], gs[j + r + q]};
#pragma unroll
          for (int q = 0; q < CH_STEP; ++q) {
            // phi(r, g) = max(a g + c r, c g + a r) on both sides
            best = __builtin_elementwise_min(best, __builtin_elementwise_max(A2 * g2[q] + cr, C2 * g2[q] + ar));
            ar += A2;
            cr += C2;
          }
          lim = min((int)best.x, (int)best.y);
        }
        tr[j] = (float)min((int)best.x, (int)best.y);
      }
      __syncthreads();
      continue;
    }
    for (int j = threadIdx.x; j < W; j += blockDim.x) {
      // columns -1 and W are background, and this column: best <= a (j + 1), a (W - j),
      // so the search below stays inside 0 .. W - 1
      int best = a * min(min(j + 1, W - j), (int)gs[j]);
      for (int r = 1; a * r < best; ++r) {
        // phi(d, g) = a max(d, g) + (b - a) min(d, g) = max(a g + c d, a d + c g)
        const int ar = a * r, cr = c * r;
        const int gl = gs[j - r], gh = gs[j + r];
        best = min(best, max(a * gl + cr, c * gl + ar));
        best = min(best, max(a * gh + cr, c * gh + ar));
      }
      tr[j] = (float)best;
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void cols_task(const uint8_t* x, int64_t pitch, float* t, int H, int W, int v0,
                                          uint32_t* sbits, int32_t* snext, int32_t* slast) {
  if (H <= 32 * CH_WORDS)
    chamfer_cols_bits(x, pitch, t, H, W, v0, sbits, snext, slast);
  else
    chamfer_cols_walk(x, pitch, t, H, W, v0);
}

__global__ void __launch_bounds__(CH_COLS_NT) chamfer_cols_kernel(const uint8_t* x, int64_t pitch, float* t, int H,
                                                                  int W) {
  __shared__ uint32_t sbits[CH_WORDS * 64];
  __shared__ int32_t snext[CH_WORDS * 64];
  __shared__ int32_t slast[CH_WORDS * 64];
  cols_task(x, pitch, t, H, W, blockIdx.x * 64, sbits, snext, slast);
}

__global__ void __launch_bounds__(CH_ROWS_NT) chamfer_rows_kernel(float* t, int64_t pitch, int H, int W, int a,
                                                                  int b) {
  extern __shared__ uint16_t gsh[];
  const int r0 = blockIdx.x * CH_ROWS_PER_TASK;
  uint16_t* gs = gsh + CH_GUARD;
  chamfer_rows(t, pitch, W, r0, min(CH_ROWS_PER_TASK, H - r0), a, b, chamfer_packed(H, W, a, b), gs);
}

__global__ void __launch_bounds__(CH_COLS_NT) chamfer_cols_batched_kernel(const ImageDesc* __restrict__ images,
                                                                          const ChamferTask* __restrict__ tasks,
                                                                          int ntasks, const uint8_t* x, float* t) {
  __shared__ uint32_t sbits[CH_WORDS * 64];
  __shared__ int32_t snext[CH_WORDS * 64];
  __shared__ int32_t slast[CH_WORDS * 64];
  for (int k = blockIdx.x; k < ntasks; k += gridDim.x) {
    const ChamferTask c = tasks[k];
    const ImageDesc im = images[c.img];
    cols_task(x + im.weight_off, im.pitch, t + im.weight_off, im.H, im.W, c.pos * 64, sbits, snext, slast);
  }
}

__global__ void __launch_bounds__(CH_ROWS_NT) chamfer_rows_batched_kernel(const ImageDesc* __restrict__ images,
                                                                          const ChamferTask* __restrict__ tasks,
                                                                          int ntasks, float* t, int a, int b) {
  extern __shared__ uint16_t gsh[];
  uint16_t* gs = gsh + CH_GUARD;
  for (int k = blockIdx.x; k < ntasks; k += gridDim.x) {
    const ChamferTask c = tasks[k];
    const ImageDesc im = images[c.img];
    chamfer_rows(t + im.weight_off, im.pitch, im.W, c.pos, min(CH_ROWS_PER_TASK, im.H - c.pos), a, b,
                 chamfer_packed(im.H, im.W, a, b), gs);
  }
}

}  // namespace

int chamfer_rows_per_task() { return CH_ROWS_PER_TASK; }

hipError_t launch_chamfer(const ImageDesc& im, const void* x, float* t, int a, int b, hipStream_t s) {
  hipLaunchKernelGGL(chamfer_cols_kernel, dim3((im.W + 63) / 64), dim3(CH_COLS_NT), 0, s, (const uint8_t*)x,
                     im.pitch, t, im.H, im.W);
  hipLaunchKernelGGL(chamfer_rows_kernel, dim3((im.H + CH_ROWS_PER_TASK - 1) / CH_ROWS_PER_TASK),
                     dim3(CH_ROWS_NT), (size_t)(im.W + 2 * CH_GUARD) * sizeof(uint16_t), s, t, im.pitch, im.H, im.W, a, b);
  return hipGetLastError();
}

hipError_t launch_chamfer_batched(const ImageDesc* d_images, const ChamferTask* d_cols, int ncols,
                                  const ChamferTask* d_rows, int nrows, int w_max, const void* x, float* t, int a,
                                  int b, int grid_cols, int grid_rows, hipStream_t s) {
  hipLaunchKernelGGL(chamfer_cols_batched_kernel, dim3(grid_cols), dim3(CH_COLS_NT), 0, s, d_images, d_cols, ncols,
                     (const uint8_t*)x, t);
  hipLaunchKernelGGL(chamfer_rows_batched_kernel, dim3(grid_rows), dim3(CH_ROWS_NT),
                     (size_t)(w_max + 2 * CH_GUARD) * sizeof(uint16_t), s, d_images, d_rows, nrows, t, a, b);
  return hipGetLastError();
}

}  // namespace itc
