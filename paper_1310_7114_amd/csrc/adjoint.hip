// Adjoint of the lattice divergence with respect to the per-pixel weights
// (Section 5 weights h; eq. (1) with the overlaps of Section 2.1 read from
// the maps):
//
//   dD/dh(y) = 2 A(y) / S_X - (2 / S_XW) K(y),
//   K(y)     = sum_k sum_c beta_kc g(c - y)   (bilinear corners c of w_k, window R)
//
// S_X = sum h A is quadratic in h (its derivative is 2A, the window being
// symmetric); S_XW = sum_k A_bil(w_k) is linear in h and A_bil(w_k) weights
// pixel y by sum_c beta_kc g(c - y). The bilinear weights factorise,
// beta_kc = bu_k(c_u) bv_k(c_v), and so does g, hence
// K(y) = sum_k a_k(y_u) b_k(y_v) with one row factor and one column factor per
// codevector.
//
// A 256-thread workgroup makes 64 x 64 pixel tiles (lane = column, wave w
// rows 16w..16w+15), a contiguous run of them, so it computes S_XW once per
// image of its run (fixed-order FP64 sum: every workgroup gets the same bits).
// Per tile it keeps only the codevectors whose corners reach the tile within R
// (compacted in k order), stages their row and column factors in LDS in
// batches of 64 and accumulates K with one FMA per pixel and codevector.
#include <algorithm>

#include "itc_device.h"

namespace itc {

constexpr int GT = 64;       // tile edge in pixels
constexpr int GNT = 256;     // threads
constexpr int GROWS = GT / (GNT / 64);  // rows per wave
constexpr int GBATCH = 64;   // codevectors per LDS batch

int grad_tiles_of(int H, int W) { return ((H + GT - 1) / GT) * ((W + GT - 1) / GT); }

template <typename T>
struct GradSmem {
  T taps[MAX_RADIUS + 1];
  T fa[GBATCH][GT];  // row factors a_k(u0 + r)
  T fb[GBATCH][GT];  // column factors b_k(v0 + c)
  int32_t list[ITC_MAX_CODEVECTORS_DEV];
  int32_t wave_count[GNT / 64];
  double red[GNT / 64];
};

// S_XW = sum_k A_bil(w_k) of one image: thread t adds k = t, t + GNT, ..., then
// a fixed-order reduction (waves by a DPP tree, then in wave order), so every
// workgroup gets the same bits.
template <typename T>
__device__ double image_sxw(const ImageDesc& im, const GradIArgs& ga, GradSmem<T>& sm) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int H = im.H, W = im.W, M = im.M;
  const T* Ap = reinterpret_cast<const T*>((const char*)ga.maps + im.map_off);
  const V2<T>* wk = reinterpret_cast<const V2<T>*>(ga.w) + im.w_off;
  double sxw = 0.0;
  for (int k = tid; k < M; k += GNT) {
    const double u = (double)wk[k].u, v = (double)wk[k].v;
    if (u > -1.0 && u < (double)H && v > -1.0 && v < (double)W) {
      const double fu0 = floor(u), fv0 = floor(v);
      const int i0 = (int)fu0, j0 = (int)fv0;
      const T fu = (T)(u - fu0), fv = (T)(v - fv0);
      T A = 0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int i = i0 + (c >> 1), j = j0 + (c & 1);
        if (i >= 0 && i < H && j >= 0 && j < W)
          A = fma_t(((c >> 1) ? fu : (T)1 - fu) * ((c & 1) ? fv : (T)1 - fv), Ap[map_index(H, i, j)], A);
      }
      sxw += (double)A;
    }
  }
  sxw = wave_sum(sxw);
  if (lane == 0) sm.red[wave] = sxw;
  __syncthreads();
  double S_XW = 0.0;
#pragma unroll
  for (int w2 = 0; w2 < GNT / 64; ++w2) S_XW += sm.red[w2];
  __syncthreads();  // red is reused
  return S_XW;
}

// dL/dh over one 64 x 64 tile at (u0, v0), given the image's S_XW.
template <typename T>
__device__ void grad_weights_tile(const ImageDesc& im, int u0, int v0, const GradIArgs& ga, double s_x,
                                  double gd, double S_XW, GradSmem<T>& sm) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int H = im.H, W = im.W, R = im.R, M = im.M;
  const T* Ap = reinterpret_cast<const T*>((const char*)ga.maps + im.map_off);
  const V2<T>* wk = reinterpret_cast<const V2<T>*>(ga.w) + im.w_off;

  // A at this lane's pixels, loaded now so that the loads overlap the work below
  const int col = v0 + lane;
  T Ay[GROWS];
#pragma unroll
  for (int r = 0; r < GROWS; ++r) {
    const int row = u0 + wave * GROWS + r;
    Ay[r] = col < W && row < H ? Ap[map_index(H, row, col)] : (T)0;
  }

  // ---- taps g[t], t = 0..R (FP64 exp rounded to the real type, as in the maps) ----
  if (tid <= R) sm.taps[tid] = (T)exp(-0.5 / (im.sigma * im.sigma) * (double)(tid * tid));

  // ---- the codevectors whose corners reach this tile within R, compacted in k order ----
  int nlist = 0;
  for (int base = 0; base < M; base += GNT) {
    const int k = base + tid;
    bool rel = false;
    if (k < M) {
      const double u = (double)wk[k].u, v = (double)wk[k].v;
      if (u > -1.0 && u < (double)H && v > -1.0 && v < (double)W) {
        const int i0 = (int)floor(u), j0 = (int)floor(v);
        rel = i0 - R <= u0 + GT - 1 && i0 + 1 + R >= u0 && j0 - R <= v0 + GT - 1 && j0 + 1 + R >= v0;
      }
    }
    const uint64_t ball = __ballot(rel);
    const int before = __builtin_amdgcn_mbcnt_hi((uint32_t)(ball >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ball, 0));
    if (lane == 0) sm.wave_count[wave] = __popcll(ball);
    __syncthreads();
    int off = nlist;
    for (int w2 = 0; w2 < wave; ++w2) off += sm.wave_count[w2];
    if (rel) sm.list[off + before] = k;
    for (int w2 = 0; w2 < GNT / 64; ++w2) nlist += sm.wave_count[w2];
    __syncthreads();
  }

  // ---- K over the tile, batch by batch of relevant codevectors ----
  T K[GROWS];
#pragma unroll
  for (int r = 0; r < GROWS; ++r) K[r] = (T)0;
  for (int b0 = 0; b0 < nlist; b0 += GBATCH) {
    const int nb = min(GBATCH, nlist - b0);
    for (int idx = tid; idx < nb * 2 * GT; idx += GNT) {
      const int kk = idx / (2 * GT), e = idx % (2 * GT);
      const int k = sm.list[b0 + kk];
      const bool row = e < GT;
      const double x = row ? (double)wk[k].u : (double)wk[k].v;
      const double f0 = floor(x);
      const int c0 = (int)f0;
      const T fr = (T)(x - f0);
      const int y = row ? u0 + e : v0 + e - GT;  // the tile row or column
      const int n = row ? H : W;
      T acc = 0;
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const int c = c0 + d, t = c > y ? c - y : y - c;
        if (c >= 0 && c < n && t <= R) acc = fma_t(d ? fr : (T)1 - fr, sm.taps[t], acc);
      }
      if (row)
        sm.fa[kk][e] = acc;
      else
        sm.fb[kk][e - GT] = acc;
    }
    __syncthreads();
    for (int kk = 0; kk < nb; ++kk) {
      const T bcol = sm.fb[kk][lane];
#pragma unroll
      for (int r = 0; r < GROWS; ++r) K[r] = fma_t(sm.fa[kk][wave * GROWS + r], bcol, K[r]);
    }
    __syncthreads();
  }

  // ---- dL/dh = dL/dD (2 A / S_X - 2 K / S_XW) ----
  const T c1 = (T)(2.0 * gd / s_x), c2 = (T)(-2.0 * gd / S_XW);
  if (col < W) {
    const int esz = im.wdtype == 0 ? 1 : (im.wdtype == 1 ? 4 : 8);
    T* g = reinterpret_cast<T*>(ga.grad_weights) + im.weight_off / esz;
#pragma unroll
    for (int r = 0; r < GROWS; ++r) {
      const int row = u0 + wave * GROWS + r;
      if (row < H) g[(size_t)row * W + col] = fma_t(c1, Ay[r], c2 * K[r]);
    }
  }
}

// Workgroup b takes the contiguous run of tiles [b per, (b + 1) per): the
// runs stay within an image for most of their length, so S_XW is computed
// once per image and run rather than once per tile.
template <typename T>
__global__ void __launch_bounds__(GNT) grad_weights_image_kernel(ImageDesc im, GradIArgs ga, int per) {
  __shared__ GradSmem<T> sm;
  const int ntv = (im.W + GT - 1) / GT, nt = ((im.H + GT - 1) / GT) * ntv;
  const double S_XW = image_sxw<T>(im, ga, sm);
  for (int i = blockIdx.x * per; i < min(nt, ((int)blockIdx.x + 1) * per); ++i) {
    grad_weights_tile<T>(im, (i / ntv) * GT, (i % ntv) * GT, ga, ga.s_x[0], ga.grad_d[0], S_XW, sm);
    __syncthreads();
  }
}

template <typename T>
__global__ void __launch_bounds__(GNT) grad_weights_tiles_kernel(const ImageDesc* __restrict__ images,
                                                                 const GradTile* __restrict__ tiles, int ntiles,
                                                                 int per, GradIArgs ga) {
  __shared__ GradSmem<T> sm;
  int cur = -1;  // image whose S_XW is held
  double S_XW = 0.0;
  for (int i = blockIdx.x * per; i < min(ntiles, ((int)blockIdx.x + 1) * per); ++i) {
    const GradTile t = tiles[i];
    const ImageDesc im = images[t.img];
    if (t.img != cur) {  // uniform
      S_XW = image_sxw<T>(im, ga, sm);
      cur = t.img;
    }
    grad_weights_tile<T>(im, t.u0, t.v0, ga, ga.s_x[t.img], ga.grad_d[t.img], S_XW, sm);
    __syncthreads();
  }
}

hipError_t launch_grad_weights(bool f64, const ImageDesc* d_images, const GradTile* d_tiles, int ntiles,
                               const GradIArgs& a, int grid, hipStream_t s, const ImageDesc* h_image) {
  if (h_image) {
    const int nt = grad_tiles_of(h_image->H, h_image->W);
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
    const int g = std::min(nt, 4 * cus), per = (nt + g - 1) / g;
    if (f64)
      hipLaunchKernelGGL(grad_weights_image_kernel<double>, dim3(g), dim3(GNT), 0, s, *h_image, a, per);
    else
      hipLaunchKernelGGL(grad_weights_image_kernel<float>, dim3(g), dim3(GNT), 0, s, *h_image, a, per);
    return hipGetLastError();
  }
  if (grid < 1 || ntiles < 1) return hipSuccess;
  const int per = (ntiles + grid - 1) / grid;
  if (f64)
    hipLaunchKernelGGL(grad_weights_tiles_kernel<double>, dim3(grid), dim3(GNT), 0, s, d_images, d_tiles, ntiles,
                       per, a);
  else
    hipLaunchKernelGGL(grad_weights_tiles_kernel<float>, dim3(grid), dim3(GNT), 0, s, d_images, d_tiles, ntiles,
                       per, a);
  return hipGetLastError();
}

}  // namespace itc
