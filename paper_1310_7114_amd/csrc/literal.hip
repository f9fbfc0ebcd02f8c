// The paper's own accelerated ITC: Algorithm 1 with the update eq. (6).
// P = X * G_xi comes from the convolution kernels (the A plane of the maps
// with sigma = xi). Every sweep then needs, per lattice codevector w_k,
//   a_k = sum_N P F,  b_k = sum_N P F x,  e_k = sum_N Q F,  d_k = sum_N Q F x
// over its window N (|x - w_k| <= R on the lattice, F the sampled G_omega),
// with Q = W * G_omega the codebook's impulse image convolved with the mask,
// and the lattice entropies V(X;W) = sum P Q = sum_k a_k and
// V(W) = sum Q^2 = sum_k e_k (each Q value is a sum of the masks of the
// codevectors whose window holds the pixel). Q is never formed:
//   e_k = sum_j K_u(j, k) K_v(j, k),  d_k = sum_j (K1_u K_v, K_u K1_v)(j, k),
//   K_u(j, k) = sum_u g(u - w_ju) g(u - w_ku),  K1_u = sum_u u g g
// over the lattice rows both windows cover (the lattice is a rectangle, so
// the 2-D overlap factorises). Away from the border K_u depends only on
// |w_ju - w_ku| (a table) and K1_u = (w_ju + w_ku)/2 K_u by symmetry.
// Then c = V(X;W)/V(W), w_k^new = (b_k - c d_k + c e_k w_k)/a_k, rounded to
// the nearest lattice point (halves upward) and clamped into the lattice.
//
// One sweep is two launches: a workgroup per codevector for the four sums
// (FP64 accumulation), then one workgroup for the entropies, D, the update
// and the stopping test. A state word lets the launches after convergence
// return at once, so the host can enqueue every sweep up front.
#include "itc_device.h"

namespace itc {

namespace {

constexpr int LIT_NT = 256;
constexpr int LIT_MAXR = 256;  // largest window radius of G_omega the host accepts

__device__ __forceinline__ double gtap(const double* g, int t) { return g[t < 0 ? -t : t]; }

// 1-D overlap of the windows of two lattice coordinates a, b on [0, n).
__device__ __forceinline__ void overlap1d(int a, int b, int n, int R, const double* g, const double* k1, double& K,
                                          double& K1) {
  const int d = a > b ? a - b : b - a;
  K = 0.0;
  K1 = 0.0;
  if (d > 2 * R) return;
  const int lo = (a > b ? a : b) - R, hi = (a < b ? a : b) + R;
  if (lo >= 0 && hi <= n - 1) {
    K = k1[d];
    K1 = 0.5 * (double)(a + b) * K;
    return;
  }
  const int l = lo < 0 ? 0 : lo, h = hi > n - 1 ? n - 1 : hi;
  for (int u = l; u <= h; ++u) {
    const double t = gtap(g, u - a) * gtap(g, u - b);
    K += t;
    K1 = fma((double)u, t, K1);
  }
}

__global__ void __launch_bounds__(LIT_NT) literal_setup_kernel(LiteralArgs la, const int32_t* w_init,
                                                               int32_t* w) {
  double* g = la.taps;
  double* k1 = la.taps + (la.R + 1);
  const double k2 = -0.5 / (la.omega * la.omega);
  for (int t = threadIdx.x; t <= la.R; t += blockDim.x) g[t] = exp(k2 * (double)(t * t));
  __syncthreads();
  for (int d = threadIdx.x; d <= 2 * la.R; d += blockDim.x) {
    double s = 0.0;
    for (int q = d - la.R; q <= la.R; ++q) s += gtap(g, q) * gtap(g, q - d);
    k1[d] = s;
  }
  for (int k = threadIdx.x; k < la.M; k += blockDim.x) {
    const int u = w_init[2 * k], v = w_init[2 * k + 1];
    w[2 * k] = u < 0 ? 0 : (u > la.H - 1 ? la.H - 1 : u);
    w[2 * k + 1] = v < 0 ? 0 : (v > la.W - 1 ? la.W - 1 : v);
  }
  if (threadIdx.x == 0) {
    *la.state = la.iters == 0 ? 1 : 0;  // 0: sweeping, 1: last D pending, 2: done
    if (la.iters_done) *la.iters_done = 0;
  }
}

// V(X) = sum P^2: block b sums rows 16b .. 16b + 15 in a fixed order.
__global__ void __launch_bounds__(LIT_NT) literal_vx_kernel(LiteralArgs la) {
  __shared__ double red[LIT_NT / 64];
  const int r0 = blockIdx.x * 16, r1 = min(r0 + 16, la.H);
  double s = 0.0;
  const int n = (r1 - r0) * la.W;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int u = r0 + i / la.W, v = i - (i / la.W) * la.W;
    const double p = (double)la.P[map_index(la.H, u, v)];
    s = fma(p, p, s);
  }
  s = block_reduce_fixed(s, red);
  if (threadIdx.x == 0) la.vx_part[blockIdx.x] = s;
}

// The four window sums of codevector k = blockIdx.x, one workgroup: lanes
// along v, the four waves taking every fourth window row, lanes along j for
// the codebook overlaps; each sum is reduced per wave by a fixed DPP tree and
// then over the waves in order.
__global__ void __launch_bounds__(LIT_NT) literal_terms_kernel(LiteralArgs la, const int32_t* __restrict__ w) {
  __shared__ double red[6][LIT_NT / 64];
  __shared__ double tap_s[3 * LIT_MAXR + 2];  // g [R + 1], then the overlaps [2R + 1]
  if (*la.state >= 2) return;
  const int k = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = LIT_NT / 64;
  for (int t = threadIdx.x; t < 3 * la.R + 2; t += LIT_NT) tap_s[t] = la.taps[t];
  __syncthreads();
  const double* g = tap_s;
  const double* k1 = tap_s + (la.R + 1);
  const int wu = w[2 * k], wv = w[2 * k + 1];
  const int R = la.R;
  const int u0 = max(wu - R, 0), u1 = min(wu + R, la.H - 1);
  const int v0 = max(wv - R, 0), v1 = min(wv + R, la.W - 1);
  // data: a, b over the window. A lane takes two columns 64 apart; each step
  // of a wave takes four of its rows, all eight loads issued before use
  // (rows past the window load the last row and weigh 0).
  double a = 0.0, bu = 0.0, bv = 0.0;
  for (int vb = v0; vb <= v1; vb += 128) {
    int vc[2];
    bool okc[2];
    double fv[2], ca[2] = {0.0, 0.0}, cu[2] = {0.0, 0.0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      vc[h] = vb + 64 * h + lane;
      okc[h] = vc[h] <= v1;
      vc[h] = okc[h] ? vc[h] : v1;
      fv[h] = okc[h] ? gtap(g, vc[h] - wv) : 0.0;
    }
    for (int ub = u0 + wave; ub <= u1; ub += 4 * NW) {
      float pv[4][2];
      double gu[4];
      int uu[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int u = ub + r * NW;
        uu[r] = u <= u1 ? u : u1;
        gu[r] = u <= u1 ? gtap(g, u - wu) : 0.0;
        pv[r][0] = la.P[map_index(la.H, uu[r], vc[0])];
        pv[r][1] = la.P[map_index(la.H, uu[r], vc[1])];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const double pf = (double)pv[r][h] * gu[r];
          ca[h] += pf;
          cu[h] = fma((double)uu[r], pf, cu[h]);
        }
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      a = fma(fv[h], ca[h], a);
      bu = fma(fv[h], cu[h], bu);
      bv = fma(fv[h] * (double)vc[h], ca[h], bv);
    }
  }
  // codebook: e, d over the other codevectors' overlapping windows (threads along j)
  double e = 0.0, du = 0.0, dv = 0.0;
  for (int j = threadIdx.x; j < la.M; j += LIT_NT) {
    double Ku, K1u, Kv, K1v;
    overlap1d(w[2 * j], wu, la.H, R, g, k1, Ku, K1u);
    if (Ku == 0.0) continue;
    overlap1d(w[2 * j + 1], wv, la.W, R, g, k1, Kv, K1v);
    e = fma(Ku, Kv, e);
    du = fma(K1u, Kv, du);
    dv = fma(Ku, K1v, dv);
  }
  const double part[6] = {wave_sum(a), wave_sum(bu), wave_sum(bv), wave_sum(e), wave_sum(du), wave_sum(dv)};
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < 6; ++q) red[q][wave] = part[q];
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double s = 0.0;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) s += red[threadIdx.x][ww];
    la.terms[6 * k + threadIdx.x] = s;
  }
}

// Entropies, D of the current codebook, then (unless this was the last D)
// the update of every codevector and the stopping test.
__global__ void __launch_bounds__(LIT_NT) literal_update_kernel(LiteralArgs la, int32_t* w, int sweep) {
  __shared__ double red[LIT_NT / 64];
  __shared__ float redf[LIT_NT / 64];
  const int st = *la.state;
  if (st >= 2) return;
  // sum_k a_k and sum_k e_k in a fixed order
  double sa = 0.0, se = 0.0;
  for (int k = threadIdx.x; k < la.M; k += blockDim.x) {
    sa += la.terms[6 * k];
    se += la.terms[6 * k + 3];
  }
  const double v_xw = block_reduce_fixed(sa, red);
  const double v_w = block_reduce_fixed(se, red);
  const double v_x = block_sum_fixed(la.vx_part, (int64_t)la.nvx, red);
  if (threadIdx.x == 0 && la.d_trace) la.d_trace[sweep] = log(v_w) + log(v_x) - 2.0 * log(v_xw);
  if (st == 1) {
    __syncthreads();
    if (threadIdx.x == 0) *la.state = 2;
    return;
  }
  const double c = v_xw / v_w;
  float step = 0.0f;
  for (int k = threadIdx.x; k < la.M; k += blockDim.x) {
    const double* t = la.terms + 6 * k;
    const double a = t[0];
    if (!(a > 0.0)) continue;
    const int ou = w[2 * k], ov = w[2 * k + 1];
    const double nu = (t[1] - c * t[4] + c * t[3] * (double)ou) / a;
    const double nv = (t[2] - c * t[5] + c * t[3] * (double)ov) / a;
    double ru = floor(nu + 0.5), rv = floor(nv + 0.5);
    ru = ru < 0.0 ? 0.0 : (ru > (double)(la.H - 1) ? (double)(la.H - 1) : ru);
    rv = rv < 0.0 ? 0.0 : (rv > (double)(la.W - 1) ? (double)(la.W - 1) : rv);
    const int iu = (int)ru, iv = (int)rv;
    step = fmaxf(step, sqrtf((float)((iu - ou) * (iu - ou) + (iv - ov) * (iv - ov))));
    w[2 * k] = iu;
    w[2 * k + 1] = iv;
  }
  step = wave_max_nonneg(step);
  if ((threadIdx.x & 63) == 0) redf[threadIdx.x >> 6] = step;
  __syncthreads();
  if (threadIdx.x == 0) {
    float smax = 0.0f;
    for (int q = 0; q < LIT_NT / 64; ++q) smax = fmaxf(smax, redf[q]);
    if (la.iters_done) *la.iters_done = sweep + 1;
    const bool conv = la.theta >= 0.0 && (double)smax <= la.theta;
    *la.state = (conv || sweep + 1 >= la.iters) ? 1 : 0;
  }
}

}  // namespace

hipError_t launch_literal(const LiteralArgs& la, const int32_t* w_init, int32_t* w_out, hipStream_t s) {
  if (la.R < 1 || la.R > LIT_MAXR) return hipErrorInvalidValue;
  hipLaunchKernelGGL(literal_setup_kernel, dim3(1), dim3(LIT_NT), 0, s, la, w_init, w_out);
  hipLaunchKernelGGL(literal_vx_kernel, dim3(la.nvx), dim3(LIT_NT), 0, s, la);
  for (int t = 0; t <= la.iters; ++t) {
    hipLaunchKernelGGL(literal_terms_kernel, dim3(la.M), dim3(LIT_NT), 0, s, la, (const int32_t*)w_out);
    hipLaunchKernelGGL(literal_update_kernel, dim3(1), dim3(LIT_NT), 0, s, la, w_out, t);
  }
  return hipGetLastError();
}

}  // namespace itc

// ---------------------------------------------------------------------------
// Algorithm 1 without a caller work buffer: the work memory is a file-scope
// device array, one per GPU, held until the process ends. Its address on the
// current device is taken with hipGetSymbolAddress at the first call on that
// device (the array's name in host code is not a device address).
// ---------------------------------------------------------------------------
#include <mutex>

namespace itc {
namespace {

constexpr size_t LITERAL_SCRATCH_BYTES = (size_t)ITC_LITERAL_SCRATCH_MIB << 20;
static __device__ __align__(256) unsigned char scratch[LITERAL_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

}  // namespace
}  // namespace itc

extern "C" itc_status itc_lattice_literal_fit_noalloc(const itc_lattice_desc* d, const void* weights, double omega,
                                                      int32_t radius_omega, int32_t M, const int32_t* w_init,
                                                      int32_t iters, double theta, int32_t* w_out, double* d_trace,
                                                      int32_t* iters_done, void* stream) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= itc::MAX_DEVICES)
    return itc::report_error(ITC_E_DEVICE, "no current HIP device");
  void* work = nullptr;
  {
    std::lock_guard<std::mutex> lock(itc::g_scratch_mu);
    if (!itc::g_scratch_ptr[dev]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(itc::scratch));
      if (e != hipSuccess || !p) return itc::report_error(ITC_E_DEVICE, "hipGetSymbolAddress of the scratch array failed");
      itc::g_scratch_ptr[dev] = p;
    }
    work = itc::g_scratch_ptr[dev];
  }
  return itc::literal_fit_with_work(d, weights, omega, radius_omega, M, w_init, iters, theta, w_out, d_trace,
                                    iters_done, work, itc::LITERAL_SCRATCH_BYTES, stream);
}
