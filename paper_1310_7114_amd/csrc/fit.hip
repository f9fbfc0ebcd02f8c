// ITC fixed-point iteration on precomputed lattice maps (eq. (4) with the data
// sums read from the convolution maps, Section 3.1; loop of Algorithm 1).
//
// One 256-thread workgroup fits one image; the codebook lives in LDS (double
// buffered, Jacobi order). Each codevector k is owned by a group of P lanes
// (P a power of two chosen from M so that the M x M work is spread over the
// workgroup): the P lanes share the bilinear map reads at w_k and split the
// sum over j of the codebook Gaussian terms, which they then combine with a
// fixed xor-shuffle tree. S_XW = sum_k A_k and S_W = sum_k C_k are reduced in
// FP64 in a fixed order, so results are bitwise reproducible and identical
// between the single-image and the batched launch.
//
// Codevector positions are held in FP64 whatever the map type: with FP32
// coordinates the rounding of w (2.4e-4 px at u ~ 2048) and of the pair
// differences w_j - w_k would dominate the error of the iteration. The
// differences and bilinear fractions are formed in FP64 and rounded once to
// the map type, in which the Gaussians and sums are evaluated.
#include "itc_device.h"

namespace itc {

constexpr int FIT_NT = 256;
constexpr int FIT_MAXPASS = ITC_MAX_CODEVECTORS_DEV / FIT_NT;

template <typename T>
struct V2 {
  T u, v;
};

__device__ __forceinline__ float gauss_unit(float d2, float k2) {
  // exp(-d2 / (2 sigma^2)) = 2^(-d2 * k2), k2 = log2(e) / (2 sigma^2)
  return __builtin_amdgcn_exp2f(-d2 * k2);
}
__device__ __forceinline__ double gauss_unit(double d2, double k2) { return exp2(-d2 * k2); }

// Lanes per codevector: minimise passes * ceil(M / P) with at most FIT_MAXPASS passes.
__device__ __forceinline__ int lanes_per_codevector(int M) {
  int bestP = 1, best = 1 << 30;
  for (int P = 1; P <= 64; P <<= 1) {
    const int slots = FIT_NT / P;
    const int passes = (M + slots - 1) / slots;
    if (passes > FIT_MAXPASS) continue;
    const int cost = passes * ((M + P - 1) / P);
    if (cost < best) {
      best = cost;
      bestP = P;
    }
  }
  return bestP;
}

struct FitImageArgs {
  const char* mbase;
  const void* w_init;
  void* w_out;
  double s_x;        // S_X of the image (used only for D)
  double* d_trace;   // [iters+1] or null
  double* d_out;     // one double or null
  int32_t* iters_done;
  double theta;
  bool write_w;
};

template <typename T>
__device__ void fit_image(const ImageDesc& im, const FitImageArgs& a, char* smem) {
  const int M = im.M;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  using P2 = V2<double>;
  P2* Wa = reinterpret_cast<P2*>(smem);
  P2* Wb = Wa + M;
  double* red = reinterpret_cast<double*>(Wb + M);  // [4 waves][2]
  double* red2 = red + 8;                           // [4 waves]

  const V2<T>* w_in = reinterpret_cast<const V2<T>*>(a.w_init) + im.w_off;
  for (int k = tid; k < M; k += FIT_NT) {
    const V2<T> w = w_in[k];
    Wa[k] = P2{(double)w.u, (double)w.v};
  }
  __syncthreads();

  const int H = im.H, W = im.W;
  const int64_t mp = im.map_pitch;
  const T* Ap = reinterpret_cast<const T*>(a.mbase + im.map_off);
  const T* Mup = Ap + (size_t)H * mp;
  const T* Mvp = Mup + (size_t)H * mp;

  const int P = lanes_per_codevector(M);
  const int slots = FIT_NT / P;
  const int npass = (M + slots - 1) / slots;
  const int grp = tid / P, p = tid % P;
  const T k2 = (T)(1.4426950408889634 / (2.0 * im.sigma * im.sigma));
  const bool need_d = a.d_trace != nullptr || a.d_out != nullptr;

  P2* Wc = Wa;
  P2* Wn = Wb;
  bool stop = false;
  int t = 0;
  for (;; ++t) {
    const bool last = (t == im.iters) || stop;
    if (last && !need_d) break;

    T Ak[FIT_MAXPASS], gu[FIT_MAXPASS], gv[FIT_MAXPASS], Eu[FIT_MAXPASS], Ev[FIT_MAXPASS];
    double sxw = 0.0, sw = 0.0;
#pragma unroll
    for (int ps = 0; ps < FIT_MAXPASS; ++ps) {
      Ak[ps] = gu[ps] = gv[ps] = Eu[ps] = Ev[ps] = (T)0;
      if (ps < npass) {
        const int k = ps * slots + grp;
        const bool own = k < M;
        const P2 wk = Wc[own ? k : 0];
        // ---- data terms: bilinear read of A, M_u, M_v at w_k ----
        T A = 0, Gu = 0, Gv = 0;
        if (own && wk.u > -1.0 && wk.u < (double)H && wk.v > -1.0 && wk.v < (double)W) {
          const double fu0 = floor(wk.u), fv0 = floor(wk.v);
          const int i0 = (int)fu0, j0 = (int)fv0;
          const T fu = (T)(wk.u - fu0), fv = (T)(wk.v - fv0);
#pragma unroll
          for (int di = 0; di < 2; ++di) {
#pragma unroll
            for (int dj = 0; dj < 2; ++dj) {
              const int i = i0 + di, j = j0 + dj;
              if (i >= 0 && i < H && j >= 0 && j < W) {
                const T b = (di ? fu : (T)1 - fu) * (dj ? fv : (T)1 - fv);
                const size_t off = (size_t)i * mp + j;
                const T av = Ap[off], mu = Mup[off], mv = Mvp[off];
                A = fma_t(b, av, A);
                // (c - w_k) A(c) - M(c) with c - w_k = (di - fu, dj - fv)
                Gu = fma_t(b, fma_t((T)di - fu, av, -mu), Gu);
                Gv = fma_t(b, fma_t((T)dj - fv, av, -mv), Gv);
              }
            }
          }
        }
        // ---- codebook terms over j = p, p + P, ... ----
        T C = 0, Cu = 0, Cv = 0;
        if (own) {
          for (int j = p; j < M; j += P) {
            const P2 wj = Wc[j];
            const T du = (T)(wj.u - wk.u), dv = (T)(wj.v - wk.v);
            const T e = gauss_unit(fma_t(du, du, dv * dv), k2);
            C += e;
            Cu = fma_t(e, du, Cu);
            Cv = fma_t(e, dv, Cv);
          }
        }
        for (int m = P >> 1; m >= 1; m >>= 1) {
          C += __shfl_xor(C, m, 64);
          Cu += __shfl_xor(Cu, m, 64);
          Cv += __shfl_xor(Cv, m, 64);
        }
        Ak[ps] = A;
        gu[ps] = Gu;
        gv[ps] = Gv;
        Eu[ps] = Cu;
        Ev[ps] = Cv;
        if (own && p == 0) {
          sxw += (double)A;
          sw += (double)C;
        }
      }
    }
    // ---- S_XW, S_W: fixed-order block reduction in FP64 ----
    sxw = wave_sum(sxw);
    sw = wave_sum(sw);
    if (lane == 0) {
      red[2 * wave] = sxw;
      red[2 * wave + 1] = sw;
    }
    __syncthreads();
    double S_XW = 0.0, S_W = 0.0;
#pragma unroll
    for (int w = 0; w < FIT_NT / 64; ++w) {
      S_XW += red[2 * w];
      S_W += red[2 * w + 1];
    }
    if (need_d) {
      const double D = log(S_W) + log(a.s_x) - 2.0 * log(S_XW);
      if (tid == 0) {
        if (a.d_trace) a.d_trace[t] = D;
        if (last && a.d_out) *a.d_out = D;
      }
    }
    if (last) break;

    // ---- Jacobi update of every owned codevector ----
    const T c = (T)(S_XW / S_W);
    float step = 0.0f;
#pragma unroll
    for (int ps = 0; ps < FIT_MAXPASS; ++ps) {
      if (ps < npass) {
        const int k = ps * slots + grp;
        if (k < M && p == 0) {
          P2 w = Wc[k];
          if (Ak[ps] != (T)0) {
            const T du = (gu[ps] - c * Eu[ps]) / Ak[ps];
            const T dv = (gv[ps] - c * Ev[ps]) / Ak[ps];
            w.u += (double)du;
            w.v += (double)dv;
            step = fmaxf(step, (float)sqrt((double)du * du + (double)dv * dv));
          }
          Wn[k] = w;
        }
      }
    }
    step = wave_max(step);
    if (lane == 0) red2[wave] = (double)step;
    __syncthreads();
    double smax = 0.0;
#pragma unroll
    for (int w = 0; w < FIT_NT / 64; ++w) smax = fmax(smax, red2[w]);
    stop = a.theta >= 0.0 && smax <= a.theta;
    P2* tmp = Wc;
    Wc = Wn;
    Wn = tmp;
  }

  if (a.write_w) {
    V2<T>* w_o = reinterpret_cast<V2<T>*>(a.w_out) + im.w_off;
    for (int k = tid; k < M; k += FIT_NT) w_o[k] = V2<T>{(T)Wc[k].u, (T)Wc[k].v};
  }
  if (tid == 0 && a.iters_done) *a.iters_done = t;
  __syncthreads();  // shared memory is reused by the next image
}

template <typename T>
__global__ void __launch_bounds__(FIT_NT) fit_image_kernel(ImageDesc im, FitArgs fa) {
  extern __shared__ __align__(16) char smem[];
  FitImageArgs a;
  a.mbase = (const char*)fa.maps;
  a.w_init = fa.w_init;
  a.w_out = fa.w_out;
  a.s_x = fa.s_x_in ? *fa.s_x_in : 1.0;
  a.d_trace = fa.d_trace;
  a.d_out = fa.d_out;
  a.iters_done = fa.iters_done;
  a.theta = fa.theta;
  a.write_w = fa.write_w != 0;
  fit_image<T>(im, a, smem);
}

template <typename T>
__global__ void __launch_bounds__(FIT_NT) fit_batched_kernel(const ImageDesc* __restrict__ images,
                                                             const int32_t* __restrict__ order, FitArgs fa) {
  extern __shared__ __align__(16) char smem[];
  double* red = reinterpret_cast<double*>(smem);
  for (int ii = blockIdx.x; ii < fa.n; ii += gridDim.x) {
    const int i = order[ii];
    const ImageDesc im = images[i];
    const T* part = reinterpret_cast<const T*>((const char*)fa.maps + im.map_off + im.part_off);
    const double s_x = block_sum_fixed(part, (int64_t)im.nstrips * im.ngroups * CONV_TW, red);
    if (threadIdx.x == 0 && fa.s_x_out) fa.s_x_out[i] = s_x;
    FitImageArgs a;
    a.mbase = (const char*)fa.maps;
    a.w_init = fa.w_init;
    a.w_out = fa.w_out;
    a.s_x = s_x;
    a.d_trace = nullptr;
    a.d_out = fa.d_out ? fa.d_out + i : nullptr;
    a.iters_done = fa.iters_done ? fa.iters_done + i : nullptr;
    a.theta = fa.theta;
    a.write_w = fa.write_w != 0;
    fit_image<T>(im, a, smem);
  }
}

template <typename T>
static size_t fit_smem(int m_max) {
  return (size_t)2 * m_max * sizeof(V2<double>) + 12 * sizeof(double) + 64;
}

int fit_blocks_per_cu(bool f64, int m_max) {
  int nb = 0;
  hipError_t e = f64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fit_batched_kernel<double>, FIT_NT,
                                                                    fit_smem<double>(m_max))
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fit_batched_kernel<float>, FIT_NT,
                                                                    fit_smem<float>(m_max));
  return e == hipSuccess ? nb : 0;
}

hipError_t launch_fit(bool f64, const ImageDesc* d_images, const int32_t* d_order, const FitArgs& a,
                      int grid, hipStream_t s, const ImageDesc* h_image) {
  if (h_image) {
    if (f64)
      hipLaunchKernelGGL(fit_image_kernel<double>, dim3(1), dim3(FIT_NT), fit_smem<double>(h_image->M), s,
                         *h_image, a);
    else
      hipLaunchKernelGGL(fit_image_kernel<float>, dim3(1), dim3(FIT_NT), fit_smem<float>(h_image->M), s,
                         *h_image, a);
    return hipGetLastError();
  }
  if (f64)
    hipLaunchKernelGGL(fit_batched_kernel<double>, dim3(grid), dim3(FIT_NT), fit_smem<double>(a.m_max), s,
                       d_images, d_order, a);
  else
    hipLaunchKernelGGL(fit_batched_kernel<float>, dim3(grid), dim3(FIT_NT), fit_smem<float>(a.m_max), s,
                       d_images, d_order, a);
  return hipGetLastError();
}

}  // namespace itc
