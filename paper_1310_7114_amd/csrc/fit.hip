// ITC fixed-point iteration on precomputed lattice maps (eq. (4) with the data
// sums read from the convolution maps, Section 3.1; loop of Algorithm 1).
//
// One 256-thread workgroup fits one image. Each codevector k is owned by a
// group of P lanes (P a power of two chosen from M, a template parameter so
// the pair loop unrolls with immediate LDS offsets): the P lanes read the maps
// bilinearly at w_k and split the sum over j of the codebook Gaussian terms,
// which they combine with a fixed cross-lane (DPP) tree. S_XW = sum_k A_k and
// S_W = sum_k C_k are reduced in FP64 in a fixed order, so results are
// bitwise reproducible and identical between the single-image and the
// batched launch.
//
// Precision: codevector positions are FP64 whatever the map type (with FP32
// coordinates the rounding of w, 2.4e-4 px near u = 2048, accumulated over
// the sweeps, would dominate the error). Owners keep their positions in
// registers; LDS holds a copy in the map type, relative to the image centre
// and scaled by s = sqrt(log2(e) / (2 sigma^2)), so that a pair's Gaussian is
// exp2(-|w_j' - w_k'|^2) and its repulsion sum is E = E'/s. Pair differences
// are one subtraction in the map type: in FP32 the rounding of the centred,
// scaled copies (at most half an ulp of s max(H, W) / 2) perturbs a near
// pair's Gaussian by a few 1e-5 relative, far below the data term's effect;
// FP64 keeps FP64 differences. The LDS codebook is padded to a multiple of
// 4P, plus one group of 4P that the pair loop reads ahead, with points at
// 1e30, whose Gaussian is exactly 0.
#include "itc_device.h"

namespace itc {

constexpr int FIT_NT = 256;
constexpr double FIT_FAR = 1e30;
// A byte offset past the end of any maps buffer (< 2 GiB with every plane
// added): buffer loads there return 0 without touching memory.
constexpr uint32_t FIT_OOB = 0x80000000u;

using P2 = V2<double>;

// Per-image status bits (the batched fit's status output).
constexpr int32_t FIT_STATUS_SUMS = 1;  // S_XW or S_W not finite: the fit stopped at the last finite codebook
constexpr int32_t FIT_STATUS_W = 2;     // a codevector step was not finite
constexpr int32_t FIT_STATUS_D = 4;     // D not finite

__device__ __forceinline__ float exp2_neg(float x) { return __builtin_amdgcn_exp2f(-x); }
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ double exp2_neg(double x) { return exp2(-x); }

// Lanes per codevector: the fewest passes the workgroup allows
// (ceil(M / FIT_NT)), then the most lanes per codevector that still fit in
// them. Many images run at once, so total work and registers (each pass
// keeps its own state) matter more than one image's sequential steps.
__host__ __device__ inline int lanes_per_codevector(int M) {
  const int passes = (M + FIT_NT - 1) / FIT_NT;
  int P = 1;
  while (P < 64 && M * (2 * P) <= FIT_NT * passes) P <<= 1;
  return P;
}

__host__ __device__ inline int padded_codebook(int M, int P) { return (M + 4 * P - 1) / (4 * P) * (4 * P); }

struct FitImageArgs {
  const char* mbase;
  const void* w_init;
  void* w_out;
  double s_x;        // S_X of the image (used only for D)
  double* d_trace;   // [iters+1] or null
  double* d_out;     // one double or null
  int32_t* iters_done;
  int32_t* status;   // FIT_STATUS_* bits of this image, or null
  double theta;
  bool write_w;
  void* grad_w;          // gradient mode: dL/dw [M][2] at w_init (no update)
  const double* grad_d;  // dL/dD (one double), gradient mode only
};

template <typename T, int P, int MAXPASS>
__device__ void fit_image(const ImageDesc& im, const FitImageArgs& a, char* smem) {
  constexpr int SLOTS = FIT_NT / P;
  const int M = im.M;
  const int Mpad = padded_codebook(M, P);
  // lane-derived values are recomputed per image: an opaque thread index
  // keeps the compiler from hoisting them out of the persistent image loop,
  // where they would stay live in registers across it
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int lane = tid & 63, wave = tid >> 6;
  const int grp = tid / P, p = tid % P;
  const int npass = (M + SLOTS - 1) / SLOTS;
  using Q2 = V2<T>;
  Q2* Wh = reinterpret_cast<Q2*>(smem);  // centred scaled positions [Mpad + 4P]
  double* red = reinterpret_cast<double*>(smem + (size_t)(Mpad + 4 * P) * sizeof(P2));  // [4 waves][2]
  double* red2 = red + 8;                                                         // [4 waves]

  const double s = sqrt(1.4426950408889634 / (2.0 * im.sigma * im.sigma));
  const double cu = 0.5 * im.H, cv = 0.5 * im.W;  // reference point of the LDS copy
  auto lds_pos = [&](double u, double v) { return Q2{(T)(s * (u - cu)), (T)(s * (v - cv))}; };
  const V2<T>* w_in = reinterpret_cast<const V2<T>*>(a.w_init) + im.w_off;

  // owned codevectors (FP64, in registers; identical in all P lanes of a group)
  double wu[MAXPASS], wv[MAXPASS];
#pragma unroll
  for (int ps = 0; ps < MAXPASS; ++ps) {
    const int k = ps * SLOTS + grp;
    wu[ps] = wv[ps] = 0.0;
    if (ps < npass && k < M) {
      const V2<T> w = w_in[k];
      wu[ps] = (double)w.u;
      wv[ps] = (double)w.v;
    }
  }
  for (int k = tid; k < Mpad + 4 * P; k += FIT_NT) {  // one padded group past Mpad: read ahead
    Q2 h{(T)FIT_FAR, (T)FIT_FAR};
    if (k < M) {
      const V2<T> w = w_in[k];
      h = lds_pos((double)w.u, (double)w.v);
    }
    Wh[k] = h;
  }
  __syncthreads();

  const int H = im.H, W = im.W;
  const uint32_t planeb = (uint32_t)(im.plane * (int64_t)sizeof(T));
  const rsrc_t mres = make_rsrc(a.mbase + im.map_off, 3u * planeb);
  const bool need_d = a.d_trace != nullptr || a.d_out != nullptr || a.status != nullptr;
  // corner values of the cell each owned codevector was last read in (key -2: none yet)
  int cell[MAXPASS];
  T cav[MAXPASS][4], cmu[MAXPASS][4], cmv[MAXPASS][4];
#pragma unroll
  for (int ps = 0; ps < MAXPASS; ++ps) {
    cell[ps] = -2;
#pragma unroll
    for (int c = 0; c < 4; ++c) cav[ps][c] = cmu[ps][c] = cmv[ps][c] = (T)0;
  }
  const Q2* wcol = Wh + p;  // this lane's column of the pair loop: j = p + P t

  bool stop = false;
  int32_t flags = 0;   // status bits (uniform except FIT_STATUS_W, combined at the end)
  int t = 0;
  for (;; ++t) {
    const bool last = (t == im.iters) || stop;
    if (last && !need_d && !a.grad_w) break;

    T Ak[MAXPASS], gu[MAXPASS], gv[MAXPASS], Eu[MAXPASS], Ev[MAXPASS];
    T dAu[MAXPASS], dAv[MAXPASS];  // slope of the bilinear interpolant of A at w_k
    double sxw = 0.0, sw = 0.0;
#pragma unroll
    for (int ps = 0; ps < MAXPASS; ++ps) {
      Ak[ps] = gu[ps] = gv[ps] = Eu[ps] = Ev[ps] = dAu[ps] = dAv[ps] = (T)0;
      if (ps < npass) {
        const int k = ps * SLOTS + grp;
        const bool own = k < M;
        const double uk = wu[ps], vk = wv[ps];
        // ---- data terms: bilinear read of A, M_u, M_v at w_k. The 12 corner
        // values of the lattice cell holding w_k stay in registers until w_k
        // enters another cell (near convergence it rarely does), so the maps
        // are read again only then. The loads are issued here and consumed
        // after the pair loop, which hides their latency. Off-lattice corners
        // load at an offset past the end of the maps, which reads 0.
        T fu = 0, fv = 0;
        {
          const bool inside = own && uk > -1.0 && uk < (double)H && vk > -1.0 && vk < (double)W;
          const double fu0 = inside ? floor(uk) : 0.0, fv0 = inside ? floor(vk) : 0.0;
          const int i0 = (int)fu0, j0 = (int)fv0;
          fu = (T)(uk - fu0);
          fv = (T)(vk - fv0);
          const int key = inside ? (i0 + 1) * (W + 2) + (j0 + 1) : -1;
          if (key != cell[ps]) {
            cell[ps] = key;
            const bool r0 = inside && i0 >= 0, r1 = inside && i0 + 1 < H;
            const bool c0 = j0 >= 0, c1 = j0 + 1 < W;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const int di = c >> 1, dj = c & 1;
              const bool ok = (di ? r1 : r0) && (dj ? c1 : c0);
              const uint32_t off = ok ? (uint32_t)map_index(H, i0 + di, j0 + dj) * (uint32_t)sizeof(T) : FIT_OOB;
              cav[ps][c] = buf_load<T>(mres, off, 0);
              cmu[ps][c] = buf_load<T>(mres, off, planeb);
              cmv[ps][c] = buf_load<T>(mres, off, 2 * planeb);
            }
          }
        }
        const T* av = cav[ps];
        const T* mu = cmu[ps];
        const T* mv = cmv[ps];
        // ---- codebook terms over j = p, p + P, ... (scaled coordinates) ----
        T C = 0, Cu = 0, Cv = 0;
        if (own) {
          const Q2 hk = lds_pos(uk, vk);
          const T hu = hk.u, hv = hk.v;
          // the next group of four is read while this one is evaluated, and
          // even and odd pairs accumulate separately: two independent chains
          T C1 = 0, Cu1 = 0, Cv1 = 0;
          Q2 nx[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) nx[u] = wcol[u * P];
          for (int jt = 0; jt < Mpad; jt += 4 * P) {
            Q2 cur[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              cur[u] = nx[u];
              nx[u] = wcol[jt + 4 * P + u * P];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const T du = cur[u].u - hu, dv = cur[u].v - hv;
              const T e = exp2_neg(fma_t(du, du, dv * dv));
              if (u & 1) {
                C1 += e;
                Cu1 = fma_t(e, du, Cu1);
                Cv1 = fma_t(e, dv, Cv1);
              } else {
                C += e;
                Cu = fma_t(e, du, Cu);
                Cv = fma_t(e, dv, Cv);
              }
            }
          }
          C += C1;
          Cu += Cu1;
          Cv += Cv1;
        }
        C = group_sum<P>(C);
        Cu = group_sum<P>(Cu);
        Cv = group_sum<P>(Cv);
        // bilinear combination: A = sum_c b_c A(c), g = sum_c b_c ((c - w_k) A(c) - M(c))
        T A = 0, Gu = 0, Gv = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int di = c >> 1, dj = c & 1;
          const T b = (di ? fu : (T)1 - fu) * (dj ? fv : (T)1 - fv);
          A = fma_t(b, av[c], A);
          Gu = fma_t(b, fma_t((T)di - fu, av[c], -mu[c]), Gu);
          Gv = fma_t(b, fma_t((T)dj - fv, av[c], -mv[c]), Gv);
        }
        // d/du and d/dv of sum_c b_c A(c): corners c = (di, dj) in (0,0),(0,1),(1,0),(1,1)
        dAu[ps] = ((T)1 - fv) * (av[2] - av[0]) + fv * (av[3] - av[1]);
        dAv[ps] = ((T)1 - fu) * (av[1] - av[0]) + fu * (av[3] - av[2]);
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
    // non-finite sums (non-finite weights or maps) end the fit at this codebook
    const bool sums_ok = isfinite(S_XW) && isfinite(S_W);  // uniform
    const bool final_eval = last || !sums_ok;
    if (!sums_ok) flags |= FIT_STATUS_SUMS;
    if (tid == 0 && (a.d_trace || (final_eval && a.d_out) || a.status)) {
      const double D = log(S_W) + log(a.s_x) - 2.0 * log(S_XW);
      if (!isfinite(D)) flags |= FIT_STATUS_D;
      if (a.d_trace) a.d_trace[t] = D;
      if (final_eval && a.d_out) *a.d_out = D;
    }
    if (a.grad_w) {  // adjoint of D at this codebook (eq. (1) differentiated through the reads)
      const double gd = *a.grad_d;
      const T ca = (T)(-2.0 * gd / S_XW);
      const T cb = (T)(2.0 * gd / (im.sigma * im.sigma * S_W) / s);  // E = E'/s
      V2<T>* gw = reinterpret_cast<V2<T>*>(a.grad_w) + im.w_off;
#pragma unroll
      for (int ps = 0; ps < MAXPASS; ++ps) {
        const int k = ps * SLOTS + grp;
        if (ps < npass && k < M && p == 0)
          gw[k] = V2<T>{fma_t(ca, dAu[ps], cb * Eu[ps]), fma_t(ca, dAv[ps], cb * Ev[ps])};
      }
      break;
    }
    if (final_eval) break;

    // ---- Jacobi update of every owned codevector (all P lanes alike) ----
    // c / s (E = E' / s), in the map type
    T cs;
    if constexpr (sizeof(T) == 4)
      cs = (T)S_XW * recip((T)S_W * (T)s);
    else
      cs = (T)(S_XW / S_W / s);
    float step = 0.0f;
#pragma unroll
    for (int ps = 0; ps < MAXPASS; ++ps) {
      if (ps < npass) {
        const int k = ps * SLOTS + grp;
        if (k < M && Ak[ps] != (T)0) {
          const T inv = recip(Ak[ps]);
          const T du = (gu[ps] - cs * Eu[ps]) * inv;
          const T dv = (gv[ps] - cs * Ev[ps]) * inv;
          if (!isfinite(du) || !isfinite(dv)) flags |= FIT_STATUS_W;
          wu[ps] += (double)du;
          wv[ps] += (double)dv;
          if (a.theta >= 0.0) step = fmaxf(step, (float)sqrt((double)du * du + (double)dv * dv));
          if (p == 0) Wh[k] = lds_pos(wu[ps], wv[ps]);
        }
      }
    }
    if (a.theta >= 0.0) {  // the largest step is needed only for the theta test
      step = wave_max_nonneg(step);
      if (lane == 0) red2[wave] = (double)step;
    }
    __syncthreads();
    if (a.theta >= 0.0) {
      double smax = 0.0;
#pragma unroll
      for (int w = 0; w < FIT_NT / 64; ++w) smax = fmax(smax, red2[w]);
      stop = smax <= a.theta;
    }
  }

  if (a.write_w) {
    V2<T>* w_o = reinterpret_cast<V2<T>*>(a.w_out) + im.w_off;
#pragma unroll
    for (int ps = 0; ps < MAXPASS; ++ps) {
      const int k = ps * SLOTS + grp;
      if (ps < npass && k < M && p == 0) w_o[k] = V2<T>{(T)wu[ps], (T)wv[ps]};
    }
  }
  if (tid == 0 && a.iters_done) *a.iters_done = t;
  if (a.status) {
    const int32_t any_w = __syncthreads_or((flags & FIT_STATUS_W) != 0);
    if (tid == 0) *a.status = (flags & ~FIT_STATUS_W) | (any_w ? FIT_STATUS_W : 0);
  }
  __syncthreads();  // shared memory is reused by the next image
}

// Passes over the owned codevectors an image needs: its codebook occupies
// ceil(M P / FIT_NT) rounds of the workgroup's lanes.
__host__ __device__ inline int fit_passes(int M) {
  const int P = lanes_per_codevector(M);
  return (M * P + FIT_NT - 1) / FIT_NT;
}

// Kernels are compiled for a bound on the passes (1, 2 or 4) so that the
// per-pass registers of codebooks up to 256 codevectors cost nothing for the
// larger ones; the lanes per codevector depend on M alone, so an image gets
// the same arithmetic from every variant.
template <typename T, int MAXPASS>
__device__ __forceinline__ void fit_dispatch(const ImageDesc& im, const FitImageArgs& a, char* smem) {
  switch (lanes_per_codevector(im.M)) {
    case 1: fit_image<T, 1, MAXPASS>(im, a, smem); break;
    case 2: fit_image<T, 2, MAXPASS>(im, a, smem); break;
    case 4: fit_image<T, 4, MAXPASS>(im, a, smem); break;
    case 8: fit_image<T, 8, MAXPASS>(im, a, smem); break;
    case 16: fit_image<T, 16, MAXPASS>(im, a, smem); break;
    case 32: fit_image<T, 32, MAXPASS>(im, a, smem); break;
    default: fit_image<T, 64, MAXPASS>(im, a, smem); break;
  }
}

template <typename T, int MAXPASS>
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
  a.status = nullptr;
  a.theta = fa.theta;
  a.write_w = fa.write_w != 0;
  a.grad_w = fa.grad_w;
  a.grad_d = fa.grad_d;
  fit_dispatch<T, MAXPASS>(im, a, smem);
}

template <typename T, int MAXPASS>
__global__ void __launch_bounds__(FIT_NT) fit_batched_kernel(const ImageDesc* __restrict__ images,
                                                             const int32_t* __restrict__ order, FitArgs fa) {
  extern __shared__ __align__(16) char smem[];
  double* red = reinterpret_cast<double*>(smem);
  for (int ii = blockIdx.x; ii < fa.n; ii += gridDim.x) {
    const int i = order[ii];
    const ImageDesc im = images[i];
    // S_X: the fixed-order sum of the FP64 partials written with the maps
    const double* sxp = reinterpret_cast<const double*>((const char*)fa.maps + im.map_off + im.part_off);
    const double s_x =
        fa.s_x_in ? fa.s_x_in[i] : block_sum_fixed(sxp, (int64_t)im.nstrips * im.nsxg * SX_SLOTS, red);
    if (threadIdx.x == 0 && fa.s_x_out) fa.s_x_out[i] = s_x;
    FitImageArgs a;
    a.mbase = (const char*)fa.maps;
    a.w_init = fa.w_init;
    a.w_out = fa.w_out;
    a.s_x = s_x;
    a.d_trace = nullptr;
    a.d_out = fa.d_out ? fa.d_out + i : nullptr;
    a.iters_done = fa.iters_done ? fa.iters_done + i : nullptr;
    a.status = fa.status ? fa.status + i : nullptr;
    a.theta = fa.theta;
    a.write_w = fa.write_w != 0;
    a.grad_w = fa.grad_w;
    a.grad_d = fa.grad_d ? fa.grad_d + i : nullptr;
    fit_dispatch<T, MAXPASS>(im, a, smem);
  }
}

// Shared memory of the fit for codebooks up to m_max: the padded scaled
// codebook (largest over every P) plus the reduction scratch.
static size_t fit_smem(int m_max) {
  int mp = 0;
  for (int P = 1; P <= 64; P <<= 1) {
    const int need = padded_codebook(m_max, P) + 4 * P;  // plus the read-ahead group
    mp = mp > need ? mp : need;
  }
  return (size_t)mp * sizeof(P2) + 12 * sizeof(double) + 64;
}

int fit_passes_of(int M) { return fit_passes(M); }

static int maxpass_bound(int np) { return np <= 1 ? 1 : (np <= 2 ? 2 : 4); }
static int maxpass_for(int m_max) { return maxpass_bound(fit_passes(m_max)); }

template <typename T, int MP>
static int fit_occupancy(int m_max) {
  int nb = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fit_batched_kernel<T, MP>, FIT_NT, fit_smem(m_max));
  return e == hipSuccess ? nb : 0;
}

int fit_blocks_per_cu(bool f64, int m_max, int max_passes) {
  switch (maxpass_bound(max_passes)) {
    case 1: return f64 ? fit_occupancy<double, 1>(m_max) : fit_occupancy<float, 1>(m_max);
    case 2: return f64 ? fit_occupancy<double, 2>(m_max) : fit_occupancy<float, 2>(m_max);
    default: return f64 ? fit_occupancy<double, 4>(m_max) : fit_occupancy<float, 4>(m_max);
  }
}

template <typename T, int MP>
static void launch_fit_t(const ImageDesc* d_images, const int32_t* d_order, const FitArgs& a, int grid,
                         hipStream_t s, const ImageDesc* h_image) {
  if (h_image)
    hipLaunchKernelGGL((fit_image_kernel<T, MP>), dim3(1), dim3(FIT_NT), fit_smem(h_image->M), s, *h_image, a);
  else
    hipLaunchKernelGGL((fit_batched_kernel<T, MP>), dim3(grid), dim3(FIT_NT), fit_smem(a.m_max), s, d_images,
                       d_order, a);
}

hipError_t launch_fit(bool f64, const ImageDesc* d_images, const int32_t* d_order, const FitArgs& a,
                      int grid, hipStream_t s, const ImageDesc* h_image) {
  // passes are bounded by the largest codebook of the launch (in the
  // gradient-only mode as well, which runs the same per-image code)
  switch (h_image ? maxpass_for(h_image->M) : (a.max_passes > 0 ? maxpass_bound(a.max_passes) : 4)) {
    case 1:
      f64 ? launch_fit_t<double, 1>(d_images, d_order, a, grid, s, h_image)
          : launch_fit_t<float, 1>(d_images, d_order, a, grid, s, h_image);
      break;
    case 2:
      f64 ? launch_fit_t<double, 2>(d_images, d_order, a, grid, s, h_image)
          : launch_fit_t<float, 2>(d_images, d_order, a, grid, s, h_image);
      break;
    default:
      f64 ? launch_fit_t<double, 4>(d_images, d_order, a, grid, s, h_image)
          : launch_fit_t<float, 4>(d_images, d_order, a, grid, s, h_image);
      break;
  }
  return hipGetLastError();
}

}  // namespace itc
