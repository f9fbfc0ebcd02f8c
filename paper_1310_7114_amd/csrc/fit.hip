// ITC fixed-point iteration on precomputed lattice maps (eq. (4) with the data
// sums read from the convolution maps, Section 3.1; loop of Algorithm 1).
//
// One 256-thread workgroup fits one image. Thread t owns codevectors
// k = t, t + 256, ...: it reads the maps bilinearly at w_k, keeps w_k in FP64
// registers and applies its update. The sum over j of the codebook Gaussian
// terms (M^2 pairs per sweep) is spread evenly over the 64 lanes of the four
// waves: the codebook is cut, by the binary digits of M, into chunks of
// 64 / P codevectors (P = 1 for every full 64, then P = 2, 4, .., 64 for the
// remaining powers of two), so that each chunk fills one wave with P lanes
// per codevector; the step sequence of all chunks (a step: one pair per lane)
// is divided into four contiguous equal parts, one per wave. A wave writes
// the P-lane sums (a fixed cross-lane DPP tree) of each chunk it visits to a
// per-(codevector, wave) slot in LDS, and the owner adds the four slots in
// wave order. S_XW = sum_k A_k and S_W = sum_k C_k are reduced in FP64 in a
// fixed order, so results are bitwise reproducible and identical between the
// single-image and the batched launch.
//
// Precision: codevector positions are FP64 whatever the map type (with FP32
// coordinates the rounding of w, 2.4e-4 px near u = 2048, accumulated over
// the sweeps, would dominate the error). LDS holds a copy in the map type,
// relative to the image centre and scaled by s = sqrt(log2(e) / (2 sigma^2)),
// so that a pair's Gaussian is exp2(-|w_j' - w_k'|^2) and its repulsion sum
// is E = E'/s. Pair differences are one subtraction in the map type: in FP32
// the rounding of the centred, scaled copies (at most half an ulp of
// s max(H, W) / 2) perturbs a near pair's Gaussian by a few 1e-5 relative, far
// below the data term's effect; FP64 keeps FP64 differences. The LDS codebook
// is padded with points at 1e30, whose Gaussian is exactly 0.
#include <type_traits>

#include "itc_device.h"

namespace itc {

constexpr int FIT_NT = 256;
constexpr int FIT_WAVES = FIT_NT / 64;
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

// Owner passes: thread t owns k = t + 256 ps for ps < ceil(M / 256).
__host__ __device__ inline int fit_passes(int M) { return (M + FIT_NT - 1) / FIT_NT; }
// LDS codebook entries: the pair loop of a chunk with P lanes per codevector
// reads 4 P ceil(M / 4P) entries, at most 256 ceil(M / 256), and one block
// of 4 P <= 256 past them (read ahead, unused).
__host__ __device__ inline int fit_codebook_len(int M) { return (M + 255) / 256 * 256 + 256; }

// Steps of a chunk with P = 2^lg lanes per codevector, in units of four.
__device__ __forceinline__ int chunk_units(int M, int lg) { return (M + (4 << lg) - 1) / (4 << lg); }

// Sums of the Gaussian terms of one codevector (scaled position hu, hv) over
// this lane's column of the LDS codebook (entries col[0], col[P], ...), in
// blocks of four entries, nun blocks. Two register sets alternate: the reads
// of the next block are issued before the arithmetic of the current one, so
// the LDS latency is hidden behind it (the scheduling barriers keep the
// compiler from sinking the reads). The read after the last block falls in
// the padding of the codebook. Even and odd entries of a block accumulate
// separately: two independent chains.
template <typename T, int P>
__device__ __forceinline__ void pair_blocks(const V2<T>* __restrict__ col, int nun, T hu, T hv, T& C, T& Cu,
                                            T& Cv) {
  T C0 = 0, Cu0 = 0, Cv0 = 0, C1 = 0, Cu1 = 0, Cv1 = 0;
  auto acc = [&](const V2<T>(&x)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const T du = x[i].u - hu, dv = x[i].v - hv;
      const T e = exp2_neg(fma_t(du, du, dv * dv));
      if (i & 1) {
        C1 += e;
        Cu1 = fma_t(e, du, Cu1);
        Cv1 = fma_t(e, dv, Cv1);
      } else {
        C0 += e;
        Cu0 = fma_t(e, du, Cu0);
        Cv0 = fma_t(e, dv, Cv0);
      }
    }
  };
  V2<T> a[4], b[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) a[i] = col[i * P];
  int u = 0;
  for (; u + 2 <= nun; u += 2) {
#pragma unroll
    for (int i = 0; i < 4; ++i) b[i] = col[(u + 1) * 4 * P + i * P];
    __builtin_amdgcn_sched_barrier(0);
    acc(a);
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = col[(u + 2) * 4 * P + i * P];
    __builtin_amdgcn_sched_barrier(0);
    acc(b);
  }
  if (u < nun) acc(a);
  C = C0 + C1;
  Cu = Cu0 + Cu1;
  Cv = Cv0 + Cv1;
}

// Sums over j = p, p + P, .. (steps [u0, u1) in units of four) of the
// Gaussian terms of codevector k, then over the P lanes of each codevector.
template <typename T, int P>
__device__ __forceinline__ void pair_chunk(const V2<T>* __restrict__ Wh, int k, int p, int u0, int u1, T& C, T& Cu,
                                           T& Cv) {
  const V2<T> hk = Wh[k];
  pair_blocks<T, P>(Wh + p + u0 * 4 * P, u1 - u0, hk.u, hk.v, C, Cu, Cv);
  C = group_sum<P>(C);
  Cu = group_sum<P>(Cu);
  Cv = group_sum<P>(Cv);
}

// The codebook's chunks: every full 64 codevectors with P = 1, then the
// remainder r = M mod 64 as at most two chunks: the largest power of two in r
// (P = 64 / that), then the rest, with the most lanes per codevector that fit
// a wave (some lanes idle). Chunk c starting at codevector k0: returns log2 P
// and its size.
__device__ __forceinline__ int chunk_lg(int M, int k0, int& size) {
  const int rem = M - k0;
  if (rem >= 64) {
    size = 64;
    return 0;
  }
  const int hb = 31 - __builtin_clz((unsigned)rem);  // floor(log2 rem)
  const bool first = (M & 63) == rem;                 // the first remainder chunk
  if (first && (rem & (rem - 1))) {
    size = 1 << hb;
    return 6 - hb;
  }
  size = rem;
  return 6 - ((rem & (rem - 1)) ? hb + 1 : hb);
}

// The pair phase of one sweep: wave `wave` walks its share of the chunk steps
// and writes each visited codevector's sums to part[(k * 4 + wave) * 3 + 0..2].
template <typename T>
__device__ __forceinline__ void pair_phase(const V2<T>* __restrict__ Wh, T* __restrict__ part, int M, int wave,
                                           int lane) {
  int units = 0;
  for (int k0 = 0, size = 0; k0 < M; k0 += size) units += chunk_units(M, chunk_lg(M, k0, size));
  const int ua = units * wave / FIT_WAVES, ub = units * (wave + 1) / FIT_WAVES;
  int cu0 = 0, k0 = 0;
  while (k0 < M && cu0 < ub) {  // uniform
    int size = 0;
    const int lg = chunk_lg(M, k0, size);
    const int nu = chunk_units(M, lg);
    const int s0 = ua > cu0 ? ua : cu0, s1 = ub < cu0 + nu ? ub : cu0 + nu;
    if (s0 < s1) {
      const int k = k0 + (lane >> lg), p = lane & ((1 << lg) - 1);
      const int u0 = s0 - cu0, u1 = s1 - cu0;
      T C = 0, Cu = 0, Cv = 0;
      switch (lg) {
        case 0: pair_chunk<T, 1>(Wh, k, p, u0, u1, C, Cu, Cv); break;
        case 1: pair_chunk<T, 2>(Wh, k, p, u0, u1, C, Cu, Cv); break;
        case 2: pair_chunk<T, 4>(Wh, k, p, u0, u1, C, Cu, Cv); break;
        case 3: pair_chunk<T, 8>(Wh, k, p, u0, u1, C, Cu, Cv); break;
        case 4: pair_chunk<T, 16>(Wh, k, p, u0, u1, C, Cu, Cv); break;
        case 5: pair_chunk<T, 32>(Wh, k, p, u0, u1, C, Cu, Cv); break;
        default: pair_chunk<T, 64>(Wh, k, p, u0, u1, C, Cu, Cv); break;
      }
      if (p == 0 && k < k0 + size) {  // lanes past the chunk read padding and are idle
        T* dst = part + ((size_t)k * FIT_WAVES + wave) * 3;
        dst[0] = C;
        dst[1] = Cu;
        dst[2] = Cv;
      }
    }
    cu0 += nu;
    k0 += size;
  }
}

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

template <typename T, int MAXPASS>
__device__ void fit_image(const ImageDesc& im, const FitImageArgs& a, char* smem) {
  const int M = im.M;
  const int WL = fit_codebook_len(M);
  // lane-derived values are recomputed per image: an opaque thread index
  // keeps the compiler from hoisting them out of the persistent image loop,
  // where they would stay live in registers across it
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: the pair phase's loops are scalar
  const int npass = fit_passes(M);
  using Q2 = V2<T>;
  Q2* Wh = reinterpret_cast<Q2*>(smem);  // centred scaled positions [WL]
  T* part = reinterpret_cast<T*>(smem + (size_t)WL * sizeof(P2));  // [M][4 waves][3]
  double* red = reinterpret_cast<double*>(smem + (size_t)WL * sizeof(P2) +
                                          ((size_t)M * FIT_WAVES * 3 * sizeof(T) + 7) / 8 * 8);  // [4 waves][2]
  double* red2 = red + 8;                                                                       // [4 waves]

  const double s = sqrt(1.4426950408889634 / (2.0 * im.sigma * im.sigma));
  const double cu = 0.5 * im.H, cv = 0.5 * im.W;  // reference point of the LDS copy
  auto lds_pos = [&](double u, double v) { return Q2{(T)(s * (u - cu)), (T)(s * (v - cv))}; };
  const V2<T>* w_in = reinterpret_cast<const V2<T>*>(a.w_init) + im.w_off;

  // owned codevectors (FP64, in registers)
  double wu[MAXPASS], wv[MAXPASS];
#pragma unroll
  for (int ps = 0; ps < MAXPASS; ++ps) {
    const int k = ps * FIT_NT + tid;
    wu[ps] = wv[ps] = 0.0;
    if (ps < npass && k < M) {
      const V2<T> w = w_in[k];
      wu[ps] = (double)w.u;
      wv[ps] = (double)w.v;
    }
  }
  for (int k = tid; k < WL; k += FIT_NT) {
    Q2 h{(T)FIT_FAR, (T)FIT_FAR};
    if (k < M) {
      const V2<T> w = w_in[k];
      h = lds_pos((double)w.u, (double)w.v);
    }
    Wh[k] = h;
  }
  // slots no wave writes (a codevector's chunk may span fewer than four waves) stay 0
  for (int i = tid; i < M * FIT_WAVES * 3; i += FIT_NT) part[i] = (T)0;
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

  bool stop = false;
  int32_t flags = 0;   // status bits (uniform except FIT_STATUS_W, combined at the end)
  int t = 0;
  for (;; ++t) {
    const bool last = (t == im.iters) || stop;
    if (last && !need_d && !a.grad_w) break;

    // ---- data terms: bilinear read of A, M_u, M_v at w_k. The 12 corner
    // values of the lattice cell holding w_k stay in registers until w_k
    // enters another cell (near convergence it rarely does), so the maps are
    // read again only then. The loads are issued before the pair phase and
    // consumed after it, which hides their latency. Off-lattice corners load
    // at an offset past the end of the maps, which reads 0.
    T fu[MAXPASS], fv[MAXPASS];
#pragma unroll
    for (int ps = 0; ps < MAXPASS; ++ps) {
      fu[ps] = fv[ps] = (T)0;
      if (ps < npass) {
        const int k = ps * FIT_NT + tid;
        const double uk = wu[ps], vk = wv[ps];
        const bool inside = k < M && uk > -1.0 && uk < (double)H && vk > -1.0 && vk < (double)W;
        const double fu0 = inside ? floor(uk) : 0.0, fv0 = inside ? floor(vk) : 0.0;
        const int i0 = (int)fu0, j0 = (int)fv0;
        fu[ps] = (T)(uk - fu0);
        fv[ps] = (T)(vk - fv0);
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
    }

    // ---- codebook terms of every codevector (scaled coordinates) ----
    pair_phase<T>(Wh, part, M, wave, lane);
    __syncthreads();

    T Ak[MAXPASS], gu[MAXPASS], gv[MAXPASS], Eu[MAXPASS], Ev[MAXPASS];
    T dAu[MAXPASS], dAv[MAXPASS];  // slope of the bilinear interpolant of A at w_k
    double sxw = 0.0, sw = 0.0;
#pragma unroll
    for (int ps = 0; ps < MAXPASS; ++ps) {
      Ak[ps] = gu[ps] = gv[ps] = Eu[ps] = Ev[ps] = dAu[ps] = dAv[ps] = (T)0;
      const int k = ps * FIT_NT + tid;
      if (ps < npass && k < M) {
        // the four waves' sums, in wave order
        const T* src = part + (size_t)k * FIT_WAVES * 3;
        T C = src[0], Cu = src[1], Cv = src[2];
#pragma unroll
        for (int w = 1; w < FIT_WAVES; ++w) {
          C += src[3 * w];
          Cu += src[3 * w + 1];
          Cv += src[3 * w + 2];
        }
        const T* av = cav[ps];
        const T* mu = cmu[ps];
        const T* mv = cmv[ps];
        // bilinear combination: A = sum_c b_c A(c), g = sum_c b_c ((c - w_k) A(c) - M(c))
        const T fuk = fu[ps], fvk = fv[ps];
        T A = 0, Gu = 0, Gv = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int di = c >> 1, dj = c & 1;
          const T b = (di ? fuk : (T)1 - fuk) * (dj ? fvk : (T)1 - fvk);
          A = fma_t(b, av[c], A);
          Gu = fma_t(b, fma_t((T)di - fuk, av[c], -mu[c]), Gu);
          Gv = fma_t(b, fma_t((T)dj - fvk, av[c], -mv[c]), Gv);
        }
        // d/du and d/dv of sum_c b_c A(c): corners c = (di, dj) in (0,0),(0,1),(1,0),(1,1)
        dAu[ps] = ((T)1 - fvk) * (av[2] - av[0]) + fvk * (av[3] - av[1]);
        dAv[ps] = ((T)1 - fuk) * (av[1] - av[0]) + fuk * (av[3] - av[2]);
        Ak[ps] = A;
        gu[ps] = Gu;
        gv[ps] = Gv;
        Eu[ps] = Cu;
        Ev[ps] = Cv;
        sxw += (double)A;
        sw += (double)C;
      }
    }
    // ---- S_XW, S_W: fixed-order block reduction in FP64 ----
    wave_sum2(sxw, sw);
    if (lane == 0) {
      red[2 * wave] = sxw;
      red[2 * wave + 1] = sw;
    }
    __syncthreads();
    double S_XW = 0.0, S_W = 0.0;
#pragma unroll
    for (int w = 0; w < FIT_WAVES; ++w) {
      S_XW += red[2 * w];
      S_W += red[2 * w + 1];
    }
    // non-finite sums (non-finite weights or maps) end the fit at this codebook
    const bool sums_ok = isfinite(S_XW) && isfinite(S_W);  // uniform
    const bool final_eval = last || !sums_ok;
    if (!sums_ok) flags |= FIT_STATUS_SUMS;
    if (tid == 0 && (a.d_trace || (final_eval && (a.d_out || a.status)))) {
      const double D = log(S_W) + log(a.s_x) - 2.0 * log(S_XW);
      if (final_eval && !isfinite(D)) flags |= FIT_STATUS_D;
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
        const int k = ps * FIT_NT + tid;
        if (ps < npass && k < M) gw[k] = V2<T>{fma_t(ca, dAu[ps], cb * Eu[ps]), fma_t(ca, dAv[ps], cb * Ev[ps])};
      }
      break;
    }
    if (final_eval) break;

    // ---- Jacobi update of every owned codevector ----
    // c / s (E = E' / s), in the map type
    T cs;
    if constexpr (sizeof(T) == 4)
      cs = (T)S_XW * recip((T)S_W * (T)s);
    else
      cs = (T)(S_XW / S_W / s);
    float step = 0.0f;
#pragma unroll
    for (int ps = 0; ps < MAXPASS; ++ps) {
      const int k = ps * FIT_NT + tid;
      if (ps < npass && k < M && Ak[ps] != (T)0) {
        const T inv = recip(Ak[ps]);
        const T du = (gu[ps] - cs * Eu[ps]) * inv;
        const T dv = (gv[ps] - cs * Ev[ps]) * inv;
        if (!isfinite(du) || !isfinite(dv)) flags |= FIT_STATUS_W;
        wu[ps] += (double)du;
        wv[ps] += (double)dv;
        if (a.theta >= 0.0) step = fmaxf(step, (float)sqrt((double)du * du + (double)dv * dv));
        Wh[k] = lds_pos(wu[ps], wv[ps]);
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
      for (int w = 0; w < FIT_WAVES; ++w) smax = fmax(smax, red2[w]);
      stop = smax <= a.theta;
    }
  }

  if (a.write_w) {
    V2<T>* w_o = reinterpret_cast<V2<T>*>(a.w_out) + im.w_off;
#pragma unroll
    for (int ps = 0; ps < MAXPASS; ++ps) {
      const int k = ps * FIT_NT + tid;
      if (ps < npass && k < M) w_o[k] = V2<T>{(T)wu[ps], (T)wv[ps]};
    }
  }
  if (tid == 0 && a.iters_done) *a.iters_done = t;
  if (a.status) {
    const int32_t any_w = __syncthreads_or((flags & FIT_STATUS_W) != 0);
    if (tid == 0) *a.status = (flags & ~FIT_STATUS_W) | (any_w ? FIT_STATUS_W : 0);
  }
  __syncthreads();  // shared memory is reused by the next image
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
  fit_image<T, MAXPASS>(im, a, smem);
}

// Waves per SIMD the batched FP32 single-pass fit is compiled for: five
// (96 registers; a few per-image values go to scratch outside the sweep
// loop) rather than the four its 110 registers allow, so five workgroups
// share a compute unit: 3-4 % faster on the 1,400 silhouettes, six 2 %.
template <typename T, int MAXPASS>
constexpr int fit_batched_min_waves() {
  return std::is_same<T, float>::value && MAXPASS == 1 ? 5 : 1;
}

// Workgroup g fits the images sched[G + 1 + sched[g]] .. sched[G + 1 + sched[g + 1] - 1]
// (G workgroups: the first G + 1 entries are the offsets of each workgroup's list).
template <typename T, int MAXPASS>
__global__ void __launch_bounds__(FIT_NT, (fit_batched_min_waves<T, MAXPASS>())) fit_batched_kernel(const ImageDesc* __restrict__ images,
                                                             const int32_t* __restrict__ sched, FitArgs fa) {
  extern __shared__ __align__(16) char smem[];
  double* red = reinterpret_cast<double*>(smem);
  const int32_t* list = sched + gridDim.x + 1;
  const int end = sched[blockIdx.x + 1];
  for (int ii = sched[blockIdx.x]; ii < end; ++ii) {
    const int i = list[ii];
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
    fit_image<T, MAXPASS>(im, a, smem);
  }
}

// Shared memory of the fit for codebooks up to m_max: the padded scaled
// codebook, the per-wave pair sums and the reduction scratch.
static size_t fit_smem(int m_max) {
  return (size_t)fit_codebook_len(m_max) * sizeof(P2) + ((size_t)m_max * FIT_WAVES * 3 * sizeof(double) + 7) / 8 * 8 +
         12 * sizeof(double) + 64;
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
static void launch_fit_t(const ImageDesc* d_images, const int32_t* d_sched, const FitArgs& a, int grid,
                         hipStream_t s, const ImageDesc* h_image) {
  if (h_image)
    hipLaunchKernelGGL((fit_image_kernel<T, MP>), dim3(1), dim3(FIT_NT), fit_smem(h_image->M), s, *h_image, a);
  else
    hipLaunchKernelGGL((fit_batched_kernel<T, MP>), dim3(grid), dim3(FIT_NT), fit_smem(a.m_max), s, d_images,
                       d_sched, a);
}

hipError_t launch_fit(bool f64, const ImageDesc* d_images, const int32_t* d_sched, const FitArgs& a,
                      int grid, hipStream_t s, const ImageDesc* h_image) {
  // passes are bounded by the largest codebook of the launch (in the
  // gradient-only mode as well, which runs the same per-image code)
  switch (h_image ? maxpass_for(h_image->M) : (a.max_passes > 0 ? maxpass_bound(a.max_passes) : 4)) {
    case 1:
      f64 ? launch_fit_t<double, 1>(d_images, d_sched, a, grid, s, h_image)
          : launch_fit_t<float, 1>(d_images, d_sched, a, grid, s, h_image);
      break;
    case 2:
      f64 ? launch_fit_t<double, 2>(d_images, d_sched, a, grid, s, h_image)
          : launch_fit_t<float, 2>(d_images, d_sched, a, grid, s, h_image);
      break;
    default:
      f64 ? launch_fit_t<double, 4>(d_images, d_sched, a, grid, s, h_image)
          : launch_fit_t<float, 4>(d_images, d_sched, a, grid, s, h_image);
      break;
  }
  return hipGetLastError();
}

}  // namespace itc
