// The fixed-point iteration of eq. (4) on the lattice maps (the loop of
// Algorithm 1) for one large image, spread over several workgroups.
//
// One launch per sweep t = 0 .. iters + 1. Workgroup g owns the codevector
// block g (S = 256 / P codevectors, P lanes each). Launch t first completes
// sweep t - 1, identically in every workgroup: it adds the workgroups' FP64
// partials of S_XW and S_W in workgroup order, forms c (and D when a trace is
// asked for), and applies the Jacobi update to every codevector from the
// per-codevector terms of sweep t - 1. It then reads the maps bilinearly at
// its own codevectors of W^t, evaluates their codebook terms against the
// whole codebook (held in LDS, centred and scaled as in the single-workgroup
// fit so that a pair's Gaussian is exp2(-|d'|^2)), and writes the terms and
// its partial sums for launch t + 1. Positions are FP64; positions, terms and
// partials are double buffered by the parity of t.
//
// Stopping: the launch that forms W^t from W^{t-1} compares the largest step
// with theta, and the launch after the final codebook writes w_out, the last
// D and the sweep count, then marks the fit done in a state word; the launches
// after it return at once. The host therefore enqueues all iters + 2 launches
// up front, with no host round trip and no grid-wide barrier, and the whole
// fit can be captured in a HIP graph. Non-finite sums S_XW or S_W end the fit
// at the codebook they were formed at, as in the single-workgroup fit.
#include "itc_device.h"

#ifndef ITC_WIDE_LANES
#define ITC_WIDE_LANES 8
#endif

namespace itc {

namespace {

constexpr int WF_NT = 256;
constexpr double WF_FAR = 1e30;
constexpr uint32_t WF_OOB = 0x80000000u;  // past the end of any maps buffer: loads read 0
constexpr int WF_TERMS = 8;               // floats per codevector: A, g_u, g_v, E'_u, E'_v, C, -, -

struct WideArgs {
  const char* maps;
  const double* s_x;     // needed only with d_trace
  const float* w_init;   // [M][2]
  float* w_out;          // [M][2]
  double* d_trace;       // [iters + 1] or null
  int32_t* iters_done;   // or null
  double theta;
  int32_t iters, M, G;
  double* pos;     // [2][M][2]
  float* terms;    // [2][M][WF_TERMS]
  double* part;    // [2][G][2]: S_XW, S_W of each workgroup
  int32_t* state;  // [0]: sweep count of the final codebook (-1: not known yet); [1]: fit done
};

__host__ __device__ inline int wide_padded(int M, int P) { return (M + 4 * P - 1) / (4 * P) * (4 * P); }

template <int P>
__global__ void __launch_bounds__(WF_NT) fit_wide_kernel(ImageDesc im, WideArgs a, int t) {
  static_assert(P >= 1 && P <= 64 && (P & (P - 1)) == 0, "lanes per codevector: a power of two up to 64");
  extern __shared__ __align__(16) char smem[];
  constexpr int S = WF_NT / P;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int M = a.M, G = a.G;
  const int Mpad = wide_padded(M, P);
  V2<float>* Wh = reinterpret_cast<V2<float>*>(smem);                                  // [Mpad]
  double* red = reinterpret_cast<double*>(smem + (size_t)Mpad * sizeof(V2<float>));    // [8]
  double* wpos = red + 8;                                                              // [M][2]

  const double s = sqrt(1.4426950408889634 / (2.0 * im.sigma * im.sigma));
  const double cu = 0.5 * im.H, cv = 0.5 * im.W;

  // ---- complete sweep t - 1 ----
  if (t == 0) {
    if (blockIdx.x == 0 && tid == 0) {
      a.state[0] = -1;
      a.state[1] = 0;
    }
    for (int k = tid; k < M; k += WF_NT) {
      wpos[2 * k] = (double)a.w_init[2 * k];
      wpos[2 * k + 1] = (double)a.w_init[2 * k + 1];
    }
  } else {
    if (a.state[1]) return;  // an earlier launch ended the fit
    const double* pp = a.part + (size_t)((t - 1) & 1) * G * 2;
    double sxw = 0.0, sw = 0.0;
    for (int g = 0; g < G; ++g) {  // workgroup order, in every thread alike
      sxw += pp[2 * g];
      sw += pp[2 * g + 1];
    }
    if (a.d_trace && blockIdx.x == 0 && tid == 0) a.d_trace[t - 1] = log(sw) + log(*a.s_x) - 2.0 * log(sxw);
    const bool sums_ok = isfinite(sxw) && isfinite(sw);
    // launch t itself may set state[0] (to t), which matters only from launch t + 1 on
    const int final_t = a.state[0];
    const double* pprev = a.pos + (size_t)((t - 1) & 1) * M * 2;
    if (t == a.iters + 1 || t == final_t + 1 || !sums_ok) {  // W^{t-1} is the final codebook
      if (blockIdx.x == 0) {
        for (int k = tid; k < M; k += WF_NT) {
          a.w_out[2 * k] = (float)pprev[2 * k];
          a.w_out[2 * k + 1] = (float)pprev[2 * k + 1];
        }
        if (tid == 0) {
          if (a.iters_done) *a.iters_done = t - 1;
          a.state[1] = 1;
        }
      }
      return;
    }
    const float cs = (float)sxw * __builtin_amdgcn_rcpf((float)sw * (float)s);  // c / s (E = E'/s)
    const float* tp = a.terms + (size_t)((t - 1) & 1) * M * WF_TERMS;
    float step = 0.0f;
    for (int k = tid; k < M; k += WF_NT) {
      double u = pprev[2 * k], v = pprev[2 * k + 1];
      const float A = tp[WF_TERMS * k];
      if (A != 0.0f) {
        const float inv = __builtin_amdgcn_rcpf(A);
        const float du = (tp[WF_TERMS * k + 1] - cs * tp[WF_TERMS * k + 3]) * inv;
        const float dv = (tp[WF_TERMS * k + 2] - cs * tp[WF_TERMS * k + 4]) * inv;
        u += (double)du;
        v += (double)dv;
        step = fmaxf(step, (float)sqrt((double)du * du + (double)dv * dv));
      }
      wpos[2 * k] = u;
      wpos[2 * k + 1] = v;
    }
    if (a.theta >= 0.0) {  // uniform
      step = wave_max_nonneg(step);
      if (lane == 0) red[wave] = (double)step;
      __syncthreads();
      double smax = 0.0;
      for (int w = 0; w < WF_NT / 64; ++w) smax = fmax(smax, red[w]);
      if (smax <= a.theta && blockIdx.x == 0 && tid == 0) a.state[0] = t;  // W^t is final
    }
  }
  __syncthreads();

  // ---- W^t: the owned positions to the work buffer, every position to LDS ----
  double* pcur = a.pos + (size_t)(t & 1) * M * 2;
  for (int k = tid; k < Mpad; k += WF_NT) {
    V2<float> h{(float)WF_FAR, (float)WF_FAR};  // padding: Gaussian exactly 0
    if (k < M) {
      const double u = wpos[2 * k], v = wpos[2 * k + 1];
      h = V2<float>{(float)(s * (u - cu)), (float)(s * (v - cv))};
      if (k / S == (int)blockIdx.x) {
        pcur[2 * k] = u;
        pcur[2 * k + 1] = v;
      }
    }
    Wh[k] = h;
  }
  __syncthreads();

  // ---- terms of the owned codevectors ----
  const int slot = tid / P, p = tid % P;
  const int k = (int)blockIdx.x * S + slot;
  const bool own = k < M;
  const int H = im.H, W = im.W;
  const uint32_t planeb = (uint32_t)(im.plane * (int64_t)sizeof(float));
  const rsrc_t mres = make_rsrc(a.maps + im.map_off, 3u * planeb);
  float av[4] = {0.f, 0.f, 0.f, 0.f}, mu[4] = {0.f, 0.f, 0.f, 0.f}, mv[4] = {0.f, 0.f, 0.f, 0.f};
  float fu = 0.f, fv = 0.f, C = 0.f, Cu = 0.f, Cv = 0.f;
  if (own) {
    const double uk = wpos[2 * k], vk = wpos[2 * k + 1];
    // bilinear corners of the cell holding w_k; off-lattice corners read 0
    const bool inside = uk > -1.0 && uk < (double)H && vk > -1.0 && vk < (double)W;
    const double fu0 = inside ? floor(uk) : 0.0, fv0 = inside ? floor(vk) : 0.0;
    const int i0 = (int)fu0, j0 = (int)fv0;
    fu = (float)(uk - fu0);
    fv = (float)(vk - fv0);
    const bool r0 = inside && i0 >= 0, r1 = inside && i0 + 1 < H;
    const bool c0 = j0 >= 0, c1 = j0 + 1 < W;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int di = c >> 1, dj = c & 1;
      const bool ok = (di ? r1 : r0) && (dj ? c1 : c0);
      const uint32_t off = ok ? (uint32_t)map_index(H, i0 + di, j0 + dj) * (uint32_t)sizeof(float) : WF_OOB;
      av[c] = buf_load<float>(mres, off, 0);
      mu[c] = buf_load<float>(mres, off, planeb);
      mv[c] = buf_load<float>(mres, off, 2 * planeb);
    }
    // codebook terms over j = p, p + P, ...: even and odd groups accumulate apart
    const float hu = (float)(s * (uk - cu)), hv = (float)(s * (vk - cv));
    float C1 = 0.f, Cu1 = 0.f, Cv1 = 0.f;
    for (int jt = 0; jt < Mpad; jt += 4 * P) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const V2<float> q = Wh[jt + u * P + p];
        const float du = q.u - hu, dv = q.v - hv;
        const float e = __builtin_amdgcn_exp2f(-__builtin_fmaf(du, du, dv * dv));
        if (u & 1) {
          C1 += e;
          Cu1 = __builtin_fmaf(e, du, Cu1);
          Cv1 = __builtin_fmaf(e, dv, Cv1);
        } else {
          C += e;
          Cu = __builtin_fmaf(e, du, Cu);
          Cv = __builtin_fmaf(e, dv, Cv);
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
  // A = sum_c b_c A(c), g = sum_c b_c ((c - w_k) A(c) - M(c))
  float A = 0.f, Gu = 0.f, Gv = 0.f;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int di = c >> 1, dj = c & 1;
    const float b = (di ? fu : 1.f - fu) * (dj ? fv : 1.f - fv);
    A = __builtin_fmaf(b, av[c], A);
    Gu = __builtin_fmaf(b, __builtin_fmaf((float)di - fu, av[c], -mu[c]), Gu);
    Gv = __builtin_fmaf(b, __builtin_fmaf((float)dj - fv, av[c], -mv[c]), Gv);
  }
  const bool writer = own && p == 0;
  if (writer) {
    float* tc = a.terms + (size_t)(t & 1) * M * WF_TERMS + (size_t)WF_TERMS * k;
    tc[0] = A;
    tc[1] = Gu;
    tc[2] = Gv;
    tc[3] = Cu;
    tc[4] = Cv;
    tc[5] = C;
  }
  // ---- the workgroup's partials of S_XW and S_W: FP64, fixed order ----
  double sxw = wave_sum(writer ? (double)A : 0.0);
  double sw = wave_sum(writer ? (double)C : 0.0);
  if (lane == 0) {  // red[] was last read before the barrier above
    red[2 * wave] = sxw;
    red[2 * wave + 1] = sw;
  }
  __syncthreads();
  if (tid == 0) {
    double tx = 0.0, tw = 0.0;
    for (int w = 0; w < WF_NT / 64; ++w) {
      tx += red[2 * w];
      tw += red[2 * w + 1];
    }
    double* pc = a.part + (size_t)(t & 1) * G * 2;
    pc[2 * blockIdx.x] = tx;
    pc[2 * blockIdx.x + 1] = tw;
  }
}

}  // namespace

// Lanes per codevector: a pair loop of M / P steps per lane against more
// workgroups, each with the per-launch fixed cost (the update of all M
// codevectors). 8 measured fastest for M = 100 and M = 500 among 4 .. 64.
constexpr int WF_P = ITC_WIDE_LANES;

int fit_wide_groups(int M) { return (M + WF_NT / WF_P - 1) / (WF_NT / WF_P); }

// Work buffer: positions [2][M][2] FP64, terms [2][M][8] FP32, partials
// [2][G][2] FP64, the state word pair.
static size_t wide_pos_bytes(int M) { return 2 * (size_t)M * 2 * sizeof(double); }
static size_t wide_terms_bytes(int M) { return 2 * (size_t)M * WF_TERMS * sizeof(float); }
static size_t wide_part_bytes(int M) { return 2 * (size_t)fit_wide_groups(M) * 2 * sizeof(double); }

size_t fit_wide_work_bytes(int M) {
  const size_t b = wide_pos_bytes(M) + wide_terms_bytes(M) + wide_part_bytes(M) + 2 * sizeof(int32_t);
  return (b + 255) / 256 * 256;
}

size_t fit_wide_smem(int M) {
  return (size_t)wide_padded(M, WF_P) * sizeof(V2<float>) + 8 * sizeof(double) +
         (size_t)M * 2 * sizeof(double);
}

hipError_t launch_fit_wide(const ImageDesc& im, const void* maps, const double* s_x, const float* w_init, int iters,
                           double theta, float* w_out, double* d_trace, int32_t* iters_done, void* work,
                           hipStream_t s) {
  const int M = im.M;
  WideArgs a;
  a.maps = (const char*)maps;
  a.s_x = s_x;
  a.w_init = w_init;
  a.w_out = w_out;
  a.d_trace = d_trace;
  a.iters_done = iters_done;
  a.theta = theta;
  a.iters = iters;
  a.M = M;
  a.G = fit_wide_groups(M);
  char* w = (char*)work;
  a.pos = (double*)w;
  a.terms = (float*)(w + wide_pos_bytes(M));
  a.part = (double*)(w + wide_pos_bytes(M) + wide_terms_bytes(M));
  a.state = (int32_t*)(w + wide_pos_bytes(M) + wide_terms_bytes(M) + wide_part_bytes(M));
  const size_t smem = fit_wide_smem(M);
  const dim3 grid(a.G), block(WF_NT);
  for (int t = 0; t <= iters + 1; ++t) {
    hipLaunchKernelGGL(fit_wide_kernel<WF_P>, grid, block, smem, s, im, a, t);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace itc
