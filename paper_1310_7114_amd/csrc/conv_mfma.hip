// Separable Gaussian convolution maps on the matrix cores, for 8-bit lattice
// weights and FP32 maps (Section 3.1: the Parzen sum of delta impulses is the
// weight image convolved with a Gaussian, whose mask factorises into 1-D
// masks). The maps are the same as the VALU kernel's:
//   A = (I *_v g) *_u g,   M_u = (I *_v g) *_u tg,   M_v = (I *_v tg) *_u g,
// with f(t) the tap at t = x_out - x_in, plus the S_X partials.
//
// Each 1-D pass is a banded Toeplitz product. Sixteen outputs along an axis
// are a 16 x K window of inputs times the K x 16 matrix T[k][n] = f(n + RA - k)
// (RA the radius rounded up to 8, f zero past the true radius), evaluated
// with v_mfma_f32_16x16x32_f16 and FP32 accumulation. FP32 accuracy comes
// from splitting operands into two FP16 parts:
//   - taps: 2^8 f(t) = hi + lo to about 2^-22 relative (the 2^8 keeps lo
//     normal for the smallest taps);
//   - row pass: the stored weights 0..255 are exact in FP16, so
//     R0 = X (g_hi + g_lo) and R1 = X (tg_hi + tg_lo) are exact products
//     summed in FP32;
//   - column pass: R0 and R1, scaled by a power of two into FP16 range, are
//     split y = y_hi + y_lo, and every map is the sum of the four products
//     T_a y_b, accumulated as a hi chain and a lo chain.
// The relative error of a map is a few 2^-22 against an FP32 direct sum's
// 2^-24 per operation.
//
// Work decomposition: a workgroup of four waves owns a strip of 64 columns
// and a segment of rows and streams down it in chunks of 16 rows. Wave w owns
// columns 16w..16w+15 in both passes, so the ring that carries row-pass
// results to the column pass is private to the wave (LDS operations of one
// wave complete in order: no barrier). Per chunk:
//   1. staging (shared): the chunk's 16 input rows with their column halo
//      are converted to FP16 into one of two LDS buffers; their global loads
//      were issued one chunk earlier. One barrier per chunk.
//   2. row pass: K/32 A-fragments (16 rows x 32 columns) times the tap
//      fragments -> R0, R1 for 16 rows x 16 columns; scaled, split and
//      written to the ring (column-major: rows contiguous, so the column
//      pass reads 8 consecutive rows per lane in one 16-byte load).
//   3. column pass, 2RA rows behind: ring fragments (K rows x 16 columns)
//      times the same tap fragments (as the A operand) -> A, M_u, M_v for 16
//      rows x 16 columns, stored coalesced along rows, and h*A summed into
//      the S_X partial of each 8-row group.
#include <type_traits>

#include "itc_device.h"

namespace itc {

namespace {

typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef _Float16 h4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

constexpr int MX_NT = 256;  // four waves; wave w owns strip columns 16w..16w+15
constexpr int MX_CH = 16;   // rows per chunk

template <int RA>
struct MxGeom {
  static_assert(RA % 8 == 0 && RA >= 8 && RA <= 32, "aligned radius");
  static constexpr int K = (16 + 2 * RA + 31) / 32 * 32;  // window of one 16-output product
  static constexpr int KS = K / 32;                         // MFMA k-steps per product
  static constexpr int J0 = 2 * RA / MX_CH;                 // chunks before the first column pass
  static constexpr int NB = J0 + 1;                         // ring blocks of 16 rows
  // Pitches in halves, chosen so that 16 lanes reading 16 bytes at one row
  // (or column) offset each hit 4 distinct banks: pitch/2 = 4 * odd dwords.
  static constexpr int RINGP = NB * MX_CH + 8;   // ring column pitch
  static constexpr int SW = 48 + K;              // staged columns (image columns v0 - RA + c)
  static constexpr int SWP = SW + 8;             // staged row pitch
  static constexpr int CC = (SW + 63) / 64;      // staged columns per lane and row
  static constexpr size_t STAGE = (size_t)MX_CH * SWP;     // halves per staging buffer
  static constexpr size_t RINGA = (size_t)CONV_TW * RINGP;  // halves per ring array
  static constexpr int RINGB = NB * MX_CH + 4;                // h byte ring column pitch (bytes)
  static constexpr size_t SMEM = (2 * STAGE + 4 * RINGA) * sizeof(_Float16) + (size_t)CONV_TW * RINGB;
  static_assert(RINGP / 2 % 8 == 4 && SWP / 2 % 8 == 4, "bank-spread pitches");
  static_assert(NB * MX_CH >= MX_CH + 2 * RA, "ring holds a column window");
  static_assert(RINGB / 4 % 2 == 1, "bank-spread byte ring");
static constexpr int MINW = (int)((160 * 1024) / SMEM) < 8 ? (int)((160 * 1024) / SMEM) : 8;
};

__device__ __forceinline__ f4_t mfma(h8_t a, h8_t b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// Split of an FP32 value into FP16 hi + lo (|x - hi - lo| <= 2^-22 |x| for
// normal parts).
struct Split16 {
  _Float16 hi, lo;
};
__device__ __forceinline__ Split16 split16(float x) {
  const _Float16 hi = (_Float16)x;
  return Split16{hi, (_Float16)(x - (float)hi)};
}

template <int RA>
__device__ __forceinline__ void mx_segment(const ImageDesc& im, int strip, int s0, int S,
                                           const char* __restrict__ wbase, char* __restrict__ mbase,
                                           _Float16* __restrict__ smem) {
  using G = MxGeom<RA>;
  _Float16* stage = smem;                  // [2][16][SWP]
  _Float16* ring = smem + 2 * G::STAGE;    // [4][64][RINGP]: R0 hi, R0 lo, R1 hi, R1 lo
  uint8_t* hring = reinterpret_cast<uint8_t*>(ring + 4 * G::RINGA);  // [64][RINGB]: stored weights

  // lane-derived values are recomputed per segment: an opaque thread index
  // keeps the compiler from hoisting them out of the persistent tile loop,
  // where they would stay live in registers across it
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n = lane & 15, q = lane >> 4;
  const int H = im.H, W = im.W;
  const int v0 = strip * CONV_TW;
  const int seg_end = min(s0 + S, H);
  const int n_out = (seg_end - s0 + MX_CH - 1) / MX_CH;
  const int nchunks = G::J0 + n_out;
  const int origin = s0 - RA;  // image row of row 0 of chunk 0

  const uint32_t rowbytes = (uint32_t)im.pitch;  // 8-bit weights
  const rsrc_t wres = make_rsrc(wbase + im.weight_off, (uint32_t)H * rowbytes);
  const rsrc_t mres = make_rsrc(mbase + im.map_off, (uint32_t)(im.part_off + (int64_t)im.nstrips * im.ngroups *
                                                                             CONV_TW * sizeof(float)));

  // ---- tap fragments: element e of lane (n, q), k-step s holds 2^8 f(t), t = n + RA - (32s + 8q + e) ----
  h8_t g_hi[G::KS], g_lo[G::KS], t_hi[G::KS], t_lo[G::KS];
  float sc1;  // row-pass outputs are scaled by sc1 = 2^-e1 into FP16 range
  float fac;  // column-pass outputs to maps
  {
    const double k2 = -0.5 / (im.sigma * im.sigma);
    const double gl = lane <= im.R ? exp(k2 * (double)(lane * lane)) : 0.0;
    // |R0|, |R1| <= 255 * 2^8 * max(sum_t g, sum_t |t| g) for 8-bit weights
    const double sg = wave_sum(lane == 0 ? gl : 2.0 * gl);
    const double stg = wave_sum(2.0 * (double)lane * gl);
    double bound = 255.0 * 256.0 * (sg > stg ? sg : stg);
    int e1 = 0;
    while (bound > 32768.0) {
      bound *= 0.5;
      ++e1;
    }
    sc1 = __builtin_ldexpf(1.0f, -e1);
#pragma unroll
    for (int s = 0; s < G::KS; ++s) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int t = n + RA - (32 * s + 8 * q + e);
        const double gv = __shfl(gl, t < 0 ? -t : t);  // |t| <= 63; zero past the radius
        float gs = (float)(256.0 * gv), ts = (float)(256.0 * (double)t * gv);
        asm volatile("" : "+v"(gs), "+v"(ts));  // split the FP32 value (no fused f64 -> f16 rounding)
        const Split16 a = split16(gs), b = split16(ts);
        g_hi[s][e] = a.hi;
        g_lo[s][e] = a.lo;
        t_hi[s][e] = b.hi;
        t_lo[s][e] = b.lo;
      }
    }
    fac = (float)(im.scale * __builtin_ldexp(1.0, e1 - 16));  // undoes the 2^8 taps twice and sc1
  }

  // ---- staging: wave w loads rows 4w..4w+3 of a chunk, staged columns lane + 64c ----
  // Lanes past the staged width or outside the image load at an offset past
  // the end of the buffer: the hardware returns 0 without a memory request.
  uint32_t xoff[G::CC];
#pragma unroll
  for (int c = 0; c < G::CC; ++c) {
    const int sc = lane + 64 * c, x = v0 - RA + sc;
    xoff[c] = sc < G::SW && x >= 0 && x < W ? (uint32_t)x : 0x80000000u;
  }
  // Loads are unconditional and rows outside the image are masked at staging
  // time, a chunk later, so that nothing waits on them in between.
  // Two chunks are in flight: set P = j & 1 holds chunk j from two chunks
  // before it is staged (P is a template constant so the sets stay in
  // registers), which leaves the loads two chunks of work to arrive.
  uint32_t pre[2][4][G::CC];
  uint32_t ymask[2] = {0u, 0u};  // bit r: fetched row 4w + r lies inside the image (uniform)
  auto fetch = [&](int j, auto P) {
    constexpr int p = decltype(P)::value;
    ymask[p] = 0u;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int y = origin + j * MX_CH + 4 * wave + r;  // uniform
      const bool yin = y >= 0 && y < H;
      ymask[p] |= yin ? 1u << r : 0u;
      const uint32_t soff = yin ? (uint32_t)y * rowbytes : 0u;
#pragma unroll
      for (int c = 0; c < G::CC; ++c) pre[p][r][c] = buf_load<uint8_t>(wres, xoff[c], soff);
    }
  };
  auto stage_chunk = [&](int j, auto P) {
    constexpr int p = decltype(P)::value;
    _Float16* xs = stage + p * G::STAGE + (4 * wave) * G::SWP + lane;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const bool yin = (ymask[p] >> r) & 1u;
#pragma unroll
      for (int c = 0; c < G::CC; ++c) {
        const uint32_t v = yin ? pre[p][r][c] : 0u;
        if (64 * c + 64 <= G::SW || lane + 64 * c < G::SW) xs[r * G::SWP + 64 * c] = (_Float16)(uint16_t)v;
      }
    }
  };

  const uint32_t mpb = (uint32_t)(im.map_pitch * sizeof(float));  // bytes per map row
  const uint32_t planeb = (uint32_t)H * mpb;
  // one descriptor per plane: the three maps share a byte offset
  const char* mimg = mbase + im.map_off;
  const rsrc_t resA = make_rsrc(mimg, planeb), resU = make_rsrc(mimg + planeb, planeb),
               resV = make_rsrc(mimg + 2 * (size_t)planeb, planeb);
  const int col = v0 + 16 * wave + n;  // this lane's output column (inside the padded pitch)
  const bool col_ok = col < W;
  const uint32_t part_base = (uint32_t)im.part_off + (uint32_t)((int64_t)strip * im.ngroups * CONV_TW * sizeof(float));
  const float hscale = (float)im.scale;
  _Float16* ring_col = ring + (size_t)(16 * wave + n) * G::RINGP;

  // Map stores are unconditional: a row outside the segment gets a byte
  // offset past the end of its plane, which the hardware discards (the
  // offset plus three rows stays below 2^32: maps are < 2 GiB). With every
  // chunk issuing the same memory operations, each wait on a load counts
  // exactly the stores issued after it.
  constexpr uint32_t MX_DISCARD = 0x80000000u;
  uint8_t* hcol = hring + (16 * wave + n) * G::RINGB;

  // One chunk: stage j, row pass j, column pass j - J0 (before the first
  // output chunk its results are discarded).
  auto chunk = [&](int j, auto P) {
    stage_chunk(j, P);
    __syncthreads();
    fetch(j + 2, P);  // past the last chunk: rows outside the image, masked

    // ---------------- row pass: chunk j -> ring block j mod NB ----------------
    {
      const _Float16* xs = stage + decltype(P)::value * G::STAGE + n * G::SWP + 16 * wave + 8 * q;
      f4_t r0 = {0.f, 0.f, 0.f, 0.f}, r1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < G::KS; ++s) {
        const h8_t a = *reinterpret_cast<const h8_t*>(xs + 32 * s);
        r0 = mfma(a, g_hi[s], r0);
        r1 = mfma(a, t_hi[s], r1);
        r0 = mfma(a, g_lo[s], r0);
        r1 = mfma(a, t_lo[s], r1);
      }
      // stored weights of rows 4q..4q+3 at this lane's column, for S_X
      const _Float16* xh = stage + decltype(P)::value * G::STAGE + (4 * q) * G::SWP + RA + 16 * wave + n;
      uint32_t hb = 0u;
#pragma unroll
      for (int i = 0; i < 4; ++i) hb |= (uint32_t)(uint16_t)xh[i * G::SWP] << (8 * i);
      h4_t h0, l0, h1, l1;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const Split16 a = split16(r0[i] * sc1), b = split16(r1[i] * sc1);
        h0[i] = a.hi;
        l0[i] = a.lo;
        h1[i] = b.hi;
        l1[i] = b.lo;
      }
      const int slot = (j % G::NB) * MX_CH + 4 * q;
      _Float16* rp = ring_col + slot;
      *reinterpret_cast<h4_t*>(rp) = h0;
      *reinterpret_cast<h4_t*>(rp + G::RINGA) = l0;
      *reinterpret_cast<h4_t*>(rp + 2 * G::RINGA) = h1;
      *reinterpret_cast<h4_t*>(rp + 3 * G::RINGA) = l1;
      *reinterpret_cast<uint32_t*>(hcol + slot) = hb;
    }
    // the column pass reads ring rows this wave has just written: keep the
    // compiler from moving LDS accesses across (the hardware keeps their order)
    __atomic_signal_fence(__ATOMIC_SEQ_CST);

    // ---------------- column pass: output rows o0..o0+15 ----------------
    {
      const int jo = j - G::J0;
      const int o0 = s0 + jo * MX_CH;
      f4_t am = {0.f, 0.f, 0.f, 0.f}, um = am, vm = am;
#pragma unroll
      for (int s = 0; s < G::KS; ++s) {
        // window rows 32s + 8q .. +7 lie in ring block jo + 2s + q/2, half q&1
        // (jo + NB = j + 1 keeps the block index non-negative)
        const int u0 = (j + 1 + 2 * s) % G::NB, u1 = (j + 2 + 2 * s) % G::NB;  // uniform
        const int blk = (q >> 1) ? u1 : u0;
        const _Float16* rp = ring_col + blk * MX_CH + 8 * (q & 1);
        const h8_t y0h = *reinterpret_cast<const h8_t*>(rp);
        const h8_t y0l = *reinterpret_cast<const h8_t*>(rp + G::RINGA);
        const h8_t y1h = *reinterpret_cast<const h8_t*>(rp + 2 * G::RINGA);
        const h8_t y1l = *reinterpret_cast<const h8_t*>(rp + 3 * G::RINGA);
        am = mfma(g_hi[s], y0h, am);
        um = mfma(t_hi[s], y0h, um);
        vm = mfma(g_hi[s], y1h, vm);
        am = mfma(g_hi[s], y0l, am);
        um = mfma(t_hi[s], y0l, um);
        vm = mfma(g_hi[s], y1l, vm);
        am = mfma(g_lo[s], y0h, am);
        um = mfma(t_lo[s], y0h, um);
        vm = mfma(g_lo[s], y1h, vm);
        am = mfma(g_lo[s], y0l, am);
        um = mfma(t_lo[s], y0l, um);
        vm = mfma(g_lo[s], y1l, vm);
      }
      // stored weights of output rows o0 + 4q .. +3: window rows RA + 4q .. +3
      // (block jo + (RA + 4q)/16, offset (RA + 4q) mod 16)
      const int hq = RA + 4 * q;
      const int hb0 = (j + 1 + RA / MX_CH) % G::NB, hb1 = (j + 2 + RA / MX_CH) % G::NB;  // uniform
      const int hblk = (RA % MX_CH + 4 * q) >= MX_CH ? hb1 : hb0;
      const uint32_t hb = *reinterpret_cast<const uint32_t*>(hcol + hblk * MX_CH + hq % MX_CH);
      // rows outside the segment (warm-up chunks, the tail of the last one)
      // are discarded; interior chunks skip the per-row tests
      const bool full = jo >= 0 && o0 + MX_CH <= seg_end;  // uniform
      const uint32_t off0 = (uint32_t)(o0 + 4 * q) * mpb + (uint32_t)col * (uint32_t)sizeof(float);
      float sx = 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = o0 + 4 * q + i;
        const bool ok = full || (row >= s0 && row < seg_end);
        const uint32_t off = ok ? off0 + (uint32_t)i * mpb : MX_DISCARD;
        const float a = am[i] * fac;
        buf_store<float>(a, resA, off, 0u);
        buf_store<float>(um[i] * fac, resU, off, 0u);
        buf_store<float>(vm[i] * fac, resV, off, 0u);
        const float h = ok ? (float)((hb >> (8 * i)) & 0xffu) : 0.f;  // zero past the width
        sx = __builtin_fmaf(h, a, sx);
      }
      // rows 8p..8p+7 of the chunk are lanes q = 2p and 2p + 1
      sx += __shfl_xor(sx, 16);
      const int grow = o0 + 8 * (q >> 1);
      const uint32_t poff = (q & 1) == 0 && grow >= s0 && grow < seg_end
                                ? part_base + (uint32_t)((grow / CONV_GROUP) * CONV_TW + 16 * wave + n) *
                                                  (uint32_t)sizeof(float)
                                : MX_DISCARD;
      buf_store<float>(sx * hscale, mres, poff, 0u);
    }
  };

  using P0 = std::integral_constant<int, 0>;
  using P1 = std::integral_constant<int, 1>;
  fetch(0, P0{});
  fetch(1, P1{});
  chunk(0, P0{});  // peeled, so that the loop is entered with the same pending operations as it repeats
  int j = 1;
  for (; j + 1 < nchunks; j += 2) {
    chunk(j, P1{});
    chunk(j + 1, P0{});
  }
  if (j < nchunks) chunk(j, P1{});
}

// Zero the rings once per workgroup: column passes of warm-up chunks read
// ring rows that no row pass of the segment has written (results discarded,
// but they must be finite).
template <int RA>
__device__ __forceinline__ void mx_clear_rings(_Float16* smem) {
  using G = MxGeom<RA>;
  uint32_t* p = reinterpret_cast<uint32_t*>(smem + 2 * G::STAGE);
  constexpr int nwords = (int)((4 * G::RINGA * sizeof(_Float16) + (size_t)CONV_TW * G::RINGB) / 4);
  for (int i = threadIdx.x; i < nwords; i += MX_NT) p[i] = 0u;
  __syncthreads();
}

template <int RA>
__global__ void __launch_bounds__(MX_NT) conv_mx_image_kernel(ImageDesc im, int S, const char* wbase,
                                                              char* mbase) {
  __shared__ __align__(16) _Float16 smem[MxGeom<RA>::SMEM / sizeof(_Float16)];
  const int strip = blockIdx.x % im.nstrips;
  const int seg = blockIdx.x / im.nstrips;
  mx_clear_rings<RA>(smem);
  mx_segment<RA>(im, strip, seg * S, S, wbase, mbase, smem);
}

template <int RA>
__global__ void __launch_bounds__(MX_NT) conv_mx_tiles_kernel(const ImageDesc* __restrict__ images,
                                                              const ConvTile* __restrict__ tiles, int ntiles,
                                                              const char* wbase, char* mbase) {
  __shared__ __align__(16) _Float16 smem[MxGeom<RA>::SMEM / sizeof(_Float16)];
  mx_clear_rings<RA>(smem);
  for (int i = blockIdx.x; i < ntiles; i += gridDim.x) {
    const ConvTile t = tiles[i];
    const ImageDesc im = images[t.img];
    mx_segment<RA>(im, t.strip, t.s0, t.S, wbase, mbase, smem);
    __syncthreads();  // the next tile restages the shared memory
  }
}

}  // namespace

int conv_mx_radius(int rclass) { return (rclass + 7) / 8 * 8; }

#define ITC_FOR_MX(X) X(8) X(16) X(24) X(32)

hipError_t launch_conv_mx_image(const ImageDesc& im, const void* w, void* m, hipStream_t s) {
  const int S = conv_segment_rows(im);
  const dim3 grid(im.nstrips * ((im.H + S - 1) / S));
#define ITC_CASE(RA)                                                                               \
  case RA:                                                                                         \
    hipLaunchKernelGGL((conv_mx_image_kernel<RA>), grid, dim3(MX_NT), 0, s, im, S, (const char*)w, \
                       (char*)m);                                                                  \
    return hipGetLastError();
  switch (conv_mx_radius(im.rclass)) { ITC_FOR_MX(ITC_CASE) default: return hipErrorInvalidValue; }
#undef ITC_CASE
}

hipError_t launch_conv_mx_tiles(int ra, const ImageDesc* d_images, const ConvTile* d_tiles, int ntiles,
                                const void* w, void* m, int grid, hipStream_t s) {
#define ITC_CASE(RA)                                                                                  \
  case RA:                                                                                            \
    hipLaunchKernelGGL((conv_mx_tiles_kernel<RA>), dim3(grid), dim3(MX_NT), 0, s, d_images, d_tiles,  \
                       ntiles, (const char*)w, (char*)m);                                             \
    return hipGetLastError();
  switch (ra) { ITC_FOR_MX(ITC_CASE) default: return hipErrorInvalidValue; }
#undef ITC_CASE
}

int conv_mx_blocks_per_cu(int ra) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
#define ITC_CASE(RA)                                                                               \
  case RA:                                                                                         \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, conv_mx_tiles_kernel<RA>, MX_NT, 0);     \
    break;
  switch (ra) { ITC_FOR_MX(ITC_CASE) default: break; }
#undef ITC_CASE
  return e == hipSuccess ? nb : 0;
}

}  // namespace itc
