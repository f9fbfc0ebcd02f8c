// Separable Gaussian convolution maps on the matrix cores, for 8-bit lattice
// weights and FP32 maps (Section 3.1: the Parzen sum of delta impulses is the
// weight image convolved with a Gaussian, whose mask factorises into 1-D
// masks). The maps are the same as the VALU kernel's:
//   A = (I *_v g) *_u g,   M_u = (I *_v g) *_u tg,   M_v = (I *_v tg) *_u g,
// with f(t) the tap at t = x_out - x_in, plus the FP64 partials of S_X.
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
//     split y = y_hi + y_lo, and every map is T_hi y_hi + T_hi y_lo +
//     T_lo y_hi; the dropped T_lo y_lo is below 2^-22 of sum |T| |y|.
// The relative error of a map is a few 2^-22 against an FP32 direct sum's
// 2^-24 per operation.
//
// Work decomposition: a workgroup of four waves owns a strip of 64 columns
// and a segment of rows (starting at a multiple of SX_ROWS) and streams down
// it in chunks of 16 rows. Wave w owns columns 16w..16w+15 (one map panel) in
// both passes, so the rings that carry row-pass results to the column pass
// are private to the wave (LDS operations of one wave complete in order: no
// barrier). Per chunk:
//   1. staging (shared): the chunk's 16 input rows with their column halo,
//      fetched MX_AHEAD (10) chunks earlier as aligned 4-byte words, are converted to
//      FP16 into one of two LDS buffers. One barrier per chunk.
//   2. row pass: K/32 A-fragments (16 rows x 32 columns) times the tap
//      fragments -> R0, R1 for 16 rows x 16 columns; scaled, split and
//      written to the ring (column-major: rows contiguous, so the column
//      pass reads 8 consecutive rows per lane in one 16-byte load); the
//      stored weights of the wave's columns go to a byte ring for S_X.
//   3. column pass, 2RA rows behind: the ring fragments are the A operand
//      and the taps the B operand, so the product is the transposed tile and
//      each lane holds four adjacent columns of one output row. A 16 x 16
//      tile of a map is then one contiguous 1 KiB of its panel, written by a
//      single 16-byte-per-lane non-temporal store; h*A is summed into an
//      FP64 partial of S_X per SX_ROWS-row group.
// A batch runs one persistent launch over the tiles of every radius class
// (sorted by radius, then cost), each workgroup walking the tile sublist of
// its XCD; a workgroup clears its shared memory when the radius of its next
// tile differs from the last one's.
#include <type_traits>
#include <utility>

#include "itc_device.h"

namespace itc {

namespace {

typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef _Float16 h4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u4_t __attribute__((ext_vector_type(4)));

constexpr int MX_NT = 256;  // four waves; wave w owns strip columns 16w..16w+15
constexpr int MX_CH = 16;   // rows per chunk
#ifndef ITC_MX_AHEAD
#define ITC_MX_AHEAD 10
#endif
// Chunks whose input loads are in flight. The memory counter that a wave
// waits on counts loads and stores in issue order, so a chunk's loads are
// complete only when the map stores issued before them are too: the depth
// also sets how many chunks of stores a wave keeps in flight. At most 63
// operations can be counted: MX_AHEAD (NI + 3) stays below that.
constexpr int MX_AHEAD = ITC_MX_AHEAD;
static_assert(MX_AHEAD >= 2 && MX_AHEAD <= 16, "prefetch depth");
// Cache policy of the map stores: non-temporal (the maps are written once
// and read much later, after every other image's maps have streamed past).
constexpr int MX_STREAM = 2;
static_assert(SX_ROWS % MX_CH == 0 && SX_SLOTS == MX_NT / 64, "one S_X slot per wave and row group");
static_assert(CONV_TW == 4 * MAP_PANEL, "a strip is four panels");

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
  static constexpr int SWD = SW / 4;             // staged 4-byte words per row
  static constexpr int SWP = SW + 8;             // staged row pitch
  static constexpr int NI = (MX_CH * SWD + MX_NT - 1) / MX_NT;  // staged words per thread and chunk
  static constexpr size_t STAGE = (size_t)MX_CH * SWP;     // halves of staged rows per buffer
  static constexpr int NDUM = NI * MX_NT - MX_CH * SWD;     // thread items past the chunk's words
  static constexpr size_t STAGEB = STAGE + 4 * NDUM;        // halves per buffer, with a slot per such item
  static constexpr size_t RINGA = (size_t)CONV_TW * RINGP;  // halves per ring array
  static constexpr int HROWS = NB * MX_CH;                   // rows of a wave's weight ring (16 bytes each)
  static constexpr size_t SMEM = (2 * STAGEB + 4 * RINGA) * sizeof(_Float16) + (size_t)4 * HROWS * 16;
  static_assert(RINGP / 2 % 8 == 4 && SWP / 2 % 8 == 4, "bank-spread pitches");
  static_assert(NB * MX_CH >= MX_CH + 2 * RA, "ring holds a column window");
  static_assert(SW % 4 == 0 && RA % 4 == 0, "word-aligned staging");
  static_assert(STAGEB % 8 == 0, "16-byte aligned staging buffers and rings");
  static_assert(MX_AHEAD * (NI + 3) <= 63, "pending memory operations within the counter's range");
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
  _Float16* stage = smem;                  // [2][STAGEB]: 16 rows of SWP halves, then the item slots
  _Float16* ring = smem + 2 * G::STAGEB;   // [4][64][RINGP]: R0 hi, R0 lo, R1 hi, R1 lo
  uint32_t* hring = reinterpret_cast<uint32_t*>(ring + 4 * G::RINGA);  // [4 waves][HROWS][4 words]

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

  const int rowbytes = (int)im.pitch;  // 8-bit weights, a multiple of 4
  const rsrc_t wres = make_rsrc(wbase + im.weight_off, (uint32_t)H * (uint32_t)rowbytes);

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

  // ---- staging: thread item i of a chunk is staged word d of row r ----
  // (r, d) = divmod(tid + 256 i, SWD); the word holds image columns
  // v0 - RA + 4d .. +3 (v0 - RA is a multiple of 8, so the word is aligned).
  // Words left of the image, rows outside it and items past the chunk load
  // at an offset past the end of the buffer: the hardware returns 0 without
  // a memory request. Bytes of a word past the width are masked to 0.
  int irow[G::NI], icol[G::NI], ioff[G::NI];
  uint32_t imask[G::NI];
#pragma unroll
  for (int i = 0; i < G::NI; ++i) {
    const int idx = tid + MX_NT * i;
    const int r = idx / G::SWD, d = idx - r * G::SWD;
    const int x = v0 - RA + 4 * d;
    const bool item = idx < MX_CH * G::SWD;
    const bool ok = item && x >= 0 && x < W;
    const int keep = W - x;  // bytes of the word inside the image
    irow[i] = ok ? r : -(1 << 20);             // never inside the image: the load reads 0
    icol[i] = x;
    // halves into a staging buffer; items past the chunk write zeros to a
    // slot of their own past the staged rows, so that the staging stores
    // are unconditional and the compiler keeps each load where it is issued
    ioff[i] = item ? r * G::SWP + 4 * d : (int)G::STAGE + 4 * (idx - MX_CH * G::SWD);
    imask[i] = !ok ? 0u : (keep >= 4 ? 0xffffffffu : (1u << (8 * keep)) - 1u);
  }
  // MX_AHEAD chunks are in flight: set P = j mod MX_AHEAD holds chunk j from
  // MX_AHEAD chunks before it is staged (P is a template constant so the sets
  // stay in registers), which leaves the loads that many chunks of work to
  // arrive.
  uint32_t pre[MX_AHEAD][G::NI];
  auto fetch = [&](int j, auto P) {
    constexpr int p = decltype(P)::value;
#pragma unroll
    for (int i = 0; i < G::NI; ++i) {
      const int y = origin + j * MX_CH + irow[i];
      const bool in = y >= 0 && y < H;
      const uint32_t off = in ? (uint32_t)(y * rowbytes + icol[i]) : 0x80000000u;
      pre[p][i] = __builtin_amdgcn_raw_buffer_load_b32(wres, off, 0, 0);
    }
  };
  auto stage_chunk = [&](auto P, auto B) {
    constexpr int p = decltype(P)::value;
    _Float16* xs = stage + decltype(B)::value * G::STAGEB;
#pragma unroll
    for (int i = 0; i < G::NI; ++i) {
      const uint32_t v = pre[p][i] & imask[i];
      h4_t h;
      h[0] = (_Float16)(float)(v & 0xffu);
      h[1] = (_Float16)(float)((v >> 8) & 0xffu);
      h[2] = (_Float16)(float)((v >> 16) & 0xffu);
      h[3] = (_Float16)(float)(v >> 24);
      *reinterpret_cast<h4_t*>(xs + ioff[i]) = h;
    }
  };

  // ---- outputs: wave w writes panel 4 strip + w, a 16 x 16 tile per chunk ----
  const int npan = im.npanels;
  const int panel = 4 * strip + wave;
  const bool pan_ok = panel < npan;  // the strip's last panels may lie past the width
  const uint32_t planeb = (uint32_t)(im.plane * (int64_t)sizeof(float));
  const char* mimg = mbase + im.map_off;
  const rsrc_t resA = make_rsrc(mimg, planeb), resU = make_rsrc(mimg + planeb, planeb),
               resV = make_rsrc(mimg + 2 * (size_t)planeb, planeb);
  // byte offset of row o of this lane's panel and columns 4q..4q+3: (panel H + o) 64 + 16 q
  const uint32_t pan_base = (uint32_t)panel * (uint32_t)H * 64u + 16u * (uint32_t)q;
  double* part = reinterpret_cast<double*>(mbase + im.map_off + im.part_off) +
                 ((int64_t)strip * im.nsxg) * SX_SLOTS + wave;
  const double hscale = im.scale;
  _Float16* ring_col = ring + (size_t)(16 * wave + n) * G::RINGP;
  uint32_t* hw = hring + wave * G::HROWS * 4;  // this wave's weight ring: [HROWS][4 words]
  constexpr uint32_t MX_DISCARD = 0x80000000u;
  double sxd = 0.0;  // this lane's share of the current S_X row group

  // One chunk: stage j, row pass j, column pass j - J0 (before the first
  // output chunk its results are discarded).
  auto chunk = [&](int j, auto P, auto B) {
    stage_chunk(P, B);
    __syncthreads();
    fetch(j + MX_AHEAD, P);  // past the last chunk: rows outside the image, masked

    // ---------------- row pass: chunk j -> ring block j mod NB ----------------
    {
      const _Float16* xs = stage + decltype(B)::value * G::STAGEB + n * G::SWP + 16 * wave + 8 * q;
      f4_t r0 = {0.f, 0.f, 0.f, 0.f}, r1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < G::KS; ++s) {
        const h8_t a = *reinterpret_cast<const h8_t*>(xs + 32 * s);
        r0 = mfma(a, g_hi[s], r0);
        r1 = mfma(a, t_hi[s], r1);
        r0 = mfma(a, g_lo[s], r0);
        r1 = mfma(a, t_lo[s], r1);
      }
      // stored weights of row n, columns 4q..4q+3 of this wave, for S_X
      const h4_t xh = *reinterpret_cast<const h4_t*>(stage + decltype(B)::value * G::STAGEB + n * G::SWP + RA +
                                                      16 * wave + 4 * q);
      uint32_t hb = 0u;
#pragma unroll
      for (int i = 0; i < 4; ++i) hb |= (uint32_t)(float)xh[i] << (8 * i);
      h4_t h0, l0, h1, l1;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const Split16 a = split16(r0[i] * sc1), b = split16(r1[i] * sc1);
        h0[i] = a.hi;
        l0[i] = a.lo;
        h1[i] = b.hi;
        l1[i] = b.lo;
      }
      const int slot = (j % G::NB) * MX_CH;
      _Float16* rp = ring_col + slot + 4 * q;
      *reinterpret_cast<h4_t*>(rp) = h0;
      *reinterpret_cast<h4_t*>(rp + G::RINGA) = l0;
      *reinterpret_cast<h4_t*>(rp + 2 * G::RINGA) = h1;
      *reinterpret_cast<h4_t*>(rp + 3 * G::RINGA) = l1;
      hw[(slot + n) * 4 + q] = hb;
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
        am = mfma(y0h, g_hi[s], am);
        um = mfma(y0h, t_hi[s], um);
        vm = mfma(y1h, g_hi[s], vm);
        am = mfma(y0l, g_hi[s], am);
        um = mfma(y0l, t_hi[s], um);
        vm = mfma(y1l, g_hi[s], vm);
        am = mfma(y0h, g_lo[s], am);
        um = mfma(y0h, t_lo[s], um);
        vm = mfma(y1h, g_lo[s], vm);
      }
      // lane (n, q) holds row o0 + n, columns 16 wave + 4q + i. Its stored
      // weights are in the weight ring at window row RA + n (block
      // jo + (RA + n)/16, row (RA + n) mod 16).
      const int wr = RA + n;
      const int hb0 = (j + 1 + RA / MX_CH) % G::NB, hb1 = (j + 2 + RA / MX_CH) % G::NB;  // uniform
      const int hblk = (RA % MX_CH + n) >= MX_CH ? hb1 : hb0;
      const uint32_t hb = hw[(hblk * MX_CH + wr % MX_CH) * 4 + q];
      const int row = o0 + n;
      const bool ok = row >= s0 && row < seg_end;  // warm-up chunks and the tail of the last one
      const uint32_t off = ok && pan_ok ? pan_base + (uint32_t)row * 64u : MX_DISCARD;
      f4_t a4, u4, v4;
      float sx = 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a4[i] = am[i] * fac;
        u4[i] = um[i] * fac;
        v4[i] = vm[i] * fac;
        sx = __builtin_fmaf((float)((hb >> (8 * i)) & 0xffu), a4[i], sx);  // zero past the width
      }
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4_t, a4), resA, off, 0, MX_STREAM);
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4_t, u4), resU, off, 0, MX_STREAM);
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4_t, v4), resV, off, 0, MX_STREAM);
      sxd += ok ? (double)sx : 0.0;
      // the last chunk of an S_X row group (or of the segment): one FP64 partial per wave
      if (jo >= 0 && ((jo + 1) % (SX_ROWS / MX_CH) == 0 || jo == n_out - 1)) {  // uniform
        const double tot = wave_sum(sxd);
        if (lane == 0) part[(int64_t)(o0 / SX_ROWS) * SX_SLOTS] = tot * hscale;
        sxd = 0.0;
      }
    }
  };

  // chunk j takes prefetch set j mod MX_AHEAD and staging buffer j mod 2;
  // the loop is unrolled over lcm(MX_AHEAD, 2) chunks so that both are
  // template constants
  constexpr int U = MX_AHEAD % 2 == 0 ? MX_AHEAD : 2 * MX_AHEAD;
  using Seq = std::make_integer_sequence<int, U>;
  auto at = [&](int j, auto I) {
    constexpr int c = 1 + decltype(I)::value;  // j = 1 mod U
    chunk(j, std::integral_constant<int, c % MX_AHEAD>{}, std::integral_constant<int, c % 2>{});
  };
  // Each prologue fetch is followed by as many (discarded) stores as a loop
  // chunk issues after its fetch, so that the loop is entered with the same
  // sequence of pending memory operations as it repeats. The compiler's
  // memory-counter waits at the loop head are the smallest over the entry and
  // the back edge: without the padding, the shorter prologue sequence would
  // cut the loads in flight in the first chunks of every loop iteration.
  for_each_index([&](auto I) {
    fetch(decltype(I)::value, I);
    asm volatile("" ::: "memory");  // keeps the padding stores distinct and in place
#pragma unroll
    for (int d = 0; d < 3; ++d) __builtin_amdgcn_raw_buffer_store_b32(0u, resA, MX_DISCARD + 16u * d, 0, 0);
    asm volatile("" ::: "memory");
  }, std::make_integer_sequence<int, MX_AHEAD>{});
  // peeled, so that the loop is entered with the same pending operations as it repeats
  chunk(0, std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{});
  int j = 1;
  for (; j + U - 1 < nchunks; j += U) for_each_index([&](auto I) { at(j + decltype(I)::value, I); }, Seq{});
  for_each_index([&](auto I) {
    if (decltype(I)::value < U - 1 && j + decltype(I)::value < nchunks) at(j + decltype(I)::value, I);
  }, Seq{});
}

// Zero the rings once per workgroup: column passes of warm-up chunks read
// ring rows that no row pass of the segment has written (results discarded,
// but they must be finite).
template <int RA>
__device__ __forceinline__ void mx_clear_rings(_Float16* smem) {
  using G = MxGeom<RA>;
  uint32_t* p = reinterpret_cast<uint32_t*>(smem + 2 * G::STAGEB);
  constexpr int nwords = (int)((4 * G::RINGA * sizeof(_Float16) + (size_t)4 * G::HROWS * 16) / 4);
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

template <int MAXRA>
constexpr size_t mx_smem_max() {
  size_t m = MxGeom<8>::SMEM;
  if constexpr (MAXRA >= 16) m = m > MxGeom<16>::SMEM ? m : MxGeom<16>::SMEM;
  if constexpr (MAXRA >= 24) m = m > MxGeom<24>::SMEM ? m : MxGeom<24>::SMEM;
  if constexpr (MAXRA >= 32) m = m > MxGeom<32>::SMEM ? m : MxGeom<32>::SMEM;
  return m;
}

// Persistent launch over the tiles of every aligned radius up to MAXRA:
// workgroup b walks the sublist of its XCD, b mod CONV_XCDS.
template <int MAXRA>
__global__ void __launch_bounds__(MX_NT) conv_mx_tiles_kernel(const ImageDesc* __restrict__ images,
                                                              const ConvTile* __restrict__ tiles, XcdSplit xs,
                                                              const char* wbase, char* mbase) {
  constexpr size_t SM = mx_smem_max<MAXRA>();
  __shared__ __align__(16) _Float16 smem[SM / sizeof(_Float16)];
  int cur = 0;  // aligned radius whose rings the shared memory holds
  const int x = blockIdx.x % CONV_XCDS, nx = gridDim.x / CONV_XCDS;
  const int end = xs.beg[x + 1];
  for (int i = xs.beg[x] + (int)blockIdx.x / CONV_XCDS; i < end; i += nx) {
    const ConvTile t = tiles[i];
    const ImageDesc im = images[t.img];
    const int ra = (im.rclass + 7) / 8 * 8;  // uniform
    if (ra != cur) {  // rings of another layout: clear them (warm-up reads must be finite)
      uint32_t* p = reinterpret_cast<uint32_t*>(smem);
      for (int k = threadIdx.x; k < (int)(SM / 4); k += MX_NT) p[k] = 0u;
      __syncthreads();
      cur = ra;
    }
    if (ra == 8) mx_segment<8>(im, t.strip, t.s0, t.S, wbase, mbase, smem);
    if constexpr (MAXRA >= 16) {
      if (ra == 16) mx_segment<16>(im, t.strip, t.s0, t.S, wbase, mbase, smem);
    }
    if constexpr (MAXRA >= 24) {
      if (ra == 24) mx_segment<24>(im, t.strip, t.s0, t.S, wbase, mbase, smem);
    }
    if constexpr (MAXRA >= 32) {
      if (ra == 32) mx_segment<32>(im, t.strip, t.s0, t.S, wbase, mbase, smem);
    }
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

hipError_t launch_conv_mx_tiles(int max_ra, const ImageDesc* d_images, const ConvTile* d_tiles, const XcdSplit& xs,
                                const void* w, void* m, int grid, hipStream_t s) {
  if (grid % CONV_XCDS != 0) return hipErrorInvalidValue;
#define ITC_CASE(RA)                                                                                  \
  case RA:                                                                                            \
    hipLaunchKernelGGL((conv_mx_tiles_kernel<RA>), dim3(grid), dim3(MX_NT), 0, s, d_images, d_tiles,  \
                       xs, (const char*)w, (char*)m);                                                 \
    return hipGetLastError();
  switch (max_ra) { ITC_FOR_MX(ITC_CASE) default: return hipErrorInvalidValue; }
#undef ITC_CASE
}

int conv_mx_blocks_per_cu(int max_ra) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
#define ITC_CASE(RA)                                                                               \
  case RA:                                                                                         \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, conv_mx_tiles_kernel<RA>, MX_NT, 0);     \
    break;
  switch (max_ra) { ITC_FOR_MX(ITC_CASE) default: break; }
#undef ITC_CASE
  return e == hipSuccess ? nb : 0;
}

}  // namespace itc
