// Separable Gaussian convolution maps of a lattice weight image (Section 3.1:
// the Parzen sum of delta impulses is the image convolved with a Gaussian; for
// small widths the 2-D mask factorises into 1-D masks). One pass produces
//   A   = (I *_v g) *_u g,   M_u = (I *_v g) *_u tg,   M_v = (I *_v tg) *_u g
// with g[t] = exp(-t^2/(2 sigma^2)), tg[t] = t g[t], |t| <= R, and FP64
// partial sums of S_X = sum I A (one per wave and SX_ROWS-row group).
//
// Work decomposition (gfx950): a workgroup of CONV_WAVES = 4 waves owns a
// strip of 64 columns (lane = column) and a segment of rows, and streams down
// it in chunks of 16 rows. Per chunk:
//   1. staging: the chunk's 16 input rows, with an R-column halo on each side,
//      are converted to the real type and written to LDS. Their global loads
//      were issued one chunk earlier into registers, behind the arithmetic;
//   2. row pass (along v): each lane makes 4 adjacent columns of R0 = I*g and
//      R1 = I*tg for one row (16 lanes per row, four rows per wave) and
//      writes them into an LDS ring holding the last 2R + 16 rows (a whole
//      number of 16-row blocks);
//   3. column pass (along u, R rows behind the row pass): wave w makes rows
//      4w..4w+3 of the chunk for its lane's column: A, M_u, M_v (12
//      accumulators). A 16-row block of the ring never wraps, and the block
//      and offset of every read are compile-time for a given w, so each read
//      is one base register plus an immediate offset. Outputs are stored in
//      the maps' panel layout; h*A is summed per lane in FP64 and per wave
//      into the S_X partial of each SX_ROWS-row group.
// Four waves per workgroup share one ring: at the LDS budget of one ring the
// chip holds twice the waves of a two-wave workgroup (the FP32 convolution of
// 64 x 1024^2 images took 0.47 ms against 0.56 ms with two), so one wave's
// LDS, scalar and memory instructions issue beside the others' FMAs. Taps
// are computed once per segment in FP64 (one lane per tap) and held in scalar
// registers; tap loops are unrolled for the class.
#include "itc_device.h"

namespace itc {

#ifndef ITC_CONV_AHEAD
#define ITC_CONV_AHEAD 1
#endif
// Chunks whose loads are in flight. A wave's memory counter counts loads and
// stores in issue order, and at most 63 of them: each chunk issues 3 KB loads
// and 3 KB stores.
constexpr int CONV_AHEAD = ITC_CONV_AHEAD;
static_assert(CONV_AHEAD >= 1 && CONV_AHEAD * 6 * CONV_KB <= 63, "pending memory operations within the counter");

template <typename T, int R>
struct ConvGeom {
  static constexpr int CH = CONV_CH;
  static constexpr int J0 = (2 * R + CH - 1) / CH;  // chunks before the first column pass
  static constexpr int NB = J0 + 1;                 // ring blocks of CH rows
  static constexpr int RING = NB * CH;              // >= 2R + CH
  static constexpr int NWIN = 2 * R + CONV_KB;      // rows a lane reads per column pass
  static constexpr int NXL = 2 * R + 4;             // row-pass inputs per lane and row
  static constexpr int XP = 2 * CONV_TW;            // staging row pitch: two staged columns per lane
  static constexpr int XW = CONV_TW + 2 * R;        // staged columns per row (<= 128)
  static constexpr size_t RING_ELEMS = (size_t)RING * CONV_TW;
  static constexpr size_t SMEM = (2 * RING_ELEMS + (size_t)CH * XP) * sizeof(T);
  static_assert(XW <= 2 * CONV_TW, "two staged columns per lane");
};

// Raw stored weight at element offset `i`, kept unconverted until staging so
// that the global load's latency hides behind a whole chunk of arithmetic.
// FP32 kernels keep 32 bits (u8 value or f32 bits; FP64 weights are narrowed
// to f32 at load), FP64 kernels keep 64 bits.
template <typename T>
struct RawOf {
  using type = uint32_t;
};
template <>
struct RawOf<double> {
  using type = uint64_t;
};

// Load of a stored weight of type WT kept as raw bits (FP64 weights are
// narrowed to f32 in FP32 kernels), and its conversion to the real type.
template <typename T, typename WT>
__device__ __forceinline__ typename RawOf<T>::type load_raw(rsrc_t r, uint32_t voff, uint32_t soff) {
  using U = typename RawOf<T>::type;
  const WT v = buf_load<WT>(r, voff, soff);
  if constexpr (sizeof(WT) == 1)
    return (U)v;
  else if constexpr (sizeof(WT) == 4)
    return (U)__builtin_bit_cast(uint32_t, v);
  else if constexpr (sizeof(U) == 8)
    return __builtin_bit_cast(uint64_t, v);
  else
    return __builtin_bit_cast(uint32_t, (float)v);
}
template <typename T, typename WT>
__device__ __forceinline__ T raw_value(typename RawOf<T>::type r) {
  if constexpr (sizeof(WT) == 1)
    return (T)(uint32_t)r;
  else if constexpr (sizeof(WT) == 4 || sizeof(r) == 4)
    return (T)__builtin_bit_cast(float, (uint32_t)r);
  else
    return (T)__builtin_bit_cast(double, (uint64_t)r);
}

// Calls f(WT{}) with WT the stored weight type: one uniform branch per call.
template <typename F>
__device__ __forceinline__ void with_weight_type(int wdtype, F&& f) {
  if (wdtype == 0)
    f(uint8_t{});
  else if (wdtype == 1)
    f(float{});
  else
    f(double{});
}

// Column pass of one wave: rows KB w .. KB w + KB - 1 of the chunk whose window starts at
// ring block `jb` (chunk index minus J0).
template <typename T, int R, int WV>
__device__ __forceinline__ void column_pass(const T* __restrict__ ring0, const T* __restrict__ ring1, int jb,
                                            int lane, const T (&g)[R + 1], const T (&tg)[R + 1],
                                            T (&a)[CONV_KB], T (&mu)[CONV_KB], T (&mv)[CONV_KB]) {
  using G = ConvGeom<T, R>;
  constexpr int KB = CONV_KB;
  constexpr int NBLK = (WV * KB + G::NWIN + CONV_CH - 1) / CONV_CH;  // blocks touched
#pragma unroll
  for (int k = 0; k < KB; ++k) a[k] = mu[k] = mv[k] = (T)0;
#pragma unroll
  for (int b = 0; b < NBLK; ++b) {
    const int slot = ((jb + b) % G::NB) * CONV_CH;
    const T* p0 = ring0 + slot * CONV_TW + lane;
    const T* p1 = ring1 + slot * CONV_TW + lane;
#pragma unroll
    for (int ii = 0; ii < CONV_CH; ++ii) {
      const int i = b * CONV_CH + ii - WV * KB;  // window row: absolute row o - R + i for output o = first + k
      if (i >= 0 && i < G::NWIN) {
        const T y = p0[ii * CONV_TW];
        const T z = p1[ii * CONV_TW];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
          const int s = k + R - i;
          if (s >= -R && s <= R) {
            const T gs = g[s < 0 ? -s : s];
            a[k] = fma_t(gs, y, a[k]);
            mv[k] = fma_t(gs, z, mv[k]);
            if (s > 0) mu[k] = fma_t(tg[s], y, mu[k]);
            if (s < 0) mu[k] = fma_t(-tg[-s], y, mu[k]);
          }
        }
      }
    }
  }
}

template <typename T, int R, typename WT>
__device__ __forceinline__ void conv_segment_t(const ImageDesc& im, int strip, int s0, int S,
                                             const char* __restrict__ wbase, char* __restrict__ mbase,
                                             char* __restrict__ smem) {
  using G = ConvGeom<T, R>;
  constexpr int CH = CONV_CH, KB = CONV_KB;
  using Raw = typename RawOf<T>::type;
  T* ring0 = reinterpret_cast<T*>(smem);
  T* ring1 = ring0 + G::RING_ELEMS;
  T* xin = ring1 + G::RING_ELEMS;

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int H = im.H, W = im.W;
  const int v0 = strip * CONV_TW;
  const int seg_end = min(s0 + S, H);
  const int n_out = (seg_end - s0 + CH - 1) / CH;
  const int nchunks = G::J0 + n_out;
  const int origin = s0 - R;                 // absolute row of relative row 0
  const int need_end = min(H, seg_end + R);  // row-pass rows at or past this are never read

  constexpr int esz = (int)sizeof(WT);
  const uint32_t rowbytes = (uint32_t)(im.pitch * esz);
  const rsrc_t wres = make_rsrc(wbase + im.weight_off, (uint32_t)H * rowbytes);
  const rsrc_t mres = make_rsrc(mbase + im.map_off, (uint32_t)(3 * im.plane * (int64_t)sizeof(T)));
  const T scale = (T)im.scale;

  // ---- taps: g[t], tg[t] for t = 0..R (zero beyond the true radius) ----
  T g[R + 1], tg[R + 1];
  {
    const double k = -0.5 / (im.sigma * im.sigma);
    const double gl = (lane <= im.R) ? exp(k * (double)(lane * lane)) : 0.0;
    const T gT = (T)gl, tgT = (T)((double)lane * gl);
#pragma unroll
    for (int t = 0; t <= R; ++t) {
      g[t] = lane_value(gT, t);
      tg[t] = lane_value(tgT, t);
    }
  }

  const uint32_t planeb = (uint32_t)(im.plane * (int64_t)sizeof(T));  // bytes per plane
  const int col = v0 + lane;
  const bool col_ok = col < W;
  const bool col_stored = col < im.npanels * MAP_PANEL;  // the strip may reach past the last panel
  // byte offset of row 0 of this lane's column in the panel layout; rows are MAP_PANEL elements apart
  const uint32_t mvoff = (uint32_t)map_index(H, 0, col) * (uint32_t)sizeof(T);
  constexpr uint32_t rowstep = MAP_PANEL * sizeof(T);
  constexpr int SPW = SX_SLOTS / CONV_WAVES;  // S_X slots per wave
  static_assert(SPW * CONV_WAVES == SX_SLOTS, "the S_X slots divide among the waves");
  double* part = reinterpret_cast<double*>(mbase + im.map_off + im.part_off) +
                 (int64_t)strip * im.nsxg * SX_SLOTS + SPW * wave;
  double sxd = 0.0;  // this lane's share of the current S_X row group

  // ---- loads of chunk j, issued CONV_AHEAD chunks before it is staged ----
  // Wave w loads rows KB w .. KB w + KB - 1 of the chunk's input (columns
  // lane and lane + 64 of the staged window) and the stored weights of its
  // own output rows of chunk j (lane's column, for S_X). Columns and rows
  // outside the image (or past the rows the segment reads) load at BUF_OOB,
  // which reads 0, so no branch or select waits on a load before its use.
  const int col0 = v0 - R + lane, col1 = col0 + CONV_TW;
  const bool ok0 = col0 >= 0 && col0 < W;
  const bool ok1 = lane + CONV_TW < G::XW && col1 >= 0 && col1 < W;
  // per-lane column terms of the offsets, and bit 31 for the lanes outside the image
  const uint32_t c0 = ok0 ? (uint32_t)col0 : 0u, c1 = ok1 ? (uint32_t)col1 : 0u, cc = col_ok ? (uint32_t)col : 0u;
  const uint32_t bad0 = (uint32_t)!ok0 << 31, bad1 = (uint32_t)!ok1 << 31, badc = (uint32_t)!col_ok << 31;
  constexpr int AH = CONV_AHEAD;
  Raw raw0[AH][KB], raw1[AH][KB], hraw[AH][KB];
  auto fetch = [&](int j, auto P) {
    constexpr int p = decltype(P)::value;
    const int y0 = origin + j * CH + wave * KB;         // input rows
    const int h0 = s0 + (j - G::J0) * CH + wave * KB;  // output rows
    {
      constexpr uint32_t es = sizeof(WT);
#pragma unroll
      for (int r = 0; r < KB; ++r) {
        const int y = y0 + r, o = h0 + r;
        // offsets below 2^31 inside the image; bit 31 set (BUF_OOB or above) outside it
        const uint32_t yout = (uint32_t)(y < 0 || y >= need_end) << 31;  // uniform
        const uint32_t oout = (uint32_t)(o < s0 || o >= seg_end) << 31;   // uniform
        const uint32_t yb = (yout ? 0u : (uint32_t)y * rowbytes) | yout;
        const uint32_t ob = (oout ? 0u : (uint32_t)o * rowbytes) | oout;
        raw0[p][r] = load_raw<T, WT>(wres, (yb + c0 * es) | bad0, 0);
        raw1[p][r] = load_raw<T, WT>(wres, (yb + c1 * es) | bad1, 0);
        hraw[p][r] = load_raw<T, WT>(wres, (ob + cc * es) | badc, 0);
      }
    }
  };
  // every lane writes both of its staged columns (columns >= XW are never
  // read) and converts the S_X weights of its output rows: set P is free
  // for the loads of a later chunk after this
  auto stage = [&](auto P, T (&hv)[KB]) {
    constexpr int p = decltype(P)::value;
    T* x = xin + wave * KB * G::XP + lane;
#pragma unroll
    for (int r = 0; r < KB; ++r) {
      x[r * G::XP] = raw_value<T, WT>(raw0[p][r]) * scale;
      x[r * G::XP + CONV_TW] = raw_value<T, WT>(raw1[p][r]) * scale;
      hv[r] = raw_value<T, WT>(hraw[p][r]);
    }
  };
  // as many (dropped) stores as a column pass makes: the prologue and the
  // warm-up chunks issue them, so that every chunk of the loop leaves the same
  // sequence of pending memory operations and the compiler's memory-counter
  // waits allow CONV_AHEAD chunks of loads in flight
  auto pad_stores = [&]() {
    asm volatile("" ::: "memory");
#pragma unroll
    for (int k = 0; k < 3 * KB; ++k) buf_store<T>((T)0, mres, BUF_OOB + 16u * k, 0);
    asm volatile("" ::: "memory");
  };

  const int rq = lane >> 4, cg = lane & 15;  // row pass: row in a set of 4, column group of 4

  auto chunk = [&](int j, auto P) {
    T hv[KB];
    stage(P, hv);
    __syncthreads();
    fetch(j + AH, P);

    // ---------------- row pass: ring rows of chunk j ----------------
    {
      const int first = origin + j * CH;
      const int slot0 = (j % G::NB) * CH;
      const bool live = first + CH > 0 && first < need_end;
#pragma unroll 1
      for (int m = 0; m < KB / 4; ++m) {
        const int r = wave * KB + rq + 4 * m;
        T r0[4], r1[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) r0[c] = r1[c] = (T)0;
        if (live) {
          const T* xr = xin + r * G::XP + 4 * cg;
          T x[G::NXL];
#pragma unroll
          for (int i = 0; i < G::NXL; ++i) x[i] = xr[i];
#pragma unroll
          for (int i = 0; i < G::NXL; ++i) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const int s = c + R - i;  // tap index t = x_out - x_in
              if (s >= -R && s <= R) {
                r0[c] = fma_t(g[s < 0 ? -s : s], x[i], r0[c]);
                if (s > 0) r1[c] = fma_t(tg[s], x[i], r1[c]);
                if (s < 0) r1[c] = fma_t(-tg[-s], x[i], r1[c]);
              }
            }
          }
        }
        T* d0 = ring0 + (slot0 + r) * CONV_TW + 4 * cg;
        T* d1 = ring1 + (slot0 + r) * CONV_TW + 4 * cg;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          d0[c] = r0[c];
          d1[c] = r1[c];
        }
      }
    }
    __syncthreads();

    // ---------------- column pass: rows KB w .. KB w + KB - 1 of output chunk j - J0 ----------------
    if (j < G::J0) {  // uniform: warm-up chunk, nothing to store
      pad_stores();
      return;
    }
    const int o0 = s0 + (j - G::J0) * CH + wave * KB;
    T a[KB], mu[KB], mv[KB];
    switch (wave) {  // uniform; the window offset of each wave is compile-time
      case 0: column_pass<T, R, 0>(ring0, ring1, j - G::J0, lane, g, tg, a, mu, mv); break;
      case 1: column_pass<T, R, 1>(ring0, ring1, j - G::J0, lane, g, tg, a, mu, mv); break;
      case 2:
        if constexpr (CONV_WAVES > 2) column_pass<T, R, 2>(ring0, ring1, j - G::J0, lane, g, tg, a, mu, mv);
        break;
      default:
        if constexpr (CONV_WAVES > 3) column_pass<T, R, 3>(ring0, ring1, j - G::J0, lane, g, tg, a, mu, mv);
        break;
    }
    // columns past the width inside the last panel are stored too (never
    // read); they carry zero weight for S_X. Rows past the segment store at
    // BUF_OOB (dropped).
    T sx = (T)0;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const bool row_ok = o0 + k < seg_end;  // uniform
      const uint32_t off = (mvoff + (uint32_t)(o0 + k) * rowstep) | ((uint32_t)!(row_ok && col_stored) << 31);
      buf_store<T>(a[k], mres, off, 0);
      buf_store<T>(mu[k], mres, off, planeb);
      buf_store<T>(mv[k], mres, off, 2 * planeb);
      if (row_ok) sx = fma_t(hv[k], a[k], sx);
    }
    sxd += (double)sx;
    // the last chunk of an S_X row group (or of the segment): wave w writes
    // the first of its slots of the group's partials and clears the others
    const int jo = j - G::J0;
    if ((jo + 1) % (SX_ROWS / CH) == 0 || jo == n_out - 1) {  // uniform
      const double tot = wave_sum(sxd);
      const int gi = (s0 + jo * CH) / SX_ROWS;
      if (lane == 0) {
        part[(int64_t)gi * SX_SLOTS] = tot * (double)im.scale;
#pragma unroll
        for (int q = 1; q < SPW; ++q) part[(int64_t)gi * SX_SLOTS + q] = 0.0;
      }
      sxd = 0.0;
    }
  };

  for_each_index([&](auto I) {
    fetch(decltype(I)::value, I);
    pad_stores();
  }, std::make_integer_sequence<int, AH>{});
  int j = 0;
  for (; j + AH <= nchunks; j += AH)
    for_each_index([&](auto I) { chunk(j + decltype(I)::value, I); }, std::make_integer_sequence<int, AH>{});
  for_each_index([&](auto I) {
    if (j + decltype(I)::value < nchunks) chunk(j + decltype(I)::value, I);
  }, std::make_integer_sequence<int, AH>{});
}

// One segment for the image's stored weight type (one uniform branch per
// segment, so the loop carries no type switch).
template <typename T, int R>
__device__ __forceinline__ void conv_segment(const ImageDesc& im, int strip, int s0, int S,
                                             const char* __restrict__ wbase, char* __restrict__ mbase,
                                             char* __restrict__ smem) {
  with_weight_type(im.wdtype, [&](auto wt) { conv_segment_t<T, R, decltype(wt)>(im, strip, s0, S, wbase, mbase, smem); });
}

// ---------------------------------------------------------------------------
// single image: one workgroup per (strip, segment); exact LDS for the class
// ---------------------------------------------------------------------------
template <typename T, int R>
__global__ void __launch_bounds__(CONV_NT) conv_image_kernel(ImageDesc im, int S, const char* wbase,
                                                             char* mbase) {
  __shared__ __align__(16) char smem[ConvGeom<T, R>::SMEM];
  const int strip = blockIdx.x % im.nstrips;
  const int seg = blockIdx.x / im.nstrips;
  conv_segment<T, R>(im, strip, seg * S, S, wbase, mbase, smem);
}

// ---------------------------------------------------------------------------
// batched: persistent workgroups of one radius class walk its tile list
// (cost-sorted by the planner, split into one sublist per XCD: block b walks
// sublist b mod CONV_XCDS, so the strips of a segment row, whose input
// windows overlap, read those lines through one L2)
// ---------------------------------------------------------------------------
template <typename T, int R>
__global__ void __launch_bounds__(CONV_NT) conv_tiles_kernel(const ImageDesc* __restrict__ images,
                                                             const ConvTile* __restrict__ tiles, XcdSplit xs,
                                                             const char* wbase, char* mbase) {
  __shared__ __align__(16) char smem[ConvGeom<T, R>::SMEM];
  const int x = blockIdx.x % CONV_XCDS, nx = gridDim.x / CONV_XCDS;
  const int end = xs.beg[x + 1];
  for (int i = xs.beg[x] + (int)blockIdx.x / CONV_XCDS; i < end; i += nx) {
    const ConvTile t = tiles[i];
    const ImageDesc im = images[t.img];
    conv_segment<T, R>(im, t.strip, t.s0, t.S, wbase, mbase, smem);
    __syncthreads();  // the next tile reuses the shared memory
  }
}

// S_X = the sum of an image's FP64 partials, in a fixed order that depends
// only on the image shape, so every path gets the same bits.
__global__ void __launch_bounds__(256) sx_total_kernel(ImageDesc im, const char* mbase, double* s_x) {
  __shared__ double red[4];
  const double* part = reinterpret_cast<const double*>(mbase + im.map_off + im.part_off);
  const double s = block_sum_fixed(part, (int64_t)im.nstrips * im.nsxg * SX_SLOTS, red);
  if (threadIdx.x == 0) *s_x = s;
}

// ---------------------------------------------------------------------------
// host-side launch helpers
// ---------------------------------------------------------------------------
#define ITC_FOR_CLASSES_F32(X) X(2) X(3) X(4) X(6) X(8) X(10) X(12) X(14) X(16) X(18) X(20) X(24) X(28) X(32)
#define ITC_FOR_CLASSES_F64(X) X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(20) X(24)

// Segment length for a single image: enough workgroups to fill the chip,
// but long enough that the 2R-row warm-up of each segment stays small; a
// multiple of SX_ROWS.
int conv_segment_rows(const ImageDesc& im) {
  const int target = 1024;  // ~4 workgroups per compute unit
  int segs = (target + im.nstrips - 1) / im.nstrips;
  int S = (im.H + segs - 1) / segs;
  const int smin = 4 * im.rclass > 64 ? 4 * im.rclass : 64;
  if (S < smin) S = smin;
  S = (S + SX_ROWS - 1) / SX_ROWS * SX_ROWS;  // segments start at multiples of the S_X row group
  return S;
}

hipError_t launch_conv_image(bool f64, const ImageDesc& im, const void* w, void* m, hipStream_t s) {
  if (conv_uses_mx(f64, im.wdtype, w, im.weight_off, im.pitch)) return launch_conv_mx_image(im, w, m, s);
  const int S = conv_segment_rows(im);
  const dim3 grid(im.nstrips * ((im.H + S - 1) / S));
#define ITC_CASE_F(RR)                                                                           \
  case RR:                                                                                      \
    hipLaunchKernelGGL((conv_image_kernel<float, RR>), grid, dim3(CONV_NT), 0, s, im, S,         \
                       (const char*)w, (char*)m);                                                \
    return hipGetLastError();
#define ITC_CASE_D(RR)                                                                           \
  case RR:                                                                                      \
    hipLaunchKernelGGL((conv_image_kernel<double, RR>), grid, dim3(CONV_NT), 0, s, im, S,        \
                       (const char*)w, (char*)m);                                                \
    return hipGetLastError();
  if (f64) {
    switch (im.rclass) { ITC_FOR_CLASSES_F64(ITC_CASE_D) default: return hipErrorInvalidValue; }
  }
  switch (im.rclass) { ITC_FOR_CLASSES_F32(ITC_CASE_F) default: return hipErrorInvalidValue; }
#undef ITC_CASE_F
#undef ITC_CASE_D
}

hipError_t launch_conv_tiles(bool f64, int rclass, const ImageDesc* d_images, const ConvTile* d_tiles,
                             const XcdSplit& xs, const void* w, void* m, int grid, hipStream_t s) {
  if (rclass >= CONV_MX_CLASS) return hipErrorInvalidValue;  // launched by launch_conv_mx_tiles
  if (grid % CONV_XCDS != 0) return hipErrorInvalidValue;
#define ITC_CASE_F(RR)                                                                              \
  case RR:                                                                                         \
    hipLaunchKernelGGL((conv_tiles_kernel<float, RR>), dim3(grid), dim3(CONV_NT), 0, s, d_images,    \
                       d_tiles, xs, (const char*)w, (char*)m);                                      \
    return hipGetLastError();
#define ITC_CASE_D(RR)                                                                              \
  case RR:                                                                                         \
    hipLaunchKernelGGL((conv_tiles_kernel<double, RR>), dim3(grid), dim3(CONV_NT), 0, s, d_images,   \
                       d_tiles, xs, (const char*)w, (char*)m);                                      \
    return hipGetLastError();
  if (f64) {
    switch (rclass) { ITC_FOR_CLASSES_F64(ITC_CASE_D) default: return hipErrorInvalidValue; }
  }
  switch (rclass) { ITC_FOR_CLASSES_F32(ITC_CASE_F) default: return hipErrorInvalidValue; }
#undef ITC_CASE_F
#undef ITC_CASE_D
}

int conv_tiles_blocks_per_cu(bool f64, int rclass) {
  if (rclass >= CONV_MX_CLASS) return conv_mx_blocks_per_cu(rclass - CONV_MX_CLASS);
  int nb = 0;
#define ITC_CASE_F(RR)                                                                               \
  case RR:                                                                                          \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, conv_tiles_kernel<float, RR>, CONV_NT, 0) != \
        hipSuccess)                                                                                 \
      return 0;                                                                                     \
    return nb;
#define ITC_CASE_D(RR)                                                                                \
  case RR:                                                                                           \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, conv_tiles_kernel<double, RR>, CONV_NT, 0) != \
        hipSuccess)                                                                                  \
      return 0;                                                                                      \
    return nb;
  if (f64) {
    switch (rclass) { ITC_FOR_CLASSES_F64(ITC_CASE_D) default: return 0; }
  }
  switch (rclass) { ITC_FOR_CLASSES_F32(ITC_CASE_F) default: return 0; }
#undef ITC_CASE_F
#undef ITC_CASE_D
}

hipError_t launch_sx_finalize(const ImageDesc& img, const void* maps, double* s_x, hipStream_t s) {
  hipLaunchKernelGGL(sx_total_kernel, dim3(1), dim3(256), 0, s, img, (const char*)maps, s_x);
  return hipGetLastError();
}

}  // namespace itc

// ---------------------------------------------------------------------------
// Debug validation: count the non-finite stored weights of images (FP32 or
// FP64 weights; 8-bit weights are always finite) into a device counter.
// ---------------------------------------------------------------------------
namespace itc {
namespace {

__device__ unsigned int g_nonfinite_count;

template <typename WT>
__device__ void count_nonfinite(const ImageDesc& im, const char* wbase) {
  const WT* w = reinterpret_cast<const WT*>(wbase + im.weight_off);
  unsigned int n = 0;
  const int64_t total = (int64_t)im.H * im.W;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t u = i / im.W, v = i - u * im.W;
    n += isfinite((double)w[u * im.pitch + v]) ? 0u : 1u;
  }
  if (n) atomicAdd(&g_nonfinite_count, n);
}

__global__ void nonfinite_images_kernel(const ImageDesc* __restrict__ images, int n, const char* wbase) {
  for (int k = 0; k < n; ++k) {
    const ImageDesc im = images[k];
    if (im.wdtype == 1) count_nonfinite<float>(im, wbase);
    if (im.wdtype == 2) count_nonfinite<double>(im, wbase);
  }
}

__global__ void nonfinite_image_kernel(ImageDesc im, const char* wbase) {
  if (im.wdtype == 1) count_nonfinite<float>(im, wbase);
  if (im.wdtype == 2) count_nonfinite<double>(im, wbase);
}

}  // namespace

hipError_t count_nonfinite_weights(const ImageDesc* h_image, const ImageDesc* d_images, int n, const void* w,
                                   unsigned int* count, hipStream_t s) {
  const unsigned int zero = 0;
  hipError_t e = hipMemcpyToSymbolAsync(HIP_SYMBOL(g_nonfinite_count), &zero, sizeof zero, 0,
                                        hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  if (h_image)
    hipLaunchKernelGGL(nonfinite_image_kernel, dim3(256), dim3(256), 0, s, *h_image, (const char*)w);
  else
    hipLaunchKernelGGL(nonfinite_images_kernel, dim3(256), dim3(256), 0, s, d_images, n, (const char*)w);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipMemcpyFromSymbolAsync(count, HIP_SYMBOL(g_nonfinite_count), sizeof *count, 0, hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

}  // namespace itc
