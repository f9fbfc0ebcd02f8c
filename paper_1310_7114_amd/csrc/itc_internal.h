// Internal declarations shared by the HIP kernels and the C-ABI host layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "itc_lattice.h"

namespace itc {

// ---------------------------------------------------------------------------
// Convolution geometry: a workgroup owns a strip of CONV_TW columns and a
// segment of rows; it streams down the segment in chunks of CONV_CH rows.
// ---------------------------------------------------------------------------
constexpr int CONV_TW = 64;     // strip width = one wave of lanes
constexpr int CONV_CH = 16;     // rows per chunk
#ifndef ITC_CONV_WAVES
#define ITC_CONV_WAVES 4
#endif
constexpr int CONV_WAVES = ITC_CONV_WAVES;  // waves per workgroup, sharing one strip
constexpr int CONV_NT = 64 * CONV_WAVES;
constexpr int CONV_KB = CONV_CH / CONV_WAVES;  // output rows per lane per chunk
constexpr int ITC_MAX_CODEVECTORS_DEV = 1024;
constexpr int MAX_RADIUS = 32;

// Supported truncation radii are rounded up to one of these classes; taps
// beyond the true radius are zero, which leaves every sum unchanged.
constexpr int kRadiusClassesF32[] = {2, 3, 4, 6, 8, 10, 12, 14, 16, 18, 20, 24, 28, 32};
constexpr int kRadiusClassesF64[] = {2, 3, 4, 6, 8, 12, 16, 20, 24};

inline int radius_class(int R, bool f64) {
  if (f64) {
    for (int c : kRadiusClassesF64)
      if (R <= c) return c;
  } else {
    for (int c : kRadiusClassesF32)
      if (R <= c) return c;
  }
  return -1;
}

// Map planes are stored in panels of MAP_PANEL columns: panel p holds
// columns MAP_PANEL p .. MAP_PANEL p + MAP_PANEL - 1 of every row, row after
// row, so a 16 x 16 output tile is one contiguous 1 KiB (FP32) block. Element
// (u, v) of a plane sits at map_index(H, u, v).
constexpr int MAP_PANEL = 16;
__host__ __device__ inline int n_panels(int W) { return (W + MAP_PANEL - 1) / MAP_PANEL; }
__host__ __device__ inline int64_t plane_elems_of(int H, int W) { return (int64_t)n_panels(W) * H * MAP_PANEL; }
__host__ __device__ inline int64_t map_index(int H, int u, int v) {
  return ((int64_t)(v / MAP_PANEL) * H + u) * MAP_PANEL + (v % MAP_PANEL);
}
__host__ __device__ inline int n_strips(int W) { return (W + CONV_TW - 1) / CONV_TW; }
// S_X = sum of FP64 partials, one per (strip, SX_ROWS-row group, slot); a
// convolution segment starts at a multiple of SX_ROWS, so every partial is
// written by exactly one workgroup, and S_X is their sum in a fixed order.
constexpr int SX_ROWS = 64;
constexpr int SX_SLOTS = 4;
__host__ __device__ inline int n_sx_groups(int H) { return (H + SX_ROWS - 1) / SX_ROWS; }
__host__ __device__ inline int64_t n_sx_partials(int H, int W) {
  return (int64_t)n_strips(W) * n_sx_groups(H) * SX_SLOTS;
}

// One image as the kernels see it. Offsets are in bytes from the batch bases.
struct ImageDesc {
  int64_t weight_off;   // stored weights of this image
  int64_t pitch;        // weight row pitch, elements
  int64_t map_off;      // maps of this image (planes A, Mu, Mv, then partials)
  int64_t plane;        // elements per map plane (panels x H x MAP_PANEL)
  int64_t part_off;     // byte offset of the FP64 S_X partials inside the maps
  int64_t w_off;        // codebook offset, codevectors
  double scale;         // h = scale * stored
  double sigma;
  int32_t H, W;
  int32_t R;            // true radius (taps beyond it are zero)
  int32_t rclass;       // compiled radius class >= R
  int32_t wdtype;       // 0 u8, 1 f32, 2 f64
  int32_t M;
  int32_t iters;
  int32_t nstrips;
  int32_t npanels;
  int32_t nsxg;         // S_X row groups
  int32_t pad_;
};

// A segment of one strip: output rows [s0, s0 + S) clipped to the image.
struct ConvTile {
  int32_t img;
  int32_t strip;
  int32_t s0;
  int32_t S;
};

// Workgroups of one launch are dealt to the chip's XCDs (each with its own
// L2) in turn: workgroup b runs on XCD b mod CONV_XCDS. A tile list split in
// CONV_XCDS sublists lets workgroup b take tiles from sublist b mod CONV_XCDS
// only, so that tiles which read the same input lines (the strips of one
// segment row, whose column halos overlap) meet in one L2. Sublist x is
// tiles [beg[x], beg[x + 1]).
constexpr int CONV_XCDS = 8;
struct XcdSplit {
  int32_t beg[CONV_XCDS + 1];
};

// Batched radius classes at or above CONV_MX_CLASS select the matrix-core
// convolution (8-bit weights, FP32 maps) with aligned radius
// class - CONV_MX_CLASS (a multiple of 8).
constexpr int CONV_MX_CLASS = 64;
// The matrix-core kernel stages rows with 4-byte loads, so every row of the
// 8-bit image must start 4-byte aligned (image base and pitch).
inline bool conv_uses_mx(bool f64, int wdtype, const void* wbase, int64_t weight_off, int64_t pitch) {
  return !f64 && wdtype == 0 && ((uintptr_t)wbase + (uint64_t)weight_off) % 4 == 0 && pitch % 4 == 0;
}
int conv_mx_radius(int rclass);

// Launchers (defined in the .hip files). All return hipError_t of the launch.
// Single image (h_image by value, all strips and segments in one grid).
hipError_t launch_conv_image(bool f64, const ImageDesc& h_image, const void* weights, void* maps,
                             hipStream_t s);
// Persistent launch over `ntiles` tiles of one radius class.
hipError_t launch_conv_tiles(bool f64, int rclass, const ImageDesc* d_images, const ConvTile* d_tiles,
                             const XcdSplit& xs, const void* weights, void* maps, int grid, hipStream_t s);
// Resident workgroups per compute unit of the persistent kernels (0 on error).
int conv_tiles_blocks_per_cu(bool f64, int rclass);
int fit_blocks_per_cu(bool f64, int m_max, int max_passes);
// Segment rows used for a single image (multiple of CONV_CH).
int conv_segment_rows(const ImageDesc& im);
hipError_t launch_conv_mx_image(const ImageDesc& h_image, const void* weights, void* maps, hipStream_t s);
// One persistent launch over matrix-core tiles of aligned radii up to max_ra
// (8, 16, 24 or 32), each workgroup walking its XCD's sublist in order
// (grid a multiple of CONV_XCDS).
hipError_t launch_conv_mx_tiles(int max_ra, const ImageDesc* d_images, const ConvTile* d_tiles, const XcdSplit& xs,
                                const void* weights, void* maps, int grid, hipStream_t s);
int conv_mx_blocks_per_cu(int max_ra);
// Debug validation (ITC_DEBUG_VALIDATE): the number of non-finite stored
// weights of one image (h_image) or of n plan images (d_images); waits for
// the stream.
hipError_t count_nonfinite_weights(const ImageDesc* h_image, const ImageDesc* d_images, int n, const void* w,
                                   unsigned int* count, hipStream_t s);
// S_X of one image: the fixed-order sum of its FP64 partials.
hipError_t launch_sx_finalize(const ImageDesc& img, const void* maps, double* s_x, hipStream_t s);
// 3-D lattices: one volume (slice, row, column) and its window radius.
struct VolumeGeom {
  int32_t D, H, W, R;
  int64_t row_pitch, slice_pitch;  // elements, of the stored weights
  double scale, sigma;
};
int volume_sx_blocks(const VolumeGeom& vg);  // FP64 partials of S_X after the planes
hipError_t launch_volume_maps(const VolumeGeom& vg, int wdtype, const void* x, float* work, float* maps,
                              double* sx_blk, double* s_x, hipStream_t s);
hipError_t launch_volume_fit(const VolumeGeom& vg, const float* maps, const double* s_x, int M, const float* w_init,
                             int iters, double theta, float* w_out, double* d_trace, int32_t* iters_done,
                             hipStream_t s);

// Young-van Vliet recursive Gaussian: coefficients, output gain and the
// zero margin appended to every line.
// Recursive Gaussian: w[n] = B x[n] + a1 w[n-1] + a2 w[n-2] + a3 w[n-3] per
// direction, output times gain; lines padded by m zeros; P = A^REC_SEG
// (row-major) for the companion matrix A of (a1, a2, a3).
constexpr int REC_SEG = 64;
struct RecCoeffs {
  double B, a1, a2, a3, gain;
  double P[9];
  int m;
};
hipError_t launch_recursive(const ImageDesc& im, const void* x, double scale, double sigma, const RecCoeffs& rc,
                            double* E1, double* E2, double* Z, void* maps, hipStream_t s);

// Algorithm 1 (eq. (6) on the lattice): device pointers into the caller's
// work buffer and the sweep parameters.
struct LiteralArgs {
  const float* P;   // A plane of the maps with sigma = xi (panel layout)
  int32_t H, W, M;
  int32_t R;        // window radius of G_omega
  int32_t iters;
  int32_t nvx;      // row blocks of the V(X) sum
  double omega, theta;
  double* taps;     // [R + 1] g, then [2R + 1] window overlaps
  double* vx_part;  // [nvx]
  double* terms;    // [6 M]: a, b_u, b_v, e, d_u, d_v
  int32_t* state;
  double* d_trace;      // [iters + 1] or null
  int32_t* iters_done;  // or null
};
hipError_t launch_literal(const LiteralArgs& la, const int32_t* w_init, int32_t* w_out, hipStream_t s);
// The body of itc_lattice_literal_fit with a work buffer of work_cap bytes
// (host layer), and the host layer's error reporting.
itc_status literal_fit_with_work(const itc_lattice_desc* d, const void* weights, double omega, int32_t radius_omega,
                                 int32_t M, const int32_t* w_init, int32_t iters, double theta, int32_t* w_out,
                                 double* d_trace, int32_t* iters_done, void* work, size_t work_cap, void* stream);
itc_status report_error(itc_status s, const char* msg);

// Chamfer transform: a task is (image, strip) for the column pass and
// (image, first row) for the row pass.
struct ChamferTask {
  int32_t img;
  int32_t pos;
};
int chamfer_rows_per_task();
hipError_t launch_chamfer(const ImageDesc& im, const void* x, float* t, int a, int b, hipStream_t s);
hipError_t launch_chamfer_batched(const ImageDesc* d_images, const ChamferTask* d_cols, int ncols,
                                  const ChamferTask* d_rows, int nrows, int w_max, const void* x, float* t, int a,
                                  int b, int grid_cols, int grid_rows, hipStream_t s);
int label_rows_per_task();
hipError_t launch_label(bool f64, const ImageDesc& im, const void* x, const void* w, int M, int32_t* lab,
                        hipStream_t s);
hipError_t launch_label_batched(const ImageDesc* d_images, const ChamferTask* d_tasks, int ntasks, int m_max,
                                const void* x, const void* w, int32_t* lab, int grid, hipStream_t s);

struct FitArgs {
  const void* maps;      // batch base of maps
  const void* w_init;    // batch base of codebooks
  void* w_out;
  double* s_x_out;       // [n] or null (batched: written from the partials)
  const double* s_x_in;  // single image: precomputed S_X (may be null when not needed)
  double* d_trace;       // single image: [iters+1] or null
  double* d_out;         // [n] or null
  int32_t* iters_done;   // [n] or null
  int32_t* status;       // [n] status bits per image, or null (batched only)
  double theta;
  int32_t n;             // images
  int32_t m_max;         // largest M (sizes the shared memory)
  int32_t write_w;       // 0: do not write w_out (divergence only)
  void* grad_w;          // non-null: gradient mode, dL/dw at w_init (same layout), no update
  const double* grad_d;  // gradient mode: dL/dD per image
  int32_t max_passes;    // largest fit_passes(M) of the launch (0: derive from m_max)
};

// Passes of the fit over an image's owned codevectors (1..4).
int fit_passes_of(int M);

// Fit of one image (h_image set: one workgroup) or of a batch: `grid`
// workgroups, workgroup g taking the images d_sched[grid + 1 + k] for k in
// [d_sched[g], d_sched[g + 1]) (the plan's schedule: grid + 1 list offsets,
// then the image indices).
hipError_t launch_fit(bool f64, const ImageDesc* d_images, const int32_t* d_sched, const FitArgs& a,
                      int grid, hipStream_t s, const ImageDesc* h_image);

// The fit of one FP32 image over several workgroups, one launch per sweep:
// workgroups used, work buffer bytes (256-byte multiple) and shared memory
// bytes for M codevectors.
int fit_wide_groups(int M);
size_t fit_wide_work_bytes(int M);
size_t fit_wide_smem(int M);
hipError_t launch_fit_wide(const ImageDesc& im, const void* maps, const double* s_x, const float* w_init, int iters,
                           double theta, float* w_out, double* d_trace, int32_t* iters_done, void* work,
                           hipStream_t s);

// dL/dh over one 64 x 64 pixel tile of an image.
struct GradTile {
  int32_t img;
  int32_t u0, v0;
  int32_t pad_;
};

struct GradIArgs {
  const void* maps;
  const void* w;          // codebooks (batch base)
  const double* s_x;      // [n] (single image: [1])
  const double* grad_d;   // [n]
  void* grad_weights;     // gradients in the real type at each image's weight element offset
  int32_t m_max;
};

// Single image when h_image is non-null (grid covers its tiles), else a
// persistent launch over `ntiles` tiles.
hipError_t launch_grad_weights(bool f64, const ImageDesc* d_images, const GradTile* d_tiles, int ntiles,
                               const GradIArgs& a, int grid, hipStream_t s, const ImageDesc* h_image);
int grad_tiles_of(int H, int W);  // tiles per image

}  // namespace itc
