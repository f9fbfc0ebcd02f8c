/*
 * itc_lattice.h -- C ABI of the MI355X (gfx950) lattice ITC library.
 *
 * Information theoretic clustering (Bauckhage & Kersting, "Efficient
 * Information Theoretic Clustering on Discrete Lattices") places M codevectors
 * w_k on a weighted lattice image I by minimising the Cauchy-Schwarz
 * divergence of eq. (1) with the fixed-point update of eq. (4). On a lattice
 * the data sums of eq. (4) are Gaussian convolutions (Section 3.1; weighted
 * data, Section 5). This library computes
 *
 *   A(x)   = sum_y I(y)             g(x - y)      (density map, "P = X * G")
 *   M_u(x) = sum_y I(y) (x_u - y_u) g(x - y)      (pixel-centred moments; the
 *   M_v(x) = sum_y I(y) (x_v - y_v) g(x - y)       u*I, v*I convolutions are
 *                                                   B = x A - M)
 *   S_X    = sum_x I(x) A(x)
 *
 * with g(d) = exp(-|d|^2 / (2 sigma^2)) on the square window |d_u|,|d_v| <= R,
 * and iterates, for every codevector k (Jacobi order, all from W_old):
 *
 *   A_k = A(w_k),  g_k = (B - A w)(w_k)              (bilinear map reads)
 *   C_k = sum_j g(w_j - w_k),  E_k = sum_j g(w_j - w_k)(w_j - w_k)   (all j)
 *   c   = S_XW / S_W,  S_XW = sum_k A_k,  S_W = sum_k C_k
 *   w_k <- w_k + (g_k - c E_k) / A_k       (w_k frozen when A_k == 0)
 *   D   = log S_W + log S_X - 2 log S_XW    (eq. (1) with tau = rho = sigma)
 *
 * This is eq. (4) with one kernel width (xi = omega = sigma/sqrt 2) and the
 * Parzen normalisations cancelled; D equals eq. (1) exactly in that reading.
 *
 * Coordinates: u = row, v = column, 0-based, pixel centres at integers.
 * Codebooks are arrays of M (u, v) pairs in the real type.
 *
 * Conventions for every entry point:
 *  - Buffers are device memory unless marked "host". The caller owns all of
 *    them; the library allocates nothing per call (plans own their device
 *    descriptor arrays, allocated once by itc_lattice_plan_create).
 *  - `stream` is a hipStream_t (NULL = the null stream). Calls enqueue work
 *    and return; results are valid after the stream is synchronised.
 *  - All argument checks run on the host before anything is enqueued. On an
 *    error nothing is enqueued, outputs are untouched and itc_last_error()
 *    gives the reason. No C++ exception crosses this boundary.
 *  - Checks that fail return ITC_E_NULL (null pointer), ITC_E_ARG (a size,
 *    width or count out of range), ITC_E_UNSUPPORTED (valid but beyond what
 *    the kernels are built for: R > 32 for FP32, R > 24 for FP64, M > 1024,
 *    an image or its maps of 2 GiB or more),
 *    ITC_E_DEVICE (a HIP launch or runtime error).
 */
#ifndef ITC_LATTICE_H
#define ITC_LATTICE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ITC_OK = 0,
  ITC_E_NULL = 1,
  ITC_E_ARG = 2,
  ITC_E_UNSUPPORTED = 3,
  ITC_E_DEVICE = 4
} itc_status;

typedef enum { ITC_U8 = 0, ITC_F32 = 1, ITC_F64 = 2 } itc_dtype;

/* Maximum supported sizes (ITC_E_UNSUPPORTED beyond them). */
#define ITC_MAX_RADIUS_F32 32
#define ITC_MAX_RADIUS_F64 24
#define ITC_MAX_CODEVECTORS 1024
#define ITC_MAX_CHAMFER_WIDTH 16384 /* widest image the chamfer transform accepts */
#define ITC_MAX_CHAMFER_HEIGHT 65535 /* tallest (column distances are kept as 16-bit integers) */
#define ITC_MAX_CHAMFER_STEP 64     /* largest orthogonal step cost of the chamfer mask */
#define ITC_MAX_LITERAL_RADIUS 256  /* largest window radius of G_omega in Algorithm 1 */

/*
 * One lattice problem. The weight image (Section 3.2 binary image, or
 * Section 5 per-pixel weights) is `height` rows of `width` stored values with
 * row pitch `pitch` elements; the weight is h = weight_scale * stored
 * (1 for 0/1 binary images, 1/255 for gray values g/255). `sigma` is the
 * Gaussian width in pixels (Section 2.1 with tau = rho = sigma); `radius` is
 * the truncation R of the window (Section 3.1 finite masks), 0 selecting
 * ceil(3 sigma). `real_dtype` selects FP32 or FP64 maps, codebooks and
 * arithmetic; S_X, S_XW, S_W and D are always accumulated in FP64.
 */
typedef struct {
  int32_t height;
  int32_t width;
  int64_t pitch;
  int32_t weight_dtype; /* itc_dtype of the stored weights */
  int32_t real_dtype;   /* ITC_F32 or ITC_F64 */
  double weight_scale;
  double sigma;
  int32_t radius;
  int32_t reserved; /* must be 0 */
} itc_lattice_desc;

/* Effective truncation radius of `d` (radius, or ceil(3 sigma) when 0); -1 if invalid. */
int32_t itc_lattice_radius(const itc_lattice_desc* d);

/*
 * Elements per map plane: ceil(width/16) panels x height x 16; -1 if
 * invalid. Each plane is stored in panels of 16 columns: element (u, v)
 * (row u, column v) is at index ((v / 16) * height + u) * 16 + v % 16, so
 * a 16 x 16 tile of a plane is one contiguous block (1 KiB in FP32).
 */
int64_t itc_lattice_plane_elems(const itc_lattice_desc* d);

/*
 * Bytes of the maps buffer for `d`, 0 if `d` is invalid. Layout (planes in
 * the real type): plane A, then plane M_u, then plane M_v, each
 * itc_lattice_plane_elems(d) elements in the panel layout above; then, 8-byte
 * aligned, a library-internal trailer of ceil(width/64) x ceil(height/64) x 4
 * FP64 partial sums of S_X. The size is a multiple of 256 bytes; the buffer
 * must be 256-byte aligned.
 */
size_t itc_lattice_maps_bytes(const itc_lattice_desc* d);

/*
 * Section 3.1 / Algorithm 1 "compute P once": the convolution maps of the
 * weight image and S_X. `weights` points at the stored image (layout in `d`),
 * `maps` at itc_lattice_maps_bytes(d) bytes (written), `s_x` at one double
 * (written). Map columns beyond `width` inside the last panel get unspecified
 * values. 8-bit weights whose rows start 4-byte aligned (base and pitch) take
 * the matrix-core convolution, others the vector-ALU one (same maps to
 * rounding).
 */
itc_status itc_lattice_precompute(const itc_lattice_desc* d, const void* weights, void* maps,
                                  double* s_x, void* stream);

/*
 * Algorithm 1's loop: `iters` Jacobi sweeps of eq. (4) from `w_init`
 * ([M][2], real type) with the data terms read from `maps` (as written by
 * itc_lattice_precompute for the same `d`). Stops early after a sweep whose
 * largest codevector step max_k ||w_k^new - w_k||_2 is <= theta (theta < 0:
 * never). Writes the final codebook to `w_out` ([M][2]; may alias w_init).
 * Optional outputs (NULL to skip): `d_trace` ([iters+1] doubles; entry t is D
 * at the codebook after t sweeps, entries past the stop are untouched),
 * `iters_done` (one int32, sweeps performed). `s_x` (from precompute) is
 * required when d_trace is requested, else may be NULL. iters == 0 copies
 * w_init to w_out and, when asked, writes D(w_init) to d_trace[0].
 * 1 <= M <= ITC_MAX_CODEVECTORS.
 */
itc_status itc_lattice_fit(const itc_lattice_desc* d, const void* maps, const double* s_x, int32_t M,
                           const void* w_init, int32_t iters, double theta, void* w_out,
                           double* d_trace, int32_t* iters_done, void* stream);

/*
 * Algorithm 1's loop as itc_lattice_fit computes it (same arguments and
 * outputs, same sweeps, theta stop and D trace), spread over several
 * workgroups for one large image: one launch per sweep, each of which first
 * reduces the previous sweep's per-workgroup FP64 partials of S_XW and S_W in
 * workgroup order, so results are reproducible run to run (they differ from
 * itc_lattice_fit's by the summation order of the codebook terms). All
 * iters + 2 launches are enqueued at once; launches after the stop return at
 * once, so the call is safe to capture in a HIP graph.
 *   work        device, itc_lattice_fit_wide_work_bytes(M) bytes, 256-byte
 *               aligned, owned by the caller; its contents on entry do not
 *               matter and are unspecified on return. Calls that overlap on
 *               one work buffer race.
 *   work_bytes  its size; smaller than required: ITC_E_ARG.
 * FP32 maps only (real_dtype ITC_F32, else ITC_E_UNSUPPORTED).
 */
itc_status itc_lattice_fit_wide(const itc_lattice_desc* d, const void* maps, const double* s_x, int32_t M,
                                const float* w_init, int32_t iters, double theta, float* w_out,
                                double* d_trace, int32_t* iters_done, void* work, size_t work_bytes,
                                void* stream);

/* Work buffer bytes itc_lattice_fit_wide needs for M codevectors; 0 if M is
 * outside 1..ITC_MAX_CODEVECTORS. */
size_t itc_lattice_fit_wide_work_bytes(int32_t M);

/*
 * Eq. (1) for codebook `w` ([M][2], real type): D = log S_W + log S_X -
 * 2 log S_XW, written to `d_out` (one double).
 */
itc_status itc_lattice_divergence(const itc_lattice_desc* d, const void* maps, const double* s_x,
                                  int32_t M, const void* w, double* d_out, void* stream);

/*
 * Adjoint of itc_lattice_divergence (the derivative of q with respect to w_k,
 * Section 3.1, with the sign and factor of the Gaussian derivative
 * (x - w_k)/sigma^2; weights as in Section 5). Given dL/dD in `grad_d` (one
 * double), writes
 *   grad_w[k]      = dL/dD * ( -(2/S_XW) grad A_bil(w_k) + (2/(sigma^2 S_W)) E_k )
 *   grad_weights(y) = dL/dD * ( 2 A(y)/S_X - (2/S_XW) K(y) ),
 *   K(y) = sum_k sum_c beta_kc g(c - y)   (bilinear corner weights of w_k, window R)
 * grad_w is [M][2] in the real type; grad_weights is height x width, row pitch
 * `width`, in the real type, the derivative with respect to the weight
 * h = weight_scale * stored. Either output may be NULL to skip it; `s_x`
 * (from precompute) is required for grad_weights.
 */
itc_status itc_lattice_divergence_backward(const itc_lattice_desc* d, const void* maps,
                                           const double* s_x, int32_t M, const void* w,
                                           const double* grad_d, void* grad_w, void* grad_weights,
                                           void* stream);

/*
 * Section 5 weighting: the chamfer distance transform T(X) of a binary image
 * (Borgefors' chamfer transforms, named there for P = T(X) * G_xi). T is the
 * least cost of an 8-connected path from each foreground pixel (stored value
 * != 0) to the background, orthogonal steps costing `a` and diagonal steps
 * `b` (3 and 4 give the usual 3-4 chamfer, T / a ~ Euclidean pixels);
 * background pixels get 0 and everything outside the lattice is background.
 *   d        height, width and pitch of the binary image; weight_dtype must be
 *            ITC_U8 (sigma and the other fields are not used);
 *   x        device, height x pitch bytes (read);
 *   t_out    device, height x pitch floats (written; columns >= width are
 *            left untouched), exact integer chamfer costs. It can be passed
 *            as an ITC_F32 weight image with the same pitch and
 *            weight_scale = 1/a.
 * Requires 1 <= a <= b <= 2a, a <= ITC_MAX_CHAMFER_STEP,
 * width <= ITC_MAX_CHAMFER_WIDTH and height <= ITC_MAX_CHAMFER_HEIGHT.
 * t_out is also the intermediate of the two passes. Asynchronous on
 * `stream`; no allocation.
 */
itc_status itc_lattice_chamfer(const itc_lattice_desc* d, const void* x, int32_t a, int32_t b,
                               float* t_out, void* stream);

/*
 * Algorithm 1 as the paper states it, with the update eq. (6): P = X * G_xi
 * once; then per sweep Q = W * G_omega with the codebook as an image of M
 * impulses, V(X;W) = sum P Q and V(W) = sum Q^2 over the lattice, and for
 * every codevector eq. (6) with G_omega(x - w_k) replaced by its sampled mask
 * F over the window |x - w_k| <= R_omega (Section 3.1). Codevectors are
 * lattice points: the value eq. (6) gives is rounded to the nearest lattice
 * point (halves upward) and clamped into the lattice. A codevector with
 * sum P F = 0 keeps its place; sweeps are Jacobi.
 *   d            the weight image and P's width: sigma = xi, radius = R_xi
 *                (0: ceil(3 xi)); real_dtype must be ITC_F32;
 *   weights      device weight image as in itc_lattice_precompute;
 *   omega        width of Q and F (> 0); radius_omega: R_omega (0: ceil(3 omega),
 *                at most ITC_MAX_LITERAL_RADIUS);
 *   w_init       device int32 [M][2] lattice points (u, v) (clamped into the
 *                lattice); w_out: device int32 [M][2] (may alias w_init);
 *   iters        sweeps (>= 0); theta: stop once no codevector moved farther
 *                than theta (< 0: run all sweeps);
 *   d_trace      device double [iters + 1] or NULL: D = log V(W) + log V(X)
 *                - 2 log V(X;W) before each sweep and after the last;
 *   iters_done   device int32 or NULL;
 *   work         device scratch of itc_lattice_literal_work_bytes(d, M,
 *                omega, radius_omega) bytes, 256-byte aligned (overwritten).
 * The paper's experiments choose omega = sqrt(N/M)/2 and xi = omega/2.
 * Asynchronous on `stream`: 2 (iters + 2) launches, no allocation.
 */
size_t itc_lattice_literal_work_bytes(const itc_lattice_desc* d, int32_t M, double omega,
                                      int32_t radius_omega);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): Algorithm 1
 * as itc_lattice_literal_fit, with the same arguments except `work`, which is
 * replaced by a library-owned scratch array of ITC_LITERAL_SCRATCH_MIB MiB per
 * GPU (held until the process ends; its address is looked up once per device
 * at the first call there). No allocation, no hipFree and no allocating
 * library routine on any call. Problems whose work memory
 * (itc_lattice_literal_work_bytes) exceeds the array return ITC_E_UNSUPPORTED
 * before anything is enqueued. Every call on a GPU uses that GPU's one array:
 * calls that overlap on one GPU (other streams, other threads) race, so the
 * caller serialises them; each call initialises what it reads. Same results
 * as itc_lattice_literal_fit, bit for bit.
 */
#define ITC_LITERAL_SCRATCH_MIB 64
itc_status itc_lattice_literal_fit_noalloc(const itc_lattice_desc* d, const void* weights, double omega,
                                           int32_t radius_omega, int32_t M, const int32_t* w_init, int32_t iters,
                                           double theta, int32_t* w_out, double* d_trace, int32_t* iters_done,
                                           void* stream);
itc_status itc_lattice_literal_fit(const itc_lattice_desc* d, const void* weights, double omega,
                                   int32_t radius_omega, int32_t M, const int32_t* w_init, int32_t iters,
                                   double theta, int32_t* w_out, double* d_trace, int32_t* iters_done,
                                   void* work, void* stream);

/*
 * Algorithm 1 as itc_lattice_literal_fit, from a density P the caller has
 * computed once: plane A of `maps`, as itc_lattice_precompute or
 * itc_lattice_precompute_recursive wrote it for `d`. The recursive maps give P
 * for any width xi = d->sigma >= 0.5 (Section 3.1: recursive filters replace
 * the masks at large widths), so the paper's widths omega = sqrt(N/M)/2,
 * xi = omega/2 run on any image; the weights are not read. `work` at
 * itc_lattice_literal_density_work_bytes(d, M, omega, radius_omega) bytes,
 * device, 256-byte aligned (overwritten); `maps` 256-byte aligned (read).
 * Other arguments, outputs and errors as itc_lattice_literal_fit; d->radius
 * and the radius limit of the masks do not apply.
 */
size_t itc_lattice_literal_density_work_bytes(const itc_lattice_desc* d, int32_t M, double omega,
                                              int32_t radius_omega);
itc_status itc_lattice_literal_fit_density(const itc_lattice_desc* d, const void* maps, double omega,
                                           int32_t radius_omega, int32_t M, const int32_t* w_init, int32_t iters,
                                           double theta, int32_t* w_out, double* d_trace, int32_t* iters_done,
                                           void* work, void* stream);

/*
 * Segments of a codebook (the shape segments of Section 4): labels(x) is the
 * index of the codevector nearest to pixel x (Euclidean; the smaller index on
 * equal distances) for every pixel of weight h(x) = weight_scale * stored > 0,
 * and -1 elsewhere. Distances are (u - w_u)^2 + (v - w_v)^2 in FP64 with two
 * rounded products and a rounded sum.
 *   d        weight image layout (sigma and radius are validated but unused);
 *   weights  device, as in itc_lattice_precompute;
 *   w        device [M][2] codebook in the real type;
 *   labels   device int32, height x pitch (written at the image's pitch).
 * Asynchronous on `stream`; no allocation.
 */
itc_status itc_lattice_label(const itc_lattice_desc* d, const void* weights, int32_t M, const void* w,
                             int32_t* labels, void* stream);

/*
 * Maps for large widths by recursive filtering (Section 3.1: for large kernel
 * widths recursive filters replace the finite masks; Deriche and van Vliet are
 * cited). Writes the same maps layout and S_X as itc_lattice_precompute, with
 * the Gaussian of width sigma replaced by Young and van Vliet's third-order
 * recursive Gaussian along v, then u (scaled to the mass of the unnormalised
 * sampled Gaussian), on the lattice grown by a one-pixel ring of zero weights
 * with every line extended by ceil(6 sigma) zeros; M = -sigma^2 grad A by
 * central differences. Cost per pixel independent of sigma; radius unused.
 * Map columns >= width are written as 0. Requires sigma >= 0.5 and
 * real_dtype ITC_F32. `maps` at itc_lattice_recursive_maps_bytes(d) bytes and
 * `work` at itc_lattice_recursive_work_bytes(d) bytes, both device and
 * 256-byte aligned; `s_x` one device double. itc_lattice_fit and
 * itc_lattice_divergence accept these maps for any sigma.
 */
size_t itc_lattice_recursive_maps_bytes(const itc_lattice_desc* d);
size_t itc_lattice_recursive_work_bytes(const itc_lattice_desc* d);
itc_status itc_lattice_precompute_recursive(const itc_lattice_desc* d, const void* weights, void* maps,
                                            double* s_x, void* work, void* stream);

/* ------------------------------------------------------------------------
 * 3-D lattices (volumes). The paper develops the method on 2-D lattices and
 * notes that it carries over to higher-dimensional ones; these entry points
 * are that carry-over with the readings of the 2-D calls (one width, cubic
 * window |d_axis| <= R, zero weights outside the lattice, trilinear reads with
 * off-lattice corners 0, Jacobi sweeps). Coordinates x = (s, u, v): slice,
 * row, column. Maps and codebooks are FP32; sums of S_X, S_XW, S_W and D FP64.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t depth, height, width; /* lattice extent, each >= 1                          */
  int32_t radius;               /* R; 0 => ceil(3 sigma); at most ITC_MAX_VOLUME_RADIUS */
  int64_t row_pitch;            /* elements between rows of the weights (>= width)   */
  int64_t slice_pitch;          /* elements between slices (>= height * row_pitch)  */
  int32_t weight_dtype;         /* itc_dtype: ITC_U8 | ITC_F32 | ITC_F64 (int32_t, so any value can be checked) */
  int32_t reserved;             /* must be 0                                         */
  double weight_scale;          /* h = weight_scale * stored                         */
  double sigma;                 /* kernel width (> 0)                                */
} itc_volume_desc;

#define ITC_MAX_VOLUME_RADIUS 32

/* Bytes of the maps buffer: planes A, M_s, M_u, M_v, each depth x height x
 * width FP32 contiguous, then library-internal FP64 block sums of S_X;
 * 0 if d is invalid. */
size_t itc_volume_maps_bytes(const itc_volume_desc* d);
/* Bytes of the work buffer of itc_volume_precompute (three FP32 volumes). */
size_t itc_volume_work_bytes(const itc_volume_desc* d);

/*
 * Section 3.1 in three dimensions: A = h * G and the moments
 * M_a(x) = sum_y h(y) (x_a - y_a) G(x - y), a = s, u, v, as chains of 1-D
 * correlations, and S_X = sum h A (one device double). `maps` and `work`
 * are device buffers of the sizes above, 256-byte aligned.
 */
itc_status itc_volume_precompute(const itc_volume_desc* d, const void* weights, void* maps, double* s_x,
                                 void* work, void* stream);

/*
 * Eq. (4) in three dimensions on the volume maps: `iters` Jacobi sweeps of M
 * codevectors (w_init, w_out: device FP32 [M][3] (s, u, v), may alias), D
 * before each sweep and after the last in d_trace (device double [iters + 1]
 * or NULL), early stop when no codevector moves farther than theta (< 0: off),
 * sweeps done in iters_done (device int32 or NULL). One workgroup.
 */
itc_status itc_volume_fit(const itc_volume_desc* d, const void* maps, const double* s_x, int32_t M,
                          const float* w_init, int32_t iters, double theta, float* w_out, double* d_trace,
                          int32_t* iters_done, void* stream);

/* ------------------------------------------------------------------------
 * Batched form: n independent images of uneven size, each with its own M,
 * sigma and iteration count, in flat device buffers. A plan is built once per
 * batch layout; its calls launch one persistent kernel each (convolution
 * over a cost-sorted tile queue; fit over a cost-sorted image queue) and
 * contain no allocation, synchronisation or memset, so they can be captured
 * into a HIP graph. Results are bitwise identical to the per-image calls on
 * the same stored images (the same convolution kernel is chosen when the
 * per-image weights pointer has the image's alignment).
 * All images must use real_dtype ITC_F32.
 * ------------------------------------------------------------------------ */
typedef struct itc_plan itc_plan;

typedef struct {
  int32_t n;                    /* number of images, >= 1 */
  const itc_lattice_desc* desc; /* host [n] */
  const int64_t* weight_off;    /* host [n]: byte offset of image i in the weights buffer */
  const int64_t* map_off;       /* host [n]: byte offset of image i's maps (256-aligned) */
  const int32_t* M;             /* host [n]: codevectors of image i */
  const int64_t* w_off;         /* host [n]: offset, in codevectors, of image i's codebook */
  const int32_t* iters;         /* host [n]: sweeps for image i */
} itc_batch;

/* Validates every image and builds the plan (copies descriptors to the device). */
itc_status itc_lattice_plan_create(const itc_batch* b, itc_plan** out);

/*
 * Convolution maps and S_X partials of every image: one persistent launch
 * per radius class. 8-bit images whose weight_off and pitch are multiples of
 * 4 take the matrix-core convolution; the weights base must then be 4-byte
 * aligned (ITC_E_ARG otherwise).
 */
itc_status itc_lattice_precompute_batched(itc_plan* p, const void* weights, void* maps, void* stream);

/*
 * Fit of every image (one persistent launch), then D at its final codebook.
 * Writes w_out (same offsets as w_init; may alias), s_x[i] and d_out[i]
 * (double [n], each may be NULL), iters_done[i] (int32 [n], may be NULL) and
 * status[i] (int32 [n], may be NULL): 0, or the sum of
 *   ITC_FIT_NONFINITE_SUMS  S_XW or S_W was not finite (non-finite weights or
 *                           maps): the image's sweeps stopped there and w_out
 *                           holds its last codebook, all of whose sums were
 *                           finite before; iters_done counts the sweeps done;
 *   ITC_FIT_NONFINITE_STEP  some codevector step was not finite;
 *   ITC_FIT_NONFINITE_D     D at the final codebook is not finite.
 * theta applies to every image (< 0: run all sweeps).
 */
#define ITC_FIT_NONFINITE_SUMS 1
#define ITC_FIT_NONFINITE_STEP 2
#define ITC_FIT_NONFINITE_D 4
itc_status itc_lattice_fit_batched(itc_plan* p, const void* maps, const void* w_init, double theta,
                                   void* w_out, double* s_x, double* d_out, int32_t* iters_done,
                                   int32_t* status, void* stream);

/* itc_lattice_precompute_batched followed by itc_lattice_fit_batched. */
itc_status itc_lattice_run_batched(itc_plan* p, const void* weights, void* maps, const void* w_init,
                                   double theta, void* w_out, double* s_x, double* d_out,
                                   int32_t* iters_done, int32_t* status, void* stream);

/*
 * Adjoint of the divergence of every image at codebooks `w` (same layout as
 * w_init), as itc_lattice_divergence_backward does for one image. `s_x` and
 * `grad_d` are double [n] (S_X of each image as written by the batched fit,
 * and dL/dD per image). grad_w has the codebook layout; grad_weights holds
 * image i's height x width gradient (row pitch width, real type) starting at
 * element offset weight_off[i] / sizeof(stored weight). Either output may be
 * NULL; s_x may be NULL when grad_weights is.
 */
itc_status itc_lattice_divergence_backward_batched(itc_plan* p, const void* maps, const double* s_x,
                                                   const void* w, const double* grad_d, void* grad_w,
                                                   void* grad_weights, void* stream);

/*
 * Chamfer transform (itc_lattice_chamfer) of every image of a plan whose
 * weights are ITC_U8. Image i is read at byte offset weight_off[i] of
 * `weights` and written at float offset weight_off[i] of `t_out` (the same
 * pitch), so t_out holds 4x the bytes of the weights buffer. Two launches.
 */
itc_status itc_lattice_chamfer_batched(itc_plan* p, const void* weights, int32_t a, int32_t b, float* t_out,
                                       void* stream);

/*
 * Segments (itc_lattice_label) of every image of a plan with its codebook
 * from `w` (the w_init layout, FP32). Image i's labels are written at int32
 * offset weight_off[i] / sizeof(stored weight) of `labels`, at its pitch.
 */
itc_status itc_lattice_label_batched(itc_plan* p, const void* weights, const void* w, int32_t* labels,
                                     void* stream);

/* Number of images in the plan, or -1 for NULL. */
int32_t itc_lattice_plan_size(const itc_plan* p);

/*
 * Tile shapes of a plan's convolution (the batched form of Section 3.1's
 * convolutions), for autotuning. The tiles of a radius class are 64-column
 * strips cut into segments of about `seg_rows` rows. Each vector-ALU class
 * runs one persistent launch with `blocks_per_cu` workgroups per compute
 * unit; the matrix-core classes share one persistent launch, with the
 * smallest `blocks_per_cu` set on any of them. The maps do not depend on the
 * shape (bitwise).
 *
 * itc_lattice_plan_conv_classes: number of classes, -1 if p is NULL.
 * itc_lattice_plan_conv_class: class c's key (stable identifier), current
 *   segment rows and workgroups per compute unit, and the most workgroups per
 *   compute unit the kernel's resources allow; any output pointer may be NULL.
 *   ITC_E_NULL for a NULL plan, ITC_E_ARG for c out of range.
 * itc_lattice_plan_set_conv_shape: sets the class with key `key` to
 *   `seg_rows` (64..4096, rounded up to a multiple of 64 per image; 0 = the
 *   default 256) and `blocks_per_cu` (1..the maximum; 0 = the maximum), and
 *   rebuilds and uploads its tile list (synchronous). ITC_E_ARG for an
 *   unknown key or out-of-range values. Plan set-up, not a per-call
 *   operation: no call on the plan may be in flight, and a graph captured
 *   before the change keeps the old launch shapes, so capture after tuning.
 */
int32_t itc_lattice_plan_conv_classes(const itc_plan* p);
/* Kernel launches of the plan's convolution (one per vector-ALU class, one for
 * all matrix-core classes together); -1 if p is NULL. */
int32_t itc_lattice_plan_conv_launches(const itc_plan* p);
itc_status itc_lattice_plan_conv_class(const itc_plan* p, int32_t c, int32_t* key, int32_t* seg_rows,
                                       int32_t* blocks_per_cu, int32_t* max_blocks_per_cu);
itc_status itc_lattice_plan_set_conv_shape(itc_plan* p, int32_t key, int32_t seg_rows, int32_t blocks_per_cu);

/* Frees the plan's device descriptors (after the work using them is done). NULL is a no-op. */
void itc_lattice_plan_destroy(itc_plan* p);

/* Static text of a status code. */
const char* itc_status_str(itc_status s);

/* Detail of the last error on the calling thread ("" if none). */
const char* itc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ITC_LATTICE_H */
