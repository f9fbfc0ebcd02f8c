// C-ABI host layer of the lattice ITC library: argument validation, image
// descriptors, batch plans and kernel launches. No allocation happens on the
// per-call paths; plans allocate their device descriptor arrays once.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "itc_internal.h"
#include "itc_lattice.h"

using itc::ConvTile;
using itc::ImageDesc;

namespace {

thread_local std::string g_last_error;

itc_status fail(itc_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

itc_status ok() {
  g_last_error.clear();
  return ITC_OK;
}

itc_status device_fail(hipError_t e, const char* where) {
  return fail(ITC_E_DEVICE, "%s: %s", where, hipGetErrorString(e));
}

size_t real_size(int dt) { return dt == ITC_F64 ? 8 : 4; }

bool env_flag(const char* name) {
  const char* v = std::getenv(name);
  return v && *v && std::strcmp(v, "0") != 0;
}

// ITC_DEBUG_VALIDATE: the precompute calls scan FP32/FP64 weights for
// non-finite values first (a synchronous kernel) and reject them.
bool debug_validate() {
  static const bool on = env_flag("ITC_DEBUG_VALIDATE");
  return on;
}

// ITC_TRACE: every entry point opens a roctx range named after it (shown by
// rocprofv3 --marker-trace). The roctx library is opened only then.
using roctx_push_t = int (*)(const char*);
using roctx_pop_t = int (*)();
roctx_push_t g_roctx_push = nullptr;
roctx_pop_t g_roctx_pop = nullptr;

bool trace_on() {
  static std::once_flag once;
  std::call_once(once, [] {
    if (!env_flag("ITC_TRACE")) return;
    for (const char* lib : {"librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so", "libroctx64.so.4"}) {
      void* h = dlopen(lib, RTLD_NOW | RTLD_LOCAL);
      if (!h) continue;
      g_roctx_push = reinterpret_cast<roctx_push_t>(dlsym(h, "roctxRangePushA"));
      g_roctx_pop = reinterpret_cast<roctx_pop_t>(dlsym(h, "roctxRangePop"));
      if (g_roctx_push && g_roctx_pop) return;
      g_roctx_push = nullptr;
      g_roctx_pop = nullptr;
    }
  });
  return g_roctx_push != nullptr;
}

struct TraceRange {
  bool on;
  explicit TraceRange(const char* name) : on(trace_on()) {
    if (on) g_roctx_push(name);
  }
  ~TraceRange() {
    if (on) g_roctx_pop();
  }
};

// Rejects FP32/FP64 weights holding a non-finite value when ITC_DEBUG_VALIDATE is set.
itc_status validate_weights(const ImageDesc* h_image, const ImageDesc* d_images, int n, bool any_float,
                            const void* weights, hipStream_t s);

int effective_radius(const itc_lattice_desc& d) {
  if (d.radius > 0) return d.radius;
  return (int)std::ceil(3.0 * d.sigma - 1e-12);
}

// Validates a descriptor; on success fills R and its compiled radius class.
// need_class: the entry point runs the mask convolution, so the window
// radius must have a compiled class (the fit, the labels and the recursive
// maps do not use it).
itc_status check_desc(const itc_lattice_desc* d, int* R_out, int* rc_out, bool need_class = true) {
  if (!d) return fail(ITC_E_NULL, "descriptor is NULL");
  if (d->height < 1 || d->width < 1)
    return fail(ITC_E_ARG, "height and width must be >= 1 (got %d x %d)", d->height, d->width);
  if (d->height > (1 << 20) || d->width > (1 << 20))
    return fail(ITC_E_ARG, "height and width must be <= 2^20 (got %d x %d)", d->height, d->width);
  if (d->pitch < d->width) return fail(ITC_E_ARG, "pitch %lld < width %d", (long long)d->pitch, d->width);
  if (d->weight_dtype < ITC_U8 || d->weight_dtype > ITC_F64)
    return fail(ITC_E_ARG, "weight_dtype %d is not ITC_U8/ITC_F32/ITC_F64", d->weight_dtype);
  if (d->real_dtype != ITC_F32 && d->real_dtype != ITC_F64)
    return fail(ITC_E_ARG, "real_dtype %d is not ITC_F32/ITC_F64", d->real_dtype);
  if (!std::isfinite(d->weight_scale)) return fail(ITC_E_ARG, "weight_scale is not finite");
  if (!(d->sigma > 0.0) || !std::isfinite(d->sigma))
    return fail(ITC_E_ARG, "sigma must be finite and > 0 (got %g)", d->sigma);
  if (d->radius < 0) return fail(ITC_E_ARG, "radius must be >= 0 (got %d)", d->radius);
  if (d->reserved != 0) return fail(ITC_E_ARG, "reserved must be 0");
  if (d->sigma > 1e6) return fail(ITC_E_UNSUPPORTED, "sigma %g too large", d->sigma);
  const int R = effective_radius(*d);
  if (R < 1) return fail(ITC_E_ARG, "radius must be >= 1 (got %d)", R);
  const bool f64 = d->real_dtype == ITC_F64;
  const int rc = itc::radius_class(R, f64);
  if (rc < 0 && need_class)
    return fail(ITC_E_UNSUPPORTED, "radius %d exceeds the compiled maximum %d for %s", R,
                f64 ? ITC_MAX_RADIUS_F64 : ITC_MAX_RADIUS_F32, f64 ? "FP64" : "FP32");
  // the kernels address one image and its maps with 32-bit byte offsets
  const uint64_t esz = d->weight_dtype == ITC_U8 ? 1 : (d->weight_dtype == ITC_F32 ? 4 : 8);
  const uint64_t img_bytes = (uint64_t)d->height * (uint64_t)d->pitch * esz;
  const uint64_t map_bytes = (uint64_t)3 * (uint64_t)itc::plane_elems_of(d->height, d->width) * (f64 ? 8 : 4) +
                             (uint64_t)itc::n_sx_partials(d->height, d->width) * 8 + 256;
  if (img_bytes >= (1ull << 31) || map_bytes >= (1ull << 31))
    return fail(ITC_E_UNSUPPORTED, "image (%llu B) or maps (%llu B) exceed 2 GiB", (unsigned long long)img_bytes,
                (unsigned long long)map_bytes);
  if (R_out) *R_out = R;
  if (rc_out) *rc_out = rc < 0 ? 0 : rc;
  return ITC_OK;
}

size_t planes_bytes(const itc_lattice_desc& d) {
  return (size_t)3 * (size_t)itc::plane_elems_of(d.height, d.width) * real_size(d.real_dtype);
}

// The FP64 S_X partials follow the planes, 8-byte aligned.
size_t part_offset(const itc_lattice_desc& d) { return (planes_bytes(d) + 7) / 8 * 8; }

size_t maps_bytes_of(const itc_lattice_desc& d) {
  return (part_offset(d) + (size_t)itc::n_sx_partials(d.height, d.width) * sizeof(double) + 255) / 256 * 256;
}

ImageDesc make_image(const itc_lattice_desc& d, int R, int rc) {
  ImageDesc im;
  std::memset(&im, 0, sizeof im);
  im.pitch = d.pitch;
  im.plane = itc::plane_elems_of(d.height, d.width);
  im.part_off = (int64_t)part_offset(d);
  im.scale = d.weight_scale;
  im.sigma = d.sigma;
  im.H = d.height;
  im.W = d.width;
  im.R = R;
  im.rclass = rc;
  im.wdtype = d.weight_dtype;
  im.nstrips = itc::n_strips(d.width);
  im.npanels = itc::n_panels(d.width);
  im.nsxg = itc::n_sx_groups(d.height);
  return im;
}

bool aligned256(const void* p) { return ((uintptr_t)p & 255u) == 0; }

itc_status validate_weights(const ImageDesc* h_image, const ImageDesc* d_images, int n, bool any_float,
                            const void* weights, hipStream_t s) {
  if (!debug_validate() || !any_float) return ITC_OK;
  unsigned int count = 0;
  const hipError_t e = itc::count_nonfinite_weights(h_image, d_images, n, weights, &count, s);
  if (e != hipSuccess) return device_fail(e, "weight validation");
  if (count) return fail(ITC_E_ARG, "the weights hold %u non-finite values (ITC_DEBUG_VALIDATE)", count);
  return ITC_OK;
}

int device_cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
    return 256;
  return n;
}

}  // namespace

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------
struct itc_plan {
  int n = 0;
  int m_max = 0;
  int max_passes = 1;  // largest fit pass count over the images
  std::vector<ImageDesc> images;
  // convolution class keys of the plan (tile shapes are set per key) and its
  // launches: one per vector-ALU class, one for every matrix-core class
  // together; launch l covers tiles [launch_begin[l], launch_end[l])
  std::vector<ConvTile> tiles;
  std::vector<int> cls;
  std::vector<int> launch_key, launch_begin, launch_end, launch_grid;
  std::vector<itc::XcdSplit> launch_split;  // XCD sublists of each launch (offsets from its first tile)
  int mx_max_ra = 0;  // largest aligned radius of the matrix-core images
  // convolution tile shape per class key (set by the autotuning hook; 0 =
  // default): target segment rows and workgroups per compute unit
  std::vector<int> key_seg, key_per;
  size_t tile_cap = 0;  // capacity of d_tiles (the most tiles any shape gives)
  // fit schedule: workgroup g of the fit launch (fit_grid workgroups) takes
  // the images fit_list[fit_begin[g] .. fit_begin[g + 1]) in turn
  std::vector<int32_t> fit_begin, fit_list;
  int fit_grid = 1;
  std::vector<itc::GradTile> gtiles;  // 64 x 64 tiles of every image, for dL/dh
  int grad_grid = 1;
  ImageDesc* d_images = nullptr;
  ConvTile* d_tiles = nullptr;
  int32_t* d_sched = nullptr;  // fit_begin then fit_list
  itc::GradTile* d_gtiles = nullptr;
  bool any_mx = false;  // some image runs the matrix-core convolution (4-byte aligned weights base)
  // chamfer transform: column-pass strips and row-pass row groups
  std::vector<itc::ChamferTask> ch_cols, ch_rows;
  bool all_u8 = true;
  int w_max = 0;
  int h_max = 0;
  itc::ChamferTask* d_ch_cols = nullptr;
  itc::ChamferTask* d_ch_rows = nullptr;
};

// Convolution tile lists of a plan: per class key (the VALU kernel's radius
// class, or CONV_MX_CLASS + aligned radius for the matrix-core kernel), every
// image's strips cut into segments of about the class's target height
// (multiples of the S_X row group), sorted by cost, most expensive first. A
// vector-ALU class is one persistent launch; the matrix-core classes share
// one persistent launch, largest radius first (a workgroup then changes its
// ring layout only a few times), with the fewest workgroups per compute unit
// any of them asks for. Every launch's tiles are split into one sublist per
// XCD: every segment row of an image (the strips whose input windows
// overlap) goes whole to the XCD with the least cost so far, so the
// overlapping input lines are read into one L2.
constexpr int PLAN_NKEYS = itc::CONV_MX_CLASS + 33;
constexpr int PLAN_SEG_DEFAULT = 256, PLAN_SEG_MIN = 64, PLAN_SEG_MAX = 4096;

// Fit schedule: the images, most expensive first, dealt to the F x C
// workgroups of the launch (F per compute unit, C units) round by round, in
// alternating directions from one round to the next, so that the most
// expensive image of one round and the cheapest of the next share a
// workgroup. Workgroup g's images form the list fit_list[fit_begin[g] ..
// fit_begin[g + 1]). Results do not depend on the schedule: each image's fit is
// the same code on one workgroup, wherever it runs.
static void fit_schedule(itc_plan* p, const std::vector<double>& cost, int C, int F) {
  const int n = p->n;
  std::vector<int32_t> sorted(n);
  std::iota(sorted.begin(), sorted.end(), 0);
  std::stable_sort(sorted.begin(), sorted.end(), [&](int a, int c) { return cost[a] > cost[c]; });
  const int grid = std::min(n, C * F);
  std::vector<std::vector<int32_t>> lists(grid);
  for (int r0 = 0; r0 < n; r0 += grid) {
    const int cnt = std::min(grid, n - r0);
    const bool rev = (r0 / grid) & 1;
    for (int q = 0; q < cnt; ++q) lists[rev ? cnt - 1 - q : q].push_back(sorted[r0 + q]);
  }
  p->fit_grid = grid;
  p->fit_begin.assign(1, 0);
  p->fit_list.clear();
  for (const auto& l : lists) {
    p->fit_list.insert(p->fit_list.end(), l.begin(), l.end());
    p->fit_begin.push_back((int32_t)p->fit_list.size());
  }
}

// The matrix-core kernel needs 4-byte aligned rows: a plan checks the image
// offsets and pitches here and the weights base at every call.
static int class_key_of(const ImageDesc& im) {
  return itc::conv_uses_mx(false, im.wdtype, nullptr, im.weight_off, im.pitch)
             ? itc::CONV_MX_CLASS + itc::conv_mx_radius(im.rclass)
             : im.rclass;
}

static int class_occupancy(const itc_plan* p, int key) {
  const int per = key >= itc::CONV_MX_CLASS ? itc::conv_mx_blocks_per_cu(p->mx_max_ra)
                                            : itc::conv_tiles_blocks_per_cu(false, key);
  return per < 1 ? 1 : per;
}

static void build_conv_tiles(itc_plan* p) {
  std::vector<std::vector<ConvTile>> by_class(PLAN_NKEYS);
  std::vector<std::vector<int64_t>> cost_of(PLAN_NKEYS);
  for (int i = 0; i < p->n; ++i) {
    const ImageDesc& im = p->images[i];
    const int key = class_key_of(im), rc = im.rclass;
    const int target = p->key_seg[key] > 0 ? p->key_seg[key] : PLAN_SEG_DEFAULT;
    int nseg = (im.H + target - 1) / target;
    int S = (im.H + nseg - 1) / nseg;
    S = (S + itc::SX_ROWS - 1) / itc::SX_ROWS * itc::SX_ROWS;
    nseg = (im.H + S - 1) / S;
    for (int sg = 0; sg < nseg; ++sg) {
      const int rows = std::min(S, im.H - sg * S);
      for (int st2 = 0; st2 < im.nstrips; ++st2) {
        by_class[key].push_back(ConvTile{i, st2, sg * S, S});
        cost_of[key].push_back((int64_t)(rows + 2 * rc) * (2 * rc + 1));
      }
    }
  }
  p->tiles.clear();
  p->cls.clear();
  p->launch_key.clear();
  p->launch_begin.clear();
  p->launch_end.clear();
  p->launch_grid.clear();
  p->launch_split.clear();
  const int cus = device_cus();
  auto append_sorted = [&](int key) {
    std::vector<int> idx(by_class[key].size());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int c) { return cost_of[key][a] > cost_of[key][c]; });
    for (int k : idx) p->tiles.push_back(by_class[key][k]);
  };
  // deal the segment rows of tiles [begin, end) (runs of tiles of one image
  // and segment, adjacent after the sort) to the XCD sublists, least loaded first
  auto deal_xcd = [&](int begin) {
    std::vector<std::vector<ConvTile>> sub(itc::CONV_XCDS);
    std::vector<int64_t> load(itc::CONV_XCDS, 0);
    for (int a = begin; a < (int)p->tiles.size();) {
      int b = a;
      int64_t cost = 0;
      while (b < (int)p->tiles.size() && p->tiles[b].img == p->tiles[a].img && p->tiles[b].s0 == p->tiles[a].s0) {
        const ImageDesc& im = p->images[p->tiles[b].img];
        const int halo = class_key_of(im) >= itc::CONV_MX_CLASS ? itc::conv_mx_radius(im.rclass) : im.rclass;
        cost += std::min(p->tiles[b].S, im.H - p->tiles[b].s0) + 2 * halo;
        ++b;
      }
      const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      sub[x].insert(sub[x].end(), p->tiles.begin() + a, p->tiles.begin() + b);
      load[x] += cost;
      a = b;
    }
    p->tiles.resize(begin);
    itc::XcdSplit xs{};
    for (int x = 0; x < itc::CONV_XCDS; ++x) {
      xs.beg[x] = (int)p->tiles.size() - begin;
      p->tiles.insert(p->tiles.end(), sub[x].begin(), sub[x].end());
    }
    xs.beg[itc::CONV_XCDS] = (int)p->tiles.size() - begin;
    return xs;
  };
  auto add_launch = [&](int key, int begin, int per) {
    const itc::XcdSplit xs = deal_xcd(begin);
    p->launch_key.push_back(key);
    p->launch_begin.push_back(begin);
    p->launch_end.push_back((int)p->tiles.size());
    // no more workgroups than tiles (rounded to whole XCD rounds), at most `per` per compute unit
    const int ntiles = (int)p->tiles.size() - begin;
    const int grid = std::min(per * cus, (ntiles + itc::CONV_XCDS - 1) / itc::CONV_XCDS * itc::CONV_XCDS);
    p->launch_grid.push_back(std::max(itc::CONV_XCDS, grid / itc::CONV_XCDS * itc::CONV_XCDS));
    p->launch_split.push_back(xs);
  };
  for (int key = 0; key < PLAN_NKEYS; ++key)
    if (!by_class[key].empty()) p->cls.push_back(key);
  for (int key = 0; key < itc::CONV_MX_CLASS; ++key) {
    if (by_class[key].empty()) continue;
    const int begin = (int)p->tiles.size();
    append_sorted(key);
    add_launch(key, begin, p->key_per[key] > 0 ? p->key_per[key] : class_occupancy(p, key));
  }
  const int begin = (int)p->tiles.size();
  int per = class_occupancy(p, itc::CONV_MX_CLASS);
  for (int key = PLAN_NKEYS - 1; key >= itc::CONV_MX_CLASS; --key) {
    if (by_class[key].empty()) continue;
    append_sorted(key);
    if (p->key_per[key] > 0) per = std::min(per, p->key_per[key]);
  }
  if ((int)p->tiles.size() > begin) add_launch(itc::CONV_MX_CLASS + p->mx_max_ra, begin, per);
}

extern "C" {

const char* itc_status_str(itc_status s) {
  switch (s) {
    case ITC_OK: return "ok";
    case ITC_E_NULL: return "null pointer";
    case ITC_E_ARG: return "invalid argument";
    case ITC_E_UNSUPPORTED: return "unsupported size";
    case ITC_E_DEVICE: return "device error";
  }
  return "unknown status";
}

const char* itc_last_error(void) { return g_last_error.c_str(); }

int32_t itc_lattice_radius(const itc_lattice_desc* d) {
  int R = 0;
  if (check_desc(d, &R, nullptr) != ITC_OK) return -1;
  return R;
}

int64_t itc_lattice_plane_elems(const itc_lattice_desc* d) {
  if (check_desc(d, nullptr, nullptr) != ITC_OK) return -1;
  return itc::plane_elems_of(d->height, d->width);
}

size_t itc_lattice_maps_bytes(const itc_lattice_desc* d) {
  if (check_desc(d, nullptr, nullptr) != ITC_OK) return 0;
  return maps_bytes_of(*d);
}

itc_status itc_lattice_precompute(const itc_lattice_desc* d, const void* weights, void* maps, double* s_x,
                                  void* stream) {
  TraceRange trace_range("itc_lattice_precompute");
  int R = 0, rc = 0;
  itc_status st = check_desc(d, &R, &rc);
  if (st != ITC_OK) return st;
  if (!weights || !maps || !s_x) return fail(ITC_E_NULL, "weights, maps and s_x must be non-NULL");
  if (!aligned256(maps)) return fail(ITC_E_ARG, "maps must be 256-byte aligned");
  const bool f64 = d->real_dtype == ITC_F64;
  const ImageDesc im = make_image(*d, R, rc);
  hipStream_t s = (hipStream_t)stream;
  st = validate_weights(&im, nullptr, 1, d->weight_dtype != ITC_U8, weights, s);
  if (st != ITC_OK) return st;
  hipError_t e = itc::launch_conv_image(f64, im, weights, maps, s);
  if (e != hipSuccess) return device_fail(e, "convolution launch");
  e = itc::launch_sx_finalize(im, maps, s_x, s);
  if (e != hipSuccess) return device_fail(e, "S_X launch");
  return ok();
}

static itc_status fit_common(const itc_lattice_desc* d, const void* maps, const double* s_x, int32_t M,
                             const void* w_init, int32_t iters, double theta, void* w_out, double* d_trace,
                             double* d_out, int32_t* iters_done, bool write_w, void* stream) {
  int R = 0, rc = 0;
  itc_status st = check_desc(d, &R, &rc, false);
  if (st != ITC_OK) return st;
  if (!maps || !w_init) return fail(ITC_E_NULL, "maps and the codebook must be non-NULL");
  if (write_w && !w_out) return fail(ITC_E_NULL, "w_out must be non-NULL");
  if ((d_trace || d_out) && !s_x) return fail(ITC_E_NULL, "s_x is required for the divergence");
  if (M < 1) return fail(ITC_E_ARG, "M must be >= 1 (got %d)", M);
  if (M > ITC_MAX_CODEVECTORS) return fail(ITC_E_UNSUPPORTED, "M %d exceeds %d", M, ITC_MAX_CODEVECTORS);
  if (iters < 0) return fail(ITC_E_ARG, "iters must be >= 0 (got %d)", iters);
  if (std::isnan(theta)) return fail(ITC_E_ARG, "theta is NaN");
  if (!aligned256(maps)) return fail(ITC_E_ARG, "maps must be 256-byte aligned");
  ImageDesc im = make_image(*d, R, rc);
  im.M = M;
  im.iters = iters;
  itc::FitArgs a;
  std::memset(&a, 0, sizeof a);
  a.maps = maps;
  a.w_init = w_init;
  a.w_out = w_out;
  a.s_x_in = s_x;
  a.d_trace = d_trace;
  a.d_out = d_out;
  a.iters_done = iters_done;
  a.theta = theta;
  a.n = 1;
  a.m_max = M;
  a.write_w = write_w ? 1 : 0;
  hipError_t e = itc::launch_fit(d->real_dtype == ITC_F64, nullptr, nullptr, a, 1, (hipStream_t)stream, &im);
  if (e != hipSuccess) return device_fail(e, "fit launch");
  return ok();
}

itc_status itc_lattice_fit(const itc_lattice_desc* d, const void* maps, const double* s_x, int32_t M,
                           const void* w_init, int32_t iters, double theta, void* w_out, double* d_trace,
                           int32_t* iters_done, void* stream) {
  TraceRange trace_range("itc_lattice_fit");
  return fit_common(d, maps, s_x, M, w_init, iters, theta, w_out, d_trace, nullptr, iters_done, true, stream);
}

size_t itc_lattice_fit_wide_work_bytes(int32_t M) {
  if (M < 1 || M > ITC_MAX_CODEVECTORS) return 0;
  return itc::fit_wide_work_bytes(M);
}

itc_status itc_lattice_fit_wide(const itc_lattice_desc* d, const void* maps, const double* s_x, int32_t M,
                                const float* w_init, int32_t iters, double theta, float* w_out, double* d_trace,
                                int32_t* iters_done, void* work, size_t work_bytes, void* stream) {
  TraceRange trace_range("itc_lattice_fit_wide");
  int R = 0, rc = 0;
  itc_status st = check_desc(d, &R, &rc, false);
  if (st != ITC_OK) return st;
  if (d->real_dtype != ITC_F32) return fail(ITC_E_UNSUPPORTED, "the wide fit takes FP32 maps only");
  if (!maps || !w_init || !w_out || !work) return fail(ITC_E_NULL, "maps, w_init, w_out and work must be non-NULL");
  if (d_trace && !s_x) return fail(ITC_E_NULL, "s_x is required for the divergence");
  if (M < 1) return fail(ITC_E_ARG, "M must be >= 1 (got %d)", M);
  if (M > ITC_MAX_CODEVECTORS) return fail(ITC_E_UNSUPPORTED, "M %d exceeds %d", M, ITC_MAX_CODEVECTORS);
  if (iters < 0) return fail(ITC_E_ARG, "iters must be >= 0 (got %d)", iters);
  if (std::isnan(theta)) return fail(ITC_E_ARG, "theta is NaN");
  if (!aligned256(maps) || !aligned256(work)) return fail(ITC_E_ARG, "maps and work must be 256-byte aligned");
  if (work_bytes < itc::fit_wide_work_bytes(M))
    return fail(ITC_E_ARG, "work buffer of %zu bytes, %zu needed", work_bytes, itc::fit_wide_work_bytes(M));
  ImageDesc im = make_image(*d, R, rc);
  im.M = M;
  im.iters = iters;
  hipError_t e = itc::launch_fit_wide(im, maps, s_x, w_init, iters, theta, w_out, d_trace, iters_done, work,
                                      (hipStream_t)stream);
  if (e != hipSuccess) return device_fail(e, "wide fit launch");
  return ok();
}

itc_status itc_lattice_divergence(const itc_lattice_desc* d, const void* maps, const double* s_x, int32_t M,
                                  const void* w, double* d_out, void* stream) {
  TraceRange trace_range("itc_lattice_divergence");
  if (!d_out) return fail(ITC_E_NULL, "d_out must be non-NULL");
  if (!s_x) return fail(ITC_E_NULL, "s_x must be non-NULL");
  return fit_common(d, maps, s_x, M, w, 0, -1.0, nullptr, nullptr, d_out, nullptr, false, stream);
}

itc_status itc_lattice_divergence_backward(const itc_lattice_desc* d, const void* maps, const double* s_x,
                                           int32_t M, const void* w, const double* grad_d, void* grad_w,
                                           void* grad_weights, void* stream) {
  TraceRange trace_range("itc_lattice_divergence_backward");
  int R = 0, rc = 0;
  itc_status st = check_desc(d, &R, &rc);
  if (st != ITC_OK) return st;
  if (!maps || !w || !grad_d) return fail(ITC_E_NULL, "maps, w and grad_d must be non-NULL");
  if (grad_weights && !s_x) return fail(ITC_E_NULL, "s_x is required for grad_weights");
  if (M < 1) return fail(ITC_E_ARG, "M must be >= 1 (got %d)", M);
  if (M > ITC_MAX_CODEVECTORS) return fail(ITC_E_UNSUPPORTED, "M %d exceeds %d", M, ITC_MAX_CODEVECTORS);
  if (!aligned256(maps)) return fail(ITC_E_ARG, "maps must be 256-byte aligned");
  const bool f64 = d->real_dtype == ITC_F64;
  ImageDesc im = make_image(*d, R, rc);
  im.M = M;
  im.iters = 0;
  hipStream_t s = (hipStream_t)stream;
  if (grad_w) {
    itc::FitArgs a;
    std::memset(&a, 0, sizeof a);
    a.maps = maps;
    a.w_init = w;
    a.theta = -1.0;
    a.n = 1;
    a.m_max = M;
    a.grad_w = grad_w;
    a.grad_d = grad_d;
    hipError_t e = itc::launch_fit(f64, nullptr, nullptr, a, 1, s, &im);
    if (e != hipSuccess) return device_fail(e, "codebook gradient launch");
  }
  if (grad_weights) {
    itc::GradIArgs g;
    std::memset(&g, 0, sizeof g);
    g.maps = maps;
    g.w = w;
    g.s_x = s_x;
    g.grad_d = grad_d;
    g.grad_weights = grad_weights;
    g.m_max = M;
    hipError_t e = itc::launch_grad_weights(f64, nullptr, nullptr, 0, g, 0, s, &im);
    if (e != hipSuccess) return device_fail(e, "weight gradient launch");
  }
  return ok();
}

// ---------------------------------------------------------------------------
// batched
// ---------------------------------------------------------------------------
itc_status itc_lattice_plan_create(const itc_batch* b, itc_plan** out) {
  TraceRange trace_range("itc_lattice_plan_create");
  if (!b || !out) return fail(ITC_E_NULL, "batch and out must be non-NULL");
  *out = nullptr;
  if (b->n < 1) return fail(ITC_E_ARG, "batch must hold >= 1 image (got %d)", b->n);
  if (!b->desc || !b->weight_off || !b->map_off || !b->M || !b->w_off || !b->iters)
    return fail(ITC_E_NULL, "batch arrays must be non-NULL");
  itc_plan* p = new (std::nothrow) itc_plan;
  if (!p) return fail(ITC_E_DEVICE, "out of host memory");
  p->n = b->n;
  p->images.resize(b->n);
  // class keys: the VALU kernel's radius class, or CONV_MX_CLASS + aligned
  // radius for the matrix-core kernel (8-bit weights)
  std::vector<double> fit_cost(b->n);
  for (int i = 0; i < b->n; ++i) {
    int R = 0, rc = 0;
    itc_status st = check_desc(&b->desc[i], &R, &rc);
    if (st != ITC_OK) {
      std::string why = g_last_error;
      delete p;
      return fail(st, "image %d: %s", i, why.c_str());
    }
    const itc_lattice_desc& d = b->desc[i];
    if (d.real_dtype != ITC_F32) {
      delete p;
      return fail(ITC_E_UNSUPPORTED, "image %d: the batched path is FP32 only", i);
    }
    if (b->M[i] < 1 || b->iters[i] < 0 || b->weight_off[i] < 0 || b->map_off[i] < 0 || b->w_off[i] < 0) {
      delete p;
      return fail(ITC_E_ARG, "image %d: M, iters and offsets must be non-negative (M >= 1)", i);
    }
    if (b->M[i] > ITC_MAX_CODEVECTORS) {
      delete p;
      return fail(ITC_E_UNSUPPORTED, "image %d: M %d exceeds %d", i, b->M[i], ITC_MAX_CODEVECTORS);
    }
    if (b->map_off[i] % 256 != 0) {
      delete p;
      return fail(ITC_E_ARG, "image %d: map_off must be a multiple of 256", i);
    }
    ImageDesc im = make_image(d, R, rc);
    im.weight_off = b->weight_off[i];
    im.map_off = b->map_off[i];
    im.w_off = b->w_off[i];
    im.M = b->M[i];
    im.iters = b->iters[i];
    p->images[i] = im;
    p->m_max = std::max(p->m_max, im.M);
    p->max_passes = std::max(p->max_passes, itc::fit_passes_of(im.M));
    p->tile_cap += (size_t)im.nstrips * (size_t)((im.H + PLAN_SEG_MIN - 1) / PLAN_SEG_MIN);
    fit_cost[i] = (double)(im.iters + 1) * im.M * (im.M + 16.0);
    for (int u0 = 0; u0 < im.H; u0 += 64)
      for (int v0 = 0; v0 < im.W; v0 += 64) p->gtiles.push_back(itc::GradTile{i, u0, v0, 0});
    p->all_u8 = p->all_u8 && im.wdtype == ITC_U8;
    p->w_max = std::max(p->w_max, im.W);
    p->h_max = std::max(p->h_max, im.H);
    for (int st2 = 0; st2 < im.nstrips; ++st2) p->ch_cols.push_back(itc::ChamferTask{i, st2});
    // row groups shared by the chamfer row pass and the labelling (equal heights, checked below)
    for (int r0 = 0; r0 < im.H; r0 += itc::chamfer_rows_per_task()) p->ch_rows.push_back(itc::ChamferTask{i, r0});
  }
  p->key_seg.assign(PLAN_NKEYS, 0);
  p->key_per.assign(PLAN_NKEYS, 0);
  for (const ImageDesc& im : p->images)
    if (class_key_of(im) >= itc::CONV_MX_CLASS) p->mx_max_ra = std::max(p->mx_max_ra, itc::conv_mx_radius(im.rclass));
  build_conv_tiles(p);
  const int cus = device_cus();
  int fper = itc::fit_blocks_per_cu(false, p->m_max, p->max_passes);
  if (fper < 1) fper = 1;
  fit_schedule(p, fit_cost, cus, fper);
  p->grad_grid = std::min((int)p->gtiles.size(), 4 * cus);
  for (const ImageDesc& im : p->images) p->any_mx = p->any_mx || class_key_of(im) >= itc::CONV_MX_CLASS;

  hipError_t e = hipMalloc(&p->d_images, sizeof(ImageDesc) * p->n);
  if (e == hipSuccess) e = hipMalloc(&p->d_tiles, sizeof(ConvTile) * std::max<size_t>(1, p->tile_cap));
  if (e == hipSuccess) e = hipMalloc(&p->d_sched, sizeof(int32_t) * (p->fit_begin.size() + p->fit_list.size()));
  if (e == hipSuccess)
    e = hipMemcpy(p->d_images, p->images.data(), sizeof(ImageDesc) * p->n, hipMemcpyHostToDevice);
  if (e == hipSuccess && !p->tiles.empty())
    e = hipMemcpy(p->d_tiles, p->tiles.data(), sizeof(ConvTile) * p->tiles.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(p->d_sched, p->fit_begin.data(), sizeof(int32_t) * p->fit_begin.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(p->d_sched + p->fit_begin.size(), p->fit_list.data(), sizeof(int32_t) * p->fit_list.size(),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&p->d_gtiles, sizeof(itc::GradTile) * p->gtiles.size());
  if (e == hipSuccess)
    e = hipMemcpy(p->d_gtiles, p->gtiles.data(), sizeof(itc::GradTile) * p->gtiles.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&p->d_ch_cols, sizeof(itc::ChamferTask) * p->ch_cols.size());
  if (e == hipSuccess)
    e = hipMemcpy(p->d_ch_cols, p->ch_cols.data(), sizeof(itc::ChamferTask) * p->ch_cols.size(),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&p->d_ch_rows, sizeof(itc::ChamferTask) * p->ch_rows.size());
  if (e == hipSuccess)
    e = hipMemcpy(p->d_ch_rows, p->ch_rows.data(), sizeof(itc::ChamferTask) * p->ch_rows.size(),
                  hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    itc_lattice_plan_destroy(p);
    return device_fail(e, "plan upload");
  }
  *out = p;
  return ok();
}

int32_t itc_lattice_plan_size(const itc_plan* p) { return p ? p->n : -1; }

int32_t itc_lattice_plan_conv_classes(const itc_plan* p) { return p ? (int32_t)p->cls.size() : -1; }

int32_t itc_lattice_plan_conv_launches(const itc_plan* p) { return p ? (int32_t)p->launch_key.size() : -1; }

itc_status itc_lattice_plan_conv_class(const itc_plan* p, int32_t c, int32_t* key, int32_t* seg_rows,
                                       int32_t* blocks_per_cu, int32_t* max_blocks_per_cu) {
  if (!p) return fail(ITC_E_NULL, "plan is NULL");
  if (c < 0 || c >= (int32_t)p->cls.size())
    return fail(ITC_E_ARG, "class index %d outside [0, %d)", c, (int)p->cls.size());
  const int k = p->cls[c];
  if (key) *key = k;
  if (seg_rows) *seg_rows = p->key_seg[k] > 0 ? p->key_seg[k] : PLAN_SEG_DEFAULT;
  if (blocks_per_cu) *blocks_per_cu = p->key_per[k] > 0 ? p->key_per[k] : class_occupancy(p, k);
  if (max_blocks_per_cu) *max_blocks_per_cu = class_occupancy(p, k);
  return ok();
}

itc_status itc_lattice_plan_set_conv_shape(itc_plan* p, int32_t key, int32_t seg_rows, int32_t blocks_per_cu) {
  if (!p) return fail(ITC_E_NULL, "plan is NULL");
  if (std::find(p->cls.begin(), p->cls.end(), key) == p->cls.end())
    return fail(ITC_E_ARG, "class key %d is not a convolution class of this plan", key);
  if (seg_rows != 0 && (seg_rows < PLAN_SEG_MIN || seg_rows > PLAN_SEG_MAX))
    return fail(ITC_E_ARG, "segment rows %d outside [%d, %d]", seg_rows, PLAN_SEG_MIN, PLAN_SEG_MAX);
  if (blocks_per_cu < 0 || blocks_per_cu > class_occupancy(p, key))
    return fail(ITC_E_ARG, "workgroups per compute unit %d outside [0, %d]", blocks_per_cu,
                class_occupancy(p, key));
  p->key_seg[key] = seg_rows;
  p->key_per[key] = blocks_per_cu;
  build_conv_tiles(p);
  if (p->tiles.size() > p->tile_cap) return fail(ITC_E_DEVICE, "tile list exceeds its capacity");
  hipError_t e = hipMemcpy(p->d_tiles, p->tiles.data(), sizeof(ConvTile) * p->tiles.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return device_fail(e, "tile upload");
  return ok();
}

itc_status itc_lattice_divergence_backward_batched(itc_plan* p, const void* maps, const double* s_x, const void* w,
                                                   const double* grad_d, void* grad_w, void* grad_weights,
                                                   void* stream) {
  TraceRange trace_range("itc_lattice_divergence_backward_batched");
  if (!p || !maps || !w || !grad_d) return fail(ITC_E_NULL, "plan, maps, w and grad_d must be non-NULL");
  if (grad_weights && !s_x) return fail(ITC_E_NULL, "s_x is required for grad_weights");
  if (!aligned256(maps)) return fail(ITC_E_ARG, "maps must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  if (grad_w) {
    itc::FitArgs a;
    std::memset(&a, 0, sizeof a);
    a.maps = maps;
    a.w_init = w;
    a.s_x_in = s_x;
    a.theta = -1.0;
    a.n = p->n;
    a.m_max = p->m_max;
    a.max_passes = p->max_passes;
    a.grad_w = grad_w;
    a.grad_d = grad_d;
    hipError_t e = itc::launch_fit(false, p->d_images, p->d_sched, a, p->fit_grid, s, nullptr);
    if (e != hipSuccess) return device_fail(e, "batched codebook gradient launch");
  }
  if (grad_weights) {
    itc::GradIArgs g;
    std::memset(&g, 0, sizeof g);
    g.maps = maps;
    g.w = w;
    g.s_x = s_x;
    g.grad_d = grad_d;
    g.grad_weights = grad_weights;
    g.m_max = p->m_max;
    hipError_t e = itc::launch_grad_weights(false, p->d_images, p->d_gtiles, (int)p->gtiles.size(), g,
                                            p->grad_grid, s, nullptr);
    if (e != hipSuccess) return device_fail(e, "batched weight gradient launch");
  }
  return ok();
}

void itc_lattice_plan_destroy(itc_plan* p) {
  if (!p) return;
  if (p->d_images) (void)hipFree(p->d_images);
  if (p->d_tiles) (void)hipFree(p->d_tiles);
  if (p->d_sched) (void)hipFree(p->d_sched);
  if (p->d_gtiles) (void)hipFree(p->d_gtiles);
  if (p->d_ch_cols) (void)hipFree(p->d_ch_cols);
  if (p->d_ch_rows) (void)hipFree(p->d_ch_rows);
  delete p;
}

itc_status itc_lattice_precompute_batched(itc_plan* p, const void* weights, void* maps, void* stream) {
  TraceRange trace_range("itc_lattice_precompute_batched");
  if (!p || !weights || !maps) return fail(ITC_E_NULL, "plan, weights and maps must be non-NULL");
  if (!aligned256(maps)) return fail(ITC_E_ARG, "maps must be 256-byte aligned");
  if (p->any_mx && (uintptr_t)weights % 4 != 0)
    return fail(ITC_E_ARG, "8-bit weights must be 4-byte aligned (the images' offsets and pitches are)");
  const itc_status vs = validate_weights(nullptr, p->d_images, p->n, !p->all_u8, weights, (hipStream_t)stream);
  if (vs != ITC_OK) return vs;
  for (size_t l = 0; l < p->launch_key.size(); ++l) {
    const int key = p->launch_key[l];
    hipError_t e =
        key >= itc::CONV_MX_CLASS
            ? itc::launch_conv_mx_tiles(key - itc::CONV_MX_CLASS, p->d_images, p->d_tiles + p->launch_begin[l],
                                        p->launch_split[l], weights, maps, p->launch_grid[l], (hipStream_t)stream)
            : itc::launch_conv_tiles(false, key, p->d_images, p->d_tiles + p->launch_begin[l], p->launch_split[l],
                                     weights, maps, p->launch_grid[l], (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "batched convolution launch");
  }
  return ok();
}

itc_status itc_lattice_fit_batched(itc_plan* p, const void* maps, const void* w_init, double theta, void* w_out,
                                   double* s_x, double* d_out, int32_t* iters_done, int32_t* status, void* stream) {
  TraceRange trace_range("itc_lattice_fit_batched");
  if (!p || !maps || !w_init || !w_out) return fail(ITC_E_NULL, "plan, maps, w_init and w_out must be non-NULL");
  if (std::isnan(theta)) return fail(ITC_E_ARG, "theta is NaN");
  if (!aligned256(maps)) return fail(ITC_E_ARG, "maps must be 256-byte aligned");
  itc::FitArgs a;
  std::memset(&a, 0, sizeof a);
  a.maps = maps;
  a.w_init = w_init;
  a.w_out = w_out;
  a.s_x_out = s_x;
  a.d_out = d_out;
  a.iters_done = iters_done;
  a.status = status;
  a.theta = theta;
  a.n = p->n;
  a.m_max = p->m_max;
  a.max_passes = p->max_passes;
  a.write_w = 1;
  hipError_t e = itc::launch_fit(false, p->d_images, p->d_sched, a, p->fit_grid, (hipStream_t)stream, nullptr);
  if (e != hipSuccess) return device_fail(e, "batched fit launch");
  return ok();
}

// Algorithm 1: the work buffer holds the maps of P (unless the caller gives
// P), then the taps and window overlaps, the V(X) row-block sums, the
// per-codevector sums and the state.
struct LiteralLayout {
  size_t maps, taps, vx, terms, state, total;
  int R, nvx;
};

static bool literal_layout(const itc_lattice_desc& d, int32_t M, double omega, int32_t radius_omega, bool with_maps,
                           LiteralLayout& L) {
  if (!(omega > 0.0) || !std::isfinite(omega)) return false;
  const double rr = std::ceil(3.0 * omega - 1e-12);
  const int R = radius_omega > 0 ? radius_omega : (rr > ITC_MAX_LITERAL_RADIUS ? ITC_MAX_LITERAL_RADIUS + 1 : (int)rr);
  if (R < 1 || R > ITC_MAX_LITERAL_RADIUS || M < 1) return false;
  L.R = R;
  L.nvx = (d.height + 15) / 16;
  L.maps = 0;
  L.taps = with_maps ? (maps_bytes_of(d) + 255) / 256 * 256 : 0;
  L.vx = L.taps + (size_t)(3 * R + 2) * sizeof(double);
  L.terms = L.vx + (size_t)L.nvx * sizeof(double);
  L.state = L.terms + (size_t)6 * M * sizeof(double);
  L.total = (L.state + 8 + 255) / 256 * 256;
  return true;
}

size_t itc_lattice_literal_work_bytes(const itc_lattice_desc* d, int32_t M, double omega, int32_t radius_omega) {
  int R = 0, rc = 0;
  if (!d || check_desc(d, &R, &rc) != ITC_OK) return 0;
  LiteralLayout L;
  if (!literal_layout(*d, M, omega, radius_omega, true, L)) return 0;
  return L.total;
}

size_t itc_lattice_literal_density_work_bytes(const itc_lattice_desc* d, int32_t M, double omega,
                                              int32_t radius_omega) {
  int R = 0, rc = 0;
  if (!d || check_desc(d, &R, &rc, false) != ITC_OK) return 0;
  LiteralLayout L;
  if (!literal_layout(*d, M, omega, radius_omega, false, L)) return 0;
  return L.total;
}

}  // extern "C"

// Algorithm 1 with P from the weights (density == NULL: the masks of width
// xi = d->sigma, written into the work buffer) or from the caller's maps
// (plane A of `density`), and a work buffer of `work_cap` bytes (the
// caller's, or the library's static scratch); ITC_E_UNSUPPORTED when the
// problem needs more.
static itc_status literal_fit_impl(const itc_lattice_desc* d, const void* weights, const void* density, double omega,
                                   int32_t radius_omega, int32_t M, const int32_t* w_init, int32_t iters, double theta,
                                   int32_t* w_out, double* d_trace, int32_t* iters_done, void* work, size_t work_cap,
                                   void* stream) {
  int R = 0, rc = 0;
  itc_status st = check_desc(d, &R, &rc, density == nullptr);
  if (st != ITC_OK) return st;
  if (!(weights || density) || !w_init || !w_out || !work)
    return fail(ITC_E_NULL, "the weights (or the density maps), w_init, w_out and work must be non-NULL");
  if (d->real_dtype != ITC_F32) return fail(ITC_E_UNSUPPORTED, "Algorithm 1 runs with real_dtype ITC_F32");
  if (!(omega > 0.0) || !std::isfinite(omega)) return fail(ITC_E_ARG, "omega must be finite and > 0 (got %g)", omega);
  if (M < 1) return fail(ITC_E_ARG, "M must be >= 1 (got %d)", M);
  if (M > ITC_MAX_CODEVECTORS) return fail(ITC_E_UNSUPPORTED, "M %d exceeds %d", M, ITC_MAX_CODEVECTORS);
  if (iters < 0) return fail(ITC_E_ARG, "iters must be >= 0 (got %d)", iters);
  if (std::isnan(theta)) return fail(ITC_E_ARG, "theta is NaN");
  if (!aligned256(work)) return fail(ITC_E_ARG, "work must be 256-byte aligned");
  if (density && !aligned256(density)) return fail(ITC_E_ARG, "the density maps must be 256-byte aligned");
  LiteralLayout L;
  if (!literal_layout(*d, M, omega, radius_omega, density == nullptr, L))
    return fail(radius_omega < 0 ? ITC_E_ARG : ITC_E_UNSUPPORTED, "omega window radius must be 1..%d",
                ITC_MAX_LITERAL_RADIUS);
  if (L.total > work_cap)
    return fail(ITC_E_UNSUPPORTED, "the problem needs %zu bytes of work memory, more than the %zu available",
                L.total, work_cap);
  hipStream_t s = (hipStream_t)stream;
  char* wb = (char*)work;
  if (!density) {
    const ImageDesc im = make_image(*d, R, rc);
    hipError_t e = itc::launch_conv_image(false, im, weights, wb + L.maps, s);
    if (e != hipSuccess) return device_fail(e, "convolution launch");
  }
  itc::LiteralArgs la;
  std::memset(&la, 0, sizeof la);
  la.P = reinterpret_cast<const float*>(density ? density : wb + L.maps);
  la.H = d->height;
  la.W = d->width;
  la.M = M;
  la.R = L.R;
  la.iters = iters;
  la.nvx = L.nvx;
  la.omega = omega;
  la.theta = theta;
  la.taps = reinterpret_cast<double*>(wb + L.taps);
  la.vx_part = reinterpret_cast<double*>(wb + L.vx);
  la.terms = reinterpret_cast<double*>(wb + L.terms);
  la.state = reinterpret_cast<int32_t*>(wb + L.state);
  la.d_trace = d_trace;
  la.iters_done = iters_done;
  hipError_t e = itc::launch_literal(la, w_init, w_out, s);
  if (e != hipSuccess) return device_fail(e, "Algorithm 1 launch");
  return ok();
}

itc_status itc::literal_fit_with_work(const itc_lattice_desc* d, const void* weights, double omega,
                                      int32_t radius_omega, int32_t M, const int32_t* w_init, int32_t iters,
                                      double theta, int32_t* w_out, double* d_trace, int32_t* iters_done, void* work,
                                      size_t work_cap, void* stream) {
  TraceRange trace_range("itc_lattice_literal_fit");
  if (!weights) return fail(ITC_E_NULL, "weights must be non-NULL");
  return literal_fit_impl(d, weights, nullptr, omega, radius_omega, M, w_init, iters, theta, w_out, d_trace,
                          iters_done, work, work_cap, stream);
}

itc_status itc::report_error(itc_status s, const char* msg) { return fail(s, "%s", msg); }

extern "C" {

itc_status itc_lattice_literal_fit(const itc_lattice_desc* d, const void* weights, double omega,
                                   int32_t radius_omega, int32_t M, const int32_t* w_init, int32_t iters,
                                   double theta, int32_t* w_out, double* d_trace, int32_t* iters_done, void* work,
                                   void* stream) {
  return itc::literal_fit_with_work(d, weights, omega, radius_omega, M, w_init, iters, theta, w_out, d_trace,
                                    iters_done, work, SIZE_MAX, stream);
}

itc_status itc_lattice_literal_fit_density(const itc_lattice_desc* d, const void* maps, double omega,
                                           int32_t radius_omega, int32_t M, const int32_t* w_init, int32_t iters,
                                           double theta, int32_t* w_out, double* d_trace, int32_t* iters_done,
                                           void* work, void* stream) {
  TraceRange trace_range("itc_lattice_literal_fit_density");
  if (!maps) return fail(ITC_E_NULL, "maps must be non-NULL");
  return literal_fit_impl(d, nullptr, maps, omega, radius_omega, M, w_init, iters, theta, w_out, d_trace,
                          iters_done, work, SIZE_MAX, stream);
}

itc_status itc_lattice_label(const itc_lattice_desc* d, const void* weights, int32_t M, const void* w,
                             int32_t* labels, void* stream) {
  TraceRange trace_range("itc_lattice_label");
  int R = 0, rc = 0;
  itc_status st = check_desc(d, &R, &rc, false);
  if (st != ITC_OK) return st;
  if (!weights || !w || !labels) return fail(ITC_E_NULL, "weights, w and labels must be non-NULL");
  if (M < 1) return fail(ITC_E_ARG, "M must be >= 1 (got %d)", M);
  if (M > ITC_MAX_CODEVECTORS) return fail(ITC_E_UNSUPPORTED, "M %d exceeds %d", M, ITC_MAX_CODEVECTORS);
  ImageDesc im = make_image(*d, R, rc);
  hipError_t e = itc::launch_label(d->real_dtype == ITC_F64, im, weights, w, M, labels, (hipStream_t)stream);
  if (e != hipSuccess) return device_fail(e, "labelling launch");
  return ok();
}

itc_status itc_lattice_label_batched(itc_plan* p, const void* weights, const void* w, int32_t* labels,
                                     void* stream) {
  TraceRange trace_range("itc_lattice_label_batched");
  if (!p || !weights || !w || !labels) return fail(ITC_E_NULL, "plan, weights, w and labels must be non-NULL");
  if (itc::label_rows_per_task() != itc::chamfer_rows_per_task())
    return fail(ITC_E_DEVICE, "row groups of the labelling and the chamfer pass differ");
  const int cus = device_cus();
  const int grid = std::min((int)p->ch_rows.size(), 8 * cus);
  hipError_t e = itc::launch_label_batched(p->d_images, p->d_ch_rows, (int)p->ch_rows.size(), p->m_max, weights, w,
                                           labels, grid, (hipStream_t)stream);
  if (e != hipSuccess) return device_fail(e, "batched labelling launch");
  return ok();
}

// ---------------------------------------------------------------------------
// recursive maps (large widths)
// ---------------------------------------------------------------------------
static itc_status check_recursive(const itc_lattice_desc* d, int* R, int* rc) {
  itc_status st = check_desc(d, R, rc, false);
  if (st != ITC_OK) return st;
  if (d->real_dtype != ITC_F32) return fail(ITC_E_UNSUPPORTED, "the recursive maps are FP32");
  if (d->sigma < 0.5) return fail(ITC_E_ARG, "the recursive Gaussian needs sigma >= 0.5 (got %g)", d->sigma);
  return ITC_OK;
}

static itc::RecCoeffs rec_coeffs(double sigma) {
  // Young & van Vliet (1995): q from sigma, then b0..b3
  const double q = sigma >= 2.5 ? 0.98711 * sigma - 0.96330 : 3.97156 - 4.14554 * std::sqrt(1.0 - 0.26891 * sigma);
  const double b0 = 1.57825 + 2.44413 * q + 1.4281 * q * q + 0.422205 * q * q * q;
  const double b1 = 2.44413 * q + 2.85619 * q * q + 1.26661 * q * q * q;
  const double b2 = -(1.4281 * q * q + 1.26661 * q * q * q);
  const double b3 = 0.422205 * q * q * q;
  itc::RecCoeffs c;
  c.B = 1.0 - (b1 + b2 + b3) / b0;
  c.a1 = b1 / b0;
  c.a2 = b2 / b0;
  c.a3 = b3 / b0;
  c.gain = std::sqrt(2.0 * M_PI) * sigma;
  c.m = (int)std::ceil(6.0 * sigma);
  // P = A^REC_SEG by repeated squaring (REC_SEG is a power of two)
  double P[9] = {c.a1, c.a2, c.a3, 1.0, 0.0, 0.0, 0.0, 1.0, 0.0};
  for (int n = 1; n < itc::REC_SEG; n *= 2) {
    double Q[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Q[3 * i + j] = P[3 * i] * P[j] + P[3 * i + 1] * P[3 + j] + P[3 * i + 2] * P[6 + j];
    std::copy(Q, Q + 9, P);
  }
  std::copy(P, P + 9, c.P);
  return c;
}

static size_t rec_e1_bytes(const itc_lattice_desc& d, int m) {
  return ((size_t)(d.width + 2 + m) * (size_t)(d.height + 2) * sizeof(double) + 255) / 256 * 256;
}
static size_t rec_e2_bytes(const itc_lattice_desc& d, int m) {
  return ((size_t)(d.height + 2 + m) * (size_t)(d.width + 2) * sizeof(double) + 255) / 256 * 256;
}
// segment states of either pass: [segments][3][columns] doubles
static size_t rec_z_bytes(const itc_lattice_desc& d, int m) {
  const size_t z1 = (size_t)((d.width + 2 + m + itc::REC_SEG - 1) / itc::REC_SEG) * (size_t)(d.height + 2);
  const size_t z2 = (size_t)((d.height + 2 + m + itc::REC_SEG - 1) / itc::REC_SEG) * (size_t)(d.width + 2);
  return (std::max(z1, z2) * 3 * sizeof(double) + 255) / 256 * 256;
}

size_t itc_lattice_recursive_maps_bytes(const itc_lattice_desc* d) {
  int R = 0, rc = 0;
  if (check_recursive(d, &R, &rc) != ITC_OK) return 0;
  return maps_bytes_of(*d);
}

size_t itc_lattice_recursive_work_bytes(const itc_lattice_desc* d) {
  int R = 0, rc = 0;
  if (check_recursive(d, &R, &rc) != ITC_OK) return 0;
  const int m = rec_coeffs(d->sigma).m;
  return rec_e1_bytes(*d, m) + rec_e2_bytes(*d, m) + rec_z_bytes(*d, m);
}

itc_status itc_lattice_precompute_recursive(const itc_lattice_desc* d, const void* weights, void* maps,
                                            double* s_x, void* work, void* stream) {
  TraceRange trace_range("itc_lattice_precompute_recursive");
  int R = 0, rc = 0;
  itc_status st = check_recursive(d, &R, &rc);
  if (st != ITC_OK) return st;
  if (!weights || !maps || !s_x || !work) return fail(ITC_E_NULL, "weights, maps, s_x and work must be non-NULL");
  if (!aligned256(maps) || !aligned256(work)) return fail(ITC_E_ARG, "maps and work must be 256-byte aligned");
  const itc::RecCoeffs c = rec_coeffs(d->sigma);
  const uint64_t e_elems = (uint64_t)(d->width + 2 + c.m) * (uint64_t)(d->height + 2 + c.m);
  if (e_elems >= (1ull << 31)) return fail(ITC_E_UNSUPPORTED, "image too large for the recursive maps");
  ImageDesc im = make_image(*d, R, rc);
  hipStream_t s = (hipStream_t)stream;
  double* E1 = (double*)work;
  double* E2 = (double*)((char*)work + rec_e1_bytes(*d, c.m));
  double* Z = (double*)((char*)E2 + rec_e2_bytes(*d, c.m));
  hipError_t e = itc::launch_recursive(im, weights, d->weight_scale, d->sigma, c, E1, E2, Z, maps, s);
  if (e != hipSuccess) return device_fail(e, "recursive maps launch");
  e = itc::launch_sx_finalize(im, maps, s_x, s);
  if (e != hipSuccess) return device_fail(e, "S_X launch");
  return ok();
}

// ---------------------------------------------------------------------------
// 3-D lattices
// ---------------------------------------------------------------------------
static itc_status check_volume(const itc_volume_desc* d, itc::VolumeGeom* vg) {
  if (!d) return fail(ITC_E_NULL, "volume descriptor is NULL");
  if (d->depth < 1 || d->height < 1 || d->width < 1)
    return fail(ITC_E_ARG, "depth, height and width must be >= 1 (got %d x %d x %d)", d->depth, d->height, d->width);
  if (d->row_pitch < d->width) return fail(ITC_E_ARG, "row_pitch %lld < width %d", (long long)d->row_pitch, d->width);
  if (d->slice_pitch < (int64_t)d->height * d->row_pitch)
    return fail(ITC_E_ARG, "slice_pitch %lld < height * row_pitch", (long long)d->slice_pitch);
  if (d->weight_dtype < ITC_U8 || d->weight_dtype > ITC_F64)
    return fail(ITC_E_ARG, "weight_dtype %d is not ITC_U8/ITC_F32/ITC_F64", d->weight_dtype);
  if (d->reserved != 0) return fail(ITC_E_ARG, "reserved must be 0");
  if (!std::isfinite(d->weight_scale)) return fail(ITC_E_ARG, "weight_scale is not finite");
  if (!(d->sigma > 0.0) || !std::isfinite(d->sigma))
    return fail(ITC_E_ARG, "sigma must be finite and > 0 (got %g)", d->sigma);
  if (d->radius < 0) return fail(ITC_E_ARG, "radius must be >= 0 (got %d)", d->radius);
  const double rr = std::ceil(3.0 * d->sigma - 1e-12);
  const int R = d->radius > 0 ? d->radius : (rr > ITC_MAX_VOLUME_RADIUS ? ITC_MAX_VOLUME_RADIUS + 1 : (int)rr);
  if (R < 1) return fail(ITC_E_ARG, "radius must be >= 1");
  if (R > ITC_MAX_VOLUME_RADIUS) return fail(ITC_E_UNSUPPORTED, "radius %d exceeds %d", R, ITC_MAX_VOLUME_RADIUS);
  static_assert(ITC_MAX_VOLUME_RADIUS == 32, "the volume kernels hold taps for radii up to 32");
  const uint64_t n = (uint64_t)d->depth * d->height * d->width;
  if (n * 4 * sizeof(float) >= (1ull << 31)) return fail(ITC_E_UNSUPPORTED, "volume maps exceed 2 GiB");
  if (vg) {
    vg->D = d->depth;
    vg->H = d->height;
    vg->W = d->width;
    vg->R = R;
    vg->row_pitch = d->row_pitch;
    vg->slice_pitch = d->slice_pitch;
    vg->scale = d->weight_scale;
    vg->sigma = d->sigma;
  }
  return ITC_OK;
}

static size_t volume_planes_bytes(const itc_volume_desc& d) {
  return (size_t)4 * d.depth * d.height * d.width * sizeof(float);
}

size_t itc_volume_maps_bytes(const itc_volume_desc* d) {
  itc::VolumeGeom vg;
  if (check_volume(d, &vg) != ITC_OK) return 0;
  return (volume_planes_bytes(*d) + (size_t)itc::volume_sx_blocks(vg) * sizeof(double) + 255) / 256 * 256;
}

size_t itc_volume_work_bytes(const itc_volume_desc* d) {
  if (check_volume(d, nullptr) != ITC_OK) return 0;
  return ((size_t)3 * d->depth * d->height * d->width * sizeof(float) + 255) / 256 * 256;
}

itc_status itc_volume_precompute(const itc_volume_desc* d, const void* weights, void* maps, double* s_x,
                                 void* work, void* stream) {
  TraceRange trace_range("itc_volume_precompute");
  itc::VolumeGeom vg;
  itc_status st = check_volume(d, &vg);
  if (st != ITC_OK) return st;
  if (!weights || !maps || !s_x || !work) return fail(ITC_E_NULL, "weights, maps, s_x and work must be non-NULL");
  if (!aligned256(maps) || !aligned256(work)) return fail(ITC_E_ARG, "maps and work must be 256-byte aligned");
  double* blk = (double*)((char*)maps + volume_planes_bytes(*d));
  hipError_t e = itc::launch_volume_maps(vg, d->weight_dtype, weights, (float*)work, (float*)maps, blk, s_x,
                                         (hipStream_t)stream);
  if (e != hipSuccess) return device_fail(e, "volume maps launch");
  return ok();
}

itc_status itc_volume_fit(const itc_volume_desc* d, const void* maps, const double* s_x, int32_t M,
                          const float* w_init, int32_t iters, double theta, float* w_out, double* d_trace,
                          int32_t* iters_done, void* stream) {
  TraceRange trace_range("itc_volume_fit");
  itc::VolumeGeom vg;
  itc_status st = check_volume(d, &vg);
  if (st != ITC_OK) return st;
  if (!maps || !s_x || !w_init || !w_out) return fail(ITC_E_NULL, "maps, s_x, w_init and w_out must be non-NULL");
  if (M < 1) return fail(ITC_E_ARG, "M must be >= 1 (got %d)", M);
  if (M > ITC_MAX_CODEVECTORS) return fail(ITC_E_UNSUPPORTED, "M %d exceeds %d", M, ITC_MAX_CODEVECTORS);
  if (iters < 0) return fail(ITC_E_ARG, "iters must be >= 0 (got %d)", iters);
  if (std::isnan(theta)) return fail(ITC_E_ARG, "theta is NaN");
  hipError_t e = itc::launch_volume_fit(vg, (const float*)maps, s_x, M, w_init, iters, theta, w_out, d_trace,
                                        iters_done, (hipStream_t)stream);
  if (e != hipSuccess) return device_fail(e, "volume fit launch");
  return ok();
}

static itc_status check_chamfer_mask(int32_t a, int32_t b) {
  if (a < 1 || a > ITC_MAX_CHAMFER_STEP || b < a || b > 2 * a)
    return fail(ITC_E_ARG, "chamfer steps need 1 <= a <= b <= 2a and a <= %d (got a=%d, b=%d)",
                ITC_MAX_CHAMFER_STEP, a, b);
  return ITC_OK;
}

itc_status itc_lattice_chamfer(const itc_lattice_desc* d, const void* x, int32_t a, int32_t b, float* t_out,
                               void* stream) {
  TraceRange trace_range("itc_lattice_chamfer");
  if (!d || !x || !t_out) return fail(ITC_E_NULL, "desc, x and t_out must be non-NULL");
  if (d->height < 1 || d->width < 1) return fail(ITC_E_ARG, "height and width must be >= 1");
  if (d->pitch < d->width) return fail(ITC_E_ARG, "pitch %lld < width %d", (long long)d->pitch, d->width);
  if (d->weight_dtype != ITC_U8) return fail(ITC_E_ARG, "the chamfer transform takes ITC_U8 images");
  if (d->width > ITC_MAX_CHAMFER_WIDTH)
    return fail(ITC_E_UNSUPPORTED, "width %d exceeds %d", d->width, ITC_MAX_CHAMFER_WIDTH);
  if (d->height > ITC_MAX_CHAMFER_HEIGHT)
    return fail(ITC_E_UNSUPPORTED, "height %d exceeds %d", d->height, ITC_MAX_CHAMFER_HEIGHT);
  if ((uint64_t)d->height * (uint64_t)d->pitch >= (1ull << 31))
    return fail(ITC_E_UNSUPPORTED, "image exceeds 2^31 elements");
  itc_status st = check_chamfer_mask(a, b);
  if (st != ITC_OK) return st;
  ImageDesc im;
  std::memset(&im, 0, sizeof im);
  im.H = d->height;
  im.W = d->width;
  im.pitch = d->pitch;
  hipError_t e = itc::launch_chamfer(im, x, t_out, a, b, (hipStream_t)stream);
  if (e != hipSuccess) return device_fail(e, "chamfer launch");
  return ok();
}

itc_status itc_lattice_chamfer_batched(itc_plan* p, const void* weights, int32_t a, int32_t b, float* t_out,
                                       void* stream) {
  TraceRange trace_range("itc_lattice_chamfer_batched");
  if (!p || !weights || !t_out) return fail(ITC_E_NULL, "plan, weights and t_out must be non-NULL");
  if (!p->all_u8) return fail(ITC_E_ARG, "the chamfer transform takes ITC_U8 images");
  if (p->w_max > ITC_MAX_CHAMFER_WIDTH)
    return fail(ITC_E_UNSUPPORTED, "width %d exceeds %d", p->w_max, ITC_MAX_CHAMFER_WIDTH);
  if (p->h_max > ITC_MAX_CHAMFER_HEIGHT)
    return fail(ITC_E_UNSUPPORTED, "height %d exceeds %d", p->h_max, ITC_MAX_CHAMFER_HEIGHT);
  itc_status st = check_chamfer_mask(a, b);
  if (st != ITC_OK) return st;
  const int cus = device_cus();
  const int gc = std::min((int)p->ch_cols.size(), 16 * cus);
  const int gr = std::min((int)p->ch_rows.size(), 8 * cus);
  hipError_t e = itc::launch_chamfer_batched(p->d_images, p->d_ch_cols, (int)p->ch_cols.size(), p->d_ch_rows,
                                             (int)p->ch_rows.size(), p->w_max, weights, t_out, a, b, gc, gr,
                                             (hipStream_t)stream);
  if (e != hipSuccess) return device_fail(e, "batched chamfer launch");
  return ok();
}

itc_status itc_lattice_run_batched(itc_plan* p, const void* weights, void* maps, const void* w_init, double theta,
                                   void* w_out, double* s_x, double* d_out, int32_t* iters_done, int32_t* status,
                                   void* stream) {
  itc_status st = itc_lattice_precompute_batched(p, weights, maps, stream);
  if (st != ITC_OK) return st;
  return itc_lattice_fit_batched(p, maps, w_init, theta, w_out, s_x, d_out, iters_done, status, stream);
}

}  // extern "C"
