// Host side of the C ABI declared in include/mcl.h.
//
// Validates arguments, carves caller-provided device workspaces, computes the
// per-step scalars in FP64 (taps, heading bookkeeping, sub-cell gate) and
// enqueues the kernels on the handle's stream.  No device allocation happens
// here; all per-state arithmetic runs in the HIP kernels.
#include <float.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mcl.h"
#include "mcl_internal.hpp"
#include "scan.hpp"

using namespace mcl;

namespace {

thread_local std::string g_err;

mcl_status fail(mcl_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

mcl_status hip_fail(hipError_t e, const char* what) {
  return fail(MCL_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                     \
  do {                                          \
    hipError_t e_ = (expr);                     \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

int round_up(int x, int m) { return (x + m - 1) / m * m; }

int resolve_radius(double sigma, int r) { return r >= 0 ? r : static_cast<int>(ceil(3.0 * sigma)); }

void gaussian_taps(double sigma, int radius, double* g) {
  double z = 0.0;
  for (int m = -radius; m <= radius; ++m) {
    const double v = sigma == 0.0 ? (m == 0 ? 1.0 : 0.0) : exp(-(m * (double)m) / (2.0 * sigma * sigma));
    g[m + radius] = v;
    z += v;
  }
  for (int i = 0; i <= 2 * radius; ++i) g[i] /= z;
}

size_t dtype_bytes(int dt) { return dt == MCL_F32 ? 4 : 2; }

// Radius of the rotated 2-D kernel (MCL_ANISOTROPIC).
int aniso_radius(const mcl_params* p) {
  return p->radius_xy >= 0 ? p->radius_xy
                           : static_cast<int>(ceil(3.0 * std::max(p->sigma_xy_cells, p->sigma_lateral_cells)));
}

mcl_status check_params(const mcl_params* p, bool need_theta) {
  if (!p) return fail(MCL_EINVAL, "params is NULL");
  if (!(p->sigma_xy_cells >= 0.0) || !isfinite(p->sigma_xy_cells))
    return fail(MCL_EINVAL, "sigma_xy_cells must be finite and >= 0");
  if (p->flags & ~0x3Fu) return fail(MCL_EINVAL, "unknown flags 0x%x", p->flags);
  if (p->flags & MCL_ANISOTROPIC) {
    // the map keeps only sigma_xy; the filter brings the lateral std-dev
    if (need_theta) {
      if (!(p->sigma_xy_cells > 0.0) || !(p->sigma_lateral_cells > 0.0) || !isfinite(p->sigma_lateral_cells))
        return fail(MCL_EINVAL, "anisotropic noise needs sigma_xy_cells > 0 and sigma_lateral_cells > 0");
      const int ra = aniso_radius(p);
      if (ra > kAnisoMaxRadius) return fail(MCL_EINVAL, "2-D blur radius %d exceeds %d", ra, kAnisoMaxRadius);
    }
  } else {
    const int rxy = resolve_radius(p->sigma_xy_cells, p->radius_xy);
    if (rxy > kMaxRadius) return fail(MCL_EINVAL, "xy blur radius %d exceeds %d", rxy, kMaxRadius);
  }
  if (need_theta) {
    if (p->n_theta < 1 || p->n_theta > kMaxTheta)
      return fail(MCL_EINVAL, "n_theta must be in [1, %d]", kMaxTheta);
    if (!(p->sigma_theta_bins >= 0.0) || !isfinite(p->sigma_theta_bins))
      return fail(MCL_EINVAL, "sigma_theta_bins must be finite and >= 0");
    const int rth = resolve_radius(p->sigma_theta_bins, p->radius_theta);
    if (rth > kMaxRadius) return fail(MCL_EINVAL, "theta blur radius %d exceeds %d", rth, kMaxRadius);
    if (p->storage < MCL_F32 || p->storage > MCL_F16) return fail(MCL_EINVAL, "unknown storage type");
    for (int i = 0; i < 7; ++i)
      if (p->launch_shape[i] < 0 || p->launch_shape[i] > 4096)
        return fail(MCL_EINVAL, "launch_shape[%d] = %d out of range", i, p->launch_shape[i]);
    const int al = p->launch_shape[6];
    if (al != 0 && (al & (al - 1)) != 0) return fail(MCL_EINVAL, "strip alignment %d is not a power of two", al);
  }
  return MCL_OK;
}

mcl_status check_desc(const mcl_map_desc* d, const mcl_params* p) {
  if (!d) return fail(MCL_EINVAL, "desc is NULL");
  if (d->width < 1 || d->height < 1 || d->width > 65536 || d->height > 65536)
    return fail(MCL_EINVAL, "map size %dx%d out of range", d->width, d->height);
  if (!(d->cell_m > 0.0) || !isfinite(d->cell_m)) return fail(MCL_EINVAL, "cell_m must be > 0");
  if (!d->occupancy) return fail(MCL_EINVAL, "occupancy is NULL");
  if (d->range_table) {
    if (d->n_dirs < 1 || d->n_dirs > kScanMaxDirs)
      return fail(MCL_EINVAL, "n_dirs must be in [1, %d]", kScanMaxDirs);
    if (!(d->max_range_m > 0.0) || !isfinite(d->max_range_m))
      return fail(MCL_EINVAL, "max_range_m must be > 0");
    // the scan kernels address the quantised table with 32-bit byte offsets
    const size_t cells = (static_cast<size_t>(d->height) * round_up(d->width, kRowAlign) + 31) / 32 * 32;
    const size_t kpad = (static_cast<size_t>(d->n_dirs) + 63) / 64 * 64;
    const size_t eb = (p && (p->flags & MCL_SCAN_F32)) ? 4 : 2;
    if (cells * kpad * eb >= (static_cast<size_t>(1) << 32))
      return fail(MCL_EINVAL, "range table of %zu bytes exceeds the 4 GiB the scan kernels address",
                  cells * kpad * eb);
  }
  return MCL_OK;
}

}  // namespace

// ---- handles -------------------------------------------------------------------

struct mcl_map_s {
  int W = 0, H = 0, pitch = 0;
  double cell = 0.0;
  double sigma_xy = 0.0;
  int rxy = 0;
  uint32_t flags = 0;
  hipStream_t stream = nullptr;
  uint8_t* occ_dev = nullptr;
  uint8_t* free8 = nullptr;
  float* mpre = nullptr;
  float* wt = nullptr;
  int64_t n_free = 0;
  ScanTable scan;  // quantised range table (scan.hpp)
};

struct StepShape {
  KernelShape k;
  int chunks = 1, chunk_len = 1, tiles_x = 1, tiles_y = 1, strip = 0;
  int blocks() const { return tiles_x * tiles_y * chunks; }
};

struct mcl_filter_s {
  mcl_map map = nullptr;
  int T = 0;
  int dtype = 0;
  int radius = 1;
  double sigma_th = 0.0;
  int rth = 0;
  hipStream_t stream = nullptr;
  void* buf[2] = {nullptr, nullptr};
  float* staging = nullptr;
  double* partials = nullptr;
  int n_partials = 0;
  FilterDev* dev = nullptr;
  float* scan_scratch = nullptr;
  int32_t* samp_list = nullptr;  // sampled update: selected cells, then positions (2 x H * pitch)
  ScanWork scanw;
  int64_t sstride = 0;
  double theta = 0.0;
  double acc_x = 0.0, acc_y = 0.0;
  double rem[kMaxTheta][2] = {};  // carried remainders of the whole-cell warp, cells
  int32_t* ishift = nullptr;      // device: whole-cell shifts of the current warp
  ShiftEntry* table_dev = nullptr;  // device: shift table of the current warp (heading counts above
                                    // kArgTableMax; smaller tables travel in the kernel arguments)
  ShiftEntry table[kMaxTheta] = {};  // host: shift table of the current warp
  float* aniso_tmp = nullptr;     // MCL_ANISOTROPIC: FP32 scratch of the theta-blurred tensor
  float* aniso_taps = nullptr;    // MCL_ANISOTROPIC: FP32 2-D taps per channel
  double sf = 0.0, sl = 0.0;      // MCL_ANISOTROPIC: std-devs along / across the heading
  int raniso = 0;                 // MCL_ANISOTROPIC: 2-D kernel radius
  double gth_sum = 1.0;           // sum of the theta taps
  int64_t steps = 0;
  StepShape shape;
  float gxy[kMaxTaps] = {};
  float gth[kMaxTaps] = {};
};

namespace {

constexpr int kReduceBlocks = 1024;

// The streaming kernel addresses one heading plane with 32-bit buffer offsets
// whose out-of-grid markers start at 2^30, so a plane must stay below 1 GiB.
bool stream_plane_ok(int W, int H, size_t eb) {
  const size_t pitch = (static_cast<size_t>(W) + kRowAlign - 1) / kRowAlign * kRowAlign;
  return pitch * static_cast<size_t>(H) * eb < (static_cast<size_t>(1) << 30);
}

// Launch shape of the step kernel, from measurements on MI355X (the numbers
// below are per step; bench-style loops of 300 steps after a warm-up).  Maps
// of fewer than 512 64 x 16 tiles: the variant-1 streaming kernel (mask in the
// y taps, theta blur before the x blur, host shift table, emit pipelined
// against the next warp), 4-row strips, 4 waves, two slice buffers, 56-column
// strips (32-byte aligned for FP32, 4-byte for 16-bit storage; 512^2 x 72
// FP32: 1280 workgroups, five waves per SIMD, 41.4 us, against 45.8 us with
// 57-column strips and 1152 workgroups and 52.6 us for the variant-0 kernel at
// its best shape).  Larger maps: the variant-0 streaming
// kernel with 16-row strips, 8 waves and one slice buffer (1024^2 x 128: FP32
// 333 us with 32-byte aligned strips, BF16 241 us with 4-byte ones; the other
// shapes and variants measured 247-379 us).  The tiled kernel remains for
// planes of 1 GiB or more, which the streaming kernels' 32-bit offsets cannot
// address.  A nonzero launch_shape in the parameters overrides the choice.
StepShape choose_shape(int W, int H, int T, int R, size_t eb, const int32_t* force) {
  StepShape s;
  const int tiled_tiles = ((W + 63) / 64) * ((H + 15) / 16);
  int sh[7] = {64, 16, 256, 0, 2, 0, kStreamAlignBytes};
  if (stream_plane_ok(W, H, eb)) {
    if (tiled_tiles < 512) {
      const int v[7] = {0, 4, 256, 1, 2, 1, eb == 4 ? 32 : 4};
      for (int i = 0; i < 7; ++i) sh[i] = v[i];
    } else {
      const int v[7] = {0, 16, 512, 1, 1, 0, eb == 4 ? 32 : 4};
      for (int i = 0; i < 7; ++i) sh[i] = v[i];
    }
  }
  bool forced = false;
  for (int i = 0; force && i < 7; ++i) forced = forced || force[i] != 0;
  if (forced) {
    for (int i = 0; i < 7; ++i) sh[i] = force[i];
    if (sh[6] == 0) sh[6] = kStreamAlignBytes;
  }
  s.k.tx = sh[0];
  s.k.ty = sh[1];
  s.k.nt = sh[2];
  s.k.nbuf = sh[0] == 0 ? sh[4] : 2;
  s.k.variant = sh[0] == 0 ? sh[5] : 0;
  s.strip = stream_strip_width(R, static_cast<int>(eb), sh[6]);
  if (s.strip <= 0) s.strip = 63 - 2 * R;
  const int strip = s.k.tx > 0 ? s.k.tx : s.strip;
  s.tiles_x = (W + strip - 1) / strip;
  s.tiles_y = (H + std::max(1, s.k.ty) - 1) / std::max(1, s.k.ty);
  const int tiles = s.tiles_x * s.tiles_y;
  int chunks = sh[3];
  if (chunks <= 0) {
    // aim for at least two workgroups per compute unit; every chunk keeps at
    // least 2R+1 channels so the recomputed halo stays below its own size
    chunks = std::max(1, (512 + tiles - 1) / tiles);
    chunks = std::min(chunks, std::max(1, T / (2 * R + 1)));
  }
  chunks = std::min(chunks, T);
  s.chunk_len = (T + chunks - 1) / chunks;
  s.chunks = (T + s.chunk_len - 1) / s.chunk_len;
  return s;
}

StepArgs make_step_args(mcl_filter f) {
  StepArgs a = {};
  const mcl_map m = f->map;
  a.buf[0] = f->buf[0];
  a.buf[1] = f->buf[1];
  a.mpre = m->mpre;
  a.wt = m->wt;
  a.partials = f->partials;
  a.dev = f->dev;
  a.W = m->W;
  a.H = m->H;
  a.pitch = m->pitch;
  a.n_theta = f->T;
  a.tiles_x = f->shape.tiles_x;
  a.tiles_y = f->shape.tiles_y;
  a.chunks = f->shape.chunks;
  a.chunk_len = f->shape.chunk_len;
  a.strip = f->shape.strip;
  a.sstride = f->sstride;
  a.dtheta = 2.0 * M_PI / f->T;
  for (int i = 0; i < kMaxTaps; ++i) {
    a.gxy[i] = f->gxy[i];
    a.gth[i] = f->gth[i];
  }
  return a;
}

ReduceArgs make_reduce_args(mcl_filter f, int mode, double factor) {
  ReduceArgs r = {};
  r.buf[0] = f->buf[0];
  r.buf[1] = f->buf[1];
  r.partials = f->partials;
  r.dev = f->dev;
  r.W = f->map->W;
  r.H = f->map->H;
  r.pitch = f->map->pitch;
  r.n_theta = f->T;
  r.sstride = f->sstride;
  r.factor = factor;
  r.mode = mode;
  return r;
}

mcl_status read_dev(mcl_filter f, FilterDev* out) {
  HIP_TRY(hipMemcpyAsync(out, f->dev, sizeof(FilterDev), hipMemcpyDeviceToHost, f->stream), "read scalars");
  HIP_TRY(hipStreamSynchronize(f->stream), "synchronize");
  return MCL_OK;
}

// Carve (or measure, when ws == nullptr) a filter workspace.
size_t carve_filter(mcl_filter f, void* ws, const mcl_map m, const mcl_params* p) {
  Carver c(ws);
  const int64_t sstride = static_cast<int64_t>(m->H) * m->pitch;
  const size_t n = static_cast<size_t>(sstride) * p->n_theta;
  const size_t eb = dtype_bytes(p->storage);
  void* b0 = c.take(n * eb);
  void* b1 = c.take(n * eb);
  float* staging = static_cast<float*>(c.take(static_cast<size_t>(m->W) * m->H * sizeof(float)));
  const int R = std::max(1, std::max(m->rxy, resolve_radius(p->sigma_theta_bins, p->radius_theta)));
  const StepShape sh = choose_shape(m->W, m->H, p->n_theta, R, eb, p->launch_shape);
  int np = std::max(sh.blocks(), std::max(kReduceBlocks, kScanMaxBlocks(m->W, m->H, m->pitch)));
  if (p->flags & MCL_ANISOTROPIC) np = std::max(np, aniso_workgroups(m->W, m->H, p->n_theta));
  double* partials = static_cast<double*>(c.take(static_cast<size_t>(np) * 3 * sizeof(double)));
  FilterDev* dev = static_cast<FilterDev*>(c.take(kDevRegionBytes));
  int32_t* ishift = static_cast<int32_t*>(c.take(2 * kMaxTheta * sizeof(int32_t)));
  ShiftEntry* table_dev = static_cast<ShiftEntry*>(c.take(kMaxTheta * sizeof(ShiftEntry)));
  float* atmp = (p->flags & MCL_ANISOTROPIC) ? static_cast<float*>(c.take(n * sizeof(float))) : nullptr;
  constexpr int kAnisoTaps = (2 * kAnisoMaxRadius + 1) * (2 * kAnisoMaxRadius + 1);
  float* ataps = (p->flags & MCL_ANISOTROPIC)
                     ? static_cast<float*>(c.take(static_cast<size_t>(p->n_theta) * kAnisoTaps * sizeof(float)))
                     : nullptr;
  float* scratch = nullptr;
  int32_t* samp = nullptr;
  if (m->scan.n_dirs > 0) {
    scratch = static_cast<float*>(c.take(n * sizeof(float)));
    samp = static_cast<int32_t*>(c.take(2 * static_cast<size_t>(sstride) * sizeof(int32_t)));
  }
  void* scanw = c.take(scan_work_bytes(p->n_theta, m->scan.kpad));
  if (f) {
    f->buf[0] = b0;
    f->buf[1] = b1;
    f->staging = staging;
    f->partials = partials;
    f->n_partials = np;
    f->dev = dev;
    f->scan_scratch = scratch;
    f->samp_list = samp;
    f->ishift = ishift;
    f->table_dev = table_dev;
    f->aniso_tmp = atmp;
    f->aniso_taps = ataps;
    f->scanw = scan_work_carve(scanw, p->n_theta, m->scan.kpad);
    f->sstride = sstride;
    f->shape = sh;
    f->radius = R;
  }
  return c.off;
}

size_t carve_map(mcl_map m, void* ws, const mcl_map_desc* d, const mcl_params* p) {
  Carver c(ws);
  const int pitch = round_up(d->width, kRowAlign);
  const size_t plane = static_cast<size_t>(d->height) * pitch;
  uint8_t* occ = static_cast<uint8_t*>(c.take(static_cast<size_t>(d->width) * d->height));
  uint8_t* free8 = static_cast<uint8_t*>(c.take(plane));
  float* mpre = static_cast<float*>(c.take(plane * sizeof(float)));
  float* wt = static_cast<float*>(c.take(plane * sizeof(float)));
  ScanTable st = scan_table_carve(c, d, pitch, (p->flags & MCL_SCAN_F32) != 0);
  if (m) {
    m->pitch = pitch;
    m->occ_dev = occ;
    m->free8 = free8;
    m->mpre = mpre;
    m->wt = wt;
    m->scan = st;
  }
  return c.off;
}

}  // namespace

// ---- ABI -----------------------------------------------------------------------

extern "C" {

const char* mcl_last_error(void) { return g_err.c_str(); }

size_t mcl_map_workspace_bytes(const mcl_map_desc* desc, const mcl_params* params) {
  if (check_desc(desc, params) != MCL_OK || check_params(params, false) != MCL_OK) return 0;
  return carve_map(nullptr, nullptr, desc, params);
}

mcl_status mcl_map_create(const mcl_map_desc* d, const mcl_params* p, void* ws, size_t ws_bytes,
                          void* stream, mcl_map* out) {
  if (!out) return fail(MCL_EINVAL, "out is NULL");
  mcl_status st = check_desc(d, p);
  if (st != MCL_OK) return st;
  if ((st = check_params(p, false)) != MCL_OK) return st;
  if (!ws) return fail(MCL_EINVAL, "workspace is NULL");
  const size_t need = carve_map(nullptr, nullptr, d, p);
  if (ws_bytes < need) return fail(MCL_ENOMEM, "map workspace needs %zu bytes, got %zu", need, ws_bytes);
  mcl_map m = new mcl_map_s();
  m->W = d->width;
  m->H = d->height;
  m->cell = d->cell_m;
  m->sigma_xy = p->sigma_xy_cells;
  // the isotropic wall weights the map keeps are not used by anisotropic
  // filters, which compute their own activation per channel
  m->rxy = std::min(kMaxRadius, resolve_radius(p->sigma_xy_cells, p->radius_xy));
  m->flags = p->flags;
  m->stream = static_cast<hipStream_t>(stream);
  carve_map(m, ws, d, p);
  int64_t nf = 0;
  for (int64_t i = 0, n = static_cast<int64_t>(m->W) * m->H; i < n; ++i) nf += d->occupancy[i] == 0;
  m->n_free = nf;
  double g[kMaxTaps];
  gaussian_taps(m->sigma_xy, m->rxy, g);
  hipError_t e = hipMemcpyAsync(m->occ_dev, d->occupancy, static_cast<size_t>(m->W) * m->H,
                                hipMemcpyHostToDevice, m->stream);
  if (e == hipSuccess)
    e = launch_map_setup(m->occ_dev, m->W, m->H, m->pitch, g, m->rxy, 1.0, m->flags, m->free8, m->mpre,
                         m->wt, m->stream);
  if (e == hipSuccess && d->range_table) {
    mcl_status ss = scan_table_build(m->scan, d, m->pitch, m->stream);
    if (ss != MCL_OK) {
      delete m;
      return ss;
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) {
    delete m;
    return hip_fail(e, "map setup");
  }
  *out = m;
  return MCL_OK;
}

void mcl_map_destroy(mcl_map m) { delete m; }

size_t mcl_filter_workspace_bytes(mcl_map map, const mcl_params* params) {
  if (!map || check_params(params, true) != MCL_OK) return 0;
  return carve_filter(nullptr, nullptr, map, params);
}

mcl_status mcl_init_belief(mcl_map map, const mcl_params* p, void* ws, size_t ws_bytes, void* stream,
                           const float* init_host, double theta0, mcl_filter* out) {
  if (!map || !out) return fail(MCL_EINVAL, "map or out is NULL");
  mcl_status st = check_params(p, true);
  if (st != MCL_OK) return st;
  if (p->sigma_xy_cells != map->sigma_xy ||
      std::min(kMaxRadius, resolve_radius(p->sigma_xy_cells, p->radius_xy)) != map->rxy ||
      p->flags != map->flags)
    return fail(MCL_EINVAL, "sigma_xy / radius_xy / flags differ from the map's");
  if (!isfinite(theta0)) return fail(MCL_EINVAL, "theta0 is not finite");
  if (!ws) return fail(MCL_EINVAL, "workspace is NULL");
  const size_t need = carve_filter(nullptr, nullptr, map, p);
  if (ws_bytes < need) return fail(MCL_ENOMEM, "filter workspace needs %zu bytes, got %zu", need, ws_bytes);
  const int64_t plane = static_cast<int64_t>(map->W) * map->H;
  float init_max = 0.f;
  if (init_host) {
    double tot = 0.0;
    for (int64_t i = 0, n = plane * p->n_theta; i < n; ++i) {
      const float v = init_host[i];
      if (!(v >= 0.0f) || !isfinite(v)) return fail(MCL_EINVAL, "init belief has a negative or non-finite value");
      tot += v;
      init_max = std::max(init_max, v);
    }
    if (!(tot > 0.0)) return fail(MCL_EINVAL, "init belief has no mass");
  } else if (map->n_free == 0) {
    return fail(MCL_EINVAL, "map has no free cell");
  }
  mcl_filter f = new mcl_filter_s();
  f->map = map;
  f->T = p->n_theta;
  f->dtype = p->storage;
  f->sigma_th = p->sigma_theta_bins;
  f->rth = resolve_radius(p->sigma_theta_bins, p->radius_theta);
  f->stream = static_cast<hipStream_t>(stream);
  f->theta = theta0;
  carve_filter(f, ws, map, p);
  // taps padded to the kernel radius (zeros beyond each axis' own radius)
  double g[kMaxTaps];
  gaussian_taps(map->sigma_xy, map->rxy, g);
  for (int m = -map->rxy; m <= map->rxy; ++m) f->gxy[f->radius + m] = static_cast<float>(g[m + map->rxy]);
  gaussian_taps(f->sigma_th, f->rth, g);
  for (int m = -f->rth; m <= f->rth; ++m) f->gth[f->radius + m] = static_cast<float>(g[m + f->rth]);
  f->gth_sum = 0.0;
  for (int m = 0; m <= 2 * f->rth; ++m) f->gth_sum += g[m];
  if (map->flags & MCL_ANISOTROPIC) {
    f->sf = p->sigma_xy_cells;
    f->sl = p->sigma_lateral_cells;
    f->raniso = aniso_radius(p);
  }
  if (!step_config_supported(f->dtype, f->radius, f->shape.k) ||
      (f->shape.k.tx == 0 && !stream_plane_ok(map->W, map->H, dtype_bytes(f->dtype)))) {
    delete f;
    return fail(MCL_EINVAL, "no kernel for this storage/radius/shape");
  }
  hipError_t e = hipSuccess;
  if (!init_host) {
    e = launch_init_uniform(f->dtype, f->buf[0], f->buf[1], map->free8, map->W, map->H, map->pitch, f->T,
                            f->sstride, f->stream);
    if (e == hipSuccess)
      e = launch_dev_init(f->dev, static_cast<double>(map->n_free) * f->T, 1.0f, f->stream);
  } else {
    const size_t eb = dtype_bytes(f->dtype);
    // a power of two that brings the largest value into [1/2, 1): exact in
    // every storage type (no rounding beyond the type's own)
    int ex = 0;
    (void)frexp(static_cast<double>(init_max), &ex);
    const float init_scale = static_cast<float>(ldexp(1.0, std::min(127, -ex)));
    e = hipMemsetAsync(f->buf[1], 0, static_cast<size_t>(f->sstride) * f->T * eb, f->stream);
    for (int k = 0; k < f->T && e == hipSuccess; ++k) {
      e = hipMemcpyAsync(f->staging, init_host + k * plane, plane * sizeof(float), hipMemcpyHostToDevice,
                         f->stream);
      // stored scaled to a peak in [1/2, 1), as every step stores it near
      // one: a sum-one belief of many states lies below the 16-bit types'
      // smallest values
      if (e == hipSuccess)
        e = launch_slice_from_f32(f->dtype, f->staging, static_cast<char*>(f->buf[0]) + k * f->sstride * eb,
                                  map->W, map->H, map->pitch, init_scale, f->stream);
    }
    if (e == hipSuccess) e = launch_dev_init(f->dev, 1.0, 1.0f, f->stream);
    if (e == hipSuccess) {
      ReduceArgs r = make_reduce_args(f, kReduceSet, 1.0);
      e = launch_reduce(f->dtype, r, kReduceBlocks, f->stream);
    }
  }
  // the upload of a host belief waits for its copies; the uniform start only
  // enqueues (device errors surface at the next synchronising call)
  if (e == hipSuccess && init_host) e = hipStreamSynchronize(f->stream);
  if (e != hipSuccess) {
    delete f;
    return hip_fail(e, "init_belief");
  }
  *out = f;
  return MCL_OK;
}

void mcl_filter_destroy(mcl_filter f) { delete f; }

// Largest whole-cell row shift of a shift table: the streaming kernels address
// the source rows of strips that no channel shifts past the grid's top edge
// without per-row checks.
static int32_t table_ny_max(const ShiftEntry* t, int n) {
  int32_t m = t[0].ny;
  for (int k = 1; k < n; ++k) m = std::max(m, t[k].ny);
  return m;
}

// Host bookkeeping of one odometry step (Sec. III-A-1, Alg. 1): the heading
// offset, the sub-cell gate's accumulated displacement, the per-channel shift
// table f->table (FP64 displacement R(psi_k) [u, v] / cell split into whole
// cells and a bilinear fraction; with MCL_INTEGER_SHIFT the whole-cell shifts
// with their carried remainders and zero fractions) and, for kernels that read
// it from device memory, the whole-cell list (written on stream s when
// dev_ishift is set).  *launch says whether a warp happens.  The arithmetic is
// FP64 in the order of the displacement formula with psi_k = theta + k 2 pi /
// n_theta.
static hipError_t plan_motion(mcl_filter f, double u, double v, double w, StepArgs& a, hipStream_t s,
                              bool* launch, bool dev_ishift) {
  const double cell = f->map->cell;
  const uint32_t flags = f->map->flags;
  double mu = u, mv = v, th = f->theta;  // motion to warp by and the heading it is expressed at
  *launch = true;
  if (flags & MCL_SUBCELL_GATE) {
    const double c = cos(f->theta), sn = sin(f->theta);
    const double ax = f->acc_x + u * c - v * sn;
    const double ay = f->acc_y + u * sn + v * c;
    f->theta += w;
    ++f->steps;
    if (hypot(ax, ay) < cell) {
      f->acc_x = ax;
      f->acc_y = ay;
      *launch = false;
      return hipSuccess;
    }
    f->acc_x = f->acc_y = 0.0;
    mu = ax;
    mv = ay;
    th = 0.0;
  } else {
    f->theta += w;
    ++f->steps;
  }
  a.u_cells = mu / cell;
  a.v_cells = mv / cell;
  a.theta_prev = th;
  a.ishift = nullptr;
  a.table = nullptr;
  const double dth = 2.0 * M_PI / f->T;
  if (flags & MCL_INTEGER_SHIFT) {
    int32_t n[2 * kMaxTheta];
    for (int k = 0; k < f->T; ++k) {
      const double psi = th + k * dth;
      const double c = cos(psi), sn = sin(psi);
      const double dx = (mu * c - mv * sn) / cell + f->rem[k][0];
      const double dy = (mu * sn + mv * c) / cell + f->rem[k][1];
      const double nx = floor(dx + 0.5), ny = floor(dy + 0.5);
      f->rem[k][0] = dx - nx;
      f->rem[k][1] = dy - ny;
      n[2 * k] = static_cast<int32_t>(nx);
      n[2 * k + 1] = static_cast<int32_t>(ny);
      f->table[k] = ShiftEntry{n[2 * k], n[2 * k + 1], 0.f, 0.f};
    }
    a.ny_max = table_ny_max(f->table, f->T);
    if (dev_ishift) {
      const hipError_t e = launch_write_shifts(n, f->T, f->ishift, s);
      if (e != hipSuccess) return e;
      a.ishift = f->ishift;
    }
    return hipSuccess;
  }
  // the bilinear warp: floor and fraction of the displacement in cells
  const double uc = a.u_cells, vc = a.v_cells;
  for (int k = 0; k < f->T; ++k) {
    const double psi = th + k * dth;
    const double c = cos(psi), sn = sin(psi);
    const double dx = uc * c - vc * sn;
    const double dy = uc * sn + vc * c;
    const double fdx = floor(dx), fdy = floor(dy);
    f->table[k] = ShiftEntry{static_cast<int32_t>(fdx), static_cast<int32_t>(fdy), static_cast<float>(dx - fdx),
                             static_cast<float>(dy - fdy)};
  }
  a.ny_max = table_ny_max(f->table, f->T);
  return hipSuccess;
}

// Launch the fused step of one filter: the streaming kernels take the shift
// table from the kernel arguments (or, above kArgTableMax channels, from the
// filter's device table, written here through kernel arguments); the tiled
// kernel computes its own.
static hipError_t launch_filter_step(mcl_filter f, StepArgs& a) {
  if (f->shape.k.tx > 0) return launch_step(f->dtype, f->radius, f->shape.k, a, nullptr, f->stream);
  if (f->T <= kArgTableMax) {
    ShiftArgs tab;
    memcpy(tab.e, f->table, static_cast<size_t>(f->T) * sizeof(ShiftEntry));
    a.table = nullptr;
    return launch_step(f->dtype, f->radius, f->shape.k, a, &tab, f->stream);
  }
  const hipError_t e = launch_write_table(f->table, f->T, f->table_dev, f->stream);
  if (e != hipSuccess) return e;
  a.table = f->table_dev;
  return launch_step(f->dtype, f->radius, f->shape.k, a, nullptr, f->stream);
}

// Arguments of the anisotropic step from the fused step's (motion, buffers)
// and the filter; theta_pre orients the noise (the heading before the step).
static AnisoArgs make_aniso_args(mcl_filter f, const StepArgs& s, double theta_pre) {
  AnisoArgs a = {};
  const mcl_map m = f->map;
  a.buf[0] = f->buf[0];
  a.buf[1] = f->buf[1];
  a.tmp = f->aniso_tmp;
  a.taps = f->aniso_taps;
  a.mpre = m->mpre;
  a.free8 = m->free8;
  a.partials = f->partials;
  a.dev = f->dev;
  a.ishift = s.ishift;
  a.W = m->W;
  a.H = m->H;
  a.pitch = m->pitch;
  a.n_theta = f->T;
  a.rxy = f->raniso;
  a.rth = f->rth;
  a.wall_normalize = (m->flags & MCL_WALL_NORMALIZE) ? 1 : 0;
  a.sstride = f->sstride;
  a.u_cells = s.u_cells;
  a.v_cells = s.v_cells;
  a.theta_prev = s.theta_prev;
  a.dtheta = s.dtheta;
  a.noise_theta = theta_pre;
  a.sf = f->sf;
  a.sl = f->sl;
  a.gth_sum = f->gth_sum;
  for (int l = -f->rth; l <= f->rth; ++l) a.gth[l + f->rth] = f->gth[f->radius + l];
  return a;
}

mcl_status mcl_step_odometry(mcl_filter f, double u, double v, double w) {
  if (!f) return fail(MCL_EINVAL, "filter is NULL");
  if (!isfinite(u) || !isfinite(v) || !isfinite(w)) return fail(MCL_EINVAL, "odometry is not finite");
  const double cell = f->map->cell;
  if (fabs(u) / cell > 1e6 || fabs(v) / cell > 1e6) return fail(MCL_EINVAL, "odometry exceeds 1e6 cells");
  StepArgs a = make_step_args(f);
  bool launch = false;
  const double theta_pre = f->theta;
  const bool aniso = (f->map->flags & MCL_ANISOTROPIC) != 0;
  HIP_TRY(plan_motion(f, u, v, w, a, f->stream, &launch, aniso || f->shape.k.tx > 0), "shift table");
  if (!launch) return MCL_OK;
  if (aniso) {
    HIP_TRY(launch_aniso_step(f->dtype, make_aniso_args(f, a, theta_pre), f->stream), "step launch");
    return MCL_OK;
  }
  HIP_TRY(launch_filter_step(f, a), "step launch");
  return MCL_OK;
}

mcl_status mcl_normalize(mcl_filter f, double* log_norm_out) {
  if (!f) return fail(MCL_EINVAL, "filter is NULL");
  FilterDev d;
  mcl_status st = read_dev(f, &d);
  if (st != MCL_OK) return st;
  if (d.status != kStatusOk) return fail(MCL_EDEGENERATE, "a step removed all probability mass");
  const double factor = f->dtype == MCL_F16 ? 1.0 / d.maxval : 1.0 / d.sum;
  ReduceArgs r = make_reduce_args(f, kReduceSet, factor);
  HIP_TRY(launch_reduce(f->dtype, r, kReduceBlocks, f->stream), "normalize launch");
  if ((st = read_dev(f, &d)) != MCL_OK) return st;
  if (log_norm_out) *log_norm_out = d.log_norm;
  if (d.status != kStatusOk) return fail(MCL_EDEGENERATE, "a step removed all probability mass");
  return MCL_OK;
}

mcl_status mcl_export_belief(mcl_filter f, float* dev_out, float* dev_map_out) {
  if (!f) return fail(MCL_EINVAL, "filter is NULL");
  if (!dev_out && !dev_map_out) return fail(MCL_EINVAL, "no output given");
  const mcl_map m = f->map;
  ReduceArgs r = make_reduce_args(f, kReduceSum, 1.0);
  HIP_TRY(launch_reduce(f->dtype, r, kReduceBlocks, f->stream), "export sum");
  // the stored buffer index lives on the device; export reads both through cur
  FilterDev d;
  mcl_status st = read_dev(f, &d);
  if (st != MCL_OK) return st;
  HIP_TRY(launch_export(f->dtype, f->buf[d.cur], m->W, m->H, m->pitch, f->T, f->sstride, f->dev, dev_out,
                        static_cast<int64_t>(m->W) * m->H, 0, dev_out ? f->T : 0, dev_map_out, f->stream),
          "export");
  return MCL_OK;
}

mcl_status mcl_export_scalars(mcl_filter f, double* dev_out) {
  if (!f || !dev_out) return fail(MCL_EINVAL, "filter or output is NULL");
  HIP_TRY(launch_export_scalars(f->dev, dev_out, f->stream), "export scalars");
  return MCL_OK;
}

mcl_status mcl_read_belief(mcl_filter f, float* host_out, mcl_pose* argmax, double* theta_offset,
                           double* log_norm) {
  if (!f) return fail(MCL_EINVAL, "filter is NULL");
  const mcl_map m = f->map;
  ReduceArgs r = make_reduce_args(f, kReduceSum, 1.0);
  HIP_TRY(launch_reduce(f->dtype, r, kReduceBlocks, f->stream), "readout sum");
  FilterDev d;
  mcl_status st = read_dev(f, &d);
  if (st != MCL_OK) return st;
  const int64_t plane = static_cast<int64_t>(m->W) * m->H;
  if (host_out) {
    for (int k = 0; k < f->T; ++k) {
      HIP_TRY(launch_export(f->dtype, f->buf[d.cur], m->W, m->H, m->pitch, f->T, f->sstride, f->dev,
                            f->staging, plane, k, k + 1, nullptr, f->stream),
              "export slice");
      HIP_TRY(hipMemcpyAsync(host_out + k * plane, f->staging, plane * sizeof(float), hipMemcpyDeviceToHost,
                             f->stream),
              "copy slice");
    }
  }
  if (argmax) {
    ReduceArgs ra = make_reduce_args(f, kReduceArgmax, 1.0);
    HIP_TRY(launch_reduce(f->dtype, ra, kReduceBlocks, f->stream), "argmax");
  }
  if ((st = read_dev(f, &d)) != MCL_OK) return st;
  if (argmax) {
    const int64_t idx = d.argmax_idx < 0 ? 0 : d.argmax_idx;
    argmax->k = static_cast<int32_t>(idx / plane);
    const int64_t rem = idx % plane;
    argmax->j = static_cast<int32_t>(rem / m->W);
    argmax->i = static_cast<int32_t>(rem % m->W);
    argmax->x_m = argmax->i * m->cell;
    argmax->y_m = argmax->j * m->cell;
    argmax->theta_rad = argmax->k * (2.0 * M_PI / f->T) + f->theta;
    argmax->prob = static_cast<double>(d.argmax_val) / d.aux[3];
  }
  if (theta_offset) *theta_offset = f->theta;
  if (log_norm) *log_norm = d.log_norm;
  if (d.status != kStatusOk) return fail(MCL_EDEGENERATE, "a step removed all probability mass");
  return MCL_OK;
}

mcl_status mcl_get_info(mcl_filter f, int sync, mcl_info* out) {
  if (!f || !out) return fail(MCL_EINVAL, "filter or out is NULL");
  memset(out, 0, sizeof(*out));
  out->width = f->map->W;
  out->height = f->map->H;
  out->n_theta = f->T;
  out->pitch = f->map->pitch;
  out->storage = f->dtype;
  out->radius = f->radius;
  out->tile_x = f->shape.k.tx;
  out->tile_y = f->shape.k.ty;
  out->theta_chunks = f->shape.chunks;
  out->workgroups = f->shape.blocks();
  out->steps = f->steps;
  out->theta_offset_rad = f->theta;
  out->state_bytes = static_cast<uint64_t>(f->map->W) * f->map->H * f->T * dtype_bytes(f->dtype);
  if (sync) {
    FilterDev d;
    mcl_status st = read_dev(f, &d);
    if (st != MCL_OK) return st;
    out->log_norm = d.log_norm;
    out->status = d.status;
    out->belief_device = f->buf[d.cur];
  } else {
    out->belief_device = nullptr;
  }
  return MCL_OK;
}

static mcl_status scan_check(mcl_filter f, const float* ranges_m, int32_t n_beams, double sigma_m, bool need_sigma) {
  if (!f) return fail(MCL_EINVAL, "filter is NULL");
  const ScanTable& t = f->map->scan;
  if (t.n_dirs == 0) return fail(MCL_ESTATE, "the map has no range table");
  if (!ranges_m) return fail(MCL_EINVAL, "ranges is NULL");
  if (n_beams != t.n_dirs) return fail(MCL_EINVAL, "n_beams %d differs from the table's %d directions", n_beams, t.n_dirs);
  if (need_sigma && (!(sigma_m > 0.0) || !isfinite(sigma_m))) return fail(MCL_EINVAL, "sigma_m must be > 0");
  for (int b = 0; b < n_beams; ++b)
    if (!isfinite(ranges_m[b])) return fail(MCL_EINVAL, "range %d is not finite", b);
  return MCL_OK;
}

static ScanLaunch scan_args(mcl_filter f) {
  const ScanTable& t = f->map->scan;
  ScanLaunch L;
  L.table = &t;
  L.work = f->scanw;
  L.buf[0] = f->buf[0];
  L.buf[1] = f->buf[1];
  L.scratch = f->scan_scratch;
  L.partials = f->partials;
  L.dev = f->dev;
  L.W = f->map->W;
  L.H = f->map->H;
  L.pitch = f->map->pitch;
  L.n_theta = f->T;
  L.dtype = f->dtype;
  L.sstride = f->sstride;
  L.theta = f->theta;
  L.stream = f->stream;
  return L;
}

static mcl_status scan_common(mcl_filter f, const float* ranges_m, int32_t n_beams, double sigma_m,
                              int32_t* dout) {
  const mcl_status st = scan_check(f, ranges_m, n_beams, sigma_m, dout == nullptr);
  if (st != MCL_OK) return st;
  HIP_TRY(scan_launch(scan_args(f), ranges_m, sigma_m, dout), "scan launch");
  return MCL_OK;
}

mcl_status mcl_apply_scan(mcl_filter f, const float* ranges_m, int32_t n_beams, double sigma_m) {
  return scan_common(f, ranges_m, n_beams, sigma_m, nullptr);
}

mcl_status mcl_apply_scan_batch(mcl_filter* const filters, const float* ranges_m, int32_t n_beams,
                                const double* sigma_m, int32_t n) {
  if (!filters || !ranges_m || !sigma_m || n < 1 || n > 65536)
    return fail(MCL_EINVAL, "filters/ranges/sigma NULL or n out of range");
  std::vector<ScanLaunch> Ls;
  Ls.reserve(n);
  for (int i = 0; i < n; ++i) {
    mcl_filter f = filters[i];
    const mcl_status st = scan_check(f, ranges_m + static_cast<int64_t>(i) * n_beams, n_beams, sigma_m[i], true);
    if (st != MCL_OK) return st;
    for (int j = 0; j < i; ++j)
      if (filters[j] == f) return fail(MCL_EINVAL, "filter %d appears twice", i);
    if (f->map != filters[0]->map) return fail(MCL_EINVAL, "filter %d is on another map", i);
    if (f->stream != filters[0]->stream) return fail(MCL_EINVAL, "filter %d is on another stream", i);
    Ls.push_back(scan_args(f));
  }
  HIP_TRY(scan_launch_batch(Ls.data(), n, ranges_m, sigma_m), "scan batch launch");
  return MCL_OK;
}

mcl_status mcl_scan_sqdist(mcl_filter f, const float* ranges_m, int32_t n_beams, int32_t* dev_out) {
  if (!dev_out) return fail(MCL_EINVAL, "dev_out is NULL");
  return scan_common(f, ranges_m, n_beams, 1.0, dev_out);
}

mcl_status mcl_apply_scan_sampled(mcl_filter f, const float* ranges_m, int32_t n_beams, double sigma_m,
                                  const uint8_t* dev_mask) {
  const mcl_status st = scan_check(f, ranges_m, n_beams, sigma_m, true);
  if (st != MCL_OK) return st;
  if (!dev_mask) return fail(MCL_EINVAL, "dev_mask is NULL");
  const int64_t cells = static_cast<int64_t>(f->map->H) * f->map->pitch;
  if (cells >= (static_cast<int64_t>(1) << 31) || cells * f->T >= (static_cast<int64_t>(1) << 31))
    return fail(MCL_EINVAL, "the sampled update supports fewer than 2^31 states");
  HIP_TRY(scan_sampled_launch(scan_args(f), ranges_m, sigma_m, dev_mask, f->samp_list, f->samp_list + cells),
          "sampled scan launch");
  return MCL_OK;
}

mcl_status mcl_sample_cells(mcl_filter f, int32_t n_samples, uint8_t* dev_mask) {
  if (!f) return fail(MCL_EINVAL, "filter is NULL");
  if (!dev_mask) return fail(MCL_EINVAL, "dev_mask is NULL");
  if (n_samples < 0) return fail(MCL_EINVAL, "n_samples must be >= 0");
  const mcl_map m = f->map;
  if (!dither_supported(m->W, m->H))
    return fail(MCL_EINVAL, "a %d x %d map is beyond the dithering kernel (H >= 4096 and W >= 8190)", m->W, m->H);
  HIP_TRY(launch_dither_source(f->dtype, f->buf[0], f->buf[1], m->W, m->H, m->pitch, f->T, f->sstride, f->partials,
                               f->dev, f->staging, f->stream),
          "belief map");
  HIP_TRY(launch_dither(f->staging, m->W, m->H, dev_mask, true, static_cast<float>(n_samples), f->dev, f->stream),
          "dithering");
  return MCL_OK;
}

mcl_status mcl_dither(const float* dev_intensity, int32_t width, int32_t height, uint8_t* dev_mask, void* stream) {
  if (width < 0 || height < 0) return fail(MCL_EINVAL, "negative size %d x %d", width, height);
  if (width == 0 || height == 0) return MCL_OK;
  if (!dev_intensity || !dev_mask) return fail(MCL_EINVAL, "NULL image or mask");
  if (!dither_supported(width, height))
    return fail(MCL_EINVAL, "a %d x %d image is beyond the dithering kernel (H >= 4096 and W >= 8190, or W * H >= 2^29)",
                width, height);
  HIP_TRY(launch_dither(dev_intensity, width, height, dev_mask, false, 1.f, nullptr,
                        static_cast<hipStream_t>(stream)),
          "dithering");
  return MCL_OK;
}

size_t mcl_match_workspace_bytes(mcl_map map, int32_t n_theta, int32_t batch) {
  if (!map || map->scan.n_dirs == 0 || n_theta < 1 || n_theta > kMaxTheta || batch < 1 || batch > 65536) return 0;
  if (static_cast<int64_t>(map->pitch) * map->H >= (static_cast<int64_t>(1) << 30)) return 0;
  return match_workspace_bytes(map->scan, map->H * map->pitch, n_theta, batch);
}

mcl_status mcl_best_match(mcl_map map, int32_t n_theta, const float* ranges_m, int32_t n_queries, int32_t batch,
                          int32_t* out_cell, int32_t* out_heading, int32_t* out_dist, void* dev_ws,
                          size_t ws_bytes, void* stream) {
  if (!map) return fail(MCL_EINVAL, "map is NULL");
  const ScanTable& t = map->scan;
  if (t.n_dirs == 0) return fail(MCL_ESTATE, "the map has no range table");
  if (n_theta < 1 || n_theta > kMaxTheta) return fail(MCL_EINVAL, "n_theta must be in [1, %d]", kMaxTheta);
  if (t.kpad > 384) return fail(MCL_EINVAL, "best_match supports tables of at most 384 directions");
  if (static_cast<int64_t>(map->pitch) * map->H >= (static_cast<int64_t>(1) << 30))
    return fail(MCL_EINVAL, "best_match supports maps of fewer than 2^30 padded cells");
  if (n_queries < 0 || batch < 1) return fail(MCL_EINVAL, "n_queries must be >= 0 and batch >= 1");
  if (n_queries > 0 && (!ranges_m || !out_cell)) return fail(MCL_EINVAL, "NULL ranges or output");
  const size_t need = mcl_match_workspace_bytes(map, n_theta, batch);
  if (need == 0) return fail(MCL_EINVAL, "batch %d x %d channels is too large", batch, n_theta);
  if (!dev_ws || ws_bytes < need) return fail(MCL_ENOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  const int N = t.n_dirs;
  for (int64_t e = 0; e < static_cast<int64_t>(n_queries) * N; ++e)
    if (!isfinite(ranges_m[e])) return fail(MCL_EINVAL, "range %lld is not finite", static_cast<long long>(e));
  const double h = t.max_range / 256.0;
  if (n_queries == 0) return MCL_OK;
  // Two pinned host staging sets: batch b + 1 is quantised on the host while
  // batch b runs on the device (the device buffers are reused in stream order).
  struct Staging {
    int16_t* zq[2] = {nullptr, nullptr};
    int32_t* sz[2] = {nullptr, nullptr};
    uint64_t* best[2] = {nullptr, nullptr};
    hipEvent_t done[2] = {nullptr, nullptr};
    hipStream_t s = nullptr;
    ~Staging() {
      if (s) (void)hipStreamSynchronize(s);  // no copy may still target the staging on an early return
      for (int i = 0; i < 2; ++i) {
        if (done[i]) (void)hipEventDestroy(done[i]);
        if (zq[i]) (void)hipHostFree(zq[i]);
        if (sz[i]) (void)hipHostFree(sz[i]);
        if (best[i]) (void)hipHostFree(best[i]);
      }
    }
  } st;
  for (int i = 0; i < 2; ++i) {
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&st.zq[i]), static_cast<size_t>(batch) * N * sizeof(int16_t)),
            "pinned staging");
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&st.sz[i]), static_cast<size_t>(batch) * sizeof(int32_t)),
            "pinned staging");
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&st.best[i]), static_cast<size_t>(batch) * sizeof(uint64_t)),
            "pinned staging");
    HIP_TRY(hipEventCreateWithFlags(&st.done[i], hipEventDisableTiming), "event");
  }
  const hipStream_t s = static_cast<hipStream_t>(stream);
  st.s = s;
  const int nbatch = (n_queries + batch - 1) / batch;
  auto quantise = [&](int bi) {
    const int q0 = bi * batch, nq = std::min(batch, n_queries - q0);
    int16_t* zq = st.zq[bi & 1];
    for (int p = 0; p < nq; ++p) {
      int32_t ss = 0;
      for (int b = 0; b < N; ++b) {
        double f = floor(static_cast<double>(ranges_m[static_cast<int64_t>(q0 + p) * N + b]) / h + 0.5);
        f = f < 0.0 ? 0.0 : (f > 256.0 ? 256.0 : f);
        const int q = static_cast<int>(f) - 128;
        zq[static_cast<size_t>(p) * N + b] = static_cast<int16_t>(q);
        ss += q * q;
      }
      st.sz[bi & 1][p] = ss;
    }
  };
  auto decode = [&](int bi) {
    const int q0 = bi * batch, nq = std::min(batch, n_queries - q0);
    for (int p = 0; p < nq; ++p) {
      const uint64_t key = st.best[bi & 1][p];
      const bool none = key == ~0ull;  // no free cell at all
      const int64_t cell = static_cast<int64_t>(key & ((1ull << 30) - 1));  // j * pitch + i
      out_cell[q0 + p] = none ? -1 : static_cast<int32_t>(cell / map->pitch * map->W + cell % map->pitch);
      if (out_heading) out_heading[q0 + p] = none ? -1 : static_cast<int32_t>((key >> 30) & 511u);
      if (out_dist) out_dist[q0 + p] = none ? -1 : static_cast<int32_t>(key >> 39);
    }
  };
  for (int bi = 0; bi < nbatch; ++bi) {
    quantise(bi);
    const int nq = std::min(batch, n_queries - bi * batch);
    HIP_TRY(match_launch(t, map->free8, map->W, map->H, map->pitch, n_theta, st.zq[bi & 1], st.sz[bi & 1], nq,
                         dev_ws, st.best[bi & 1], s),
            "best match");
    HIP_TRY(hipEventRecord(st.done[bi & 1], s), "event");
    if (bi > 0) {
      HIP_TRY(hipEventSynchronize(st.done[(bi - 1) & 1]), "best match");
      decode(bi - 1);
    }
  }
  HIP_TRY(hipEventSynchronize(st.done[(nbatch - 1) & 1]), "best match");
  decode(nbatch - 1);
  return MCL_OK;
}

mcl_status mcl_difficulty(mcl_map map, const int32_t* query_cells, const int32_t* best_cells, int32_t n,
                          double threshold_m, double* out) {
  if (!map || !out) return fail(MCL_EINVAL, "NULL map or output");
  if (n < 0 || (n > 0 && (!query_cells || !best_cells))) return fail(MCL_EINVAL, "bad query list");
  if (!(threshold_m >= 0.0)) return fail(MCL_EINVAL, "threshold must be >= 0");
  const int64_t cells = static_cast<int64_t>(map->W) * map->H;
  int64_t far = 0;
  for (int32_t e = 0; e < n; ++e) {
    const int64_t q = query_cells[e], b = best_cells[e];
    if (q < 0 || q >= cells) return fail(MCL_EINVAL, "query cell %lld outside the map", static_cast<long long>(q));
    if (b < 0 || b >= cells) {
      ++far;
      continue;
    }
    const double di = static_cast<double>(q % map->W - b % map->W), dj = static_cast<double>(q / map->W - b / map->W);
    if (map->cell * hypot(di, dj) > threshold_m) ++far;
  }
  *out = n > 0 ? static_cast<double>(far) / n : 0.0;
  return MCL_OK;
}

// One batch parameter slot, the same layout on the host and the device: the
// job table, the first-workgroup offsets of every group and the jobs' shift
// tables.
struct SlotLayout {
  size_t args_off = 0, first_off = 0, tables_off = 0, bytes = 0;
};
static SlotLayout slot_layout(int32_t n) {
  auto up = [](size_t x) { return (x + 255) & ~static_cast<size_t>(255); };
  SlotLayout l;
  l.args_off = 0;
  l.first_off = up(static_cast<size_t>(n) * sizeof(StepArgs));
  l.tables_off = up(l.first_off + static_cast<size_t>(2 * n + 2) * sizeof(int32_t));
  l.bytes = up(l.tables_off + static_cast<size_t>(n) * kMaxTheta * sizeof(ShiftEntry));
  return l;
}

struct BatchGroup {
  int dtype, radius;
  KernelShape k;
  int job0, first0, njobs, blocks, max_theta;
};

static mcl_status check_batch(mcl_filter* const filters, const double* uvw, int32_t n) {
  if (!filters || !uvw || n < 1 || n > 65536) return fail(MCL_EINVAL, "filters/uvw NULL or n out of range");
  for (int i = 0; i < n; ++i) {
    if (!filters[i]) return fail(MCL_EINVAL, "filter %d is NULL", i);
    for (int j = 0; j < i; ++j)
      if (filters[j] == filters[i]) return fail(MCL_EINVAL, "filter %d appears twice", i);
    const double* o = uvw + 3 * i;
    if (!isfinite(o[0]) || !isfinite(o[1]) || !isfinite(o[2])) return fail(MCL_EINVAL, "odometry %d not finite", i);
    const double cell = filters[i]->map->cell;
    if (fabs(o[0]) / cell > 1e6 || fabs(o[1]) / cell > 1e6) return fail(MCL_EINVAL, "odometry %d too large", i);
  }
  return MCL_OK;
}

// One filter's launch in a batch.
struct BatchJob {
  StepArgs a;
  int dtype, radius;
  KernelShape k;
  mcl_filter f;
};

// Host side of one batched step: each filter's bookkeeping as in
// mcl_step_odometry (a filter whose sub-cell gate does not fire takes no
// launch; anisotropic filters launch their own passes on s), then the job
// table, offsets and shift tables written into `host` (laid out as
// slot_layout(n)) with device pointers into `dev`.  jobs and groups are
// caller storage for n entries each (nothing is allocated here); *ngroups =
// launch groups, *used = bytes to copy.
static mcl_status plan_batch(mcl_filter* const filters, const double* uvw, int32_t n, hipStream_t s, char* host,
                             char* dev, BatchJob* jobs, BatchGroup* groups, int* ngroups, size_t* used) {
  int njobs = 0;
  for (int i = 0; i < n; ++i) {
    mcl_filter f = filters[i];
    const double u = uvw[3 * i], v = uvw[3 * i + 1], w = uvw[3 * i + 2];
    StepArgs a = make_step_args(f);
    bool launch = false;
    const double theta_pre = f->theta;
    const bool aniso = (f->map->flags & MCL_ANISOTROPIC) != 0;
    HIP_TRY(plan_motion(f, u, v, w, a, s, &launch, aniso || f->shape.k.tx > 0), "shift table");
    if (!launch) continue;
    if (aniso) {
      HIP_TRY(launch_aniso_step(f->dtype, make_aniso_args(f, a, theta_pre), s), "step launch");
      continue;
    }
    jobs[njobs++] = BatchJob{a, f->dtype, f->radius, f->shape.k, f};
  }
  *ngroups = 0;
  *used = 0;
  if (njobs == 0) return MCL_OK;
  auto same = [](const BatchJob& x, const BatchJob& y) {
    return x.dtype == y.dtype && x.radius == y.radius && x.k == y.k;
  };
  auto less = [](const BatchJob& x, const BatchJob& y) {
    if (x.dtype != y.dtype) return x.dtype < y.dtype;
    if (x.radius != y.radius) return x.radius < y.radius;
    return x.k < y.k;
  };
  // stable insertion sort by kernel group (no temporary buffer)
  for (int i = 1; i < njobs; ++i) {
    const BatchJob x = jobs[i];
    int j = i;
    while (j > 0 && less(x, jobs[j - 1])) {
      jobs[j] = jobs[j - 1];
      --j;
    }
    jobs[j] = x;
  }
  const SlotLayout lay = slot_layout(n);
  StepArgs* args = reinterpret_cast<StepArgs*>(host + lay.args_off);
  int32_t* first = reinterpret_cast<int32_t*>(host + lay.first_off);
  ShiftEntry* tables = reinterpret_cast<ShiftEntry*>(host + lay.tables_off);
  const ShiftEntry* tables_dev = reinterpret_cast<const ShiftEntry*>(dev + lay.tables_off);
  int nfirst = 0, ntab = 0, ng = 0;
  for (int i = 0; i < njobs; ++i) {
    if (i == 0 || !same(jobs[i], jobs[i - 1])) {
      if (ng > 0) first[nfirst++] = groups[ng - 1].blocks;
      groups[ng++] = BatchGroup{jobs[i].dtype, jobs[i].radius, jobs[i].k, i, nfirst, 0, 0, 0};
    }
    BatchGroup& g = groups[ng - 1];
    first[nfirst++] = g.blocks;
    args[i] = jobs[i].a;
    if (jobs[i].k.tx == 0) {
      // the streaming kernels read the job's shift table from the slot
      args[i].table = tables_dev + ntab;
      memcpy(tables + ntab, jobs[i].f->table, static_cast<size_t>(jobs[i].f->T) * sizeof(ShiftEntry));
      ntab += jobs[i].f->T;
    }
    g.blocks += jobs[i].a.tiles_x * jobs[i].a.tiles_y * jobs[i].a.chunks;
    g.max_theta = std::max(g.max_theta, static_cast<int>(jobs[i].a.n_theta));
    ++g.njobs;
  }
  first[nfirst++] = groups[ng - 1].blocks;
  *ngroups = ng;
  *used = lay.tables_off + static_cast<size_t>(ntab) * sizeof(ShiftEntry);
  return MCL_OK;
}

static hipError_t launch_groups(const BatchGroup* groups, int ngroups, char* dev, int32_t n, hipStream_t s) {
  const SlotLayout lay = slot_layout(n);
  const StepArgs* args_dev = reinterpret_cast<const StepArgs*>(dev + lay.args_off);
  const int32_t* first_dev = reinterpret_cast<const int32_t*>(dev + lay.first_off);
  for (int i = 0; i < ngroups; ++i) {
    const BatchGroup& g = groups[i];
    const hipError_t e = launch_step_batch(g.dtype, g.radius, g.k, args_dev + g.job0, first_dev + g.first0, g.njobs,
                                           g.blocks, g.max_theta, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

size_t mcl_batch_workspace_bytes(int32_t max_filters) {
  if (max_filters < 1 || max_filters > 65536) return 0;
  return 2 * slot_layout(max_filters).bytes;
}

mcl_status mcl_step_batch(mcl_filter* const filters, const double* uvw, int32_t n, void* dev_ws, size_t ws_bytes,
                          void* stream) {
  mcl_status st = check_batch(filters, uvw, n);
  if (st != MCL_OK) return st;
  if (!dev_ws) return fail(MCL_EINVAL, "workspace is NULL");
  const SlotLayout lay = slot_layout(n);
  if (ws_bytes < lay.bytes) return fail(MCL_ENOMEM, "batch workspace needs %zu bytes", lay.bytes);
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<char> host(lay.bytes);
  std::vector<BatchJob> jobs(n);
  std::vector<BatchGroup> groups(n);
  int ngroups = 0;
  size_t used = 0;
  char* dev = static_cast<char*>(dev_ws);
  if ((st = plan_batch(filters, uvw, n, s, host.data(), dev, jobs.data(), groups.data(), &ngroups, &used)) != MCL_OK)
    return st;
  if (ngroups == 0) return MCL_OK;
  // a copy from pageable memory: the host buffer may be released on return
  HIP_TRY(hipMemcpyAsync(dev, host.data(), used, hipMemcpyHostToDevice, s), "batch jobs upload");
  HIP_TRY(launch_groups(groups.data(), ngroups, dev, n, s), "batch launch");
  return MCL_OK;
}

}  // extern "C"

// ---- batched steps without allocation -------------------------------------------------
// The job table of mcl_step_batch_noalloc lives in this file-scope device
// array (one copy per GPU, held until the process ends) and its host staging
// in a file-scope host array; calls share both, under a host lock.
namespace {
constexpr int32_t kNoallocMaxFilters = 256;
constexpr size_t kNoallocBytes = 1u << 21;  // >= slot_layout(kNoallocMaxFilters).bytes (checked below)
constexpr int kNoallocMaxDevices = 64;
}  // namespace
static __device__ __align__(256) char scratch[kNoallocBytes];
static char noalloc_host[kNoallocBytes];
static BatchJob noalloc_jobs[kNoallocMaxFilters];
static BatchGroup noalloc_groups[kNoallocMaxFilters];
static char* noalloc_dev[kNoallocMaxDevices];  // device address of `scratch` per device, set once
static std::mutex noalloc_mutex;

// Device address of `scratch` on the current device (the array's host-side
// name is not a device address), looked up once per device.
static mcl_status noalloc_scratch(char** out) {
  int device = -1;
  HIP_TRY(hipGetDevice(&device), "current device");
  if (device < 0 || device >= kNoallocMaxDevices) return fail(MCL_EDEVICE, "device %d beyond %d", device, kNoallocMaxDevices);
  if (!noalloc_dev[device]) {
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "scratch symbol address");
    noalloc_dev[device] = static_cast<char*>(ptr);
  }
  *out = noalloc_dev[device];
  return MCL_OK;
}

extern "C" mcl_status mcl_step_batch_noalloc(mcl_filter* const filters, const double* uvw, int32_t n, void* stream) {
  static_assert(kNoallocBytes >= 256 * (sizeof(StepArgs) + 2 * sizeof(int32_t) + kMaxTheta * sizeof(ShiftEntry)) + 1024,
                "the static job table holds kNoallocMaxFilters filters");
  if (n > kNoallocMaxFilters)
    return fail(MCL_EINVAL, "%d filters: the static job table holds at most %d", n, kNoallocMaxFilters);
  mcl_status st = check_batch(filters, uvw, n);
  if (st != MCL_OK) return st;
  const SlotLayout lay = slot_layout(n);
  if (lay.bytes > kNoallocBytes) return fail(MCL_EINVAL, "job table of %zu bytes exceeds %zu", lay.bytes, kNoallocBytes);
  std::lock_guard<std::mutex> lock(noalloc_mutex);
  char* dev = nullptr;
  if ((st = noalloc_scratch(&dev)) != MCL_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int ngroups = 0;
  size_t used = 0;
  if ((st = plan_batch(filters, uvw, n, s, noalloc_host, dev, noalloc_jobs, noalloc_groups, &ngroups, &used)) != MCL_OK)
    return st;
  if (ngroups == 0) return MCL_OK;
  // the whole used part of the table is rewritten on every call (nothing in
  // it needs to start at zero); the copy from pageable memory completes
  // before the host buffer is reused by the next call
  HIP_TRY(hipMemcpyAsync(dev, noalloc_host, used, hipMemcpyHostToDevice, s), "batch jobs upload");
  HIP_TRY(launch_groups(noalloc_groups, ngroups, dev, n, s), "batch launch");
  return MCL_OK;
}

// ---- graph-replayed batches (serving) ------------------------------------------------
struct mcl_batch_s {
  int32_t max_filters = 0;
  hipStream_t stream = nullptr;
  SlotLayout lay;
  char* dev[2] = {nullptr, nullptr};   // device parameter slots (caller's workspace)
  char* host[2] = {nullptr, nullptr};  // pinned host parameter slots
  hipEvent_t done[2] = {nullptr, nullptr};
  bool pending[2] = {false, false};
  int next = 0;
  struct Graph {
    std::vector<int64_t> key;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<Graph> graphs[2];
  int64_t captures = 0, replays = 0;
  ~mcl_batch_s() {
    for (int i = 0; i < 2; ++i) {
      for (Graph& g : graphs[i])
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
      if (done[i]) (void)hipEventDestroy(done[i]);
      if (host[i]) (void)hipHostFree(host[i]);
    }
  }
};

namespace {
constexpr size_t kBatchGraphCache = 32;  // instantiated graphs kept per slot
}

extern "C" {

mcl_status mcl_batch_create(int32_t max_filters, void* dev_ws, size_t ws_bytes, void* stream, mcl_batch* out) {
  if (!out) return fail(MCL_EINVAL, "out is NULL");
  const size_t need = mcl_batch_workspace_bytes(max_filters);
  if (need == 0) return fail(MCL_EINVAL, "max_filters out of range");
  if (!dev_ws) return fail(MCL_EINVAL, "workspace is NULL");
  if (!stream) return fail(MCL_EINVAL, "graph capture needs a stream other than the default (NULL) stream");
  if (ws_bytes < need) return fail(MCL_ENOMEM, "batch workspace needs %zu bytes, got %zu", need, ws_bytes);
  mcl_batch b = new mcl_batch_s();
  b->max_filters = max_filters;
  b->stream = static_cast<hipStream_t>(stream);
  b->lay = slot_layout(max_filters);
  for (int i = 0; i < 2; ++i) {
    b->dev[i] = static_cast<char*>(dev_ws) + i * b->lay.bytes;
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&b->host[i]), b->lay.bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done[i], hipEventDisableTiming);
    if (e != hipSuccess) {
      delete b;
      return hip_fail(e, "batch slots");
    }
  }
  *out = b;
  return MCL_OK;
}

void mcl_batch_destroy(mcl_batch b) {
  if (!b) return;
  for (int i = 0; i < 2; ++i)
    if (b->pending[i]) (void)hipEventSynchronize(b->done[i]);
  delete b;
}

mcl_status mcl_batch_step(mcl_batch b, mcl_filter* const filters, const double* uvw, int32_t n) {
  if (!b) return fail(MCL_EINVAL, "batch is NULL");
  mcl_status st = check_batch(filters, uvw, n);
  if (st != MCL_OK) return st;
  if (n > b->max_filters) return fail(MCL_EINVAL, "%d filters, the batch holds at most %d", n, b->max_filters);
  const int slot = b->next;
  // the slot's previous replay must have read its parameters
  if (b->pending[slot]) HIP_TRY(hipEventSynchronize(b->done[slot]), "batch slot wait");
  b->pending[slot] = false;
  std::vector<BatchJob> jobs(n);
  std::vector<BatchGroup> groups(n);
  int ngroups = 0;
  size_t used = 0;
  if ((st = plan_batch(filters, uvw, n, b->stream, b->host[slot], b->dev[slot], jobs.data(), groups.data(), &ngroups,
                       &used)) != MCL_OK)
    return st;
  if (ngroups == 0) return MCL_OK;
  groups.resize(ngroups);
  b->next ^= 1;
  // the graph depends on the launch structure and the copied size, not on the
  // parameters, which the copy node reads from the pinned slot at every replay
  std::vector<int64_t> key = {n, static_cast<int64_t>(used)};
  for (const BatchGroup& g : groups) {
    const int64_t k[] = {g.dtype, g.radius, g.k.tx, g.k.ty, g.k.nt, g.k.nbuf, g.k.variant, g.job0, g.first0,
                         g.njobs, g.blocks, g.max_theta};
    key.insert(key.end(), k, k + 12);
  }
  std::vector<mcl_batch_s::Graph>& cache = b->graphs[slot];
  hipGraphExec_t exec = nullptr;
  for (mcl_batch_s::Graph& g : cache)
    if (g.key == key) exec = g.exec;
  if (!exec) {
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "graph capture");
    hipError_t e = hipMemcpyAsync(b->dev[slot], b->host[slot], used, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = launch_groups(groups.data(), ngroups, b->dev[slot], n, b->stream);
    const hipError_t e2 = hipStreamEndCapture(b->stream, &graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    if (cache.size() >= kBatchGraphCache) {
      // the oldest graph of this slot: its last replay was waited for above
      (void)hipGraphExecDestroy(cache.front().exec);
      cache.erase(cache.begin());
    }
    cache.push_back(mcl_batch_s::Graph{key, exec});
    ++b->captures;
  }
  HIP_TRY(hipGraphLaunch(exec, b->stream), "graph launch");
  HIP_TRY(hipEventRecord(b->done[slot], b->stream), "batch slot event");
  b->pending[slot] = true;
  ++b->replays;
  return MCL_OK;
}

mcl_status mcl_batch_counts(mcl_batch b, int64_t* captures, int64_t* replays) {
  if (!b) return fail(MCL_EINVAL, "batch is NULL");
  if (captures) *captures = b->captures;
  if (replays) *replays = b->replays;
  return MCL_OK;
}

}  // extern "C"
