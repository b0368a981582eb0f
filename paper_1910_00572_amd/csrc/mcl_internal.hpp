// Internal definitions shared by the host library and the HIP kernels.
// Nothing here is part of the public ABI (include/mcl.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcl {

constexpr int kMaxRadius = 4;                 // largest blur radius the kernels support
constexpr int kMaxTaps = 2 * kMaxRadius + 1;
constexpr int kMaxTheta = 360;                // heading channels per filter
constexpr int kRowAlign = 8;                  // row pitch multiple (16 bytes of 16-bit storage)
constexpr int kStatusOk = 0;
constexpr int kStatusDegenerate = 3;

// Device-resident scalars of one filter.  Written only by the last workgroup of
// a launch (or by setup kernels), read by the next launch on the same stream.
struct FilterDev {
  double log_norm;     // ln of the product of kept masses since initialisation
  double lnsum;        // ln(sum of the stored buffer)
  double sum;          // sum of the stored buffer
  double aux[4];       // scan: [0] = M*, [1] = ln(stored value at the best state), [2] = D at it
  float scale;         // factor the next update applies on load (1 / max of the stored buffer)
  float maxval;        // max of the stored buffer
  int32_t cur;         // which of the two belief buffers holds the state
  int32_t status;      // sticky: kStatusOk or kStatusDegenerate
  uint32_t counter;    // arrival counter of the last-workgroup reduction
  uint32_t pad0;
  int64_t argmax_idx;  // flat (k, j, i) index of the readout argmax
  float argmax_val;
  float pad1;
  // sampled observation update
  int32_t nsel;        // cells in the sample list (appended by the compaction, cleared by the update)
  int32_t dstar;       // smallest squared distance over the sampled states (INT32_MAX: no sample)
  float dither_total;  // FP32 sum of the belief map the dithering scales by
  int32_t pad2;
};

// Last-workgroup reductions.  Each workgroup publishes its partial results
// with device-coherent stores (they bypass the per-XCD L2), waits for them to
// complete, and then counts itself in; the workgroup that arrives last reads
// every partial with device-coherent loads.  The wait orders the stores
// before the count without an acquire-release fence, which on this part
// writes back and invalidates the whole L2 of the XCD for every workgroup
// (about 30 ns each, measured).  Counting is two-level: workgroups count in
// one of kArriveGroups group counters (256 bytes apart, so they are served
// in parallel), and the last of each group counts in dev->counter; counts on
// one address are served one at a time (about 11 ns each).
constexpr int kArriveGroups = 16;
constexpr int kArriveStride = 64;  // uint32 between group counters
constexpr size_t kDevBytes = (sizeof(FilterDev) + 255) / 256 * 256;
// FilterDev plus its group counters, as carved from a workspace.
constexpr size_t kDevRegionBytes = kDevBytes + kArriveGroups * kArriveStride * sizeof(uint32_t);

__device__ inline void publish(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// blk: this workgroup's index among the nblocks that reduce into dev.
__device__ inline bool arrive_last(FilterDev* dev, uint32_t blk, uint32_t nblocks) {
  __builtin_amdgcn_s_waitcnt(0);  // the partials above are complete
  const uint32_t groups = nblocks < kArriveGroups ? nblocks : kArriveGroups;
  const uint32_t g = blk % groups;
  const uint32_t gsize = (nblocks - g + groups - 1) / groups;  // workgroups with this residue
  uint32_t* cg = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(dev) + kDevBytes) + g * kArriveStride;
  if (__hip_atomic_fetch_add(cg, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != gsize - 1) return false;
  __hip_atomic_store(cg, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // the whole group is in
  return __hip_atomic_fetch_add(&dev->counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == groups - 1;
}

// Warp of one heading channel: source offset (nx, ny) in whole cells and the
// bilinear fractions (fx, fy) of the displacement R(psi_k) [u, v] / cell,
// computed on the host in FP64 (floor and remainder) and rounded to FP32.
struct ShiftEntry {
  int32_t nx, ny;
  float fx, fy;
};
// Heading counts up to this many pass their shift table in the kernel
// arguments of a single-filter step (16 bytes per channel).
constexpr int kArgTableMax = 128;
struct ShiftArgs {
  ShiftEntry e[kArgTableMax];
};

// Everything one step of one filter needs.  Passed by value for a single
// filter, or from device memory for a batch.
struct StepArgs {
  void* buf[2];               // belief buffers, storage type, [k][j][pitch]
  const float* mpre;          // pre-blur traversability, [j][pitch] (0 outside the grid)
  const float* wt;            // post-blur weights M / G(B_0), [j][pitch]
  double* partials;           // 2 doubles per workgroup
  FilterDev* dev;
  int32_t W, H, pitch, n_theta;
  int32_t tiles_x, tiles_y, chunks, chunk_len;
  int32_t strip;              // streaming kernel: output columns per strip
  int32_t ny_max;             // streaming kernels: largest whole-cell row shift of the table's channels
  int64_t sstride;            // elements per heading slice (H * pitch)
  double u_cells, v_cells;    // odometry in cells, robot frame
  double theta_prev, dtheta;  // heading offset before the step, 2 pi / n_theta
  float gxy[kMaxTaps];        // x/y taps, centred at index R of the kernel radius
  float gth[kMaxTaps];        // theta taps
  const int32_t* ishift;      // tiled kernel: whole-cell shifts (nx, ny) per channel, or null: computed from u, v
  const ShiftEntry* table;    // streaming kernels: per-channel shift table in device memory, or null
                              // (then the table travels in the kernel arguments)
};

// Odometry step with anisotropic, heading-rotated noise (aniso.hip).
constexpr int kAnisoMaxRadius = 6;  // 2-D kernel radius, cells
struct AnisoArgs {
  void* buf[2];
  float* tmp;                 // FP32 scratch, [k][j][pitch]
  float* taps;                // FP32 2-D taps, [k][(2 rxy + 1)^2], written by the first kernel
  const float* mpre;          // pre-blur traversability, [j][pitch]
  const uint8_t* free8;       // free cells, [j][pitch] (0 outside the grid)
  double* partials;           // 2 doubles per workgroup of the second pass
  FilterDev* dev;
  const int32_t* ishift;      // whole-cell shifts per channel, or null
  int32_t W, H, pitch, n_theta;
  int32_t rxy, rth;           // 2-D kernel radius; theta radius
  int32_t wall_normalize;
  int64_t sstride;
  double u_cells, v_cells;    // motion to warp by, cells, at heading theta_prev
  double theta_prev, dtheta;
  double noise_theta;         // heading of channel 0 that orients the noise (pre-step)
  double sf, sl;              // std-devs along and across the heading, cells
  double gth_sum;             // sum of the theta taps
  float gth[kMaxTaps];        // theta taps, index l + rth
};
hipError_t launch_aniso_step(int dtype, const AnisoArgs& a, hipStream_t s);
int aniso_workgroups(int W, int H, int n_theta);

// Gaussian taps of the map's x/y blur (FP64, index m + radius).
struct MapTaps {
  double g[kMaxTaps];
};

// Generic pass over a stored belief with a last-workgroup reduction.
struct ReduceArgs {
  void* buf[2];
  double* partials;
  FilterDev* dev;
  int32_t W, H, pitch, n_theta;
  int64_t sstride;
  double factor;              // multiply the stored buffer in place by this (1 = read only)
  int32_t mode;               // kReduceSet / kReduceArgmax
};
constexpr int kReduceSet = 0;     // sum/max -> dev (sum, lnsum, scale, maxval)
constexpr int kReduceArgmax = 1;  // argmax -> dev (argmax_idx, argmax_val)
constexpr int kReduceSum = 2;     // sum -> dev->aux[3] only (export normaliser)

// Bump allocator over a caller-provided buffer; with base == nullptr it only
// measures.  Every region starts on a 256-byte boundary.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  void* take(size_t bytes) {
    off = (off + 255) & ~static_cast<size_t>(255);
    void* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
};

// ---- launchers (defined in the .hip files) -----------------------------------
// Return hipSuccess or the launch error.
// Output columns per strip of the streaming kernel.  Lanes R+1 .. 63-R can
// hold outputs; the strip is trimmed to a multiple of `align_bytes` of
// storage so that, with strips starting at multiples of the strip width,
// every output row store covers whole aligned segments and no two strips
// write into the same segment.
constexpr int stream_strip_width(int R, int elt_bytes, int align_bytes) {
  const int al = align_bytes > elt_bytes ? align_bytes / elt_bytes : 1;
  return ((63 - 2 * R) / al) * al;
}
constexpr int kStreamAlignBytes = 32;

// Launch shape of the step kernel.  tx > 0: tiled kernel with tx x ty tiles
// and nt threads.  tx == 0: streaming kernel with ty-row strips, nt / 64
// waves and nbuf source-slice buffers.
// variant (streaming kernel only): 0 = x blur by lane shifts before the
// theta ring, 1 = mask folded into the y taps, theta blur first and the x
// blur through a per-wave LDS row, host shift table.
struct KernelShape {
  int tx = 64, ty = 16, nt = 256, nbuf = 2, variant = 0;
  bool operator==(const KernelShape& o) const {
    return tx == o.tx && ty == o.ty && nt == o.nt && nbuf == o.nbuf && variant == o.variant;
  }
  bool operator<(const KernelShape& o) const {
    if (tx != o.tx) return tx < o.tx;
    if (ty != o.ty) return ty < o.ty;
    if (nt != o.nt) return nt < o.nt;
    if (nbuf != o.nbuf) return nbuf < o.nbuf;
    return variant < o.variant;
  }
};
// tab: the shift table of a single-filter step when n_theta <= kArgTableMax
// and a.table is null (variant 1); ignored otherwise.
hipError_t launch_step(int dtype, int radius, const KernelShape& k, const StepArgs& a, const ShiftArgs* tab,
                       hipStream_t s);
// jobs_dev[0..njobs) with first_dev[j] = first workgroup of job j (first_dev[njobs] = total);
// max_theta = the largest heading count among the jobs.
hipError_t launch_step_batch(int dtype, int radius, const KernelShape& k, const StepArgs* jobs_dev,
                             const int32_t* first_dev, int32_t njobs, int32_t total_blocks, int32_t max_theta,
                             hipStream_t s);
bool step_config_supported(int dtype, int radius, const KernelShape& k);

hipError_t launch_map_setup(const uint8_t* occ_dev, int W, int H, int pitch, const double* gxy,
                            int rxy, double gth_sum, uint32_t flags, uint8_t* free8, float* mpre,
                            float* wt, hipStream_t s);
hipError_t launch_init_uniform(int dtype, void* buf0, void* buf1, const uint8_t* free8, int W, int H,
                               int pitch, int n_theta, int64_t sstride, hipStream_t s);
// dst_slice = src * factor, converted to the storage type (pitch layout).
hipError_t launch_slice_from_f32(int dtype, const float* src, void* dst_slice, int W, int H,
                                 int pitch, float factor, hipStream_t s);
hipError_t launch_reduce(int dtype, const ReduceArgs& a, int nblocks, hipStream_t s);
hipError_t launch_export(int dtype, const void* buf, int W, int H, int pitch, int n_theta,
                         int64_t sstride, const FilterDev* dev, float* out, int64_t out_slice_stride,
                         int k_begin, int k_end, float* map_out, hipStream_t s);
hipError_t launch_dev_init(FilterDev* dev, double sum, float maxval, hipStream_t s);
// out[0] = log-normaliser, out[1] = sticky status (device, two doubles).
hipError_t launch_export_scalars(const FilterDev* dev, double* out, hipStream_t s);
// Write n[0 .. 2*count) (whole-cell shifts, nx ny per channel) to device memory
// through the kernel's arguments: no host-side synchronisation.
hipError_t launch_write_shifts(const int32_t* n, int count, int32_t* dst, hipStream_t s);
// Write a shift table t[0 .. count) to device memory through kernel
// arguments (kArgTableMax entries per launch).
hipError_t launch_write_table(const ShiftEntry* t, int count, ShiftEntry* dst, hipStream_t s);

// Floyd-Steinberg sample selection (sample.hip).  src: H x W dense FP32,
// either the intensity itself (scaled == false) or the belief map, turned into
// min(1, n_samples * m / total) with the total from dev->dither_total.
// dither_supported() says whether a W x H image fits the kernel's LDS ring.
bool dither_supported(int W, int H);
hipError_t launch_dither(const float* src, int W, int H, uint8_t* mask, bool scaled, float n_samples,
                         const FilterDev* dev, hipStream_t s);
// Belief map max_k B of the stored belief into out (H x W dense FP32) and the
// FP32-rounded FP64 sum of it into dev->dither_total.
hipError_t launch_dither_source(int dtype, const void* buf0, const void* buf1, int W, int H, int pitch,
                                int n_theta, int64_t sstride, double* partials, FilterDev* dev, float* out,
                                hipStream_t s);

}  // namespace mcl
