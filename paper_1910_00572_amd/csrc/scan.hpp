// Dense range-scan observation update: device tables and host entry points.
#pragma once

#include "../../include/mcl.h"
#include "mcl_internal.hpp"

namespace mcl {

constexpr int kScanMaxDirs = 1024;

// Quantised range table of a map (built once by scan_table_build).
struct ScanTable {
  int n_dirs = 0;          // 0 = the map has no range table
  int kpad = 0;            // n_dirs rounded up to the GEMM depth granule
  double max_range = 0.0;
  bool f32 = false;        // operands stored as FP32 instead of BF16
  void* rq = nullptr;      // centred counts (bf16 or f32), H*pitch cells x kpad, MFMA-tiled (scan.hip)
  size_t rq_bytes = 0;
  int32_t* sr = nullptr;   // [H*pitch] sum over directions of rq^2
  float* stage = nullptr;  // FP32 upload staging
  size_t stage_elems = 0;
};

// Per-filter scan scratch (circulant operand, per-tile partials).
struct ScanWork {
  void* c = nullptr;       // [n_theta_pad][kpad] circulant scan operand
};

// Partials the scan needs: one per 128-cell tile of pass 1, two per pass-2 block
// (the sampled update needs at most 256 + 2 * 2048).
inline int kScanMaxBlocks(int W, int H, int pitch) {
  (void)W;
  return static_cast<int>((static_cast<int64_t>(H) * pitch + 127) / 128) + 2048;
}

// Everything one scan update needs from the filter handle.
struct ScanLaunch {
  const ScanTable* table;
  ScanWork work;
  void* buf[2];
  float* scratch;     // FP32, n_theta * H * pitch
  double* partials;
  FilterDev* dev;
  int W, H, pitch, n_theta, dtype;
  int64_t sstride;
  double theta;       // heading offset at the time of the scan
  hipStream_t stream;
};

// Enqueue the scan update (dout == nullptr) or the diagnostic distance output.
hipError_t scan_launch(const ScanLaunch& L, const float* ranges_m, double sigma_m, int32_t* dout);
// Enqueue the scan updates of n filters of one map on Ls[0].stream: ranges_m
// holds n scans of the table's n_dirs beams, sigma_m one std-dev per filter.
// Each filter's result is bitwise that of scan_launch.
hipError_t scan_launch_batch(const ScanLaunch* Ls, int n, const float* ranges_m, const double* sigma_m);
// Enqueue the sampled update on the cells of `mask` (H x W dense, nonzero =
// selected).  list and pos: H * pitch int32 each (sample list and positions).
hipError_t scan_sampled_launch(const ScanLaunch& L, const float* ranges_m, double sigma_m, const uint8_t* mask,
                               int32_t* list, int32_t* pos);
// Best match of nq quantised query scans over every free state (map
// difficulty), enqueued on s: copies the queries in, runs the product and
// copies best_host[p] = (D << 39) | (k << 30) | cell out (cell = j * pitch + i).  The host
// buffers must stay valid (and be pinned for the copies to be asynchronous)
// until the stream has reached that point.
size_t match_workspace_bytes(const ScanTable& t, int cells, int n_theta, int batch);
hipError_t match_launch(const ScanTable& t, const uint8_t* free8, int W, int H, int pitch, int n_theta,
                        const int16_t* zq_host, const int32_t* sz_host, int nq, void* ws, uint64_t* best_host,
                        hipStream_t s);
size_t scan_work_bytes(int n_theta, int kpad);
ScanWork scan_work_carve(void* base, int n_theta, int kpad);
ScanTable scan_table_carve(Carver& c, const mcl_map_desc* d, int pitch, bool f32);
mcl_status scan_table_build(ScanTable& t, const mcl_map_desc* d, int pitch, hipStream_t s);

}  // namespace mcl

