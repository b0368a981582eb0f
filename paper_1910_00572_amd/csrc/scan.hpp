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
  void* rq = nullptr;      // [H*pitch][kpad] centred counts (bf16 or f32)
  int32_t* sr = nullptr;   // [H*pitch] sum over directions of rq^2
  float* stage = nullptr;  // FP32 upload staging
  size_t stage_elems = 0;
};

// Per-filter scan scratch (circulant operand, per-tile partials).
struct ScanWork {
  void* c = nullptr;       // [n_theta_pad][kpad] circulant scan operand
  int32_t* zs = nullptr;   // device copy of the quantised scan and offsets
};

inline int kScanMaxBlocks(int W, int H, int pitch) {
  (void)W;
  return static_cast<int>((static_cast<int64_t>(H) * pitch + 255) / 256);
}
size_t scan_work_bytes(int n_theta, int kpad);
ScanWork scan_work_carve(void* base, int n_theta, int kpad);
ScanTable scan_table_carve(Carver& c, const mcl_map_desc* d, int pitch, bool f32);
mcl_status scan_table_build(ScanTable& t, const mcl_map_desc* d, int pitch, hipStream_t s);

}  // namespace mcl

mcl_status scan_apply(mcl_filter f, const float* ranges_m, int32_t n_beams, double sigma_m);
mcl_status scan_sqdist(mcl_filter f, const float* ranges_m, int32_t n_beams, int32_t* dev_out);
