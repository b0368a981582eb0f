// Floyd-Steinberg sample selection of the belief map (Sec. III-B, dithering).
//
// The sampled observation update compares a scan against a subset of the
// states only: the cells an error-diffusion dithering of the belief map
// m(i, j) = max_k B (Sec. III-A, last paragraph) selects.  The intensity is
// I = min(1, N m / sum m), so that about N cells come out selected.
//
// Floyd-Steinberg diffusion visits the cells in raster order and pushes the
// quantisation error of a cell to its right neighbour (7/16) and to the
// below-left, below and below-right neighbours (3/16, 5/16, 1/16).  Every
// decision depends on all cells before it, so the work is a wavefront: with
// phases of K steps and cell (i, j) at step i + (K + 1) j, every cell of the
// row above that sends error to (i, j) is handled at least K steps earlier,
// i.e. in an earlier phase, and only the left neighbour lies in the same
// phase, on the same thread.  A thread owns whole rows; the errors of a row
// reach the thread of the next row through a small LDS ring of the row's last
// columns, and one barrier (LDS only) separates phases.
//
// The error a cell receives is summed in the order raster order delivers it
// (below-right push of (i-1, j-1), below push of (i, j-1), below-left push of
// (i+1, j-1), right push of (i-1, j)), every product and sum an FP32
// operation rounded to nearest with no fused multiply-add, so the selection
// equals the raster-order selection bit for bit.
#include <float.h>
#include <math.h>

#include <algorithm>

#include "mcl_internal.hpp"

namespace mcl {
namespace {

constexpr int kDitherMaxThreads = 1024;
constexpr int kDitherMaxLds = 65536;  // bytes of the LDS error ring
constexpr int kDitherMaxSlots = 4;    // rows one thread has in flight at most

// Columns of a row kept in the ring: the row below reads columns i0-1 .. i0+K
// while this row writes i0+K+1 .. i0+2K, so 2K + 2 must be distinct.
constexpr int ring_cols(int K) {
  int d = 1;
  while (d < 2 * K + 2) d *= 2;
  return d;
}

struct DitherArgs {
  const float* src;     // H x W dense: intensity, or the belief map (scaled)
  uint8_t* mask;        // H x W dense output, 1 = selected
  const FilterDev* dev; // scaled: the FP32 total of the belief map
  int32_t W, H;
  int32_t ring;         // rows of the error ring (power of two)
  int32_t scaled;
  float n;              // requested sample count (scaled)
  int32_t phases;       // phases to run (a multiple of the prefetch depth)
  uint32_t cells;       // W * H
};

// One thread per row slot; slot s of thread t holds rows t + nt (s + MAXA q).
// PF = phases between the load of a source value and its use.
template <int K, int MAXA, int PF>
__global__ __launch_bounds__(kDitherMaxThreads) void dither_kernel(DitherArgs a) {
#pragma clang fp contract(off)
  constexpr int D = ring_cols(K);
  extern __shared__ float ering[];
  const int t = threadIdx.x, nt = blockDim.x;
  const int W = a.W, H = a.H;
  const int rmask = a.ring - 1;
  const int span = nt * MAXA;        // rows between consecutive rows of one slot
  const int wrap = (K + 1) * span;   // columns a slot moves back when it takes its next row
  // unscaled: I = img exactly (1 * img / 1); a non-positive total gives I = 0
  const float total_in = a.scaled ? a.dev->dither_total : 1.f;
  const bool tpos = total_in > 0.f;
  const float total = tpos ? total_in : 1.f;
  const float nsamp = a.scaled ? a.n : 1.f;
  const bool clamp = a.scaled != 0;
  const float w7 = 7.f / 16.f, w3 = 3.f / 16.f, w5 = 5.f / 16.f, w1 = 1.f / 16.f;
  // Offsets past the end of a buffer read zero and drop stores, so loads and
  // stores of cells outside the image need no branch.
  const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(a.src), static_cast<short>(0), static_cast<int>(a.cells * 4u), 0x00020000);
  const __amdgpu_buffer_rsrc_t rmask_out = __builtin_amdgcn_make_buffer_rsrc(
      a.mask, static_cast<short>(0), static_cast<int>(a.cells), 0x00020000);
  constexpr uint32_t kOut = 0x80000000u;  // at or past the end of both buffers

  int row[MAXA], col[MAXA];    // current row and first column of the phase
  int prow[MAXA], pcol[MAXA];  // the same, PF phases ahead (loads in flight)
  float eleft[MAXA];           // error of the previous cell of the row
  float pf[PF][MAXA][K];       // source values, loaded PF phases ahead
#pragma unroll
  for (int s = 0; s < MAXA; ++s) {
    row[s] = prow[s] = t + nt * s;
    col[s] = pcol[s] = -(K + 1) * row[s];
    eleft[s] = 0.f;
  }
  auto advance = [&](int& r, int& c) {
    c += K;
    const bool done = c >= W;
    r = done ? r + span : r;
    c = done ? c - wrap : c;
  };
  auto load_phase = [&](float (&dst)[MAXA][K]) {
#pragma unroll
    for (int s = 0; s < MAXA; ++s) {
#pragma unroll
      for (int c = 0; c < K; ++c) {
        const int i = pcol[s] + c;
        const bool ok = i >= 0 && i < W && prow[s] < H;
        dst[s][c] = __builtin_bit_cast(
            float, __builtin_amdgcn_raw_buffer_load_b32(rsrc, ok ? static_cast<uint32_t>(prow[s] * W + i) * 4u : kOut, 0, 0));
      }
      advance(prow[s], pcol[s]);
    }
  };
#pragma unroll
  for (int u = 0; u < PF; ++u) load_phase(pf[u]);

  for (int p0 = 0; p0 < a.phases; p0 += PF) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
#pragma unroll
      for (int s = 0; s < MAXA; ++s) {
        const int j = row[s], i0 = col[s];
        // row above, columns i0-1 .. i0+K (written in earlier phases)
        const float* up = ering + ((j - 1) & rmask) * D;
        float ua[K + 2];
#pragma unroll
        for (int c = 0; c < K + 2; ++c) ua[c] = up[(i0 - 1 + c) & (D - 1)];
        const bool has_up = j > 0 && j < H;
#pragma unroll
        for (int c = 0; c < K; ++c) {
          const int i = i0 + c;
          const bool act = i >= 0 && i < W && j < H;
          const float q = (nsamp * pf[u][s][c]) / total;
          const float I = clamp ? (tpos ? fminf(1.f, q) : 0.f) : q;
          const float p1 = w1 * ua[c], p5 = w5 * ua[c + 1], p3 = w3 * ua[c + 2], p7 = w7 * eleft[s];
          float err = 0.f;
          const float e1 = err + p1;
          err = (has_up && i >= 1) ? e1 : err;
          const float e5 = err + p5;
          err = has_up ? e5 : err;
          const float e3 = err + p3;
          err = (has_up && i + 1 < W) ? e3 : err;
          const float e7 = err + p7;
          err = i >= 1 ? e7 : err;
          const float v = I + err;
          const bool sel = v >= 0.5f;
          const float e = v - (sel ? 1.f : 0.f);
          eleft[s] = e;
          // only cells of the image write: a ring row's entries may still be
          // read for the row it held before, until its new row starts
          if (act) ering[(j & rmask) * D + (i & (D - 1))] = e;
          __builtin_amdgcn_raw_buffer_store_b8(static_cast<uint8_t>(sel ? 1 : 0), rmask_out,
                                               act ? static_cast<uint32_t>(j * W + i) : kOut, 0, 0);
        }
        advance(row[s], col[s]);
      }
      // loads for PF phases ahead reuse this phase's registers
      load_phase(pf[u]);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    }
  }
}

// Belief map of the stored belief and its FP64 sum (rounded to FP32).
template <typename T>
__device__ inline float to_f32(T v) {
  return static_cast<float>(v);
}
template <>
__device__ inline float to_f32<__bf16>(__bf16 v) {
  return __uint_as_float(static_cast<uint32_t>(__builtin_bit_cast(uint16_t, v)) << 16);
}

constexpr int kSrcThreads = 256;
constexpr int kSrcMaxBlocks = 1024;

template <typename T>
__global__ __launch_bounds__(kSrcThreads) void dither_source_kernel(const void* buf0, const void* buf1, int W,
                                                                   int pitch, int n_theta, int64_t sstride,
                                                                   uint32_t cells, double* partials,
                                                                   FilterDev* dev, float* out) {
  __shared__ double rs[kSrcThreads];
  __shared__ int last_flag;
  const int t = threadIdx.x;
  const T* bel = static_cast<const T*>(dev->cur ? buf1 : buf0);
  double s = 0.0;
  for (uint32_t e = blockIdx.x * kSrcThreads + t; e < cells; e += gridDim.x * kSrcThreads) {
    const uint32_t j = e / static_cast<uint32_t>(W), i = e - j * static_cast<uint32_t>(W);
    const T* p = bel + static_cast<int64_t>(j) * pitch + i;
    float m = 0.f;
#pragma unroll 8
    for (int k = 0; k < n_theta; ++k) m = fmaxf(m, to_f32<T>(p[k * sstride]));
    out[e] = m;
    s += static_cast<double>(m);
  }
  rs[t] = s;
  __syncthreads();
  for (int st = kSrcThreads / 2; st > 0; st >>= 1) {
    if (t < st) rs[t] += rs[t + st];
    __syncthreads();
  }
  if (t == 0) {
    partials[blockIdx.x] = rs[0];
    const uint32_t prev = __hip_atomic_fetch_add(&dev->counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last_flag = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!last_flag) return;
  double ts = 0.0;
  for (int b = t; b < static_cast<int>(gridDim.x); b += kSrcThreads)
    ts += __hip_atomic_load(&partials[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  rs[t] = ts;
  __syncthreads();
  for (int st = kSrcThreads / 2; st > 0; st >>= 1) {
    if (t < st) rs[t] += rs[t + st];
    __syncthreads();
  }
  if (t == 0) {
    dev->dither_total = static_cast<float>(rs[0]);
    __hip_atomic_store(&dev->counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Launch geometry of the dithering kernel for a W x H image.
struct DitherPlan {
  int K = 0, slots = 0, threads = 0, ring = 0;
  size_t lds = 0;
  bool ok = false;
};

int next_pow2(int x) {
  int p = 1;
  while (p < x) p *= 2;
  return p;
}

DitherPlan plan_for(int W, int H, int K) {
  DitherPlan p;
  p.K = K;
  // rows that are active at once (a slot moves to its next row (K+1) span columns back)
  const int64_t need = std::min<int64_t>(H, (static_cast<int64_t>(W) + K - 1 + K) / (K + 1));
  const int64_t nt = std::min<int64_t>(kDitherMaxThreads, (need + 63) / 64 * 64);
  const int64_t slots = (need + nt - 1) / nt;
  // ring rows: a row's entries are reused by row j + ring only after row j + 1 is done
  const int64_t rows = std::min<int64_t>(H, 1 + (static_cast<int64_t>(W) + K - 1 + K) / (K + 1));
  if (slots > kDitherMaxSlots || rows > (1 << 20)) return p;
  p.ring = next_pow2(static_cast<int>(rows));
  p.lds = static_cast<size_t>(p.ring) * ring_cols(K) * sizeof(float);
  p.slots = static_cast<int>(slots < 1 ? 1 : slots);
  p.threads = static_cast<int>(nt < 64 ? 64 : nt);
  p.ok = p.lds <= kDitherMaxLds;
  return p;
}

// Prefer three steps per phase (fewer barriers); fall back to one when the
// three-step ring would not fit.
DitherPlan choose_plan(int W, int H) {
  DitherPlan p = plan_for(W, H, 3);
  if (!p.ok) p = plan_for(W, H, 1);
  return p;
}

template <int K, int MAXA>
hipError_t launch_k(const DitherArgs& a0, const DitherPlan& p, hipStream_t s) {
  constexpr int PF = K == 1 ? 16 : 4;
  DitherArgs a = a0;
  const int64_t last = static_cast<int64_t>(a.W - 1) + static_cast<int64_t>(K + 1) * (a.H - 1);
  const int64_t phases = last / K + 1;
  a.phases = static_cast<int32_t>((phases + PF - 1) / PF * PF);
  hipLaunchKernelGGL((dither_kernel<K, MAXA, PF>), dim3(1), dim3(p.threads), p.lds, s, a);
  return hipGetLastError();
}

}  // namespace

bool dither_supported(int W, int H) {
  if (W < 1 || H < 1) return false;
  // 32-bit byte offsets of the FP32 source, with room for the out-of-range marker
  if (static_cast<int64_t>(W) * H >= (static_cast<int64_t>(1) << 29)) return false;
  return choose_plan(W, H).ok;
}

hipError_t launch_dither(const float* src, int W, int H, uint8_t* mask, bool scaled, float n_samples,
                         const FilterDev* dev, hipStream_t s) {
  const DitherPlan p = choose_plan(W, H);
  if (!p.ok) return hipErrorInvalidValue;
  DitherArgs a = {};
  a.src = src;
  a.mask = mask;
  a.dev = dev;
  a.W = W;
  a.H = H;
  a.ring = p.ring;
  a.scaled = scaled ? 1 : 0;
  a.n = n_samples;
  a.cells = static_cast<uint32_t>(static_cast<int64_t>(W) * H);
  if (p.K == 3) {
    switch (p.slots) {
      case 1: return launch_k<3, 1>(a, p, s);
      case 2: return launch_k<3, 2>(a, p, s);
      default: return launch_k<3, 4>(a, p, s);
    }
  }
  switch (p.slots) {
    case 1: return launch_k<1, 1>(a, p, s);
    case 2: return launch_k<1, 2>(a, p, s);
    default: return launch_k<1, 4>(a, p, s);
  }
}

hipError_t launch_dither_source(int dtype, const void* buf0, const void* buf1, int W, int H, int pitch,
                                int n_theta, int64_t sstride, double* partials, FilterDev* dev, float* out,
                                hipStream_t s) {
  const uint32_t cells = static_cast<uint32_t>(static_cast<int64_t>(W) * H);
  const int blocks = static_cast<int>(std::min<int64_t>(kSrcMaxBlocks, (cells + kSrcThreads - 1) / kSrcThreads));
  switch (dtype) {
    case 0: hipLaunchKernelGGL(dither_source_kernel<float>, dim3(blocks), dim3(kSrcThreads), 0, s, buf0, buf1, W, pitch, n_theta, sstride, cells, partials, dev, out); break;
    case 1: hipLaunchKernelGGL(dither_source_kernel<__bf16>, dim3(blocks), dim3(kSrcThreads), 0, s, buf0, buf1, W, pitch, n_theta, sstride, cells, partials, dev, out); break;
    case 2: hipLaunchKernelGGL(dither_source_kernel<_Float16>, dim3(blocks), dim3(kSrcThreads), 0, s, buf0, buf1, W, pitch, n_theta, sstride, cells, partials, dev, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mcl
