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
  const float* src;     // H x W dense intensity
  uint8_t* mask;        // H x W dense output, 1 = selected
  int32_t W, H;
  int32_t ring;         // rows of the error ring (power of two)
  int32_t rstride;      // floats between ring rows: ring_cols(K), or one more (odd, no bank conflicts)
  int32_t phases;       // phases to run (a multiple of the prefetch depth)
  uint32_t cells;       // W * H
};

// One thread per row slot; slot s of thread t holds rows t + nt (s + MAXA q).
// PF = phases between the load of an intensity and its use.
//
// Borders cost no tests: error from outside the image is an exact zero in
// the ring (row -1 is a ring row that stays zero until row 0 is done; each
// row writes zero to its column -1 in the phase that holds it and to column
// W when it ends; the left error is reset when a slot takes a new row).  Adding a zero
// changes no nonzero sum and a zero's sign changes no decision, so the
// selection is the one that skips those terms.
template <int K, int MAXA, int PF>
__global__ __launch_bounds__(kDitherMaxThreads) void dither_kernel(DitherArgs a) {
#pragma clang fp contract(off)
  constexpr int D = ring_cols(K);
  extern __shared__ float ering[];
  const int t = threadIdx.x, nt = blockDim.x;
  const int W = a.W, H = a.H;
  const int rmask = a.ring - 1;
  const int RS = a.rstride;
  const int span = nt * MAXA;        // rows between consecutive rows of one slot
  const int wrap = (K + 1) * span;   // columns a slot moves back when it takes its next row
  const float w7 = 7.f / 16.f, w3 = 3.f / 16.f, w5 = 5.f / 16.f, w1 = 1.f / 16.f;
  // Offsets past the end of a buffer read zero and drop stores, so loads and
  // stores of cells outside the image need no branch.
  const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(a.src), static_cast<short>(0), static_cast<int>(a.cells * 4u), 0x00020000);
  const __amdgpu_buffer_rsrc_t rmask_out = __builtin_amdgcn_make_buffer_rsrc(
      a.mask, static_cast<short>(0), static_cast<int>(a.cells), 0x00020000);
  constexpr uint32_t kOut = 0x80000000u;  // at or past the end of both buffers

  for (int x = t; x < a.ring * RS; x += nt) ering[x] = 0.f;

  int row[MAXA], col[MAXA];    // current row and first column of the phase
  int prow[MAXA], pcol[MAXA];  // the same, PF phases ahead (loads in flight)
  float eleft[MAXA];           // error of the previous cell of the row
  float pf[PF][MAXA][K];       // intensities, loaded PF phases ahead
#pragma unroll
  for (int s = 0; s < MAXA; ++s) {
    row[s] = prow[s] = t + nt * s;
    col[s] = pcol[s] = -(K + 1) * row[s];
    eleft[s] = 0.f;
  }
  // a row is done once its phase starts past column W (column W itself is
  // still visited, to write the zero the row below reads there)
  auto advance = [&](int& r, int& c) -> bool {
    c += K;
    const bool done = c > W;
    r = done ? r + span : r;
    c = done ? c - wrap : c;
    return done;
  };
  auto load_phase = [&](float (&dst)[MAXA][K]) {
#pragma unroll
    for (int s = 0; s < MAXA; ++s) {
      const uint32_t rb = static_cast<uint32_t>(prow[s]) * static_cast<uint32_t>(W);
#pragma unroll
      for (int c = 0; c < K; ++c) {
        const int i = pcol[s] + c;
        const bool ok = i >= 0 && i < W && prow[s] < H;
        dst[s][c] = __builtin_bit_cast(
            float, __builtin_amdgcn_raw_buffer_load_b32(rsrc, ok ? (rb + static_cast<uint32_t>(i)) * 4u : kOut, 0, 0));
      }
      advance(prow[s], pcol[s]);
    }
  };
#pragma unroll
  for (int u = 0; u < PF; ++u) load_phase(pf[u]);
  __syncthreads();  // ring cleared

  for (int p0 = 0; p0 < a.phases; p0 += PF) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
#pragma unroll
      for (int s = 0; s < MAXA; ++s) {
        const int j = row[s], i0 = col[s];
        // row above, columns i0-1 .. i0+K (written in earlier phases)
        const float* up = ering + ((j - 1) & rmask) * RS;
        float* me = ering + (j & rmask) * RS;
        float ua[K + 2];
#pragma unroll
        for (int c = 0; c < K + 2; ++c) ua[c] = up[(i0 - 1 + c) & (D - 1)];
        const bool live_row = j < H;
        const bool starts = i0 < 0 && i0 + K >= 0;  // this phase holds column -1
        const uint32_t rb = static_cast<uint32_t>(j) * static_cast<uint32_t>(W);
#pragma unroll
        for (int c = 0; c < K; ++c) {
          const int i = i0 + c;
          const bool act = live_row && i >= 0 && i < W;
          // arrival order: below-right push of (i-1, j-1), below of (i, j-1),
          // below-left of (i+1, j-1), right of (i-1, j).  The oracle starts
          // from +0; starting from the first product differs only in the sign
          // of a zero sum.
          const float err = ((w1 * ua[c] + w5 * ua[c + 1]) + w3 * ua[c + 2]) + w7 * eleft[s];
          const float v = pf[u][s][c] + err;
          const bool sel = v >= 0.5f;
          const float e = act ? v - (sel ? 1.f : 0.f) : 0.f;
          eleft[s] = e;
          if (live_row && (act || i == W || (starts && i < 0))) me[i & (D - 1)] = e;
          __builtin_amdgcn_raw_buffer_store_b8(static_cast<uint8_t>(sel ? 1 : 0), rmask_out,
                                               act ? rb + static_cast<uint32_t>(i) : kOut, 0, 0);
        }
        if (advance(row[s], col[s])) eleft[s] = 0.f;
      }
      // loads for PF phases ahead reuse this phase's registers
      load_phase(pf[u]);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    }
  }
}

// One-wave variant: no LDS and no barrier.  Lane l takes rows l, l + 64,
// l + 128, ... in turn, K cells per phase, cell (i, j) at step i + (K+1) j as
// above.  The row below needs, in its next phase, this row's errors at its
// columns i0-1 .. i0+K: the last two cells of this lane's phase before last
// and the K cells of its last phase.  Each lane keeps those K + 2 values and
// the lane below reads them by a one-lane rotation of the wave (lane 0, which
// holds row 64 m, reads lane 63, which holds row 64 m - 1).  Cells outside the
// image (columns < 0 or >= W, rows >= H) carry error zero, so the rows above
// row 0 and the borders need no tests.  A lane moves to its next row once that
// row's first step falls in the phase; with 63 (K+1) >= W + 2K + 2 the row
// below has by then stopped reading the old row, and the lane above moved on
// only after this lane's row stopped reading it.  The arithmetic and its order
// are those of dither_kernel.
template <int K, int PF>
__global__ __launch_bounds__(64) void dither_wave_kernel(DitherArgs a) {
#pragma clang fp contract(off)
  const int l = threadIdx.x;
  const int W = a.W, H = a.H;
  const float w7 = 7.f / 16.f, w3 = 3.f / 16.f, w5 = 5.f / 16.f, w1 = 1.f / 16.f;
  const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(a.src), static_cast<short>(0), static_cast<int>(a.cells * 4u), 0x00020000);
  const __amdgpu_buffer_rsrc_t rmask_out = __builtin_amdgcn_make_buffer_rsrc(
      a.mask, static_cast<short>(0), static_cast<int>(a.cells), 0x00020000);
  constexpr uint32_t kOut = 0x80000000u;  // at or past the end of both buffers
  constexpr int kRowStep = 64 * (K + 1);  // steps between two rows of one lane

  int j = l, jf = l;            // row of this phase; row of the phase being prefetched
  int next = kRowStep + (K + 1) * l, nextf = next;  // first step of the lane's next row
  float hist[K + 2], elast[K];
#pragma unroll
  for (int c = 0; c < K + 2; ++c) hist[c] = 0.f;
#pragma unroll
  for (int c = 0; c < K; ++c) elast[c] = 0.f;
  float eleft = 0.f;
  float pf[PF][K];
  // Intensities of phase q: every cell of the phase with a column >= 0 has a
  // non-negative offset (W >= K), so one out-of-range marker per phase covers
  // phases without such a cell; a cell outside the image reads a value it
  // never uses.
  auto load_phase = [&](int q, float (&dst)[K]) {
    if (q * K + K - 1 >= nextf) {
      jf += 64;
      nextf += kRowStep;
    }
    const int base = jf * W + (q * K - (K + 1) * jf);
    const uint32_t off = base >= 0 ? static_cast<uint32_t>(base) * 4u : kOut;
#pragma unroll
    for (int c = 0; c < K; ++c)
      dst[c] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rsrc, off + 4u * c, 0, 0));
  };
#pragma unroll
  for (int u = 0; u < PF; ++u) load_phase(u, pf[u]);

  for (int p0 = 0; p0 < a.phases; p0 += PF) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int p = p0 + u;
      if (p * K + K - 1 >= next) {
        j += 64;
        next += kRowStep;
      }
      // columns i0-1 .. i0+K of the row above, from the lane above
      float ua[K + 2];
#pragma unroll
      for (int c = 0; c < K + 2; ++c)  // wave_ror:1, every lane has a source
        ua[c] = __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, hist[c]), 0x13C, 0xf, 0xf,
                                                                   true));
      const int i0 = p * K - (K + 1) * j;
      // a row past the last reads as a column past the end; the empty asm
      // keeps the limit a plain register, so each cell is tested with one
      // vector compare (left visible, the compiler splits the test into a
      // per-cell compare and a scalar AND with the row condition)
      uint32_t wlim = j < H ? static_cast<uint32_t>(W) : 0u;
      asm volatile("" : "+v"(wlim));
      // mask byte of cell c: offset base + c, the c in the instruction's scalar
      // offset; a cell outside the image selects kOut - c instead.  At 16
      // cells per phase the compiler's schedule of that form measured slower
      // (1240 against 913 us at 1024 x 1024), so that width adds per cell.
      constexpr bool kScalarOffset = K != 16;
      const uint32_t rb = static_cast<uint32_t>(j) * static_cast<uint32_t>(W);
      const uint32_t base = rb + static_cast<uint32_t>(i0);
      float ecur[K];
#pragma unroll
      for (int c = 0; c < K; ++c) {
        const int i = i0 + c;
        const bool act = static_cast<uint32_t>(i) < wlim;
        const float err = ((w1 * ua[c] + w5 * ua[c + 1]) + w3 * ua[c + 2]) + w7 * eleft;
        const float v = pf[u][c] + err;
        const bool sel = v >= 0.5f;
        const float e = act ? v - (sel ? 1.f : 0.f) : 0.f;
        eleft = e;
        ecur[c] = e;
        if constexpr (kScalarOffset)
          __builtin_amdgcn_raw_buffer_store_b8(static_cast<uint8_t>(sel ? 1 : 0), rmask_out,
                                               act ? base : kOut - static_cast<uint32_t>(c), c, 0);
        else
          __builtin_amdgcn_raw_buffer_store_b8(static_cast<uint8_t>(sel ? 1 : 0), rmask_out,
                                               act ? rb + static_cast<uint32_t>(i) : kOut, 0, 0);
      }
      hist[0] = elast[K - 2];
      hist[1] = elast[K - 1];
#pragma unroll
      for (int c = 0; c < K; ++c) {
        hist[c + 2] = ecur[c];
        elast[c] = ecur[c];
      }
      load_phase(p + PF, pf[u]);
    }
  }
}

// I = min(1, n m / total) in place (FP32 product and quotient rounded to
// nearest; a total that is not positive gives I = 0).
__global__ void intensity_kernel(float* __restrict__ m, uint32_t cells, float n, const FilterDev* __restrict__ dev) {
  const float total = dev->dither_total;
  const bool tpos = total > 0.f;
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < cells; e += gridDim.x * blockDim.x)
    m[e] = tpos ? fminf(1.f, (n * m[e]) / total) : 0.f;
}

// Belief map of the stored belief and its FP64 sum (rounded to FP32).
// A thread takes a run of four cells of a row (the pitch is a multiple of
// eight) and reads the run's heading planes kSrcBatch at a time, the loads
// of a batch all in flight.
constexpr int kSrcThreads = 256;
constexpr int kSrcMaxBlocks = 1024;
constexpr int kSrcBatch = 24;

template <typename T>
__device__ inline void load_run(const T* p, float v[4]);
template <>
__device__ inline void load_run<float>(const float* p, float v[4]) {
  const float4 q = *reinterpret_cast<const float4*>(p);
  v[0] = q.x;
  v[1] = q.y;
  v[2] = q.z;
  v[3] = q.w;
}
template <>
__device__ inline void load_run<__bf16>(const __bf16* p, float v[4]) {
  const uint2 q = *reinterpret_cast<const uint2*>(p);
  v[0] = __uint_as_float(q.x << 16);
  v[1] = __uint_as_float(q.x & 0xffff0000u);
  v[2] = __uint_as_float(q.y << 16);
  v[3] = __uint_as_float(q.y & 0xffff0000u);
}
template <>
__device__ inline void load_run<_Float16>(const _Float16* p, float v[4]) {
  typedef __attribute__((__vector_size__(4 * sizeof(_Float16)))) _Float16 h4;
  const h4 q = *reinterpret_cast<const h4*>(p);
  for (int i = 0; i < 4; ++i) v[i] = static_cast<float>(q[i]);
}

template <typename T>
__global__ __launch_bounds__(kSrcThreads) void dither_source_kernel(const void* buf0, const void* buf1, int W,
                                                                   int pitch, int n_theta, int64_t sstride,
                                                                   int runs, double* partials, FilterDev* dev,
                                                                   float* out) {
  __shared__ double rs[kSrcThreads];
  __shared__ int last_flag;
  const int t = threadIdx.x;
  const T* bel = static_cast<const T*>(dev->cur ? buf1 : buf0);
  const int rpr = pitch / 4;  // runs per row
  double s = 0.0;
  for (int q = blockIdx.x * kSrcThreads + t; q < runs; q += gridDim.x * kSrcThreads) {
    const int j = q / rpr, i0 = 4 * (q - j * rpr);
    const T* p = bel + static_cast<int64_t>(j) * pitch + i0;
    float m[4] = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < n_theta; k0 += kSrcBatch) {
      float v[kSrcBatch][4];
#pragma unroll
      for (int b = 0; b < kSrcBatch; ++b) {
        const int k = min(k0 + b, n_theta - 1);  // repeats of the last plane leave the max unchanged
        load_run<T>(p + k * sstride, v[b]);
      }
#pragma unroll
      for (int b = 0; b < kSrcBatch; ++b)
#pragma unroll
        for (int c = 0; c < 4; ++c) m[c] = fmaxf(m[c], v[b][c]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (i0 + c < W) {
        out[static_cast<int64_t>(j) * W + i0 + c] = m[c];
        s += static_cast<double>(m[c]);
      }
    }
  }
  rs[t] = s;
  __syncthreads();
  for (int st = kSrcThreads / 2; st > 0; st >>= 1) {
    if (t < st) rs[t] += rs[t + st];
    __syncthreads();
  }
  if (t == 0) {
    publish(&partials[blockIdx.x], rs[0]);
    last_flag = arrive_last(dev, blockIdx.x, gridDim.x);
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
  int K = 0, slots = 0, threads = 0, ring = 0, rstride = 0;
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
  // rows in flight at once: a slot takes its next row (K+1) span columns
  // back, once its current row is past column W
  const int64_t need = std::min<int64_t>(H, (static_cast<int64_t>(W) + K + K) / (K + 1));
  const int64_t nt = std::min<int64_t>(kDitherMaxThreads, (need + 63) / 64 * 64);
  const int64_t slots = (need + nt - 1) / nt;
  // ring rows: row j + ring first writes (its column -1, at step
  // (K+1)(j+ring) - 1) in a later phase than row j + 1 last reads row j
  // (step (K+1)(j+1) + W - 1); without reuse one more row, so that row -1
  // reads a ring row that stays zero
  const int64_t rows = std::min<int64_t>(static_cast<int64_t>(H) + 1,
                                         1 + (static_cast<int64_t>(W) + K + K) / (K + 1));
  if (slots > kDitherMaxSlots || rows > (1 << 20)) return p;
  p.ring = next_pow2(static_cast<int>(rows));
  // consecutive threads hold consecutive ring rows: an odd row stride puts
  // their accesses on distinct banks (a power-of-two stride shares banks
  // among every eighth lane); kept unpadded where the padding would not fit
  p.rstride = ring_cols(K) + 1;
  p.lds = static_cast<size_t>(p.ring) * p.rstride * sizeof(float);
  if (p.lds > kDitherMaxLds) {
    p.rstride = ring_cols(K);
    p.lds = static_cast<size_t>(p.ring) * p.rstride * sizeof(float);
  }
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

// Cells per phase of the one-wave kernel for width W: the smallest of 8, 16
// and 32 with 63 (K+1) >= W + 2K + 2 (and K <= W); 0 if none.
int wave_k(int W) {
  for (int K : {8, 16, 32})
    if (K <= W && 63 * (K + 1) >= W + 2 * K + 2) return K;
  return 0;
}

template <int K>
hipError_t launch_wave(const DitherArgs& a0, hipStream_t s) {
  constexpr int PF = 128 / K;  // loads in flight about PF phases ahead
  DitherArgs a = a0;
  const int64_t last = static_cast<int64_t>(a.W) - 1 + static_cast<int64_t>(K + 1) * (a.H - 1);
  const int64_t phases = last / K + 1;
  a.phases = static_cast<int32_t>((phases + PF - 1) / PF * PF);
  hipLaunchKernelGGL((dither_wave_kernel<K, PF>), dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

template <int K, int MAXA>
hipError_t launch_k(const DitherArgs& a0, const DitherPlan& p, hipStream_t s) {
  constexpr int PF = K == 1 ? 16 : 4;
  DitherArgs a = a0;
  // the last visit is the zero write at column W of the last row
  const int64_t last = static_cast<int64_t>(a.W) + static_cast<int64_t>(K + 1) * (a.H - 1);
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
  a.W = W;
  a.H = H;
  a.ring = p.ring;
  a.rstride = p.rstride;
  a.cells = static_cast<uint32_t>(static_cast<int64_t>(W) * H);
  if (scaled) {
    // the belief map in src becomes the intensity, in place
    const int blocks = static_cast<int>(std::min<int64_t>(1024, (a.cells + 255) / 256));
    hipLaunchKernelGGL(intensity_kernel, dim3(blocks), dim3(256), 0, s, const_cast<float*>(src), a.cells, n_samples, dev);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  switch (wave_k(W)) {
    case 8: return launch_wave<8>(a, s);
    case 16: return launch_wave<16>(a, s);
    case 32: return launch_wave<32>(a, s);
    default: break;
  }
  if (p.K == 3) {
    if (p.slots == 1) return launch_k<3, 1>(a, p, s);
    return launch_k<3, 2>(a, p, s);
  }
  return launch_k<1, 4>(a, p, s);
}

hipError_t launch_dither_source(int dtype, const void* buf0, const void* buf1, int W, int H, int pitch,
                                int n_theta, int64_t sstride, double* partials, FilterDev* dev, float* out,
                                hipStream_t s) {
  const int runs = static_cast<int>(static_cast<int64_t>(H) * pitch / 4);
  const int blocks = std::max(1, std::min(kSrcMaxBlocks, (runs + kSrcThreads - 1) / kSrcThreads));
  switch (dtype) {
    case 0: hipLaunchKernelGGL(dither_source_kernel<float>, dim3(blocks), dim3(kSrcThreads), 0, s, buf0, buf1, W, pitch, n_theta, sstride, runs, partials, dev, out); break;
    case 1: hipLaunchKernelGGL(dither_source_kernel<__bf16>, dim3(blocks), dim3(kSrcThreads), 0, s, buf0, buf1, W, pitch, n_theta, sstride, runs, partials, dev, out); break;
    case 2: hipLaunchKernelGGL(dither_source_kernel<_Float16>, dim3(blocks), dim3(kSrcThreads), 0, s, buf0, buf1, W, pitch, n_theta, sstride, runs, partials, dev, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mcl
