// Dense range-scan observation update on the matrix cores (gfx950).
//
// The observation update of eq. (sensor update) multiplies the belief by a
// per-beam Gaussian range likelihood and renormalises.  With ranges quantised
// to h = max_range / 256 (centred counts in [-128, 128], exact in BF16), the
// squared distance of the scan to the expected ranges of state (cell, k) is
//   D = sum_b (z_b - r[cell, (b + s_k) mod N])^2 = Sz - 2 X + Sr[cell],
//   X[cell, k] = sum_beta r[cell, beta] C[beta, k],  C[beta, k] = z[(beta - s_k) mod N],
// so the cross term X is a dense (cells x N) by (N x Theta) product.  Every
// partial sum is an integer below 2^24, so the FP32 accumulation of the MFMA
// is exact and D matches a direct integer evaluation bit for bit.
//
// Pass 1 (scan_gemm): X on MFMA (v_mfma_f32_32x32x16_bf16, or the FP32
//   32x32x2 form), epilogue D -> L = ln B - c D, per-tile reference state
//   (largest L), tile-relative L - L_ref written in FP32 (both terms formed
//   from exact integers and logs of stored values, so no large cancellation),
//   and the tile's L_ref in FP64.  The last workgroup takes M* = max L_ref.
// Pass 2 (scan_apply): B = exp(L - M*) with max one, stored in place, sum/max
//   reduction; the last workgroup updates the log-normaliser by
//   ln sum B + M* - ln(sum of the previous stored belief).
#include <float.h>
#include <math.h>

#include <algorithm>

#include "scan.hpp"

namespace mcl {
namespace {

constexpr int kTileCells = 128;  // cells per GEMM workgroup (4 waves x 32)
constexpr int kNChunk = 4;       // 32-wide N blocks held in accumulators at once
constexpr int kScanThreads = 256;
constexpr int kScanApplyBlocks = 1024;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

struct ScanArgs {
  const void* rq;       // [cells][kpad] quantised table (bf16 or f32)
  const int32_t* sr;    // [cells] sum of squares per cell
  const void* ct;       // [npad][kpad] circulant operand (same type as rq)
  void* buf[2];         // belief buffers (current one chosen by dev->cur)
  float* lrel;          // [n_theta][cells] tile-relative log-likelihood
  int32_t* dout;        // diagnostic: dense D [n_theta][H][W] (mode 1)
  double* partials;     // [tiles] reference L (pass 1), then 2 per pass-2 block
  FilterDev* dev;
  int32_t cells, n_theta, npad, kpad, W, pitch;
  int64_t sstride;
  int32_t sz;           // sum of squared scan counts
  float c;              // h^2 / (2 sigma^2)
  int32_t tiles;        // number of pass-1 workgroups
};

template <typename T>
__device__ inline float ld_belief(const T* p) {
  return static_cast<float>(*p);
}
template <>
__device__ inline float ld_belief<__bf16>(const __bf16* p) {
  return __uint_as_float(static_cast<uint32_t>(*reinterpret_cast<const uint16_t*>(p)) << 16);
}

// ---- circulant operand ---------------------------------------------------------
struct CtArgs {
  void* ct;
  int32_t n_dirs, n_theta, npad, kpad, f32;
  int16_t zq[kScanMaxDirs];
  int16_t s[kMaxTheta];
};

__global__ void build_ct_kernel(CtArgs a) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.npad * a.kpad) return;
  const int k = idx / a.kpad, beta = idx % a.kpad;
  float v = 0.f;
  if (k < a.n_theta && beta < a.n_dirs) {
    int b = (beta - a.s[k]) % a.n_dirs;
    if (b < 0) b += a.n_dirs;
    v = static_cast<float>(a.zq[b]);
  }
  if (a.f32)
    static_cast<float*>(a.ct)[idx] = v;
  else
    static_cast<__bf16*>(a.ct)[idx] = static_cast<__bf16>(v);
}

// ---- pass 1: cross term on MFMA + likelihood epilogue ----------------------------------
// One wave: 32 cells x (up to kNChunk*32) channels.  OP = __bf16 or float.
template <typename OP>
struct Mfma;

template <>
struct Mfma<__bf16> {
  static constexpr int KSTEP = 16;  // depth per instruction
  __device__ static inline void step(const __bf16* arow, const __bf16* brow, int k0, int half, f32x16& acc) {
    const bf16x8 a = *reinterpret_cast<const bf16x8*>(arow + k0 + 8 * half);
    const bf16x8 b = *reinterpret_cast<const bf16x8*>(brow + k0 + 8 * half);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
};

template <>
struct Mfma<float> {
  // Four 32x32x2 instructions per 8-deep chunk.  The depth order inside a
  // chunk is permuted identically for both operands (lane half h supplies
  // depth k0 + 4h + s at sub-step s); the sum is exact, so order is free.
  static constexpr int KSTEP = 8;
  __device__ static inline void step(const float* arow, const float* brow, int k0, int half, f32x16& acc) {
    const float4 a = *reinterpret_cast<const float4*>(arow + k0 + 4 * half);
    const float4 b = *reinterpret_cast<const float4*>(brow + k0 + 4 * half);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b.z, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b.w, acc, 0, 0, 0);
  }
};

// Accumulator layout of a 32x32 MFMA: lane l holds column (l % 32); register
// 4g + i holds row 8g + 4(l / 32) + i.  Rows are cells, columns channels.
// With at most kNChunk*32 channels the accumulators stay in registers between
// the search for the tile's reference state and the write of L - L_ref; more
// channels recompute the product once.
template <typename OP, typename T, int MODE>
__global__ __launch_bounds__(kScanThreads) void scan_gemm_kernel(ScanArgs a) {
  __shared__ float red_v[kScanThreads];
  __shared__ int red_i[kScanThreads];
  __shared__ int red_d[kScanThreads];
  __shared__ float red_lb[kScanThreads];
  __shared__ double red_m[kScanThreads];
  __shared__ int last_flag;
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const int half = lane >> 5, col = lane & 31;
  const int cell0 = blockIdx.x * kTileCells + wv * 32;
  const OP* rq = static_cast<const OP*>(a.rq);
  const OP* ct = static_cast<const OP*>(a.ct);
  FilterDev* dev = a.dev;
  const T* bel = static_cast<const T*>(a.buf[dev->cur]);
  const int arow_cell = min(cell0 + col, a.cells - 1);
  const OP* arow = rq + static_cast<int64_t>(arow_cell) * a.kpad;
  const int nblocks = a.npad / 32;
  const int nchunks = (nblocks + kNChunk - 1) / kNChunk;

  f32x16 acc[kNChunk];
  auto compute = [&](int nc) {
    const int nb0 = nc * kNChunk;
#pragma unroll
    for (int b = 0; b < kNChunk; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[b][i] = 0.f;
    for (int k0 = 0; k0 < a.kpad; k0 += Mfma<OP>::KSTEP) {
#pragma unroll
      for (int b = 0; b < kNChunk; ++b)
        if (nb0 + b < nblocks) {
          const OP* brow = ct + static_cast<int64_t>((nb0 + b) * 32 + col) * a.kpad;
          Mfma<OP>::step(arow, brow, k0, half, acc[b]);
        }
    }
  };
  // visit(k, cell, d) for every valid (channel, cell) of the accumulators
  auto epilogue = [&](int nc, auto&& visit) {
#pragma unroll
    for (int b = 0; b < kNChunk; ++b) {
      const int k = (nc * kNChunk + b) * 32 + col;
      if (nc * kNChunk + b >= nblocks || k >= a.n_theta) continue;
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int cell = cell0 + 8 * g + 4 * half + i;
          if (cell < a.cells) visit(k, cell, a.sz - 2 * static_cast<int>(acc[b][4 * g + i]) + a.sr[cell]);
        }
    }
  };

  if (MODE == 1) {
    const int H = a.cells / a.pitch;
    for (int nc = 0; nc < nchunks; ++nc) {
      compute(nc);
      epilogue(nc, [&](int k, int cell, int d) {
        const int j = cell / a.pitch, x = cell % a.pitch;
        if (x < a.W) a.dout[(static_cast<int64_t>(k) * H + j) * a.W + x] = d;
      });
    }
    return;
  }

  // search: largest L = ln B - c D (FP32 estimate; ties -> lowest index)
  float best = -INFINITY, best_lb = 0.f;
  int best_idx = -1, best_d = 0;
  for (int nc = 0; nc < nchunks; ++nc) {
    compute(nc);
    epilogue(nc, [&](int k, int cell, int d) {
      const float bv = ld_belief<T>(bel + static_cast<int64_t>(k) * a.sstride + cell);
      if (bv > 0.f) {
        const float lb = logf(bv);
        const float L = lb - a.c * static_cast<float>(d);
        const int idx = k * kTileCells + (cell - static_cast<int>(blockIdx.x) * kTileCells);
        if (L > best || (L == best && idx < best_idx)) {
          best = L;
          best_idx = idx;
          best_d = d;
          best_lb = lb;
        }
      }
    });
  }
  red_v[t] = best;
  red_i[t] = best_idx;
  red_d[t] = best_d;
  red_lb[t] = best_lb;
  __syncthreads();
  for (int st = kScanThreads / 2; st > 0; st >>= 1) {
    if (t < st) {
      const float o = red_v[t + st];
      const int oi = red_i[t + st];
      if (oi >= 0 && (red_i[t] < 0 || o > red_v[t] || (o == red_v[t] && oi < red_i[t]))) {
        red_v[t] = o;
        red_i[t] = oi;
        red_d[t] = red_d[t + st];
        red_lb[t] = red_lb[t + st];
      }
    }
    __syncthreads();
  }
  const bool has_ref = red_i[0] >= 0;
  const int ref_d = red_d[0];
  const float ref_lb = red_lb[0];
  if (t == 0) {
    // L_ref in FP64 from the stored value and the exact integer distance
    a.partials[blockIdx.x] = has_ref ? static_cast<double>(ref_lb) - static_cast<double>(a.c) * ref_d : -INFINITY;
  }
  // write L - L_ref for every state of the tile
  for (int nc = 0; nc < nchunks; ++nc) {
    if (nchunks > 1) compute(nc);
    epilogue(nc, [&](int k, int cell, int d) {
      const int64_t e = static_cast<int64_t>(k) * a.sstride + cell;
      const float bv = ld_belief<T>(bel + e);
      float lr = -INFINITY;
      if (bv > 0.f && has_ref) lr = (logf(bv) - ref_lb) - a.c * static_cast<float>(d - ref_d);
      a.lrel[e] = lr;
    });
  }

  // last workgroup: M* = max over tiles
  __syncthreads();
  if (t == 0) {
    const uint32_t prev = __hip_atomic_fetch_add(&dev->counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last_flag = (prev == static_cast<uint32_t>(gridDim.x - 1));
  }
  __syncthreads();
  if (!last_flag) return;
  double m = -INFINITY;
  for (int b = t; b < static_cast<int>(gridDim.x); b += kScanThreads)
    m = fmax(m, __hip_atomic_load(&a.partials[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  red_m[t] = m;
  __syncthreads();
  for (int st = kScanThreads / 2; st > 0; st >>= 1) {
    if (t < st) red_m[t] = fmax(red_m[t], red_m[t + st]);
    __syncthreads();
  }
  if (t == 0) {
    dev->aux[0] = red_m[0];
    if (!(red_m[0] > -INFINITY)) dev->status = kStatusDegenerate;
    __hip_atomic_store(&dev->counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---- pass 2: exponentiate, store, renormalise ------------------------------------------
template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(ScanArgs a) {
  __shared__ double rs[kScanThreads];
  __shared__ float rm[kScanThreads];
  __shared__ int last_flag;
  const int t = threadIdx.x;
  FilterDev* dev = a.dev;
  const double mstar = dev->aux[0];
  if (!(mstar > -INFINITY)) return;  // degenerate: keep the belief (uniform across the grid)
  T* bel = static_cast<T*>(a.buf[dev->cur]);
  double* part = a.partials + a.tiles;
  const int64_t n = static_cast<int64_t>(a.n_theta) * a.sstride;
  float s = 0.f, mx = 0.f;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(kScanThreads) + t; e < n;
       e += static_cast<int64_t>(gridDim.x) * kScanThreads) {
    const int cell = static_cast<int>(e % a.sstride);
    const double mt = a.partials[cell / kTileCells];
    float v = 0.f;
    if (mt > -INFINITY) v = expf(a.lrel[e] + static_cast<float>(mt - mstar));
    const T st = static_cast<T>(v);
    bel[e] = st;
    const float vs = static_cast<float>(st);
    s += vs;
    mx = fmaxf(mx, vs);
  }
  rs[t] = static_cast<double>(s);
  rm[t] = mx;
  __syncthreads();
  for (int st = kScanThreads / 2; st > 0; st >>= 1) {
    if (t < st) {
      rs[t] += rs[t + st];
      rm[t] = fmaxf(rm[t], rm[t + st]);
    }
    __syncthreads();
  }
  if (t == 0) {
    part[2 * blockIdx.x] = rs[0];
    part[2 * blockIdx.x + 1] = static_cast<double>(rm[0]);
    const uint32_t prev = __hip_atomic_fetch_add(&dev->counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last_flag = (prev == static_cast<uint32_t>(gridDim.x - 1));
  }
  __syncthreads();
  if (!last_flag) return;
  double ts = 0.0;
  float tm = 0.f;
  for (int b = t; b < static_cast<int>(gridDim.x); b += kScanThreads) {
    ts += __hip_atomic_load(&part[2 * b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    tm = fmaxf(tm, static_cast<float>(__hip_atomic_load(&part[2 * b + 1], __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT)));
  }
  rs[t] = ts;
  rm[t] = tm;
  __syncthreads();
  for (int st = kScanThreads / 2; st > 0; st >>= 1) {
    if (t < st) {
      rs[t] += rs[t + st];
      rm[t] = fmaxf(rm[t], rm[t + st]);
    }
    __syncthreads();
  }
  if (t == 0) {
    const double tot = rs[0];
    const float m = rm[0];
    if (!(tot > 0.0) || !isfinite(tot) || !(m > 0.f)) {
      dev->status = kStatusDegenerate;
    } else {
      dev->log_norm += log(tot) + mstar - dev->lnsum;
      dev->lnsum = log(tot);
      dev->sum = tot;
      dev->maxval = m;
      dev->scale = 1.0f / m;
    }
    __hip_atomic_store(&dev->counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---- map table: quantise ranges ---------------------------------------------------------
template <typename OP>
__global__ void quantize_kernel(const float* __restrict__ src, OP* __restrict__ rq, int32_t* __restrict__ sr, int W,
                                int pitch, int j0, int rows, int n_dirs, int kpad, double h) {
  const int local = blockIdx.x * blockDim.x + threadIdx.x;
  if (local >= rows * pitch) return;
  const int j = j0 + local / pitch, x = local % pitch;
  const int64_t cell = static_cast<int64_t>(j) * pitch + x;
  OP* out = rq + cell * kpad;
  int32_t ss = 0;
  for (int b = 0; b < kpad; ++b) {
    int q = 0;
    if (x < W && b < n_dirs) {
      const double r = static_cast<double>(src[(static_cast<int64_t>(local / pitch) * W + x) * n_dirs + b]);
      double f = floor(r / h + 0.5);
      f = f < 0.0 ? 0.0 : (f > 256.0 ? 256.0 : f);
      q = static_cast<int>(f) - 128;
    }
    out[b] = static_cast<OP>(static_cast<float>(q));
    ss += q * q;
  }
  sr[cell] = ss;
}

int round_up_i(int x, int m) { return (x + m - 1) / m * m; }

}  // namespace

// ---- host entry points ---------------------------------------------------------------------
size_t scan_work_bytes(int n_theta, int kpad) {
  if (kpad == 0) return 0;
  const int npad = round_up_i(n_theta, 32);
  return static_cast<size_t>(npad) * kpad * sizeof(float);
}

ScanWork scan_work_carve(void* base, int n_theta, int kpad) {
  ScanWork w;
  (void)n_theta;
  w.c = kpad ? base : nullptr;
  return w;
}

ScanTable scan_table_carve(Carver& c, const mcl_map_desc* d, int pitch, bool f32) {
  ScanTable t;
  if (!d->range_table) return t;
  t.n_dirs = d->n_dirs;
  t.kpad = round_up_i(d->n_dirs, 32);
  t.max_range = d->max_range_m;
  t.f32 = f32;
  const size_t cells = static_cast<size_t>(d->height) * pitch;
  t.rq = c.take(cells * t.kpad * (f32 ? 4 : 2));
  t.sr = static_cast<int32_t*>(c.take(cells * sizeof(int32_t)));
  t.stage_elems = std::max<size_t>(static_cast<size_t>(d->width) * d->n_dirs, 1u << 22);
  t.stage = static_cast<float*>(c.take(t.stage_elems * sizeof(float)));
  return t;
}

mcl_status scan_table_build(ScanTable& t, const mcl_map_desc* d, int pitch, hipStream_t s) {
  if (t.n_dirs == 0) return MCL_OK;
  const int W = d->width, H = d->height;
  const size_t row_elems = static_cast<size_t>(W) * d->n_dirs;
  const int rows_per = static_cast<int>(std::max<size_t>(1, t.stage_elems / row_elems));
  const double h = d->max_range_m / 256.0;
  for (int j0 = 0; j0 < H; j0 += rows_per) {
    const int rows = std::min(rows_per, H - j0);
    hipError_t e = hipMemcpyAsync(t.stage, d->range_table + static_cast<size_t>(j0) * row_elems,
                                  rows * row_elems * sizeof(float), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return MCL_EDEVICE;
    const int n = rows * pitch;
    if (t.f32)
      hipLaunchKernelGGL(quantize_kernel<float>, dim3((n + 255) / 256), dim3(256), 0, s, t.stage,
                         static_cast<float*>(t.rq), t.sr, W, pitch, j0, rows, d->n_dirs, t.kpad, h);
    else
      hipLaunchKernelGGL(quantize_kernel<__bf16>, dim3((n + 255) / 256), dim3(256), 0, s, t.stage,
                         static_cast<__bf16*>(t.rq), t.sr, W, pitch, j0, rows, d->n_dirs, t.kpad, h);
    if (hipGetLastError() != hipSuccess) return MCL_EDEVICE;
    // the staging buffer is reused by the next chunk
    if (hipStreamSynchronize(s) != hipSuccess) return MCL_EDEVICE;
  }
  return MCL_OK;
}

}  // namespace mcl

namespace mcl {

hipError_t scan_launch(const ScanLaunch& L, const float* ranges_m, double sigma_m, int32_t* dout) {
  const ScanTable& t = *L.table;
  const int N = t.n_dirs;
  const double h = t.max_range / 256.0;
  CtArgs ca;
  ca.ct = L.work.c;
  ca.n_dirs = N;
  ca.n_theta = L.n_theta;
  ca.npad = round_up_i(L.n_theta, 32);
  ca.kpad = t.kpad;
  ca.f32 = t.f32 ? 1 : 0;
  int64_t sz = 0;
  for (int b = 0; b < N; ++b) {
    double f = floor(static_cast<double>(ranges_m[b]) / h + 0.5);
    f = f < 0.0 ? 0.0 : (f > 256.0 ? 256.0 : f);
    const int q = static_cast<int>(f) - 128;
    ca.zq[b] = static_cast<int16_t>(q);
    sz += q * q;
  }
  const double dth = 2.0 * M_PI / L.n_theta;
  const double step = 2.0 * M_PI / N;
  for (int k = 0; k < L.n_theta; ++k) {
    long s = static_cast<long>(floor((L.theta + k * dth) / step + 0.5)) % N;
    if (s < 0) s += N;
    ca.s[k] = static_cast<int16_t>(s);
  }
  const int nct = ca.npad * ca.kpad;
  hipLaunchKernelGGL(build_ct_kernel, dim3((nct + 255) / 256), dim3(256), 0, L.stream, ca);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;

  ScanArgs a = {};
  a.rq = t.rq;
  a.sr = t.sr;
  a.ct = L.work.c;
  a.buf[0] = L.buf[0];
  a.buf[1] = L.buf[1];
  a.lrel = L.scratch;
  a.dout = dout;
  a.partials = L.partials;
  a.dev = L.dev;
  a.cells = L.H * L.pitch;
  a.n_theta = L.n_theta;
  a.npad = ca.npad;
  a.kpad = t.kpad;
  a.W = L.W;
  a.pitch = L.pitch;
  a.sstride = L.sstride;
  a.sz = static_cast<int32_t>(sz);
  a.c = static_cast<float>(h * h / (2.0 * sigma_m * sigma_m));
  a.tiles = (a.cells + kTileCells - 1) / kTileCells;
  const dim3 g1(a.tiles), b1(kScanThreads);
#define MCL_GEMM(OP, T, MODE) hipLaunchKernelGGL((scan_gemm_kernel<OP, T, MODE>), g1, b1, 0, L.stream, a)
  if (dout) {
    if (t.f32) MCL_GEMM(float, float, 1);
    else MCL_GEMM(__bf16, float, 1);
    return hipGetLastError();
  }
  switch (L.dtype * 2 + (t.f32 ? 1 : 0)) {
    case 0: MCL_GEMM(__bf16, float, 0); break;
    case 1: MCL_GEMM(float, float, 0); break;
    case 2: MCL_GEMM(__bf16, __bf16, 0); break;
    case 3: MCL_GEMM(float, __bf16, 0); break;
    case 4: MCL_GEMM(__bf16, _Float16, 0); break;
    case 5: MCL_GEMM(float, _Float16, 0); break;
    default: return hipErrorInvalidValue;
  }
#undef MCL_GEMM
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int blocks2 = kScanApplyBlocks;
  switch (L.dtype) {
    case 0: hipLaunchKernelGGL(scan_apply_kernel<float>, dim3(blocks2), dim3(kScanThreads), 0, L.stream, a); break;
    case 1: hipLaunchKernelGGL(scan_apply_kernel<__bf16>, dim3(blocks2), dim3(kScanThreads), 0, L.stream, a); break;
    case 2: hipLaunchKernelGGL(scan_apply_kernel<_Float16>, dim3(blocks2), dim3(kScanThreads), 0, L.stream, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int scan_tiles(int cells) { return (cells + kTileCells - 1) / kTileCells; }

}  // namespace mcl
