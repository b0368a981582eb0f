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
constexpr int kMaxNChunk = 4;    // 32-wide channel blocks held in accumulators at once, at most
constexpr int kScanThreads = 256;
constexpr int kScanApplyBlocks = 1024;  // pass-2 workgroups at most (two partials each)

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
  uint32_t rq_bytes;    // size of the tiled table
};

// Four consecutive stored beliefs (16-byte aligned for FP32, 8-byte for 16-bit storage).
template <typename T>
__device__ inline void load4(const T* p, float v[4]);
template <>
__device__ inline void load4<float>(const float* p, float v[4]) {
  const float4 q = *reinterpret_cast<const float4*>(p);
  v[0] = q.x;
  v[1] = q.y;
  v[2] = q.z;
  v[3] = q.w;
}
template <>
__device__ inline void load4<__bf16>(const __bf16* p, float v[4]) {
  const uint2 q = *reinterpret_cast<const uint2*>(p);
  v[0] = __uint_as_float(q.x << 16);
  v[1] = __uint_as_float(q.x & 0xffff0000u);
  v[2] = __uint_as_float(q.y << 16);
  v[3] = __uint_as_float(q.y & 0xffff0000u);
}
template <>
__device__ inline void load4<_Float16>(const _Float16* p, float v[4]) {
  typedef __attribute__((__vector_size__(4 * sizeof(_Float16)))) _Float16 h4;
  const h4 q = *reinterpret_cast<const h4*>(p);
  for (int i = 0; i < 4; ++i) v[i] = static_cast<float>(q[i]);
}
// Store four values rounded to the storage type (round to nearest even);
// returns the stored values as FP32 in v.
template <typename T>
__device__ inline void store4(T* p, float v[4]) {
  typedef __attribute__((__vector_size__(4 * sizeof(T)))) T t4;
  t4 q;
  for (int i = 0; i < 4; ++i) {
    q[i] = static_cast<T>(v[i]);
    v[i] = static_cast<float>(q[i]);
  }
  *reinterpret_cast<t4*>(p) = q;
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
//
// The range table is stored in the order the matrix-core A operand is read
// ("MFMA-tiled"): for every group of 32 cells and every depth step of KSTEP,
// the 64 lanes' 16-byte operands lie contiguously (lane l = cell l % 32,
// depth half l / 32).  One A load per step is then a single coalesced 1 KB
// read, and the whole table is read once per scan.
template <typename OP>
struct Mfma;

template <>
struct Mfma<__bf16> {
  static constexpr int KSTEP = 16;  // depth per instruction
  static constexpr int HALF = 8;    // depth per lane
  using Vec = bf16x8;
  __device__ static inline void mma(const Vec& av, const Vec& bv, f32x16& acc) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
  }
};

template <>
struct Mfma<float> {
  // Four 32x32x2 instructions per 8-deep chunk.  The depth order inside a
  // chunk is permuted identically for both operands (lane half h supplies
  // depth k0 + 4h + s at sub-step s); the sum is exact, so order is free.
  static constexpr int KSTEP = 8;
  static constexpr int HALF = 4;
  using Vec = float4;
  __device__ static inline void mma(const Vec& av, const Vec& bv, f32x16& acc) {
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, bv.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.y, bv.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.z, bv.z, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.w, bv.w, acc, 0, 0, 0);
  }
};

// Element offset of table entry (cell, beta) in the MFMA-tiled layout:
// [depth step][32-cell group][lane][HALF].  Step-major order makes the waves
// that run at the same time (same step, neighbouring groups) read one
// contiguous stretch of memory, spread over all HBM channels.
template <typename OP>
__host__ __device__ inline int64_t tiled_offset(int64_t cell, int beta, int64_t ngroups) {
  constexpr int KSTEP = Mfma<OP>::KSTEP, HALF = Mfma<OP>::HALF;
  const int64_t group = cell >> 5;
  const int r = static_cast<int>(cell & 31);
  const int step = beta / KSTEP, k = beta % KSTEP;
  const int lane = r + 32 * (k / HALF);
  return ((step * ngroups + group) * 64 + lane) * HALF + (k % HALF);
}

// Accumulator layout of a 32x32 MFMA: lane l holds column (l % 32); register
// 4g + i holds row 8g + 4(l / 32) + i.  Rows are cells, columns channels, so
// a lane owns runs of four consecutive cells of one channel: the epilogue
// reads the belief and writes L in 16-byte (FP32) pieces.  With at most
// kNChunk*32 channels the accumulators and ln B stay in registers between
// the search for the tile's reference state and the write of L - L_ref; more
// channels recompute the product once.
//
// BL: the whole circulant operand (every channel block, depth KPAD) is staged
// once per workgroup in LDS, in the order the MFMA reads it ([block][depth
// step][lane]), so the four waves share it instead of each streaming it from
// L2; only when all blocks fit one pass (nblocks == NCH) and KPAD > 0.
template <typename OP, typename T, int MODE, int NCH, int KPAD, bool BL = false>
__device__ __forceinline__ void scan_gemm_body(const ScanArgs& a, const int tile, const int ntiles,
                                               const bool stage = true) {
  constexpr int kNChunk = NCH;  // 32-wide channel blocks held in accumulators at once
  static_assert(!BL || KPAD > 0, "the staged operand needs a compile-time depth");
  __shared__ float red_v[kScanThreads];
  __shared__ int red_i[kScanThreads];
  __shared__ int red_d[kScanThreads];
  __shared__ float red_lb[kScanThreads];
  __shared__ double red_m[kScanThreads];
  __shared__ int last_flag;
  constexpr int KSTEP = Mfma<OP>::KSTEP, HALF = Mfma<OP>::HALF;
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const int half = lane >> 5, col = lane & 31;
  const int cell0 = tile * kTileCells + wv * 32;
  const OP* ct = static_cast<const OP*>(a.ct);
  FilterDev* dev = a.dev;
  const T* bel = static_cast<const T*>(a.buf[dev->cur]);
  // this wave's 32-cell group of the tiled table (padded to whole groups)
  const int64_t ngroups = (a.cells + 31) / 32;
  const OP* agroup = static_cast<const OP*>(a.rq) + (static_cast<int64_t>(cell0 >> 5) * 64 + lane) * HALF;
  const int64_t astep = ngroups * 64 * HALF;  // elements between depth steps
  const int nblocks = a.npad / 32;
  const int nchunks = (nblocks + kNChunk - 1) / kNChunk;

  using Vec = typename Mfma<OP>::Vec;
  constexpr int KSB = KPAD > 0 ? KPAD / KSTEP : 1;  // depth steps of the staged operand
  __shared__ Vec bsh[BL ? NCH * KSB * 64 : 1];
  if (BL && stage) {
    // 16-byte pieces of the [npad][kpad] operand, column by column (the
    // global reads are contiguous), written to their MFMA-order slots
    constexpr int PPC = KPAD / HALF;  // pieces per column
    const __amdgpu_buffer_rsrc_t rsb = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<OP*>(ct), static_cast<short>(0), static_cast<int>(a.npad * a.kpad * sizeof(OP)), 0x00020000);
    for (int e = t; e < NCH * 32 * PPC; e += kScanThreads) {
      const int c = e / PPC, pc = e - c * PPC;
      const int st = (pc * HALF) / KSTEP, hf = ((pc * HALF) % KSTEP) / HALF;
      bsh[((c >> 5) * KSB + st) * 64 + hf * 32 + (c & 31)] = __builtin_bit_cast(
          Vec, __builtin_amdgcn_raw_buffer_load_b128(rsb, static_cast<uint32_t>(e * 16), 0, 0));
    }
    __syncthreads();
  }

  f32x16 acc[kNChunk];
  // Depth loop.  The operands of a step are loaded four steps ahead (a ring
  // of four register sets): the A pieces stream from HBM, the B pieces (the
  // small circulant operand) come from the caches.  The loop is unrolled by four
  // with compile-time buffer indices and has no branch; the scheduling
  // barriers keep the compiler from sinking loads down to their use, which
  // would expose the memory latency at every step.  Loads past the last step
  // repeat the last step's address and are never used.  Channel blocks past
  // the last one (a final partial chunk) repeat the last block's operand; the
  // epilogue ignores them.
  constexpr int PA = 4;               // prefetch depth (steps)
  constexpr int EB = sizeof(OP);
  const int nsteps = a.kpad / KSTEP;  // a multiple of PA: kpad is a multiple of 64
  // Operands come through raw buffer descriptors: the per-step offsets go
  // into the scalar offset (A: one 1 KB piece per wave and step) or the
  // instruction's immediate offset (B), so the depth loop needs no vector
  // address registers.  All offsets lie inside the tables.
  const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void*>(a.rq), static_cast<short>(0), static_cast<int>(a.rq_bytes), 0x00020000);
  const uint32_t va = static_cast<uint32_t>(((cell0 >> 5) * 64 + lane) * HALF * EB);
  const uint32_t astep_bytes = static_cast<uint32_t>(astep * EB);
  const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<OP*>(ct), static_cast<short>(0), static_cast<int>(a.npad * a.kpad * EB), 0x00020000);
  auto load_a = [&](int step, Vec& v) {
    const uint32_t so = static_cast<uint32_t>(min(step, nsteps - 1)) * astep_bytes;
    v = __builtin_bit_cast(Vec, __builtin_amdgcn_raw_buffer_load_b128(ra, va, so, 0));
  };
  auto load_b = [&](int nc, int step, Vec (&v)[kNChunk]) {
    if constexpr (BL) {
      const int st = min(step, KSB - 1);
#pragma unroll
      for (int b = 0; b < kNChunk; ++b) v[b] = bsh[(b * KSB + st) * 64 + lane];
      return;
    }
    const uint32_t so = static_cast<uint32_t>(min(step, nsteps - 1) * KSTEP * EB);
#pragma unroll
    for (int b = 0; b < kNChunk; ++b) {
      const int nb = min(nc * kNChunk + b, nblocks - 1);
      const uint32_t vb = static_cast<uint32_t>(((nb * 32 + col) * a.kpad + HALF * half) * EB);
      v[b] = __builtin_bit_cast(Vec, __builtin_amdgcn_raw_buffer_load_b128(rb, vb, so, 0));
    }
  };
  auto compute = [&](int nc) {
#pragma unroll
    for (int b = 0; b < kNChunk; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[b][i] = 0.f;
    Vec abuf[PA];
    Vec bbuf[PA][kNChunk];
#pragma unroll
    for (int u = 0; u < PA; ++u) {
      load_a(u, abuf[u]);
      load_b(nc, u, bbuf[u]);
    }
    if constexpr (KPAD > 0) {
      // depth known at compile time: the whole loop is unrolled, so the
      // compiler's wait counters track every load exactly (a loop back edge
      // makes it wait for all outstanding loads at the top of each trip)
      constexpr int KS = KPAD / KSTEP;
#pragma unroll
      for (int st = 0; st < KS; st += PA) {
#pragma unroll
        for (int u = 0; u < PA; ++u) {
#pragma unroll
          for (int b = 0; b < kNChunk; ++b) Mfma<OP>::mma(abuf[u], bbuf[u][b], acc[b]);
          __builtin_amdgcn_sched_barrier(0);
          if (st + u + PA < KS) {
            load_a(st + u + PA, abuf[u]);
            load_b(nc, st + u + PA, bbuf[u]);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    } else {
      for (int st = 0; st < nsteps; st += PA) {
#pragma unroll
        for (int u = 0; u < PA; ++u) {
#pragma unroll
          for (int b = 0; b < kNChunk; ++b) Mfma<OP>::mma(abuf[u], bbuf[u][b], acc[b]);
          __builtin_amdgcn_sched_barrier(0);
          load_a(st + u + PA, abuf[u]);
          load_b(nc, st + u + PA, bbuf[u]);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
  };
  // visit(b, g, k, cb) for every valid run of four cells cb.. of channel k
  auto quads = [&](int nc, auto&& visit) {
#pragma unroll
    for (int b = 0; b < kNChunk; ++b) {
      const int k = (nc * kNChunk + b) * 32 + col;
      if (nc * kNChunk + b >= nblocks || k >= a.n_theta) continue;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int cb = cell0 + 8 * g + 4 * half;  // a.cells is a multiple of 8: runs are whole
        if (cb < a.cells) visit(b, g, k, cb);
      }
    }
  };
  auto dist = [&](int b, int g, int i, int sr) { return a.sz - 2 * static_cast<int>(acc[b][4 * g + i]) + sr; };

  if (MODE == 1) {
    const int H = a.cells / a.pitch;
    for (int nc = 0; nc < nchunks; ++nc) {
      compute(nc);
      quads(nc, [&](int b, int g, int k, int cb) {
        const int4 sr4 = *reinterpret_cast<const int4*>(a.sr + cb);
        const int srv[4] = {sr4.x, sr4.y, sr4.z, sr4.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int cell = cb + i;
          const int j = cell / a.pitch, x = cell % a.pitch;
          if (x < a.W) a.dout[(static_cast<int64_t>(k) * H + j) * a.W + x] = dist(b, g, i, srv[i]);
        }
      });
    }
    return;
  }

  // search: largest L = ln B - c D (FP32 estimate; ties -> lowest index).
  // ln B is computed once per state and kept for the write pass.
  float lbk[kNChunk][4][4];
  int srv[4][4];
  auto load_b4 = [&](int b, int g, int k, int cb) {
    load4<T>(bel + static_cast<int64_t>(k) * a.sstride + cb, lbk[b][g]);
  };
  auto to_log = [&](int b, int g) {
#pragma unroll
    for (int i = 0; i < 4; ++i) lbk[b][g][i] = lbk[b][g][i] > 0.f ? logf(lbk[b][g][i]) : -INFINITY;
  };
  float best = -INFINITY, best_lb = 0.f;
  int best_idx = -1, best_d = 0;
  for (int nc = 0; nc < nchunks; ++nc) {
    compute(nc);
    if (nc == 0) {
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int cb = min(cell0 + 8 * g + 4 * half, a.cells - 4);
        const int4 sr4 = *reinterpret_cast<const int4*>(a.sr + cb);
        srv[g][0] = sr4.x;
        srv[g][1] = sr4.y;
        srv[g][2] = sr4.z;
        srv[g][3] = sr4.w;
      }
    }
    quads(nc, load_b4);
    quads(nc, [&](int b, int g, int k, int cb) {
      to_log(b, g);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float lb = lbk[b][g][i];
        if (lb > -INFINITY) {
          const int d = dist(b, g, i, srv[g][i]);
          const float L = lb - a.c * static_cast<float>(d);
          const int idx = k * kTileCells + (cb + i - static_cast<int>(tile) * kTileCells);
          if (L > best || (L == best && idx < best_idx)) {
            best = L;
            best_idx = idx;
            best_d = d;
            best_lb = lb;
          }
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
    publish(&a.partials[tile], has_ref ? static_cast<double>(ref_lb) - static_cast<double>(a.c) * ref_d : -INFINITY);
  }
  // write L - L_ref for every state of the tile (both terms are differences
  // of nearby quantities: no large cancellation)
  for (int nc = 0; nc < nchunks; ++nc) {
    if (nchunks > 1) compute(nc);
    quads(nc, [&](int b, int g, int k, int cb) {
      if (nchunks > 1) {
        load_b4(b, g, k, cb);
        to_log(b, g);
      }
      float lr[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float lb = lbk[b][g][i];
        lr[i] = (lb > -INFINITY && has_ref) ? (lb - ref_lb) - a.c * static_cast<float>(dist(b, g, i, srv[g][i]) - ref_d)
                                            : -INFINITY;
      }
      *reinterpret_cast<float4*>(a.lrel + static_cast<int64_t>(k) * a.sstride + cb) = make_float4(lr[0], lr[1], lr[2], lr[3]);
    });
  }

  // last workgroup: M* = max over tiles
  __syncthreads();
  if (t == 0) {
    last_flag = arrive_last(dev, tile, ntiles);
  }
  __syncthreads();
  if (!last_flag) return;
  double m = -INFINITY;
  for (int b = t; b < ntiles; b += kScanThreads)
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

template <typename OP, typename T, int MODE, int NCH, int KPAD, bool BL = false>
__global__ __launch_bounds__(kScanThreads) void scan_gemm_kernel(ScanArgs a) {
  scan_gemm_body<OP, T, MODE, NCH, KPAD, BL>(a, blockIdx.x, gridDim.x);
}

// Persistent form of the staged-operand pass: a workgroup stages the
// circulant operand once and then takes tiles blockIdx.x, + gridDim.x, ...
// (two workgroups per compute unit fit the staged operand).  Every tile is
// computed and published exactly as by scan_gemm_kernel.
constexpr int kScanPersistBlocks = 512;
template <typename OP, typename T, int NCH>
__global__ __launch_bounds__(kScanThreads) void scan_gemm_persist_kernel(ScanArgs a, int ntiles) {
  bool stage = true;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    scan_gemm_body<OP, T, 0, NCH, 384, true>(a, tile, ntiles, stage);
    stage = false;
  }
}

// The scans of several filters of one map in one launch: every workgroup
// takes its 128-cell tile of the table for each filter in turn, so the tile
// is read from memory once and from the caches for the other filters.
constexpr int kScanBatchMax = 16;
struct ScanJobs {
  ScanArgs a[kScanBatchMax];
  int32_t n;
};

template <typename OP, typename T, int NCH, int KPAD, bool BL>
__global__ __launch_bounds__(kScanThreads) void scan_gemm_batch_kernel(ScanJobs jobs) {
  for (int j = 0; j < jobs.n; ++j) {
    scan_gemm_body<OP, T, 0, NCH, KPAD, BL>(jobs.a[j], blockIdx.x, gridDim.x);
    __syncthreads();  // shared arrays are reused by the next filter
  }
}

// ---- pass 2: exponentiate, store, renormalise ------------------------------------------
// Grid (bx, channel): block (bx, k) walks runs of four cells of plane k with
// a stride of gridDim.x runs, so every access is a 16-byte (FP32) piece and
// the tile of a cell is a shift, not a 64-bit division.
template <typename T>
__device__ __forceinline__ void scan_apply_body(const ScanArgs& a, const int bx, const int nbx, const int k) {
  __shared__ double rs[kScanThreads];
  __shared__ float rm[kScanThreads];
  __shared__ int last_flag;
  const int t = threadIdx.x;
  FilterDev* dev = a.dev;
  const double mstar = dev->aux[0];
  if (!(mstar > -INFINITY)) return;  // degenerate: keep the belief (uniform across the grid)
  const int blk = k * nbx + bx;
  const int nblk = nbx * a.n_theta;
  T* plane = static_cast<T*>(a.buf[dev->cur]) + static_cast<int64_t>(k) * a.sstride;
  const float* lplane = a.lrel + static_cast<int64_t>(k) * a.sstride;
  double* part = a.partials + a.tiles;
  const int nquads = static_cast<int>(a.sstride / 4);
  float s = 0.f, mx = 0.f;
  for (int q = bx * kScanThreads + t; q < nquads; q += nbx * kScanThreads) {
    const int cell = 4 * q;
    const double mt = a.partials[cell / kTileCells];
    const float4 lr = *reinterpret_cast<const float4*>(lplane + cell);
    const float off = static_cast<float>(mt - mstar);
    const bool live = mt > -INFINITY;
    float v[4] = {live ? expf(lr.x + off) : 0.f, live ? expf(lr.y + off) : 0.f, live ? expf(lr.z + off) : 0.f,
                  live ? expf(lr.w + off) : 0.f};
    store4<T>(plane + cell, v);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      s += v[i];
      mx = fmaxf(mx, v[i]);
    }
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
    publish(&part[2 * blk], rs[0]);
    publish(&part[2 * blk + 1], static_cast<double>(rm[0]));
    last_flag = arrive_last(dev, static_cast<uint32_t>(blk), static_cast<uint32_t>(nblk));
  }
  __syncthreads();
  if (!last_flag) return;
  double ts = 0.0;
  float tm = 0.f;
  for (int b = t; b < nblk; b += kScanThreads) {
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

template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(ScanArgs a) {
  scan_apply_body<T>(a, blockIdx.x, gridDim.x, blockIdx.y);
}

// pass 2 of several filters: blockIdx.z is the filter, blockIdx.y the channel
template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_apply_batch_kernel(ScanJobs jobs) {
  const ScanArgs& a = jobs.a[blockIdx.z];
  if (static_cast<int>(blockIdx.y) >= a.n_theta) return;
  scan_apply_body<T>(a, blockIdx.x, gridDim.x, blockIdx.y);
}

// ---- sampled observation update ---------------------------------------------------------
// The update of eq. (sensor update) on the states of the cells a selection
// mask holds (the Floyd-Steinberg samples of the belief map, Sec. III-B).  A
// state that is not sampled takes the likelihood of the best-matching sample,
// so unsampled states keep their stored value and a sampled state is
// multiplied by exp(-c (D - D*)), D* the smallest distance over the samples.
//
//   compact  mask -> list of the selected cells (any order) and, for every
//            cell of the pitch layout, its position in the list (-1: not
//            selected)
//   pass 1   D of every sampled state on the matrix cores: the dense product
//            restricted to the listed rows of the range table (each lane
//            gathers its own 16-byte operand pieces); D* by a last-workgroup
//            reduction.  D is stored per (list position, channel).
//   pass 2a  sampled states are multiplied in place, their old values kept
//            where D was
//   pass 2b  the whole belief is read once for its sum and max; the last
//            workgroup updates the log-normaliser by ln sum - c D* -
//            ln(previous sum), or, if no mass is left, puts the old values
//            back and flags the filter degenerate.
struct SampledArgs {
  const void* rq;       // MFMA-tiled range table
  const int32_t* sr;    // [cells] sum of squares per cell
  const void* ct;       // [npad][kpad] circulant operand
  void* buf[2];
  const uint8_t* mask;  // H x W dense selection
  int32_t* list;        // [nsel] selected cells (pitch layout)
  int32_t* pos;         // [cells] position in the list, -1 = not selected
  int32_t* dsc;         // [nsel][n_theta] D (pass 1), then the old value as FP32 bits (pass 2)
  double* partials;     // pass 1: one per workgroup; pass 2b: two per workgroup after them
  FilterDev* dev;
  int32_t cells, n_theta, npad, kpad, W, H, pitch;
  int64_t sstride;
  int32_t sz;           // sum of squared scan counts
  float c;              // h^2 / (2 sigma^2), FP32 (factors)
  double c64;           // the same in FP64 (log-normaliser)
  int32_t p1_blocks;    // pass-1 workgroups (offset of the pass-2 partials)
  uint32_t rq_bytes;
};

constexpr int kCompactThreads = 256;
constexpr int kCompactMaxBlocks = 1024;

// One workgroup per stretch of cells, a wave per quarter of it: a counting
// pass, one atomic per workgroup for the list offset, then the writing pass
// (the mask bytes come from the caches the second time).
__global__ __launch_bounds__(kCompactThreads) void compact_kernel(SampledArgs a, int per_wave) {
  __shared__ int wcount[kCompactThreads / 64];
  __shared__ int bbase;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const uint32_t n = static_cast<uint32_t>(a.cells);
  const uint32_t w0 = (blockIdx.x * (kCompactThreads / 64) + wv) * static_cast<uint32_t>(per_wave) * 64u;
  auto selected = [&](uint32_t cell) {
    const uint32_t j = cell / static_cast<uint32_t>(a.pitch), i = cell - j * static_cast<uint32_t>(a.pitch);
    return cell < n && i < static_cast<uint32_t>(a.W) && a.mask[j * static_cast<uint32_t>(a.W) + i] != 0;
  };
  int cnt = 0;
  for (int it = 0; it < per_wave; ++it) cnt += __popcll(__ballot(selected(w0 + it * 64u + lane)));
  if (lane == 0) wcount[wv] = cnt;
  __syncthreads();
  if (t == 0) {
    int tot = 0;
    for (int w = 0; w < kCompactThreads / 64; ++w) tot += wcount[w];
    bbase = tot > 0 ? __hip_atomic_fetch_add(&a.dev->nsel, tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
  }
  __syncthreads();
  int off = bbase;
  for (int w = 0; w < wv; ++w) off += wcount[w];
  const uint64_t below = (1ull << lane) - 1ull;
  for (int it = 0; it < per_wave; ++it) {
    const uint32_t cell = w0 + it * 64u + lane;
    const bool sel = selected(cell);
    const uint64_t bal = __ballot(sel);
    const int idx = off + __popcll(bal & below);
    if (sel) a.list[idx] = static_cast<int32_t>(cell);
    if (cell < n) a.pos[cell] = sel ? idx : -1;
    off += __popcll(bal);
  }
}

// Pass 1.  One work item = 32 listed cells x one 32-channel block.  With the
// depth known at compile time (KPAD > 0) the depth loop is unrolled and its
// operand loads run PA steps ahead.
template <typename OP, int KPAD>
__global__ __launch_bounds__(kScanThreads) void sampled_gemm_kernel(SampledArgs a) {
  __shared__ int red[kScanThreads / 64];
  __shared__ double red_d[kScanThreads];
  __shared__ int last_flag;
  constexpr int KSTEP = Mfma<OP>::KSTEP, HALF = Mfma<OP>::HALF, EB = sizeof(OP);
  using Vec = typename Mfma<OP>::Vec;
  constexpr int PA = 8;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int half = lane >> 5, col = lane & 31;
  FilterDev* dev = a.dev;
  const int nsel = __hip_atomic_load(&dev->nsel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int nblocks = a.npad / 32;
  const int items = (nsel + 31) / 32 * nblocks;
  const int64_t ngroups = (a.cells + 31) / 32;
  const uint32_t astep_bytes = static_cast<uint32_t>(ngroups * 64 * HALF * EB);
  const int nsteps = KPAD > 0 ? KPAD / KSTEP : a.kpad / KSTEP;  // a multiple of 4
  const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void*>(a.rq), static_cast<short>(0), static_cast<int>(a.rq_bytes), 0x00020000);
  const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void*>(a.ct), static_cast<short>(0), static_cast<int>(a.npad * a.kpad * EB), 0x00020000);
  int dmin = INT32_MAX;
  for (int it = blockIdx.x * (kScanThreads / 64) + wv; it < items; it += gridDim.x * (kScanThreads / 64)) {
    const int grp = it / nblocks, nb = it - grp * nblocks;
    const int cell = a.list[min(grp * 32 + col, nsel - 1)];
    const uint32_t va = static_cast<uint32_t>(((cell >> 5) * 64 + (cell & 31) + 32 * half) * HALF * EB);
    const uint32_t vb = static_cast<uint32_t>(((nb * 32 + col) * a.kpad + HALF * half) * EB);
    auto load = [&](int st, Vec& av, Vec& bv) {
      const int sc = min(st, nsteps - 1);
      av = __builtin_bit_cast(Vec, __builtin_amdgcn_raw_buffer_load_b128(ra, va, static_cast<uint32_t>(sc) * astep_bytes, 0));
      bv = __builtin_bit_cast(Vec, __builtin_amdgcn_raw_buffer_load_b128(rb, vb, static_cast<uint32_t>(sc * KSTEP * EB), 0));
    };
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.f;
    if constexpr (KPAD > 0) {
      constexpr int KS = KPAD / KSTEP;
      constexpr int P = PA < KS ? PA : KS;
      Vec abuf[P], bbuf[P];
#pragma unroll
      for (int u = 0; u < P; ++u) load(u, abuf[u], bbuf[u]);
#pragma unroll
      for (int st = 0; st < KS; ++st) {
        Mfma<OP>::mma(abuf[st % P], bbuf[st % P], acc);
        __builtin_amdgcn_sched_barrier(0);
        if (st + P < KS) load(st + P, abuf[st % P], bbuf[st % P]);
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
      constexpr int P = 4;
      Vec abuf[P], bbuf[P];
#pragma unroll
      for (int u = 0; u < P; ++u) load(u, abuf[u], bbuf[u]);
      for (int st = 0; st < nsteps; st += P) {
#pragma unroll
        for (int u = 0; u < P; ++u) {
          Mfma<OP>::mma(abuf[u], bbuf[u], acc);
          __builtin_amdgcn_sched_barrier(0);
          load(st + u + P, abuf[u], bbuf[u]);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    // rows are list positions, columns channels (accumulator layout of the dense pass)
    const int srv = a.sr[cell];
    const int k = nb * 32 + col;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rho = 8 * g + 4 * half + i;
        const int sr_r = __shfl(srv, rho);
        const int r = grp * 32 + rho;
        if (r < nsel && k < a.n_theta) {
          const int d = a.sz - 2 * static_cast<int>(acc[4 * g + i]) + sr_r;
          a.dsc[static_cast<int64_t>(r) * a.n_theta + k] = d;
          dmin = min(dmin, d);
        }
      }
    }
  }
  // D* over the grid
  for (int o = 32; o > 0; o >>= 1) dmin = min(dmin, __shfl_xor(dmin, o));
  if (lane == 0) red[wv] = dmin;
  __syncthreads();
  if (t == 0) {
    int m = red[0];
    for (int w = 1; w < kScanThreads / 64; ++w) m = min(m, red[w]);
    publish(&a.partials[blockIdx.x], static_cast<double>(m));
    last_flag = arrive_last(dev, blockIdx.x, gridDim.x);
  }
  __syncthreads();
  if (!last_flag) return;
  double m = static_cast<double>(INT32_MAX);
  for (int b = t; b < static_cast<int>(gridDim.x); b += kScanThreads)
    m = fmin(m, __hip_atomic_load(&a.partials[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  red_d[t] = m;
  __syncthreads();
  for (int st = kScanThreads / 2; st > 0; st >>= 1) {
    if (t < st) red_d[t] = fmin(red_d[t], red_d[t + st]);
    __syncthreads();
  }
  if (t == 0) {
    dev->dstar = static_cast<int32_t>(red_d[0]);
    __hip_atomic_store(&dev->counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Pass 2a.  One thread per sampled state (list position r, channel k):
// multiply the stored value in place by exp(-c (D - D*)) and keep the old
// value where D was.
template <typename T>
__global__ __launch_bounds__(kScanThreads) void sampled_scale_kernel(SampledArgs a) {
  FilterDev* dev = a.dev;
  const int dstar = dev->dstar;
  if (dstar == INT32_MAX) return;  // no sample
  const int nsel = __hip_atomic_load(&dev->nsel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  T* bel = static_cast<T*>(a.buf[dev->cur]);
  float* old = reinterpret_cast<float*>(a.dsc);
  const int n = nsel * a.n_theta;  // below 2^31: checked on the host
  for (int e = blockIdx.x * kScanThreads + threadIdx.x; e < n; e += gridDim.x * kScanThreads) {
    const int r = e / a.n_theta, k = e - r * a.n_theta;
    T* p = bel + static_cast<int64_t>(k) * a.sstride + a.list[r];
    const float v = static_cast<float>(*p);
    const int d = a.dsc[e];
    old[e] = v;
    *p = static_cast<T>(v * expf(-a.c * static_cast<float>(d - dstar)));
  }
}

// Pass 2b.  Sum and max of the whole stored belief (padding cells hold zero),
// streamed flat: a thread reads four runs of four values per round, a wave a
// contiguous stretch.  The last workgroup updates the filter scalars, or
// puts the old sampled values back if no mass is left.
template <typename T>
__global__ __launch_bounds__(kScanThreads) void sampled_apply_kernel(SampledArgs a) {
  __shared__ double rs[kScanThreads];
  __shared__ float rm[kScanThreads];
  __shared__ int last_flag;
  constexpr int U = 4;
  const int t = threadIdx.x;
  const int nthr = kScanThreads;
  FilterDev* dev = a.dev;
  const int dstar = dev->dstar;
  if (dstar == INT32_MAX) return;  // no sample: no update (uniform across the grid)
  T* bel = static_cast<T*>(a.buf[dev->cur]);
  float* old = reinterpret_cast<float*>(a.dsc);
  const int blk = blockIdx.x, nblk = gridDim.x;
  double* part = a.partials + a.p1_blocks;
  const int64_t nruns = a.sstride / 4 * a.n_theta;
  double s = 0.0;
  float mx = 0.f;
  for (int64_t b = static_cast<int64_t>(blockIdx.x) * kScanThreads * U + t; b < nruns;
       b += static_cast<int64_t>(gridDim.x) * kScanThreads * U) {
    float v[U][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = b + static_cast<int64_t>(u) * kScanThreads;
      if (i < nruns) load4<T>(bel + 4 * i, v[u]);
      else v[u][0] = v[u][1] = v[u][2] = v[u][3] = 0.f;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      s += static_cast<double>((v[u][0] + v[u][1]) + (v[u][2] + v[u][3]));
      mx = fmaxf(mx, fmaxf(fmaxf(v[u][0], v[u][1]), fmaxf(v[u][2], v[u][3])));
    }
  }
  rs[t] = s;
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
    publish(&part[2 * blk], rs[0]);
    publish(&part[2 * blk + 1], static_cast<double>(rm[0]));
    last_flag = arrive_last(dev, static_cast<uint32_t>(blk), static_cast<uint32_t>(nblk));
  }
  __syncthreads();
  if (!last_flag) return;
  double ts = 0.0;
  float tm = 0.f;
  for (int b = t; b < nblk; b += nthr) {
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
  const double tot = rs[0];
  const float m = rm[0];
  const bool degenerate = !(tot > 0.0) || !isfinite(tot) || !(m > 0.f);
  const int nsel = __hip_atomic_load(&dev->nsel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (degenerate) {
    // every sampled state went to zero and nothing else holds mass: restore
    const int64_t n = static_cast<int64_t>(nsel) * a.n_theta;
    for (int64_t e = t; e < n; e += nthr) {
      const int r = static_cast<int>(e / a.n_theta), k = static_cast<int>(e - static_cast<int64_t>(r) * a.n_theta);
      bel[static_cast<int64_t>(k) * a.sstride + a.list[r]] = static_cast<T>(old[e]);
    }
  }
  if (t == 0) {
    if (degenerate) {
      dev->status = kStatusDegenerate;
    } else {
      dev->log_norm += log(tot) - a.c64 * static_cast<double>(dstar) - dev->lnsum;
      dev->lnsum = log(tot);
      dev->sum = tot;
      dev->maxval = m;
      dev->scale = 1.0f / m;
    }
    dev->nsel = 0;
    __hip_atomic_store(&dev->counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---- best match of many scans over every free state (map difficulty) ------------------
// For a batch of query scans, the free cell q and heading k whose expected scan
// is closest (smallest exact D, heading offset 0): the dense product of the
// range table with the circulant columns of every (query, heading), reduced by
// min instead of exponentiated.  A 64-bit key (D, k, cell) orders the
// candidates as the stated tie rule does (lowest k * H * W + q: the padded
// cell index j * pitch + i has the dense order on candidate cells), so one
// min suffices.  The product kernel stores each workgroup's minimum per
// column; a second pass takes the minimum per query (a min is order-free, so
// the result does not depend on scheduling).
struct MatchArgs {
  const void* rq;          // MFMA-tiled range table
  const int32_t* sr;       // [cells] sum of squares
  const uint8_t* free8;    // [cells] free cells (pitch layout; 0 outside the grid)
  const void* ct;          // circulant columns (column = query * n_theta + k), MFMA-tiled per 32 columns
  const int32_t* sz;       // [batch] sum of squared counts of each query
  uint32_t* keys;          // [tiles][ncols_pad]: per workgroup and column, min of (D << 7 | local cell)
  uint64_t* best;          // [batch]
  int32_t cells, pitch, W, n_theta, ncols, ncols_pad, kpad, tiles;
  uint32_t rq_bytes;
  uint64_t inv_theta;      // ceil(2^40 / n_theta): column / n_theta = (column * inv_theta) >> 40
};

constexpr uint64_t kNoKey = ~0ull;

// column / n_theta without a division: exact for columns below 2^24 (the
// column operand's 2 GiB limit keeps them there) and n_theta <= 360: the
// product stays below 2^64 and the reciprocal's rounding error below 2^-16 <
// 1 / n_theta
__device__ inline int col_query(int c, uint64_t inv_theta) {
  return static_cast<int>((static_cast<uint64_t>(c) * inv_theta) >> 40);
}

// One workgroup: 128 cells (32 per wave, A operand in registers for the whole
// depth) against every column block of the batch.  A block of 32 columns is
// loaded once per workgroup into LDS, double buffered, in the order the MFMA
// reads it ([depth step][lane]), so all four waves share it.  Within the
// workgroup a candidate is a 32-bit key (D << 7 | local cell); D < 2^25 for
// any table of at most 384 directions, so the key is exact.  Per block, one
// wave in turn takes the minimum over the four waves and stores it.
template <typename OP, int KPAD>
__global__ __launch_bounds__(kScanThreads) void match_gemm_kernel(MatchArgs a) {
  constexpr int KSTEP = Mfma<OP>::KSTEP, HALF = Mfma<OP>::HALF, EB = sizeof(OP);
  constexpr int KS = KPAD / KSTEP;
  constexpr int BLK = KS * 64;                // 16-byte pieces in one 32-column block
  constexpr int PER = BLK / kScanThreads;     // pieces each thread stages per block
  constexpr int PB = 4;                       // LDS read-ahead in depth steps
  static_assert(BLK % kScanThreads == 0, "block not divisible among the threads");
  using Vec = typename Mfma<OP>::Vec;
  __shared__ Vec bs[2][BLK];
  __shared__ uint32_t wmin[2][kScanThreads / 64][32];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int half = lane >> 5, col = lane & 31;
  const int cell0 = blockIdx.x * kTileCells + wv * 32;
  const int64_t ngroups = (a.cells + 31) / 32;
  const uint32_t astep_bytes = static_cast<uint32_t>(ngroups * 64 * HALF * EB);
  const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void*>(a.rq), static_cast<short>(0), static_cast<int>(a.rq_bytes), 0x00020000);
  const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void*>(a.ct), static_cast<short>(0), static_cast<int>(a.ncols_pad * a.kpad * EB), 0x00020000);
  const int ncb = a.ncols_pad / 32;
  // stage column block 0
  {
    Vec v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u)
      v[u] = __builtin_bit_cast(Vec, __builtin_amdgcn_raw_buffer_load_b128(rb, static_cast<uint32_t>((t + u * kScanThreads) * 16), 0, 0));
#pragma unroll
    for (int u = 0; u < PER; ++u) bs[0][t + u * kScanThreads] = v[u];
  }
  // this wave's 32 cells: the A operand stays in registers for every column
  Vec av[KS];
  const uint32_t va = static_cast<uint32_t>(((cell0 >> 5) * 64 + lane) * HALF * EB);
#pragma unroll
  for (int st = 0; st < KS; ++st)
    av[st] = __builtin_bit_cast(Vec, __builtin_amdgcn_raw_buffer_load_b128(ra, va, static_cast<uint32_t>(st) * astep_bytes, 0));
  // the lane's 16 accumulator rows: (Sr << 7 | local cell) and whether the cell is a candidate
  uint32_t rbase[16];
  uint32_t okmask = 0;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int lc = wv * 32 + 8 * g + 4 * half + i;
      const int cell = blockIdx.x * kTileCells + lc;
      const int x = cell % a.pitch;
      const bool ok = cell < a.cells && x < a.W && a.free8[min(cell, a.cells - 1)] != 0;
      rbase[4 * g + i] = (static_cast<uint32_t>(a.sr[min(cell, a.cells - 1)]) << 7) | static_cast<uint32_t>(lc);
      okmask |= ok ? (1u << (4 * g + i)) : 0u;
    }
  }
  __syncthreads();
  // One column block per call.  The loads of block cb + 2 are issued here and
  // stored to LDS one call later, so each has a whole block's work to arrive;
  // block cb + 1 (loaded one call ago) is stored to the other LDS buffer.
  // ncb is even (the host pads the columns to 64), so the loop below runs
  // the calls in pairs with compile-time register sets.
  auto block = [&](int cb, Vec (&ld)[PER], Vec (&stv)[PER]) {
#pragma unroll
    for (int u = 0; u < PER; ++u)
      ld[u] = __builtin_bit_cast(Vec, __builtin_amdgcn_raw_buffer_load_b128(
                  rb, static_cast<uint32_t>(((cb + 2) * BLK + t + u * kScanThreads) * 16), 0, 0));
    const Vec* B = bs[cb & 1];
    Vec bf[PB];
#pragma unroll
    for (int u = 0; u < PB; ++u) bf[u] = B[u * 64 + lane];
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.f;
#pragma unroll
    for (int st = 0; st < KS; ++st) {
      Mfma<OP>::mma(av[st], bf[st % PB], acc);
      if (st + PB < KS) bf[st % PB] = B[(st + PB) * 64 + lane];
    }
    // column of this lane; key = (Sz + Sr - 2X) << 7 | local cell, exact in 32 bits
    const int c = cb * 32 + col;
    const int p = c < a.ncols ? col_query(c, a.inv_theta) : 0;
    const uint32_t sz7 = static_cast<uint32_t>(a.sz[p]) << 7;
    uint32_t m = ~0u;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const uint32_t key = rbase[r] + sz7 - (static_cast<uint32_t>(static_cast<int>(acc[r])) << 8);
      m = ((okmask >> r) & 1u) && key < m ? key : m;
    }
    const uint32_t o = __shfl_xor(m, 32);  // the other 16 rows of the same column
    m = o < m ? o : m;
    if (half == 0) wmin[cb & 1][wv][col] = m;
#pragma unroll
    for (int u = 0; u < PER; ++u) bs[(cb + 1) & 1][t + u * kScanThreads] = stv[u];
    __syncthreads();
    if (wv == (cb & 3) && lane < 32) {
      // the workgroup's minimum per column, stored for the per-query pass
      uint32_t w = wmin[cb & 1][0][lane];
#pragma unroll
      for (int v = 1; v < kScanThreads / 64; ++v) w = wmin[cb & 1][v][lane] < w ? wmin[cb & 1][v][lane] : w;
      a.keys[static_cast<int64_t>(blockIdx.x) * a.ncols_pad + cb * 32 + lane] = w;
    }
  };
  Vec nxA[PER], nxB[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u)
    nxA[u] = __builtin_bit_cast(Vec, __builtin_amdgcn_raw_buffer_load_b128(
                 rb, static_cast<uint32_t>((BLK + t + u * kScanThreads) * 16), 0, 0));
  for (int cb = 0; cb < ncb; cb += 2) {
    block(cb, nxB, nxA);
    block(cb + 1, nxA, nxB);
  }
}

// Per query: the minimum over workgroups and headings of the 64-bit key
// (D << 39) | (k << 30) | cell, cell in the padded layout (its order is the
// dense order on candidate cells).  Grid (queries, kReduceChunks): each
// workgroup takes one share of the product's workgroups and folds its
// minimum into best[query] with a 64-bit atomic min (order-free).
constexpr int kReduceChunks = 16;
__global__ __launch_bounds__(kScanThreads) void match_reduce_kernel(MatchArgs a) {
  __shared__ uint64_t red[kScanThreads];
  const int t = threadIdx.x, p = blockIdx.x;
  uint64_t m = kNoKey;
  const int64_t n = static_cast<int64_t>(a.tiles) * a.n_theta;
  const int64_t e0 = n * blockIdx.y / gridDim.y, e1 = n * (blockIdx.y + 1) / gridDim.y;
  const bool recip = n < (int64_t{1} << 24);  // (tile, k) from e without a 64-bit division
  for (int64_t e = e0 + t; e < e1; e += kScanThreads) {
    const int tile = recip ? col_query(static_cast<int>(e), a.inv_theta) : static_cast<int>(e / a.n_theta);
    const int k = static_cast<int>(e - static_cast<int64_t>(tile) * a.n_theta);
    const uint32_t w = a.keys[static_cast<int64_t>(tile) * a.ncols_pad + static_cast<int64_t>(p) * a.n_theta + k];
    if (w == ~0u) continue;
    const uint64_t key = (static_cast<uint64_t>(w >> 7) << 39) | (static_cast<uint64_t>(k) << 30) |
                         static_cast<uint64_t>(tile * kTileCells + static_cast<int>(w & 127u));
    m = key < m ? key : m;
  }
  red[t] = m;
  __syncthreads();
  for (int st = kScanThreads / 2; st > 0; st >>= 1) {
    if (t < st && red[t + st] < red[t]) red[t] = red[t + st];
    __syncthreads();
  }
  if (t == 0 && red[0] != kNoKey) __hip_atomic_fetch_min(a.best + p, red[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Circulant columns of a batch of queries: C[p * n_theta + k][beta] = zq_p[(beta - s_k) mod N],
// stored in the order the product kernel stages them.
struct MatchCtArgs {
  void* ct;
  const int16_t* zq;        // [batch][n_dirs]
  uint64_t* best;           // [nq], set to all ones
  int32_t n_dirs, n_theta, ncols, ncols_pad, kpad, f32, nq;
  int16_t s[kMaxTheta];
};

// One thread per 16-byte piece: HALF consecutive depths of one column, which
// the MFMA-tiled order keeps together ([block][depth step][lane half][column][HALF]).
template <typename OP>
__device__ inline void match_ct_piece(const MatchCtArgs& a, int64_t piece) {
  constexpr int KSTEP = Mfma<OP>::KSTEP, HALF = Mfma<OP>::HALF;
  const int ppc = a.kpad / HALF;  // pieces per column
  const int c = static_cast<int>(piece / ppc), beta0 = static_cast<int>(piece - static_cast<int64_t>(c) * ppc) * HALF;
  const int st = beta0 / KSTEP, hf = (beta0 - st * KSTEP) / HALF;
  const int64_t dst = (static_cast<int64_t>(c / 32) * (a.kpad / KSTEP) + st) * 64 + hf * 32 + (c & 31);
  float v[HALF];
  const bool live = c < a.ncols;
  const int p = live ? c / a.n_theta : 0, k = live ? c - p * a.n_theta : 0;
  int b = (beta0 - a.s[k]) % a.n_dirs;
  if (b < 0) b += a.n_dirs;
#pragma unroll
  for (int h = 0; h < HALF; ++h) {
    v[h] = live && beta0 + h < a.n_dirs ? static_cast<float>(a.zq[static_cast<int64_t>(p) * a.n_dirs + b]) : 0.f;
    b = b + 1 == a.n_dirs ? 0 : b + 1;
  }
  typename Mfma<OP>::Vec out;
  if constexpr (sizeof(OP) == 4) {
    out = make_float4(v[0], v[1], v[2], v[3]);
  } else {
#pragma unroll
    for (int h = 0; h < HALF; ++h) out[h] = static_cast<OP>(v[h]);
  }
  static_cast<typename Mfma<OP>::Vec*>(a.ct)[dst] = out;
}

__global__ void match_ct_kernel(MatchCtArgs a) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx < a.nq) a.best[idx] = kNoKey;
  const int64_t pieces = static_cast<int64_t>(a.ncols_pad) * a.kpad / (a.f32 ? Mfma<float>::HALF : Mfma<__bf16>::HALF);
  if (idx >= pieces) return;
  if (a.f32)
    match_ct_piece<float>(a, idx);
  else
    match_ct_piece<__bf16>(a, idx);
}

// ---- map table: quantise ranges ---------------------------------------------------------
template <typename OP>
__global__ void quantize_kernel(const float* __restrict__ src, OP* __restrict__ rq, int32_t* __restrict__ sr, int W,
                                int pitch, int j0, int rows, int n_dirs, int kpad, double h, int64_t ngroups) {
  const int local = blockIdx.x * blockDim.x + threadIdx.x;
  if (local >= rows * pitch) return;
  const int j = j0 + local / pitch, x = local % pitch;
  const int64_t cell = static_cast<int64_t>(j) * pitch + x;
  int32_t ss = 0;
  for (int b = 0; b < kpad; ++b) {
    int q = 0;
    if (x < W && b < n_dirs) {
      const double r = static_cast<double>(src[(static_cast<int64_t>(local / pitch) * W + x) * n_dirs + b]);
      double f = floor(r / h + 0.5);
      f = f < 0.0 ? 0.0 : (f > 256.0 ? 256.0 : f);
      q = static_cast<int>(f) - 128;
    }
    rq[tiled_offset<OP>(cell, b, ngroups)] = static_cast<OP>(static_cast<float>(q));
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
  t.kpad = round_up_i(d->n_dirs, 64);  // whole groups of four depth steps (depth loop)
  t.max_range = d->max_range_m;
  t.f32 = f32;
  const size_t cells = static_cast<size_t>(d->height) * pitch;
  const size_t cells_pad = (cells + 31) / 32 * 32;  // whole 32-cell groups of the tiled layout
  t.rq_bytes = cells_pad * t.kpad * (f32 ? 4 : 2);
  t.rq = c.take(t.rq_bytes);
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
  // the padding cells of the last 32-cell group stay zero
  if (hipMemsetAsync(t.rq, 0, t.rq_bytes, s) != hipSuccess) return MCL_EDEVICE;
  for (int j0 = 0; j0 < H; j0 += rows_per) {
    const int rows = std::min(rows_per, H - j0);
    hipError_t e = hipMemcpyAsync(t.stage, d->range_table + static_cast<size_t>(j0) * row_elems,
                                  rows * row_elems * sizeof(float), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return MCL_EDEVICE;
    const int n = rows * pitch;
    if (t.f32)
      hipLaunchKernelGGL(quantize_kernel<float>, dim3((n + 255) / 256), dim3(256), 0, s, t.stage,
                         static_cast<float*>(t.rq), t.sr, W, pitch, j0, rows, d->n_dirs, t.kpad, h,
                         (static_cast<int64_t>(H) * pitch + 31) / 32);
    else
      hipLaunchKernelGGL(quantize_kernel<__bf16>, dim3((n + 255) / 256), dim3(256), 0, s, t.stage,
                         static_cast<__bf16*>(t.rq), t.sr, W, pitch, j0, rows, d->n_dirs, t.kpad, h,
                         (static_cast<int64_t>(H) * pitch + 31) / 32);
    if (hipGetLastError() != hipSuccess) return MCL_EDEVICE;
    // the staging buffer is reused by the next chunk
    if (hipStreamSynchronize(s) != hipSuccess) return MCL_EDEVICE;
  }
  return MCL_OK;
}

}  // namespace mcl

namespace mcl {

namespace {

// Quantise the scan, compute the beam offsets s_k of every channel and build
// the circulant operand C; returns the sum of squared scan counts in *sz.
hipError_t build_ct(const ScanLaunch& L, const float* ranges_m, CtArgs& ca, int64_t* sz_out) {
  const ScanTable& t = *L.table;
  const int N = t.n_dirs;
  const double h = t.max_range / 256.0;
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
  *sz_out = sz;
  return hipGetLastError();
}

}  // namespace

namespace {

// Arguments of both passes for one filter, after its circulant operand.
ScanArgs scan_args_for(const ScanLaunch& L, const CtArgs& ca, int64_t sz, double sigma_m, int32_t* dout) {
  const ScanTable& t = *L.table;
  const double h = t.max_range / 256.0;
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
  a.rq_bytes = static_cast<uint32_t>(t.rq_bytes);
  return a;
}

}  // namespace

hipError_t scan_launch(const ScanLaunch& L, const float* ranges_m, double sigma_m, int32_t* dout) {
  const ScanTable& t = *L.table;
  const double h = t.max_range / 256.0;
  CtArgs ca;
  int64_t sz = 0;
  hipError_t e = build_ct(L, ranges_m, ca, &sz);
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
  a.rq_bytes = static_cast<uint32_t>(t.rq_bytes);
  const dim3 g1(a.tiles), b1(kScanThreads);
  // channel blocks per pass: all of them when they fit (no recomputation)
  const int nch = std::min(kMaxNChunk, ca.npad / 32);
  // BF16 operands, depth 384, at most three blocks in one pass: the operand
  // (at most 72 KB) is staged in LDS, two workgroups per compute unit, each
  // staging it once for all its tiles
  const bool stage_b = !dout && !t.f32 && t.kpad == 384 && ca.npad / 32 <= 3;
  if (stage_b) {
    const dim3 gp(std::min(a.tiles, kScanPersistBlocks));
    switch (L.dtype * 8 + nch) {
#define MCL_GEMM_BL(DT, T_)                                                                                   \
  case DT * 8 + 1: hipLaunchKernelGGL((scan_gemm_persist_kernel<__bf16, T_, 1>), gp, b1, 0, L.stream, a, a.tiles); break; \
  case DT * 8 + 2: hipLaunchKernelGGL((scan_gemm_persist_kernel<__bf16, T_, 2>), gp, b1, 0, L.stream, a, a.tiles); break; \
  case DT * 8 + 3: hipLaunchKernelGGL((scan_gemm_persist_kernel<__bf16, T_, 3>), gp, b1, 0, L.stream, a, a.tiles); break;
      MCL_GEMM_BL(0, float)
      MCL_GEMM_BL(1, __bf16)
      MCL_GEMM_BL(2, _Float16)
#undef MCL_GEMM_BL
      default: return hipErrorInvalidValue;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // depth 384 (321..384 directions, e.g. 360) has a fully unrolled depth loop
#define MCL_GEMM_K(OP, T, MODE, KP)                                                                    \
  switch (nch) {                                                                                       \
    case 1: hipLaunchKernelGGL((scan_gemm_kernel<OP, T, MODE, 1, KP>), g1, b1, 0, L.stream, a); break;  \
    case 2: hipLaunchKernelGGL((scan_gemm_kernel<OP, T, MODE, 2, KP>), g1, b1, 0, L.stream, a); break;  \
    case 3: hipLaunchKernelGGL((scan_gemm_kernel<OP, T, MODE, 3, KP>), g1, b1, 0, L.stream, a); break;  \
    default: hipLaunchKernelGGL((scan_gemm_kernel<OP, T, MODE, 4, KP>), g1, b1, 0, L.stream, a); break; \
  }
#define MCL_GEMM(OP, T, MODE)                                \
  do {                                                       \
    if (MODE == 0 && t.kpad == 384) {                        \
      MCL_GEMM_K(OP, T, MODE, (MODE == 0 ? 384 : 0))         \
    } else {                                                 \
      MCL_GEMM_K(OP, T, MODE, 0)                             \
    }                                                        \
  } while (0)
  if (dout) {
    if (t.f32) MCL_GEMM(float, float, 1);
    else MCL_GEMM(__bf16, float, 1);
    return hipGetLastError();
  }
  if (!stage_b) switch (L.dtype * 2 + (t.f32 ? 1 : 0)) {
    case 0: MCL_GEMM(__bf16, float, 0); break;
    case 1: MCL_GEMM(float, float, 0); break;
    case 2: MCL_GEMM(__bf16, __bf16, 0); break;
    case 3: MCL_GEMM(float, __bf16, 0); break;
    case 4: MCL_GEMM(__bf16, _Float16, 0); break;
    case 5: MCL_GEMM(float, _Float16, 0); break;
    default: return hipErrorInvalidValue;
  }
#undef MCL_GEMM
#undef MCL_GEMM_K
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // pass 2: at most kScanApplyBlocks workgroups (two partials each)
  const dim3 g2(std::max(1, std::min(64, kScanApplyBlocks / L.n_theta)), L.n_theta);
  switch (L.dtype) {
    case 0: hipLaunchKernelGGL(scan_apply_kernel<float>, g2, dim3(kScanThreads), 0, L.stream, a); break;
    case 1: hipLaunchKernelGGL(scan_apply_kernel<__bf16>, g2, dim3(kScanThreads), 0, L.stream, a); break;
    case 2: hipLaunchKernelGGL(scan_apply_kernel<_Float16>, g2, dim3(kScanThreads), 0, L.stream, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t scan_launch_batch(const ScanLaunch* Ls, int n, const float* ranges_m, const double* sigma_m) {
  if (n < 1) return hipSuccess;
  const ScanTable& t = *Ls[0].table;
  const hipStream_t stream = Ls[0].stream;
  // circulant operands, then the filters grouped by storage type and heading
  // count (the kernels' template arguments and the pass-2 grid, which sets the
  // reduction order: each filter reduces as it would alone), kScanBatchMax per
  // launch
  std::vector<std::pair<int64_t, int>> order;  // (group key, filter)
  std::vector<ScanArgs> args(n);
  for (int i = 0; i < n; ++i) {
    CtArgs ca;
    int64_t sz = 0;
    const hipError_t e = build_ct(Ls[i], ranges_m + static_cast<int64_t>(i) * t.n_dirs, ca, &sz);
    if (e != hipSuccess) return e;
    args[i] = scan_args_for(Ls[i], ca, sz, sigma_m[i], nullptr);
    order.push_back({static_cast<int64_t>(Ls[i].dtype) * 4096 + Ls[i].n_theta, i});
  }
  std::stable_sort(order.begin(), order.end(),
                   [](const std::pair<int64_t, int>& x, const std::pair<int64_t, int>& y) { return x.first < y.first; });
  for (size_t g0 = 0; g0 < order.size();) {
    size_t g1 = g0;
    while (g1 < order.size() && order[g1].first == order[g0].first && g1 - g0 < kScanBatchMax) ++g1;
    ScanJobs jobs = {};
    jobs.n = static_cast<int32_t>(g1 - g0);
    int max_theta = 0;
    for (size_t q = g0; q < g1; ++q) {
      jobs.a[q - g0] = args[order[q].second];
      max_theta = std::max(max_theta, jobs.a[q - g0].n_theta);
    }
    const int dtype = Ls[order[g0].second].dtype;
    const ScanArgs& a0 = jobs.a[0];
    const dim3 g1d(a0.tiles), b1(kScanThreads);
    const int nch = std::min(kMaxNChunk, a0.npad / 32);
    const bool stage_b = !t.f32 && t.kpad == 384 && a0.npad / 32 <= 3;
    if (stage_b) {
      switch (dtype * 8 + nch) {
#define MCL_GEMMB_BL(DT, T_)                                                                                               \
  case DT * 8 + 1: hipLaunchKernelGGL((scan_gemm_batch_kernel<__bf16, T_, 1, 384, true>), g1d, b1, 0, stream, jobs); break; \
  case DT * 8 + 2: hipLaunchKernelGGL((scan_gemm_batch_kernel<__bf16, T_, 2, 384, true>), g1d, b1, 0, stream, jobs); break; \
  case DT * 8 + 3: hipLaunchKernelGGL((scan_gemm_batch_kernel<__bf16, T_, 3, 384, true>), g1d, b1, 0, stream, jobs); break;
        MCL_GEMMB_BL(0, float)
        MCL_GEMMB_BL(1, __bf16)
        MCL_GEMMB_BL(2, _Float16)
#undef MCL_GEMMB_BL
        default: return hipErrorInvalidValue;
      }
    } else {
#define MCL_GEMMB_K(OP, T_, KP)                                                                                          \
  switch (nch) {                                                                                                        \
    case 1: hipLaunchKernelGGL((scan_gemm_batch_kernel<OP, T_, 1, KP, false>), g1d, b1, 0, stream, jobs); break;        \
    case 2: hipLaunchKernelGGL((scan_gemm_batch_kernel<OP, T_, 2, KP, false>), g1d, b1, 0, stream, jobs); break;        \
    case 3: hipLaunchKernelGGL((scan_gemm_batch_kernel<OP, T_, 3, KP, false>), g1d, b1, 0, stream, jobs); break;        \
    default: hipLaunchKernelGGL((scan_gemm_batch_kernel<OP, T_, 4, KP, false>), g1d, b1, 0, stream, jobs); break;       \
  }
#define MCL_GEMMB(OP, T_)          \
  do {                              \
    if (t.kpad == 384) {            \
      MCL_GEMMB_K(OP, T_, 384)      \
    } else {                        \
      MCL_GEMMB_K(OP, T_, 0)        \
    }                               \
  } while (0)
      switch (dtype * 2 + (t.f32 ? 1 : 0)) {
        case 0: MCL_GEMMB(__bf16, float); break;
        case 1: MCL_GEMMB(float, float); break;
        case 2: MCL_GEMMB(__bf16, __bf16); break;
        case 3: MCL_GEMMB(float, __bf16); break;
        case 4: MCL_GEMMB(__bf16, _Float16); break;
        case 5: MCL_GEMMB(float, _Float16); break;
        default: return hipErrorInvalidValue;
      }
#undef MCL_GEMMB
#undef MCL_GEMMB_K
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // pass 2: the per-filter grid of scan_launch, the filter in z
    const dim3 g2(std::max(1, std::min(64, kScanApplyBlocks / max_theta)), max_theta, jobs.n);
    switch (dtype) {
      case 0: hipLaunchKernelGGL(scan_apply_batch_kernel<float>, g2, dim3(kScanThreads), 0, stream, jobs); break;
      case 1: hipLaunchKernelGGL(scan_apply_batch_kernel<__bf16>, g2, dim3(kScanThreads), 0, stream, jobs); break;
      case 2: hipLaunchKernelGGL(scan_apply_batch_kernel<_Float16>, g2, dim3(kScanThreads), 0, stream, jobs); break;
      default: return hipErrorInvalidValue;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    g0 = g1;
  }
  return hipSuccess;
}

hipError_t scan_sampled_launch(const ScanLaunch& L, const float* ranges_m, double sigma_m, const uint8_t* mask,
                               int32_t* list, int32_t* pos) {
  const ScanTable& t = *L.table;
  const double h = t.max_range / 256.0;
  CtArgs ca;
  int64_t sz = 0;
  hipError_t e = build_ct(L, ranges_m, ca, &sz);
  if (e != hipSuccess) return e;
  SampledArgs a = {};
  a.rq = t.rq;
  a.sr = t.sr;
  a.ct = L.work.c;
  a.buf[0] = L.buf[0];
  a.buf[1] = L.buf[1];
  a.mask = mask;
  a.list = list;
  a.pos = pos;
  a.dsc = reinterpret_cast<int32_t*>(L.scratch);
  a.partials = L.partials;
  a.dev = L.dev;
  a.cells = L.H * L.pitch;
  a.n_theta = L.n_theta;
  a.npad = ca.npad;
  a.kpad = t.kpad;
  a.W = L.W;
  a.H = L.H;
  a.pitch = L.pitch;
  a.sstride = L.sstride;
  a.sz = static_cast<int32_t>(sz);
  a.c64 = h * h / (2.0 * sigma_m * sigma_m);
  a.c = static_cast<float>(a.c64);
  a.rq_bytes = static_cast<uint32_t>(t.rq_bytes);
  // compaction: at most kCompactMaxBlocks workgroups, at least four rounds of 64 cells per wave
  const int64_t waves_needed = (static_cast<int64_t>(a.cells) + 255) / 256;
  const int64_t g0 = std::min<int64_t>(kCompactMaxBlocks, (waves_needed + 3) / 4);
  const int per_wave = static_cast<int>((a.cells + g0 * 4 * 64 - 1) / (g0 * 4 * 64));
  hipLaunchKernelGGL(compact_kernel, dim3(static_cast<int>(g0)), dim3(kCompactThreads), 0, L.stream, a, per_wave);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  a.p1_blocks = std::min(256, std::max(1, (a.cells + 127) / 128));
  const dim3 g1(a.p1_blocks), b1(kScanThreads);
  if (t.f32) {
    if (t.kpad == 384) hipLaunchKernelGGL((sampled_gemm_kernel<float, 384>), g1, b1, 0, L.stream, a);
    else hipLaunchKernelGGL((sampled_gemm_kernel<float, 0>), g1, b1, 0, L.stream, a);
  } else {
    if (t.kpad == 384) hipLaunchKernelGGL((sampled_gemm_kernel<__bf16, 384>), g1, b1, 0, L.stream, a);
    else hipLaunchKernelGGL((sampled_gemm_kernel<__bf16, 0>), g1, b1, 0, L.stream, a);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // pass 2: scale the sampled states, then the sum/max stream
  if (static_cast<int64_t>(a.cells) * L.n_theta >= (static_cast<int64_t>(1) << 31)) return hipErrorInvalidValue;
  const int g2a = std::max(1, std::min(1024, (a.cells / 8 * L.n_theta + kScanThreads - 1) / kScanThreads));
  const int64_t runs = L.sstride / 4 * L.n_theta;
  const int g2b = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(2048, (runs + 4 * kScanThreads - 1) / (4 * kScanThreads))));
  switch (L.dtype) {
    case 0:
      hipLaunchKernelGGL(sampled_scale_kernel<float>, dim3(g2a), dim3(kScanThreads), 0, L.stream, a);
      hipLaunchKernelGGL(sampled_apply_kernel<float>, dim3(g2b), dim3(kScanThreads), 0, L.stream, a);
      break;
    case 1:
      hipLaunchKernelGGL(sampled_scale_kernel<__bf16>, dim3(g2a), dim3(kScanThreads), 0, L.stream, a);
      hipLaunchKernelGGL(sampled_apply_kernel<__bf16>, dim3(g2b), dim3(kScanThreads), 0, L.stream, a);
      break;
    case 2:
      hipLaunchKernelGGL(sampled_scale_kernel<_Float16>, dim3(g2a), dim3(kScanThreads), 0, L.stream, a);
      hipLaunchKernelGGL(sampled_apply_kernel<_Float16>, dim3(g2b), dim3(kScanThreads), 0, L.stream, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t match_workspace_bytes(const ScanTable& t, int cells, int n_theta, int batch) {
  if (t.n_dirs == 0 || batch < 1) return 0;
  const int64_t tiles = (static_cast<int64_t>(cells) + kTileCells - 1) / kTileCells;
  const int64_t ncols_pad = round_up_i(batch * n_theta, 64);  // an even number of 32-column blocks
  const int64_t ct_bytes = ncols_pad * t.kpad * (t.f32 ? 4 : 2);
  if (ct_bytes >= (int64_t{1} << 31)) return 0;  // the column operand is addressed with 31-bit offsets
  Carver c(nullptr);
  c.take(static_cast<size_t>(ct_bytes));
  c.take(static_cast<size_t>(batch) * t.n_dirs * sizeof(int16_t));
  c.take(static_cast<size_t>(batch) * sizeof(int32_t));
  c.take(static_cast<size_t>(batch) * sizeof(uint64_t));
  c.take(static_cast<size_t>(tiles * ncols_pad) * sizeof(uint32_t));
  return c.off;
}

hipError_t match_launch(const ScanTable& t, const uint8_t* free8, int W, int H, int pitch, int n_theta,
                        const int16_t* zq_host, const int32_t* sz_host, int nq, void* ws, uint64_t* best_host,
                        hipStream_t s) {
  const int cells = H * pitch;
  const int ncols = nq * n_theta, ncols_pad = round_up_i(ncols, 64);
  const int tiles = (cells + kTileCells - 1) / kTileCells;
  Carver c(ws);
  void* ct = c.take(static_cast<size_t>(ncols_pad) * t.kpad * (t.f32 ? 4 : 2));
  int16_t* zq = static_cast<int16_t*>(c.take(static_cast<size_t>(nq) * t.n_dirs * sizeof(int16_t)));
  int32_t* sz = static_cast<int32_t*>(c.take(static_cast<size_t>(nq) * sizeof(int32_t)));
  uint64_t* best = static_cast<uint64_t*>(c.take(static_cast<size_t>(nq) * sizeof(uint64_t)));
  uint32_t* keys = static_cast<uint32_t*>(c.take(static_cast<size_t>(tiles) * ncols_pad * sizeof(uint32_t)));
  hipError_t e = hipMemcpyAsync(zq, zq_host, static_cast<size_t>(nq) * t.n_dirs * sizeof(int16_t),
                                hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  if ((e = hipMemcpyAsync(sz, sz_host, static_cast<size_t>(nq) * sizeof(int32_t), hipMemcpyHostToDevice, s)) !=
      hipSuccess)
    return e;
  MatchCtArgs ca = {};
  ca.ct = ct;
  ca.zq = zq;
  ca.n_dirs = t.n_dirs;
  ca.n_theta = n_theta;
  ca.ncols = ncols;
  ca.ncols_pad = ncols_pad;
  ca.kpad = t.kpad;
  ca.f32 = t.f32 ? 1 : 0;
  ca.best = best;
  ca.nq = nq;
  const double step = 2.0 * M_PI / t.n_dirs, dth = 2.0 * M_PI / n_theta;
  for (int k = 0; k < n_theta; ++k) {
    long v = static_cast<long>(floor((0.0 + k * dth) / step + 0.5)) % t.n_dirs;
    if (v < 0) v += t.n_dirs;
    ca.s[k] = static_cast<int16_t>(v);
  }
  // one thread per 16-byte piece of the operand, and at least one per query (best[] reset)
  const int64_t nct = std::max<int64_t>(static_cast<int64_t>(ncols_pad) * t.kpad / (t.f32 ? 4 : 8), nq);
  hipLaunchKernelGGL(match_ct_kernel, dim3(static_cast<unsigned>((nct + 255) / 256)), dim3(256), 0, s, ca);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  MatchArgs a = {};
  a.rq = t.rq;
  a.sr = t.sr;
  a.free8 = free8;
  a.ct = ct;
  a.sz = sz;
  a.keys = keys;
  a.best = best;
  a.tiles = tiles;
  a.cells = cells;
  a.pitch = pitch;
  a.W = W;
  a.n_theta = n_theta;
  a.ncols = ncols;
  a.ncols_pad = ncols_pad;
  a.kpad = t.kpad;
  a.rq_bytes = static_cast<uint32_t>(t.rq_bytes);
  a.inv_theta = ((uint64_t{1} << 40) + static_cast<uint64_t>(n_theta) - 1) / static_cast<uint64_t>(n_theta);
  // the A operand is held in registers for the whole table depth (at most 384)
#define MCL_MATCH(KP)                                                                                   \
  case KP:                                                                                              \
    if (t.f32) hipLaunchKernelGGL((match_gemm_kernel<float, KP>), dim3(tiles), dim3(kScanThreads), 0, s, a); \
    else hipLaunchKernelGGL((match_gemm_kernel<__bf16, KP>), dim3(tiles), dim3(kScanThreads), 0, s, a);      \
    break;
  switch (t.kpad) {
    MCL_MATCH(64)
    MCL_MATCH(128)
    MCL_MATCH(192)
    MCL_MATCH(256)
    MCL_MATCH(320)
    MCL_MATCH(384)
    default: return hipErrorInvalidValue;
  }
#undef MCL_MATCH
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(match_reduce_kernel, dim3(nq, kReduceChunks), dim3(kScanThreads), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return hipMemcpyAsync(best_host, best, static_cast<size_t>(nq) * sizeof(uint64_t), hipMemcpyDeviceToHost, s);
}

int scan_tiles(int cells) { return (cells + kTileCells - 1) / kTileCells; }

}  // namespace mcl
