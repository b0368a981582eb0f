// Odometry step with anisotropic, heading-rotated motion noise.
//
// Eq. (Gaussian kernel) with the covariance R(psi) diag(sf^2, sl^2) R(psi)^T
// rotated to a channel's heading: forward noise sf along (cos psi, sin psi),
// lateral noise sl across it.  The kernel of output channel k is that 2-D
// Gaussian at psi_k = theta + k dTheta times the circular theta Gaussian, so
// the 3-D blur is the theta blur followed by one rotated 2-D blur per
// channel; the kernel activation G(B_0, k) of Alg. 1 depends on k too.
//
//   aniso_taps_kernel   each channel's rotated 2-D taps (FP64, normalised)
//   aniso_theta_kernel  warp (Sec. III-A-1, bilinear or whole-cell), pre-blur
//                       mask and circular theta blur -> FP32 scratch
//   aniso_xy_kernel     per channel (eight to a workgroup): rotated 2-D blur of the scratch and of
//                       the free mask (the activation), post-blur mask and
//                       M / G(B_0, k), store, sum/max; the last workgroup
//                       renormalises as the fused step does
//
// The rotated kernel is not separable, so this path trades the fused step's
// register pipeline for two plain passes with LDS tiles.
#include <float.h>
#include <math.h>

#include "mcl_internal.hpp"

namespace mcl {
namespace {

template <typename T>
__device__ inline float ld(const T* p) {
  return static_cast<float>(*p);
}
template <>
__device__ inline float ld<__bf16>(const __bf16* p) {
  return __uint_as_float(static_cast<uint32_t>(__builtin_bit_cast(uint16_t, *p)) << 16);
}

constexpr int kThThreads = 256;

// Per-channel displacement in cells, split into integer and fractional parts,
// exactly as the fused step does (FP64), or the host's whole-cell shifts.
__device__ inline void channel_shift(const AnisoArgs& a, int k, int& nx, int& ny, float& fx, float& fy) {
  if (a.ishift) {
    nx = a.ishift[2 * k];
    ny = a.ishift[2 * k + 1];
    fx = fy = 0.f;
    return;
  }
  double sn, cs;
  sincos(a.theta_prev + k * a.dtheta, &sn, &cs);
  const double dx = a.u_cells * cs - a.v_cells * sn;
  const double dy = a.u_cells * sn + a.v_cells * cs;
  const double fdx = floor(dx), fdy = floor(dy);
  nx = static_cast<int>(fdx);
  ny = static_cast<int>(fdy);
  fx = static_cast<float>(dx - fdx);
  fy = static_cast<float>(dy - fdy);
}

// Taps of every channel's rotated Gaussian, FP64, normalised to sum 1, stored
// FP32 as taps[k][(n + r) d + m + r].  Grid n_theta, one workgroup per channel.
__global__ __launch_bounds__(kThThreads) void aniso_taps_kernel(AnisoArgs a) {
  __shared__ double tsum[kThThreads];
  const int t = threadIdx.x, k = blockIdx.x;
  const int r = a.rxy, d = 2 * r + 1;
  double cs, sn;
  sincos(a.noise_theta + k * a.dtheta, &sn, &cs);
  double w[1 + (2 * kAnisoMaxRadius + 1) * (2 * kAnisoMaxRadius + 1) / kThThreads];
  double part = 0.0;
  int u = 0;
  for (int e = t; e < d * d; e += kThThreads, ++u) {
    const int n = e / d - r, m = e % d - r;
    const double al = cs * m + sn * n, ac = -sn * m + cs * n;
    const double q = al * al / (a.sf * a.sf) + ac * ac / (a.sl * a.sl);
    w[u] = exp(-0.5 * q);
    part += w[u];
  }
  tsum[t] = part;
  __syncthreads();
  for (int st = kThThreads / 2; st > 0; st >>= 1) {
    if (t < st) tsum[t] += tsum[t + st];
    __syncthreads();
  }
  const double z = tsum[0];
  u = 0;
  for (int e = t; e < d * d; e += kThThreads, ++u) a.taps[k * d * d + e] = static_cast<float>(w[u] / z);
}

// Raw-buffer reads of one stored value (zero outside the descriptor).
template <typename T>
__device__ inline float ld_buf(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ inline float ld_buf<float>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ inline float ld_buf<__bf16>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __uint_as_float(static_cast<uint32_t>(__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0)) << 16);
}
template <>
__device__ inline float ld_buf<_Float16>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return static_cast<float>(__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0)));
}
// Offsets into one heading plane below 1 GiB: a row part below 2^30, or 2^30
// for a row outside the grid, plus a column part below 2^30, or 2^31 for a
// column outside; the sum is out of the plane's range exactly when either is.
constexpr uint32_t kThRowOut = 1u << 30;
constexpr uint32_t kThColOut = 1u << 31;

// Warp, pre-blur mask and circular theta blur into the FP32 scratch.  Grid
// (pitch / kThThreads, H): one cell per thread, streaming through the
// channels.  Each channel's warped value is computed once and kept in a
// shift register of the last 2 RTH + 1 channels; output channel k is emitted
// when channel k + RTH has arrived.  The next channel's four source values
// are loaded before the current one is combined.  BUF (planes below 1 GiB):
// the source values come through a buffer descriptor per plane, the two row
// offsets in scalar registers (the row is the workgroup's), so only the two
// column tests run per lane.
template <typename T, int RTH, bool BUF>
__global__ __launch_bounds__(kThThreads) void aniso_theta_kernel(AnisoArgs a) {
  constexpr int NTAP = 2 * RTH + 1;
  constexpr int EB = static_cast<int>(sizeof(T));
  __shared__ int snx[kMaxTheta], sny[kMaxTheta];
  __shared__ float sfx[kMaxTheta], sfy[kMaxTheta];
  const int t = threadIdx.x;
  const int i = blockIdx.x * kThThreads + t;
  const int j = blockIdx.y;
  const int n = a.n_theta, rth = RTH;
  for (int k = t; k < n; k += kThThreads) channel_shift(a, k, snx[k], sny[k], sfx[k], sfy[k]);
  __syncthreads();
  if (i >= a.pitch) return;
  const FilterDev* dev = a.dev;
  const T* __restrict__ bin = static_cast<const T*>(a.buf[dev->cur]);
  const float scale = dev->scale;
  const bool inside = i < a.W;
  const float mp = inside ? a.mpre[static_cast<int64_t>(j) * a.pitch + i] * scale : 0.f;
  float* __restrict__ out = a.tmp + static_cast<int64_t>(j) * a.pitch + i;
  // the four source values of channel c (zero outside the grid) and their weights
  const uint32_t row_bytes = static_cast<uint32_t>(a.pitch) * EB;
  const uint32_t plane_bytes = static_cast<uint32_t>(a.sstride) * EB;  // below 2^30 when BUF
  auto fetch = [&](int c, float v[4]) {
    const int nx = __builtin_amdgcn_readfirstlane(snx[c]), ny = __builtin_amdgcn_readfirstlane(sny[c]);
    const T* plane = bin + static_cast<int64_t>(c) * a.sstride;
    if constexpr (BUF) {
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<T*>(plane), static_cast<short>(0), static_cast<int>(plane_bytes), 0x00020000);
      uint32_t coff[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int ii = i - nx - q;
        coff[q] = static_cast<unsigned>(ii) < static_cast<unsigned>(a.W) ? static_cast<uint32_t>(ii) * EB : kThColOut;
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int jj = j - ny - b;
        const uint32_t roff = static_cast<unsigned>(jj) < static_cast<unsigned>(a.H) ? static_cast<uint32_t>(jj) * row_bytes
                                                                                     : kThRowOut;
#pragma unroll
        for (int q = 0; q < 2; ++q) v[2 * b + q] = ld_buf<T>(rs, coff[q], roff);
      }
      return;
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int jj = j - ny - b;
      const bool oky = jj >= 0 && jj < a.H;
      const int jc = min(max(jj, 0), a.H - 1);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int ii = i - nx - q;
        const bool ok = oky && ii >= 0 && ii < a.W;
        const int ic = min(max(ii, 0), a.W - 1);
        const float x = ld<T>(plane + static_cast<int64_t>(jc) * a.pitch + ic);
        v[2 * b + q] = ok ? x : 0.f;
      }
    }
  };
  float ring[NTAP];
#pragma unroll
  for (int l = 0; l < NTAP; ++l) ring[l] = 0.f;
  const int total = n + 2 * rth;  // channels -rth .. n - 1 + rth
  int c = (n - rth % n) % n;
  float v[4];
  fetch(c, v);
  for (int e = 0; e < total; ++e) {
    const float fx = sfx[c], fy = sfy[c];
    const int cn = c + 1 == n ? 0 : c + 1;
    float vn[4];
    fetch(cn, vn);  // past the last channel this reads a valid plane and is discarded
    const float s = ((1.f - fx) * v[0] + fx * v[1]) * (1.f - fy) + ((1.f - fx) * v[2] + fx * v[3]) * fy;
#pragma unroll
    for (int l = NTAP - 1; l > 0; --l) ring[l] = ring[l - 1];
    ring[0] = inside ? s * mp : 0.f;
    if (e >= 2 * rth) {
      // ring[l] holds channel (k + rth - l): output k = e - 2 rth
      float acc = 0.f;
#pragma unroll
      for (int l = 0; l < NTAP; ++l) acc += a.gth[l] * ring[l];
      out[static_cast<int64_t>(e - 2 * rth) * a.sstride] = acc;
    }
    c = cn;
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = vn[q];
  }
}

constexpr int kXyTx = 64, kXyTy = 16, kXyThreads = 256;
constexpr int kXyRows = kXyTy / (kXyThreads / kXyTx);  // outputs per thread, down a column
constexpr int kXyChannels = 8;                          // channels per workgroup

template <typename T>
__device__ inline T store_t(float v) {
  return static_cast<T>(v);
}

// Grid (tiles_x, tiles_y, channel groups): one 64 x 16 output tile for up to
// kXyChannels consecutive channels.  The free-mask tile is loaded once; the
// scratch tile of the next channel is loaded into registers while the current
// one is blurred from LDS (double buffered, one barrier per channel).  Each
// thread computes a column of four outputs, so a row it reads from LDS serves
// up to four of them.  One sum/max reduction per workgroup.
template <typename T, int R>
__global__ __launch_bounds__(kXyThreads) void aniso_xy_kernel(AnisoArgs a) {
  constexpr int D = 2 * R + 1;
  constexpr int LW = kXyTx + 2 * R, LH = kXyTy + 2 * R, NL = LW * LH;
  constexpr int PER = (NL + kXyThreads - 1) / kXyThreads;
  __shared__ float ts[2][NL];
  __shared__ float ms[NL];
  __shared__ float gs[2][D * D];
  __shared__ double red_s[kXyThreads];
  __shared__ float red_m[kXyThreads];
  __shared__ int last_flag;
  const int t = threadIdx.x;
  const int k0 = blockIdx.z * kXyChannels;
  const int k1 = min(a.n_theta, k0 + kXyChannels);
  const int x0 = blockIdx.x * kXyTx, y0 = blockIdx.y * kXyTy;
  FilterDev* dev = a.dev;
  const int cur = dev->cur;
  const float scale = dev->scale;
  T* __restrict__ bout = static_cast<T*>(a.buf[cur ^ 1]);

  // this thread's share of the halo tile: grid offsets (or -1 outside the grid)
  int64_t off[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = t + u * kXyThreads;
    const int ly = e / LW, lx = e - ly * LW;
    const int gy = y0 + ly - R, gx = x0 + lx - R;
    const bool in = e < NL && gy >= 0 && gy < a.H && gx >= 0 && gx < a.W;
    off[u] = in ? static_cast<int64_t>(gy) * a.pitch + gx : -1;
  }
  // loads from a clamped (valid) address, then a select: no branches around them
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const float v = static_cast<float>(a.free8[off[u] >= 0 ? off[u] : 0]);
    if (t + u * kXyThreads < NL) ms[t + u * kXyThreads] = off[u] >= 0 ? v : 0.f;
  }
  // the next channel's scratch tile and taps, held in registers until stored
  float pre[PER];
  float tap = 0.f;
  auto fetch = [&](int k) {
    const float* __restrict__ src = a.tmp + static_cast<int64_t>(k) * a.sstride;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const float v = src[off[u] >= 0 ? off[u] : 0];
      pre[u] = off[u] >= 0 ? v : 0.f;
    }
    tap = a.taps[k * D * D + (t < D * D ? t : 0)];
  };
  auto put = [&](int b) {
#pragma unroll
    for (int u = 0; u < PER; ++u)
      if (t + u * kXyThreads < NL) ts[b][t + u * kXyThreads] = pre[u];
    if (t < D * D) gs[b][t] = tap;
  };
  fetch(k0);
  put(0);

  const int ox = t % kXyTx, oy0 = (t / kXyTx) * kXyRows;
  double s = 0.0;
  float mx = 0.f;
  for (int k = k0; k < k1; ++k) {
    const int b = (k - k0) & 1;
    __syncthreads();
    if (k + 1 < k1) fetch(k + 1);
    // out(i, j) = sum_{m, n} g[n][m] s(i - m, j - n): LDS row ly holds j - n + R,
    // column lx holds i - m + R
    const float* g = gs[b];
    float tv[kXyRows], av[kXyRows];
#pragma unroll
    for (int q = 0; q < kXyRows; ++q) tv[q] = av[q] = 0.f;
    // one tap column at a time (not unrolled), so only 2R + 1 taps and one
    // column of LDS values are live
#pragma unroll 1
    for (int m = -R; m <= R; ++m) {
      float gc[D];
#pragma unroll
      for (int n = 0; n < D; ++n) gc[n] = g[n * D + m + R];
      const float* tcol = ts[b] + oy0 * LW + ox + R - m;
      const float* mcol = ms + oy0 * LW + ox + R - m;
#pragma unroll
      for (int dy = 0; dy < kXyRows + 2 * R; ++dy) {
        const float vt = tcol[dy * LW], vm = mcol[dy * LW];
#pragma unroll
        for (int q = 0; q < kXyRows; ++q) {
          const int nn = q + R - dy;  // row offset n of this input for output q
          if (nn >= -R && nn <= R) {
            tv[q] += gc[nn + R] * vt;
            av[q] += gc[nn + R] * vm;
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kXyRows; ++q) {
      const int gy = y0 + oy0 + q, gx = x0 + ox;
      if (gy < a.H && gx < a.W) {
        const bool free = ms[(oy0 + q + R) * LW + ox + R] > 0.f;
        float u = 0.f;
        if (free) u = a.wall_normalize ? tv[q] / (av[q] * a.gth_sum) : tv[q];
        const T qv = store_t<T>(u);
        bout[static_cast<int64_t>(k) * a.sstride + static_cast<int64_t>(gy) * a.pitch + gx] = qv;
        const float uq = static_cast<float>(qv);
        s += static_cast<double>(uq);
        mx = fmaxf(mx, uq);
      }
    }
    if (k + 1 < k1) put(b ^ 1);
  }
  red_s[t] = s;
  red_m[t] = mx;
  __syncthreads();
  for (int st = kXyThreads / 2; st > 0; st >>= 1) {
    if (t < st) {
      red_s[t] += red_s[t + st];
      red_m[t] = fmaxf(red_m[t], red_m[t + st]);
    }
    __syncthreads();
  }
  const int blk = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  const int nblk = gridDim.x * gridDim.y * gridDim.z;
  if (t == 0) {
    publish(&a.partials[2 * blk], red_s[0]);
    publish(&a.partials[2 * blk + 1], static_cast<double>(red_m[0]));
    last_flag = arrive_last(dev, static_cast<uint32_t>(blk), static_cast<uint32_t>(nblk));
  }
  __syncthreads();
  if (!last_flag) return;
  double ts2 = 0.0;
  float tm = 0.f;
  for (int b = t; b < nblk; b += kXyThreads) {
    ts2 += __hip_atomic_load(&a.partials[2 * b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    tm = fmaxf(tm, static_cast<float>(__hip_atomic_load(&a.partials[2 * b + 1], __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT)));
  }
  red_s[t] = ts2;
  red_m[t] = tm;
  __syncthreads();
  for (int st = kXyThreads / 2; st > 0; st >>= 1) {
    if (t < st) {
      red_s[t] += red_s[t + st];
      red_m[t] = fmaxf(red_m[t], red_m[t + st]);
    }
    __syncthreads();
  }
  if (t == 0) {
    const double tot = red_s[0];
    const float m = red_m[0];
    if (!(tot > 0.0) || !isfinite(tot) || !(m > 0.f)) {
      dev->status = kStatusDegenerate;  // keep the previous belief (cur unchanged)
    } else {
      dev->log_norm += log(tot) - log(static_cast<double>(scale)) - dev->lnsum;
      dev->lnsum = log(tot);
      dev->sum = tot;
      dev->maxval = m;
      const double sc = 1.0 / static_cast<double>(m);
      dev->scale = sc > static_cast<double>(FLT_MAX) ? FLT_MAX : static_cast<float>(sc);
      dev->cur = cur ^ 1;
    }
    __hip_atomic_store(&dev->counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <typename T>
hipError_t launch_typed(const AnisoArgs& a, hipStream_t s) {
  const dim3 g1((a.pitch + kThThreads - 1) / kThThreads, a.H);
  const dim3 g2((a.W + kXyTx - 1) / kXyTx, (a.H + kXyTy - 1) / kXyTy, (a.n_theta + kXyChannels - 1) / kXyChannels);
  hipLaunchKernelGGL(aniso_taps_kernel, dim3(a.n_theta), dim3(kThThreads), 0, s, a);
  const bool buf = static_cast<uint64_t>(a.sstride) * sizeof(T) < (static_cast<uint64_t>(1) << 30);
#define MCL_THETA(R_)                                                                         \
  case R_:                                                                                    \
    if (buf)                                                                                  \
      hipLaunchKernelGGL((aniso_theta_kernel<T, R_, true>), g1, dim3(kThThreads), 0, s, a);  \
    else                                                                                      \
      hipLaunchKernelGGL((aniso_theta_kernel<T, R_, false>), g1, dim3(kThThreads), 0, s, a); \
    break;
  static_assert(kMaxRadius == 4, "instantiate aniso_theta_kernel for every theta radius");
  switch (a.rth) {
    MCL_THETA(0)
    MCL_THETA(1)
    MCL_THETA(2)
    MCL_THETA(3)
    MCL_THETA(4)
    default: return hipErrorInvalidValue;
  }
#undef MCL_THETA
  switch (a.rxy) {
    case 0: hipLaunchKernelGGL((aniso_xy_kernel<T, 0>), g2, dim3(kXyThreads), 0, s, a); break;
    case 1: hipLaunchKernelGGL((aniso_xy_kernel<T, 1>), g2, dim3(kXyThreads), 0, s, a); break;
    case 2: hipLaunchKernelGGL((aniso_xy_kernel<T, 2>), g2, dim3(kXyThreads), 0, s, a); break;
    case 3: hipLaunchKernelGGL((aniso_xy_kernel<T, 3>), g2, dim3(kXyThreads), 0, s, a); break;
    case 4: hipLaunchKernelGGL((aniso_xy_kernel<T, 4>), g2, dim3(kXyThreads), 0, s, a); break;
    case 5: hipLaunchKernelGGL((aniso_xy_kernel<T, 5>), g2, dim3(kXyThreads), 0, s, a); break;
    case 6: hipLaunchKernelGGL((aniso_xy_kernel<T, 6>), g2, dim3(kXyThreads), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

int aniso_workgroups(int W, int H, int n_theta) {
  return ((W + kXyTx - 1) / kXyTx) * ((H + kXyTy - 1) / kXyTy) * ((n_theta + kXyChannels - 1) / kXyChannels);
}

hipError_t launch_aniso_step(int dtype, const AnisoArgs& a, hipStream_t s) {
  static_assert(kAnisoMaxRadius == 6, "instantiate aniso_xy_kernel for every radius");
  if (a.rxy < 0 || a.rxy > kAnisoMaxRadius || a.rth < 0 || a.rth > kMaxRadius || !a.taps) return hipErrorInvalidValue;
  switch (dtype) {
    case 0: return launch_typed<float>(a, s);
    case 1: return launch_typed<__bf16>(a, s);
    case 2: return launch_typed<_Float16>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mcl
