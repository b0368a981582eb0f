// Odometry step with anisotropic, heading-rotated motion noise.
//
// Eq. (Gaussian kernel) with the covariance R(psi) diag(sf^2, sl^2) R(psi)^T
// rotated to a channel's heading: forward noise sf along (cos psi, sin psi),
// lateral noise sl across it.  The kernel of output channel k is that 2-D
// Gaussian at psi_k = theta + k dTheta times the circular theta Gaussian, so
// the 3-D blur is the theta blur followed by one rotated 2-D blur per
// channel; the kernel activation G(B_0, k) of Alg. 1 depends on k too.
//
//   aniso_theta_kernel  warp (Sec. III-A-1, bilinear or whole-cell), pre-blur
//                       mask and circular theta blur -> FP32 scratch
//   aniso_xy_kernel     per channel: rotated 2-D blur of the scratch and of
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

// Grid (columns / kThThreads, H, n_theta): one output (k, j, i) per thread.
// The shifts of the 2 rth + 1 source channels are computed once per workgroup.
template <typename T>
__global__ __launch_bounds__(kThThreads) void aniso_theta_kernel(AnisoArgs a) {
  __shared__ int snx[kMaxTaps], sny[kMaxTaps];
  __shared__ float sfx[kMaxTaps], sfy[kMaxTaps];
  const int t = threadIdx.x;
  const int i = blockIdx.x * kThThreads + t;
  const int j = blockIdx.y, k = blockIdx.z;
  const int nl = 2 * a.rth + 1;
  if (t < nl) {
    int ks = (k - (t - a.rth)) % a.n_theta;
    if (ks < 0) ks += a.n_theta;
    channel_shift(a, ks, snx[t], sny[t], sfx[t], sfy[t]);
  }
  __syncthreads();
  if (i >= a.pitch) return;
  const FilterDev* dev = a.dev;
  const T* __restrict__ bin = static_cast<const T*>(a.buf[dev->cur]);
  const float scale = dev->scale;
  float acc = 0.f;
  if (i < a.W) {
    for (int l = 0; l < nl; ++l) {
      int ks = (k - (l - a.rth)) % a.n_theta;
      if (ks < 0) ks += a.n_theta;
      const int nx = snx[l], ny = sny[l];
      const float fx = sfx[l], fy = sfy[l];
      const T* plane = bin + static_cast<int64_t>(ks) * a.sstride;
      float s = 0.f;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int jj = j - ny - b;
        const float wy = b ? fy : 1.f - fy;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const int ii = i - nx - c;
          const float wx = c ? fx : 1.f - fx;
          if (jj >= 0 && jj < a.H && ii >= 0 && ii < a.W)
            s += (wx * wy) * ld<T>(plane + static_cast<int64_t>(jj) * a.pitch + ii);
        }
      }
      acc += a.gth[l] * (s * scale);
    }
    acc *= a.mpre[static_cast<int64_t>(j) * a.pitch + i];
  }
  a.tmp[static_cast<int64_t>(k) * a.sstride + static_cast<int64_t>(j) * a.pitch + i] = acc;
}

constexpr int kXyTx = 64, kXyTy = 16, kXyThreads = 256;

template <typename T>
__device__ inline T store_t(float v) {
  return static_cast<T>(v);
}

// Grid (tiles_x, tiles_y, n_theta): one 64 x 16 output tile of one channel.
template <typename T>
__global__ __launch_bounds__(kXyThreads) void aniso_xy_kernel(AnisoArgs a) {
  constexpr int MAXD = 2 * kAnisoMaxRadius + 1;
  constexpr int LW = kXyTx + 2 * kAnisoMaxRadius, LH = kXyTy + 2 * kAnisoMaxRadius;
  __shared__ float ts[LH * LW];
  __shared__ float ms[LH * LW];
  __shared__ float taps[MAXD * MAXD];
  __shared__ double tsum[kXyThreads];
  __shared__ double red_s[kXyThreads];
  __shared__ float red_m[kXyThreads];
  __shared__ int last_flag;
  const int t = threadIdx.x;
  const int r = a.rxy, d = 2 * r + 1;
  const int lw = kXyTx + 2 * r, lh = kXyTy + 2 * r;
  const int k = blockIdx.z;
  const int x0 = blockIdx.x * kXyTx, y0 = blockIdx.y * kXyTy;
  FilterDev* dev = a.dev;
  const int cur = dev->cur;
  const float scale = dev->scale;
  T* __restrict__ bout = static_cast<T*>(a.buf[cur ^ 1]);

  // taps of this channel's rotated Gaussian, FP64, normalised to sum 1
  double cs, sn;
  sincos(a.noise_theta + k * a.dtheta, &sn, &cs);
  double w = 0.0;
  for (int e = t; e < d * d; e += kXyThreads) {
    const int n = e / d - r, m = e % d - r;
    const double al = cs * m + sn * n, ac = -sn * m + cs * n;
    const double q = al * al / (a.sf * a.sf) + ac * ac / (a.sl * a.sl);
    w += exp(-0.5 * q);
  }
  tsum[t] = w;
  // scratch and free-mask tiles with a halo of r cells (zero outside the grid)
  const float* __restrict__ src = a.tmp + static_cast<int64_t>(k) * a.sstride;
  for (int e = t; e < lw * lh; e += kXyThreads) {
    const int ly = e / lw, lx = e % lw;
    const int gy = y0 + ly - r, gx = x0 + lx - r;
    const bool in = gy >= 0 && gy < a.H && gx >= 0 && gx < a.W;
    const int64_t o = static_cast<int64_t>(gy) * a.pitch + gx;
    ts[ly * LW + lx] = in ? src[o] : 0.f;
    ms[ly * LW + lx] = in ? static_cast<float>(a.free8[o]) : 0.f;
  }
  __syncthreads();
  for (int st = kXyThreads / 2; st > 0; st >>= 1) {
    if (t < st) tsum[t] += tsum[t + st];
    __syncthreads();
  }
  const double z = tsum[0];
  for (int e = t; e < d * d; e += kXyThreads) {
    const int n = e / d - r, m = e % d - r;
    const double al = cs * m + sn * n, ac = -sn * m + cs * n;
    const double q = al * al / (a.sf * a.sf) + ac * ac / (a.sl * a.sl);
    taps[e] = static_cast<float>(exp(-0.5 * q) / z);
  }
  __syncthreads();

  // four outputs per thread: out(i, j) = sum_{m, n} g[n][m] s(i - m, j - n)
  double s = 0.0;
  float mx = 0.f;
  for (int o = t; o < kXyTx * kXyTy; o += kXyThreads) {
    const int oy = o / kXyTx, ox = o % kXyTx;
    const int gy = y0 + oy, gx = x0 + ox;
    if (gy >= a.H || gx >= a.W) continue;
    float tv = 0.f, av = 0.f;
    for (int n = -r; n <= r; ++n) {
      const float* trow = ts + (oy + r - n) * LW + (ox + r);
      const float* mrow = ms + (oy + r - n) * LW + (ox + r);
      const float* g = taps + (n + r) * d + r;
      for (int m = -r; m <= r; ++m) {
        tv += g[m] * trow[-m];
        av += g[m] * mrow[-m];
      }
    }
    const bool free = ms[(oy + r) * LW + ox + r] > 0.f;
    float u = 0.f;
    if (free) u = a.wall_normalize ? tv / (av * a.gth_sum) : tv;
    const T q = store_t<T>(u);
    bout[static_cast<int64_t>(k) * a.sstride + static_cast<int64_t>(gy) * a.pitch + gx] = q;
    const float uq = static_cast<float>(q);
    s += static_cast<double>(uq);
    mx = fmaxf(mx, uq);
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

}  // namespace

int aniso_workgroups(int W, int H, int n_theta) {
  return ((W + kXyTx - 1) / kXyTx) * ((H + kXyTy - 1) / kXyTy) * n_theta;
}

hipError_t launch_aniso_step(int dtype, const AnisoArgs& a, hipStream_t s) {
  if (a.rxy < 0 || a.rxy > kAnisoMaxRadius || a.rth < 0 || a.rth > kMaxRadius) return hipErrorInvalidValue;
  const dim3 g1((a.pitch + kThThreads - 1) / kThThreads, a.H, a.n_theta);
  const dim3 g2((a.W + kXyTx - 1) / kXyTx, (a.H + kXyTy - 1) / kXyTy, a.n_theta);
  switch (dtype) {
    case 0:
      hipLaunchKernelGGL(aniso_theta_kernel<float>, g1, dim3(kThThreads), 0, s, a);
      hipLaunchKernelGGL(aniso_xy_kernel<float>, g2, dim3(kXyThreads), 0, s, a);
      break;
    case 1:
      hipLaunchKernelGGL(aniso_theta_kernel<__bf16>, g1, dim3(kThThreads), 0, s, a);
      hipLaunchKernelGGL(aniso_xy_kernel<__bf16>, g2, dim3(kXyThreads), 0, s, a);
      break;
    case 2:
      hipLaunchKernelGGL(aniso_theta_kernel<_Float16>, g1, dim3(kThThreads), 0, s, a);
      hipLaunchKernelGGL(aniso_xy_kernel<_Float16>, g2, dim3(kXyThreads), 0, s, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mcl
