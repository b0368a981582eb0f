// Setup, readout and normalisation kernels around the fused step.
//
//   map_setup     traversability M, kernel activation G(B_0) and the post-blur
//                 weights M / G(B_0) of Alg. 1 (FP64 arithmetic, FP32 result)
//   init_uniform  B_0 = 1 on free cells of every channel (uniform up to scale)
//   slice_from_f32  upload path of an explicit initial belief
//   reduce        in-place rescale + sum/max, or argmax with lowest-index ties,
//                 finished by the last workgroup (deterministic order)
//   export        normalised FP32 copy (sums to one) and the belief map
//                 max_k B (Sec. III-A, last paragraph)
#include <float.h>
#include <math.h>

#include "mcl_internal.hpp"

namespace mcl {
namespace {

template <typename T>
__device__ inline float to_f32(T v) {
  return static_cast<float>(v);
}
template <>
__device__ inline float to_f32<__bf16>(__bf16 v) {
  return __uint_as_float(static_cast<uint32_t>(__builtin_bit_cast(uint16_t, v)) << 16);
}

__global__ void map_setup_kernel(const uint8_t* __restrict__ occ, int W, int H, int pitch, MapTaps taps,
                                 int rxy, double gth_sum, uint32_t flags, uint8_t* __restrict__ free8,
                                 float* __restrict__ mpre, float* __restrict__ wt) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= pitch || y >= H) return;
  const int64_t o = static_cast<int64_t>(y) * pitch + x;
  const bool inside = x < W;
  const bool fr = inside && occ[static_cast<int64_t>(y) * W + x] == 0;
  free8[o] = fr ? 1 : 0;
  mpre[o] = (flags & 1u) ? (fr ? 1.f : 0.f) : (inside ? 1.f : 0.f);
  float w = 0.f;
  if (fr) {
    if (flags & 2u) {
      double A = 0.0;
      for (int n = -rxy; n <= rxy; ++n) {
        const int yy = y - n;
        if (yy < 0 || yy >= H) continue;
        double row = 0.0;
        for (int m = -rxy; m <= rxy; ++m) {
          const int xx = x - m;
          if (xx < 0 || xx >= W) continue;
          if (occ[static_cast<int64_t>(yy) * W + xx] == 0) row += taps.g[m + rxy];
        }
        A += taps.g[n + rxy] * row;
      }
      A *= gth_sum;
      w = static_cast<float>(1.0 / A);
    } else {
      w = 1.f;
    }
  }
  wt[o] = w;
}

template <typename T>
__global__ void init_uniform_kernel(T* __restrict__ b0, T* __restrict__ b1, const uint8_t* __restrict__ free8,
                                    int64_t plane, int64_t n) {
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    b0[e] = static_cast<T>(free8[e % plane] ? 1.f : 0.f);
    b1[e] = static_cast<T>(0.f);
  }
}

template <typename T>
__global__ void slice_from_f32_kernel(const float* __restrict__ src, T* __restrict__ dst, int W, int H,
                                      int pitch, float factor) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= pitch || y >= H) return;
  const float v = x < W ? src[static_cast<int64_t>(y) * W + x] * factor : 0.f;
  dst[static_cast<int64_t>(y) * pitch + x] = static_cast<T>(v);
}

constexpr int kRedThreads = 256;

template <typename T>
__global__ __launch_bounds__(kRedThreads) void reduce_kernel(ReduceArgs a) {
  __shared__ double rs[kRedThreads];
  __shared__ float rm[kRedThreads];
  __shared__ int64_t ri[kRedThreads];
  __shared__ int last_flag;
  const int t = threadIdx.x;
  FilterDev* dev = a.dev;
  T* buf = static_cast<T*>(a.buf[dev->cur]);
  const int64_t n = a.sstride * a.n_theta;
  const int nblk = gridDim.x;
  double s = 0.0;
  float mx = 0.f;
  int64_t mi = INT64_MAX;
  const bool rescale = a.mode == kReduceSet && a.factor != 1.0;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(kRedThreads) + t; e < n;
       e += static_cast<int64_t>(nblk) * kRedThreads) {
    float v = to_f32<T>(buf[e]);
    if (rescale) {
      const T nv = static_cast<T>(static_cast<float>(static_cast<double>(v) * a.factor));
      buf[e] = nv;
      v = to_f32<T>(nv);
    }
    if (a.mode == kReduceArgmax) {
      const int64_t k = e / a.sstride, rem = e % a.sstride;
      const int64_t j = rem / a.pitch, i = rem % a.pitch;
      if (i < a.W) {
        const int64_t flat = (k * a.H + j) * a.W + i;
        if (v > mx || (v == mx && flat < mi)) {
          mx = v;
          mi = flat;
        }
      }
    } else {
      s += static_cast<double>(v);
      mx = fmaxf(mx, v);
    }
  }
  rs[t] = s;
  rm[t] = mx;
  ri[t] = mi;
  __syncthreads();
  for (int st = kRedThreads / 2; st > 0; st >>= 1) {
    if (t < st) {
      rs[t] += rs[t + st];
      const float o = rm[t + st];
      const int64_t oi = ri[t + st];
      if (o > rm[t] || (o == rm[t] && oi < ri[t])) {
        rm[t] = o;
        ri[t] = oi;
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    publish(&a.partials[3 * blockIdx.x], rs[0]);
    publish(&a.partials[3 * blockIdx.x + 1], static_cast<double>(rm[0]));
    publish(&a.partials[3 * blockIdx.x + 2], static_cast<double>(ri[0]));
    last_flag = arrive_last(dev, blockIdx.x, static_cast<uint32_t>(nblk));
  }
  __syncthreads();
  if (!last_flag) return;
  s = 0.0;
  mx = 0.f;
  mi = INT64_MAX;
  for (int b = t; b < nblk; b += kRedThreads) {
    s += __hip_atomic_load(&a.partials[3 * b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const float o = static_cast<float>(__hip_atomic_load(&a.partials[3 * b + 1], __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT));
    const int64_t oi = static_cast<int64_t>(
        __hip_atomic_load(&a.partials[3 * b + 2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (a.mode == kReduceArgmax) {
      if (o > mx || (o == mx && oi < mi)) {
        mx = o;
        mi = oi;
      }
    } else {
      mx = fmaxf(mx, o);
    }
  }
  rs[t] = s;
  rm[t] = mx;
  ri[t] = mi;
  __syncthreads();
  for (int st = kRedThreads / 2; st > 0; st >>= 1) {
    if (t < st) {
      rs[t] += rs[t + st];
      const float o = rm[t + st];
      const int64_t oi = ri[t + st];
      if (o > rm[t] || (o == rm[t] && oi < ri[t])) {
        rm[t] = o;
        ri[t] = oi;
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    if (a.mode == kReduceArgmax) {
      dev->argmax_idx = ri[0];
      dev->argmax_val = rm[0];
    } else if (a.mode == kReduceSum) {
      dev->aux[3] = rs[0];
    } else {
      const double tot = rs[0];
      const float m = rm[0];
      if (!(tot > 0.0) || !isfinite(tot) || !(m > 0.f)) {
        dev->status = kStatusDegenerate;
      } else {
        dev->sum = tot;
        dev->lnsum = log(tot);
        dev->maxval = m;
        const double sc = 1.0 / static_cast<double>(m);
        dev->scale = sc > static_cast<double>(FLT_MAX) ? FLT_MAX : static_cast<float>(sc);
      }
    }
    __hip_atomic_store(&dev->counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <typename T>
__global__ void export_kernel(const T* __restrict__ buf, int W, int H, int pitch, int64_t sstride,
                              const FilterDev* __restrict__ dev, float* __restrict__ out,
                              int64_t out_slice_stride, int k_begin) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  const int k = k_begin + blockIdx.z;
  if (x >= W) return;
  const double inv = 1.0 / dev->aux[3];
  const float v = to_f32<T>(buf[k * sstride + static_cast<int64_t>(y) * pitch + x]);
  out[(k - k_begin) * out_slice_stride + static_cast<int64_t>(y) * W + x] =
      static_cast<float>(static_cast<double>(v) * inv);
}

template <typename T>
__global__ void belief_map_kernel(const T* __restrict__ buf, int W, int H, int pitch, int n_theta,
                                  int64_t sstride, const FilterDev* __restrict__ dev, float* __restrict__ out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= W) return;
  float m = 0.f;
  for (int k = 0; k < n_theta; ++k)
    m = fmaxf(m, to_f32<T>(buf[k * sstride + static_cast<int64_t>(y) * pitch + x]));
  out[static_cast<int64_t>(y) * W + x] = static_cast<float>(static_cast<double>(m) / dev->aux[3]);
}

struct ShiftList {
  int32_t n[2 * kMaxTheta];
};

__global__ void write_shifts_kernel(ShiftList l, int count, int32_t* __restrict__ dst) {
  for (int i = threadIdx.x; i < 2 * count; i += blockDim.x) dst[i] = l.n[i];
}

__global__ void write_table_kernel(ShiftArgs t, int count, ShiftEntry* __restrict__ dst) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) dst[i] = t.e[i];
}

__global__ void export_scalars_kernel(const FilterDev* dev, double* out) {
  out[0] = dev->log_norm;
  out[1] = static_cast<double>(dev->status);
}

__global__ void dev_init_kernel(FilterDev* dev, double sum, float maxval) {
  FilterDev d = {};
  d.log_norm = 0.0;
  d.sum = sum;
  d.lnsum = log(sum);
  d.maxval = maxval;
  d.scale = 1.0f / maxval;
  d.cur = 0;
  d.status = kStatusOk;
  d.counter = 0;
  d.argmax_idx = -1;
  *dev = d;
  uint32_t* cg = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(dev) + kDevBytes);
  for (int i = 0; i < kArriveGroups * kArriveStride; ++i) cg[i] = 0u;
}

template <typename T>
const T* as(const void* p) {
  return static_cast<const T*>(p);
}

}  // namespace

hipError_t launch_map_setup(const uint8_t* occ_dev, int W, int H, int pitch, const double* gxy, int rxy,
                            double gth_sum, uint32_t flags, uint8_t* free8, float* mpre, float* wt,
                            hipStream_t s) {
  MapTaps taps = {};
  for (int i = 0; i <= 2 * rxy; ++i) taps.g[i] = gxy[i];
  dim3 grid((pitch + 255) / 256, H);
  hipLaunchKernelGGL(map_setup_kernel, grid, dim3(256), 0, s, occ_dev, W, H, pitch, taps, rxy, gth_sum,
                     flags, free8, mpre, wt);
  return hipGetLastError();
}

hipError_t launch_init_uniform(int dtype, void* buf0, void* buf1, const uint8_t* free8, int W, int H,
                               int pitch, int n_theta, int64_t sstride, hipStream_t s) {
  (void)W;
  const int64_t n = sstride * n_theta;
  const int64_t plane = static_cast<int64_t>(H) * pitch;
  const int blocks = static_cast<int>((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
  switch (dtype) {
    case 0:
      hipLaunchKernelGGL(init_uniform_kernel<float>, dim3(blocks), dim3(256), 0, s, static_cast<float*>(buf0),
                         static_cast<float*>(buf1), free8, plane, n);
      break;
    case 1:
      hipLaunchKernelGGL(init_uniform_kernel<__bf16>, dim3(blocks), dim3(256), 0, s,
                         static_cast<__bf16*>(buf0), static_cast<__bf16*>(buf1), free8, plane, n);
      break;
    case 2:
      hipLaunchKernelGGL(init_uniform_kernel<_Float16>, dim3(blocks), dim3(256), 0, s,
                         static_cast<_Float16*>(buf0), static_cast<_Float16*>(buf1), free8, plane, n);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_slice_from_f32(int dtype, const float* src, void* dst, int W, int H, int pitch, float factor,
                                 hipStream_t s) {
  dim3 grid((pitch + 255) / 256, H);
  switch (dtype) {
    case 0: hipLaunchKernelGGL(slice_from_f32_kernel<float>, grid, dim3(256), 0, s, src, static_cast<float*>(dst), W, H, pitch, factor); break;
    case 1: hipLaunchKernelGGL(slice_from_f32_kernel<__bf16>, grid, dim3(256), 0, s, src, static_cast<__bf16*>(dst), W, H, pitch, factor); break;
    case 2: hipLaunchKernelGGL(slice_from_f32_kernel<_Float16>, grid, dim3(256), 0, s, src, static_cast<_Float16*>(dst), W, H, pitch, factor); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_reduce(int dtype, const ReduceArgs& a, int nblocks, hipStream_t s) {
  switch (dtype) {
    case 0: hipLaunchKernelGGL(reduce_kernel<float>, dim3(nblocks), dim3(kRedThreads), 0, s, a); break;
    case 1: hipLaunchKernelGGL(reduce_kernel<__bf16>, dim3(nblocks), dim3(kRedThreads), 0, s, a); break;
    case 2: hipLaunchKernelGGL(reduce_kernel<_Float16>, dim3(nblocks), dim3(kRedThreads), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_export(int dtype, const void* buf, int W, int H, int pitch, int n_theta, int64_t sstride,
                         const FilterDev* dev, float* out, int64_t out_slice_stride, int k_begin, int k_end,
                         float* map_out, hipStream_t s) {
  dim3 grid((W + 255) / 256, H, k_end - k_begin);
  if (k_end > k_begin) {
    switch (dtype) {
      case 0: hipLaunchKernelGGL(export_kernel<float>, grid, dim3(256), 0, s, as<float>(buf), W, H, pitch, sstride, dev, out, out_slice_stride, k_begin); break;
      case 1: hipLaunchKernelGGL(export_kernel<__bf16>, grid, dim3(256), 0, s, as<__bf16>(buf), W, H, pitch, sstride, dev, out, out_slice_stride, k_begin); break;
      case 2: hipLaunchKernelGGL(export_kernel<_Float16>, grid, dim3(256), 0, s, as<_Float16>(buf), W, H, pitch, sstride, dev, out, out_slice_stride, k_begin); break;
      default: return hipErrorInvalidValue;
    }
  }
  if (map_out) {
    dim3 g2((W + 255) / 256, H);
    switch (dtype) {
      case 0: hipLaunchKernelGGL(belief_map_kernel<float>, g2, dim3(256), 0, s, as<float>(buf), W, H, pitch, n_theta, sstride, dev, map_out); break;
      case 1: hipLaunchKernelGGL(belief_map_kernel<__bf16>, g2, dim3(256), 0, s, as<__bf16>(buf), W, H, pitch, n_theta, sstride, dev, map_out); break;
      case 2: hipLaunchKernelGGL(belief_map_kernel<_Float16>, g2, dim3(256), 0, s, as<_Float16>(buf), W, H, pitch, n_theta, sstride, dev, map_out); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

hipError_t launch_write_shifts(const int32_t* n, int count, int32_t* dst, hipStream_t s) {
  if (count < 1 || count > kMaxTheta) return hipErrorInvalidValue;
  ShiftList l;
  for (int i = 0; i < 2 * count; ++i) l.n[i] = n[i];
  hipLaunchKernelGGL(write_shifts_kernel, dim3(1), dim3(256), 0, s, l, count, dst);
  return hipGetLastError();
}

hipError_t launch_write_table(const ShiftEntry* t, int count, ShiftEntry* dst, hipStream_t s) {
  if (count < 1 || count > kMaxTheta) return hipErrorInvalidValue;
  for (int k0 = 0; k0 < count; k0 += kArgTableMax) {
    const int n = count - k0 < kArgTableMax ? count - k0 : kArgTableMax;
    ShiftArgs a;
    for (int i = 0; i < n; ++i) a.e[i] = t[k0 + i];
    hipLaunchKernelGGL(write_table_kernel, dim3(1), dim3(128), 0, s, a, n, dst + k0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_export_scalars(const FilterDev* dev, double* out, hipStream_t s) {
  hipLaunchKernelGGL(export_scalars_kernel, dim3(1), dim3(1), 0, s, dev, out);
  return hipGetLastError();
}

hipError_t launch_dev_init(FilterDev* dev, double sum, float maxval, hipStream_t s) {
  hipLaunchKernelGGL(dev_init_kernel, dim3(1), dim3(1), 0, s, dev, sum, maxval);
  return hipGetLastError();
}

}  // namespace mcl
