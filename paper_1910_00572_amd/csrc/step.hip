// Fused odometry step of the belief-tensor filter for gfx950.
//
// One launch applies Alg. 1 to the whole tensor and renormalises:
//   S  = M_pre (.) warp_k(s * B_k)            bilinear per-channel shift (Sec. III-A-1)
//   T  = g_theta *_theta g_y *_y g_x *_x S    separable Gaussian (Sec. III-A-2)
//   B' = W_post (.) T                         W_post = M / G(B_0)   (Sec. III-A-3)
// followed by the sum / max reduction that renormalises the belief (the eta
// of eq. sensor update, applied after every step) and a lazily applied scale
// s = 1 / max that keeps 16-bit storage in range.
//
// Design (2.5-D stencil): a workgroup owns an output tile of TX x TY cells
// and streams through the heading channels.  For every channel it
//   P1  stages the shifted source window (TY+2R+1 rows) from HBM into LDS,
//       realigned so the fractional shift reads aligned 16-byte words;
//   P2  applies the bilinear weights and the pre-blur mask -> S in LDS;
//   P3  blurs along y -> LDS;   P4  blurs along x -> registers;
//   P5  keeps the last 2R+1 channels in a register ring and emits the
//       theta-blurred, masked, wall-normalised output of channel j-R.
// The next channel's window is loaded into registers while P2-P4 run.  Each
// state is read from HBM once (plus the halo, shared through L2) and written
// once.  The circular theta blur starts R channels early and runs R late,
// wrapping the channel index.  The sum/max reduction is finished by the last
// workgroup to arrive (atomic counter), so a step is a single launch whose
// result does not depend on workgroup timing.
#include <float.h>
#include <math.h>

#include <type_traits>

#include "mcl_internal.hpp"

namespace mcl {
namespace {

// ---- storage types -------------------------------------------------------------
template <typename T>
struct Store;

template <>
struct Store<float> {
  static constexpr int VEC = 4;  // elements per 16-byte word
  __device__ static inline void unpack(const uint4& r, float* o) {
    o[0] = __uint_as_float(r.x);
    o[1] = __uint_as_float(r.y);
    o[2] = __uint_as_float(r.z);
    o[3] = __uint_as_float(r.w);
  }
  __device__ static inline void store4(float* p, const float* v) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
  }
};

template <>
struct Store<__bf16> {
  static constexpr int VEC = 8;
  __device__ static inline void unpack(const uint4& r, float* o) {
    const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      o[2 * i] = __uint_as_float(w[i] << 16);
      o[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
    }
  }
  __device__ static inline uint32_t pack2(float a, float b) {
    const uint32_t lo = __builtin_bit_cast(uint16_t, static_cast<__bf16>(a));
    const uint32_t hi = __builtin_bit_cast(uint16_t, static_cast<__bf16>(b));
    return lo | (hi << 16);
  }
  __device__ static inline void store4(__bf16* p, const float* v) {
    *reinterpret_cast<uint2*>(p) = make_uint2(pack2(v[0], v[1]), pack2(v[2], v[3]));
  }
};

template <>
struct Store<_Float16> {
  static constexpr int VEC = 8;
  __device__ static inline void unpack(const uint4& r, float* o) {
    const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      o[2 * i] = static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(w[i] & 0xffffu)));
      o[2 * i + 1] = static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(w[i] >> 16)));
    }
  }
  __device__ static inline uint32_t pack2(float a, float b) {
    const uint32_t lo = __builtin_bit_cast(uint16_t, static_cast<_Float16>(a));
    const uint32_t hi = __builtin_bit_cast(uint16_t, static_cast<_Float16>(b));
    return lo | (hi << 16);
  }
  __device__ static inline void store4(_Float16* p, const float* v) {
    *reinterpret_cast<uint2*>(p) = make_uint2(pack2(v[0], v[1]), pack2(v[2], v[3]));
  }
};

// Spread consecutive workgroups over the 8 XCDs so that each XCD (own L2)
// receives a contiguous band of tiles: neighbouring tiles share halo rows.
__device__ inline int xcd_remap(int b, int n) {
  constexpr int X = 8;
  const int q = n / X, r = n % X;
  const int x = b % X, i = b / X;
  return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Wave priority by progress through a workgroup's G channel groups.  The
// instruction arbiter of a SIMD prefers higher-priority waves and, among
// equals, older ones, so without this the oldest workgroups on a compute unit
// run ahead, finish first and leave the last ones to run alone at low
// occupancy.  Lowering the priority as a wave advances (3 for its first
// quarter of groups, then 2, 1, 0) lets lagging waves catch up: the
// workgroups sharing a compute unit advance together and finish together.
// Used by the variant-1 streaming kernel, whose 512 x 512 x 72 step it takes
// from 47.7 to 44.8 us; the variant-0 kernel of the 1024 x 1024 x 128 step
// ran slower with it (333 to 364 us), so it does not use it.
struct ProgressPriority {
  int q1, q2, q3;
  __device__ explicit ProgressPriority(int G) : q1(G / 4), q2(G / 2), q3((3 * G) / 4) {
    __builtin_amdgcn_s_setprio(3);
  }
  __device__ void at(int g) const {
    if (g >= q3) __builtin_amdgcn_s_setprio(0);
    else if (g >= q2) __builtin_amdgcn_s_setprio(1);
    else if (g >= q1) __builtin_amdgcn_s_setprio(2);
  }
};

// A batch's job table (StepArgs per job, first workgroup per job) is read
// through the constant address space with a wave-uniform index: the compiler
// then uses scalar loads into scalar registers, as for kernel arguments.
// Read through plain global pointers it treats the loaded arguments as
// per-lane values and moves the step's whole address arithmetic to the vector
// unit (the batched step ran at about half the speed of the single one).
typedef const __attribute__((address_space(4))) int32_t* ConstI32;
typedef const __attribute__((address_space(4))) StepArgs* ConstArgs;

// Job of global workgroup g: the largest j with first[j] <= g (uniform).
__device__ inline int find_job(const int32_t* __restrict__ first_p, int njobs, int g) {
  const ConstI32 first = (ConstI32)first_p;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  return __builtin_amdgcn_readfirstlane(lo);
}

// The arguments of job j, read in place through the constant address space
// (the step bodies take their argument type as a template parameter), and the
// workgroup's block index within the job.
__device__ inline const __attribute__((address_space(4))) StepArgs& job_args(const StepArgs* __restrict__ jobs,
                                                                            const int32_t* __restrict__ first,
                                                                            int j, int g, int& blk) {
  blk = g - ((ConstI32)first)[j];
  return ((ConstArgs)jobs)[j];
}

// Run by every thread of the last workgroup to arrive: reduce all partials in
// a fixed order and update the filter scalars (renormalisation bookkeeping).
template <int NT, typename Args>
__device__ void finalize_step(Args& a, FilterDev* dev, int nblk, float scale, int cur, double* red_s,
                              float* red_m) {
  const int t = threadIdx.x;
  double s = 0.0;
  float mx = 0.f;
  for (int b = t; b < nblk; b += NT) {
    s += __hip_atomic_load(&a.partials[2 * b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    mx = fmaxf(mx, static_cast<float>(__hip_atomic_load(&a.partials[2 * b + 1], __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT)));
  }
  red_s[t] = s;
  red_m[t] = mx;
  __syncthreads();
#pragma unroll
  for (int st = NT / 2; st > 0; st >>= 1) {
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

template <typename T, int R, int TX, int TY, int NT, typename Args = const StepArgs>
__device__ __forceinline__ void step_body(Args& a, const int blk, const int nblk) {
  constexpr int VEC = Store<T>::VEC;
  constexpr int RQ = 4;                      // x halo of the S/Y region, one quad
  constexpr int SC = TX + 2 * RQ;            // S/Y region width
  constexpr int SCP = SC + 4;                // LDS row pitch (floats)
  constexpr int SR = TY + 2 * R;             // S rows
  constexpr int WR = SR + 1;                 // source-window rows
  constexpr int NV = (SC + VEC) / VEC;       // 16-byte words per window row
  constexpr int NRAW = WR * NV;
  constexpr int IPT1 = (NRAW + NT - 1) / NT;
  constexpr int NQ = SC / 4;                 // quads per S/Y row
  constexpr int NS = (SR / 2) * NQ;          // P2 items: 2 rows x 1 quad
  constexpr int IPT2 = (NS + NT - 1) / NT;
  constexpr int NYI = (TY / 2) * NQ;         // P3 items: 2 rows x 1 quad
  constexpr int IPT3 = (NYI + NT - 1) / NT;
  constexpr int OQ = TX / 4;
  constexpr int NP = TY * OQ;                // P4 items: 1 row x 1 quad
  constexpr int IPT4 = NP / NT;
  constexpr int RING = 2 * R + 1;
  static_assert(NP % NT == 0, "output quads must divide evenly");
  static_assert(SC % VEC == 0 && TY % 2 == 0, "tile shape");
  static_assert(R >= 1 && R <= kMaxRadius, "radius");
  static_assert((NT & (NT - 1)) == 0, "power-of-two workgroup");

  __shared__ __attribute__((aligned(16))) float rawL[WR][SC + 8];
  __shared__ __attribute__((aligned(16))) float sL[SR][SCP];
  __shared__ __attribute__((aligned(16))) float yL[TY][SCP];
  __shared__ int pnx[kMaxTheta], pny[kMaxTheta];
  __shared__ float pfx[kMaxTheta], pfy[kMaxTheta];
  __shared__ double red_s[NT];
  __shared__ float red_m[NT];
  __shared__ int last_flag;

  const int t = threadIdx.x;
  const int W = a.W, H = a.H, pitch = a.pitch, nth = a.n_theta;
  (void)W;
  const int64_t sstride = a.sstride;
  const int tiles_x = a.tiles_x;
  const int ntile = tiles_x * a.tiles_y;
  const int chunk = blk / ntile, tile = blk % ntile;
  const int x0 = (tile % tiles_x) * TX;
  const int y0 = (tile / tiles_x) * TY;
  const int kbeg = chunk * a.chunk_len;
  const int kend = min(nth, kbeg + a.chunk_len);
  FilterDev* dev = a.dev;
  const int cur = dev->cur;
  const float scale = dev->scale;
  const T* __restrict__ bin = static_cast<const T*>(a.buf[cur]);
  T* __restrict__ bout = static_cast<T*>(a.buf[cur ^ 1]);
  const double u = a.u_cells, v = a.v_cells, th0 = a.theta_prev, dth = a.dtheta;

  // Per-channel displacement R(theta + k dtheta) [u, v] in cells, split into
  // integer and fractional parts (FP64, once per workgroup); or whole-cell
  // shifts given by the host.
  for (int k = t; k < nth; k += NT) {
    if (a.ishift) {
      pnx[k] = a.ishift[2 * k];
      pny[k] = a.ishift[2 * k + 1];
      pfx[k] = 0.f;
      pfy[k] = 0.f;
      continue;
    }
    double sn, cs;
    sincos(th0 + k * dth, &sn, &cs);
    const double dx = u * cs - v * sn;
    const double dy = u * sn + v * cs;
    const double fdx = floor(dx), fdy = floor(dy);
    pnx[k] = static_cast<int>(fdx);
    pny[k] = static_cast<int>(fdy);
    pfx[k] = static_cast<float>(dx - fdx);
    pfy[k] = static_cast<float>(dy - fdy);
  }
  float gx[RING], gt[RING];
#pragma unroll
  for (int l = 0; l < RING; ++l) {
    gx[l] = a.gxy[l];
    gt[l] = a.gth[l];
  }

  // Pre-blur mask of this thread's P2 items, wall weights of its outputs.
  float mreg[IPT2][2][4];
#pragma unroll
  for (int i = 0; i < IPT2; ++i) {
    const int id = t + i * NT;
    const int srp = id / NQ, q = id % NQ;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int y = y0 - R + 2 * srp + s;
      const int x = x0 - RQ + 4 * q;
      float4 mv = make_float4(0.f, 0.f, 0.f, 0.f);
      if (id < NS && y >= 0 && y < H && x >= 0 && x < pitch)
        mv = *reinterpret_cast<const float4*>(a.mpre + static_cast<int64_t>(y) * pitch + x);
      mreg[i][s][0] = mv.x;
      mreg[i][s][1] = mv.y;
      mreg[i][s][2] = mv.z;
      mreg[i][s][3] = mv.w;
    }
  }
  float wreg[IPT4][4];
  int64_t ooff[IPT4];
  bool ostore[IPT4];
#pragma unroll
  for (int i = 0; i < IPT4; ++i) {
    const int id = t + i * NT;
    const int yr = id / OQ, oq = id % OQ;
    const int y = y0 + yr, x = x0 + 4 * oq;
    ostore[i] = (y < H) && (x < pitch);
    ooff[i] = static_cast<int64_t>(y) * pitch + x;
    float4 wv = make_float4(0.f, 0.f, 0.f, 0.f);
    if (ostore[i]) wv = *reinterpret_cast<const float4*>(a.wt + ooff[i]);
    wreg[i][0] = wv.x * scale;
    wreg[i][1] = wv.y * scale;
    wreg[i][2] = wv.z * scale;
    wreg[i][3] = wv.w * scale;
  }

  float ring[IPT4][RING][4];
  float psum = 0.f, pmax = 0.f;
  const int jbeg = kbeg - R;
  const int count = (kend - kbeg) + 2 * R;

  auto phys = [nth](int j) {
    int k = j % nth;
    return k < 0 ? k + nth : k;
  };

  uint4 pre[IPT1];
  auto issue_loads = [&](int j) {
    const int kp = phys(j);
    const int colbase = x0 - RQ - pnx[kp] - 1;
    const int xa = colbase - (((colbase % VEC) + VEC) % VEC);
    const int rowbase = y0 - R - pny[kp] - 1;
    const T* base = bin + static_cast<int64_t>(kp) * sstride;
#pragma unroll
    for (int i = 0; i < IPT1; ++i) {
      const int id = t + i * NT;
      const int r = id / NV, vv = id % NV;
      const int gy = rowbase + r;
      const int gxe = xa + vv * VEC;
      pre[i] = make_uint4(0u, 0u, 0u, 0u);
      if (id < NRAW && static_cast<unsigned>(gy) < static_cast<unsigned>(H) && gxe >= 0 && gxe < pitch)
        pre[i] = *reinterpret_cast<const uint4*>(base + static_cast<int64_t>(gy) * pitch + gxe);
    }
  };

  __syncthreads();  // shift table ready
  issue_loads(jbeg);

  for (int jj = 0; jj < count; jj += RING) {
#pragma unroll
    for (int p = 0; p < RING; ++p) {
      const int jrel = jj + p;
      if (jrel < count) {
        const int j = jbeg + jrel;
        const int kp = phys(j);
        const float fx = pfx[kp], fy = pfy[kp];
        {
          // P1: window registers -> LDS as loaded (aligned 16-byte writes,
          // conflict-free); the misalignment is resolved in P2.
#pragma unroll
          for (int i = 0; i < IPT1; ++i) {
            const int id = t + i * NT;
            if (id < NRAW) {
              const int r = id / NV, vv = id % NV;
              float vals[VEC];
              Store<T>::unpack(pre[i], vals);
#pragma unroll
              for (int e = 0; e < VEC; e += 4)
                *reinterpret_cast<float4*>(&rawL[r][vv * VEC + e]) =
                    make_float4(vals[e], vals[e + 1], vals[e + 2], vals[e + 3]);
            }
          }
        }
        __syncthreads();
        if (jrel + 1 < count) issue_loads(j + 1);

        // P2: bilinear weights and pre-blur mask -> S.  S column c reads window
        // columns c + m (weight fx) and c + m + 1, m = window misalignment
        // (uniform): two aligned 16-byte reads per row, then a compile-time
        // selection for m mod 4.
        {
          const int colbase = x0 - RQ - pnx[kp] - 1;
          const int m = ((colbase % VEC) + VEC) % VEC;
          const int mh = m >> 2, ml = m & 3;
          auto p2 = [&](auto mlc) {
            constexpr int ML = decltype(mlc)::value;
#pragma unroll
            for (int i = 0; i < IPT2; ++i) {
              const int id = t + i * NT;
              if (id < NS) {
                const int srp = id / NQ, q = id % NQ;
                const int c0 = 4 * (q + mh);
                float xr[3][4];
#pragma unroll
                for (int rr = 0; rr < 3; ++rr) {
                  const float4 a4 = *reinterpret_cast<const float4*>(&rawL[2 * srp + rr][c0]);
                  const float4 b4 = *reinterpret_cast<const float4*>(&rawL[2 * srp + rr][c0 + 4]);
                  const float wv[8] = {a4.x, a4.y, a4.z, a4.w, b4.x, b4.y, b4.z, b4.w};
#pragma unroll
                  for (int e = 0; e < 4; ++e) xr[rr][e] = fmaf(fx, wv[ML + e] - wv[ML + e + 1], wv[ML + e + 1]);
                }
#pragma unroll
                for (int sidx = 0; sidx < 2; ++sidx) {
                  float sv[4];
#pragma unroll
                  for (int e = 0; e < 4; ++e)
                    sv[e] = fmaf(fy, xr[sidx][e] - xr[sidx + 1][e], xr[sidx + 1][e]) * mreg[i][sidx][e];
                  *reinterpret_cast<float4*>(&sL[2 * srp + sidx][4 * q]) = make_float4(sv[0], sv[1], sv[2], sv[3]);
                }
              }
            }
          };
          switch (ml) {
            case 0: p2(std::integral_constant<int, 0>()); break;
            case 1: p2(std::integral_constant<int, 1>()); break;
            case 2: p2(std::integral_constant<int, 2>()); break;
            default: p2(std::integral_constant<int, 3>()); break;
          }
        }
        __syncthreads();

        // P3: blur along y, two output rows per item.
#pragma unroll
        for (int i = 0; i < IPT3; ++i) {
          const int id = t + i * NT;
          if (id < NYI) {
            const int yrp = id / NQ, q = id % NQ;
            float a0[4] = {0.f, 0.f, 0.f, 0.f}, a1[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int l = 0; l <= 2 * R + 1; ++l) {
              const float4 s4 = *reinterpret_cast<const float4*>(&sL[2 * yrp + l][4 * q]);
              const float sv[4] = {s4.x, s4.y, s4.z, s4.w};
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                if (l <= 2 * R) a0[e] = fmaf(gx[l], sv[e], a0[e]);
                if (l >= 1) a1[e] = fmaf(gx[l - 1], sv[e], a1[e]);
              }
            }
            *reinterpret_cast<float4*>(&yL[2 * yrp][4 * q]) = make_float4(a0[0], a0[1], a0[2], a0[3]);
            *reinterpret_cast<float4*>(&yL[2 * yrp + 1][4 * q]) = make_float4(a1[0], a1[1], a1[2], a1[3]);
          }
        }
        __syncthreads();

        // P4: blur along x into the ring slot of this channel.
#pragma unroll
        for (int i = 0; i < IPT4; ++i) {
          const int id = t + i * NT;
          const int yr = id / OQ, oq = id % OQ;
          float yv[12];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const float4 y4 = *reinterpret_cast<const float4*>(&yL[yr][4 * oq + 4 * c]);
            yv[4 * c] = y4.x;
            yv[4 * c + 1] = y4.y;
            yv[4 * c + 2] = y4.z;
            yv[4 * c + 3] = y4.w;
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            float acc = 0.f;
#pragma unroll
            for (int l = 0; l < RING; ++l) acc = fmaf(gx[l], yv[RQ - R + e + l], acc);
            ring[i][p][e] = acc;
          }
        }

        // P5: theta blur of channel j - R, post-blur weights, store, reduce.
        if (jrel >= 2 * R) {
          const int ko = phys(j - R);
          T* obase = bout + static_cast<int64_t>(ko) * sstride;
#pragma unroll
          for (int i = 0; i < IPT4; ++i) {
            float o[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              float acc = 0.f;
#pragma unroll
              for (int l = 0; l < RING; ++l) acc = fmaf(gt[l], ring[i][(p - 2 * R + l + RING) % RING][e], acc);
              o[e] = acc * wreg[i][e];
              psum += o[e];
              pmax = fmaxf(pmax, o[e]);
            }
            if (ostore[i]) Store<T>::store4(obase + ooff[i], o);
          }
        }
      }
    }
  }

  // Workgroup partial (fixed tree), then the last workgroup to arrive
  // reduces all partials in a fixed order and updates the filter scalars.
  red_s[t] = static_cast<double>(psum);
  red_m[t] = pmax;
  __syncthreads();
  static_assert((NT & (NT - 1)) == 0, "the tree reduction needs a power-of-two workgroup");
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (t < s) {
      red_s[t] += red_s[t + s];
      red_m[t] = fmaxf(red_m[t], red_m[t + s]);
    }
    __syncthreads();
  }
  if (t == 0) {
    publish(&a.partials[2 * blk], red_s[0]);
    publish(&a.partials[2 * blk + 1], static_cast<double>(red_m[0]));
    last_flag = arrive_last(dev, static_cast<uint32_t>(blk), static_cast<uint32_t>(nblk));
  }
  __syncthreads();
  if (!last_flag) return;

  finalize_step<NT>(a, dev, nblk, scale, cur, red_s, red_m);
}

// ---- streaming variant ------------------------------------------------------------
// One wave owns a strip of 64 consecutive columns (lane = column) and streams
// the TY + 2R + 1 source rows of a channel through registers: the bilinear
// x neighbour comes from the adjacent lane (DPP wave shift), the y
// interpolation, mask and y blur run down a register window, and the x blur
// uses DPP shifts of the y-blurred rows.  Lanes R+1 .. R+strip hold the
// strip's outputs (strip <= 63 - 2R, a multiple of 32 bytes of storage, so
// strips never share a 32-byte segment of an output row).  The waves of a
// workgroup take consecutive channels; the theta blur reads a ring of
// 2R + 2 WAVES channel results in LDS (layout [slot][lane][row], 16-byte
// reads of four rows), with one barrier per group of WAVES channels.  The
// next group's source rows are loaded while the current group is computed.
//
// Rows are read and written through one raw buffer descriptor per heading
// plane; a row or column outside the grid gets an out-of-range offset, and
// the hardware returns 0 for (and drops stores to) out-of-range offsets, so
// the borders need no branch.
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit data (gfx9 family)

template <typename T>
struct Elt;
template <>
struct Elt<float> {
  static constexpr int BYTES = 4;
  // the b32 buffer builtins move raw 32-bit words: bit-cast, never convert
  __device__ static inline float load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
  }
  __device__ static inline void store(float v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, 0);
  }
};
template <>
struct Elt<__bf16> {
  static constexpr int BYTES = 2;
  __device__ static inline float load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __uint_as_float(static_cast<uint32_t>(__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0)) << 16);
  }
  __device__ static inline void store(float v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, static_cast<__bf16>(v)), r, off, 0, 0);
  }
};
template <>
struct Elt<_Float16> {
  static constexpr int BYTES = 2;
  __device__ static inline float load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return static_cast<float>(__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0)));
  }
  __device__ static inline void store(float v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, static_cast<_Float16>(v)), r, off, 0, 0);
  }
};

__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), static_cast<short>(0), static_cast<int>(bytes),
                                           kRsrcWord3);
}

// Byte offsets into one heading plane (H * pitch elements, below 1 GiB, one
// descriptor): a row part below 2^30 for rows inside the grid and 2^30 for
// rows outside, plus a column part below 2^30 for columns inside the row and
// 2^31 outside.  The sum stays below 2^32 and is out of range (the load
// returns 0, the store is dropped) exactly when the row or the column is.
constexpr uint32_t kRowOut = 1u << 30;
constexpr uint32_t kColOut = 1u << 31;

template <typename T>
__device__ inline float load_row(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ inline float load_row<float>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ inline float load_row<__bf16>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __uint_as_float(static_cast<uint32_t>(__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0)) << 16);
}
template <>
__device__ inline float load_row<_Float16>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return static_cast<float>(__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0)));
}
template <typename T>
__device__ inline void store_row(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ inline void store_row<float>(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, 0);
}
template <>
__device__ inline void store_row<__bf16>(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, static_cast<__bf16>(v)), r, voff, soff, 0);
}
template <>
__device__ inline void store_row<_Float16>(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, static_cast<_Float16>(v)), r, voff, soff, 0);
}

// Row addressing of a strip's source slices: interior strips address rows
// from each slice's first row without per-row checks.
template <bool B>
struct RowMode {
  static constexpr bool interior = B;
};

// lane i receives lane i-1 / i+1; lanes without a source receive 0
__device__ inline float from_left(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x138, 0xf, 0xf, true));
}
__device__ inline float from_right(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xf, 0xf, true));
}

// x blur of one row held one column per lane, sum over m of g[R + m] v(x + m)
// with g[R + m] = g[R - m].  Each side is summed Horner-style towards the
// centre, a_m = a_{m+1}(shifted one lane) + g[R + m] v, so that every lane
// shift is folded into an add (no separate lane moves); the products and
// sums are rounded separately so the shifts stay on the added operand.
// With UNIT the centre tap is taken as one (the caller scaled the taps).
template <int R, bool UNIT>
__device__ inline float x_blur_shifted_sums(float v, const float (&g)[2 * R + 1]) {
#pragma clang fp contract(off)
  float gv[R + 1];
  gv[0] = UNIT ? v : g[R] * v;
#pragma unroll
  for (int m = 1; m <= R; ++m) gv[m] = g[R + m] * v;
  float al = gv[R], ar = gv[R];
#pragma unroll
  for (int m = R - 1; m >= 1; --m) {
    al = from_left(al) + gv[m];
    ar = from_right(ar) + gv[m];
  }
  return (from_left(al) + gv[0]) + from_right(ar);
}

template <typename T, int R, int TY, int WAVES, int NBUF, typename Args = const StepArgs>
__device__ __forceinline__ void stream_body(Args& a, const ShiftEntry* __restrict__ tab, const int blk,
                                            const int nblk) {
  constexpr int NT = 64 * WAVES;
  constexpr int NS = TY + 2 * R;   // S rows
  constexpr int NR = NS + 1;       // source rows
  constexpr int GW = WAVES;        // channels per group (one per wave)
  // Ring slots: a group's emit reads 2R + GW channels.  With up to four waves
  // the ring also holds the next group's GW channels, so the next process
  // may start before every wave has finished emitting (one barrier per
  // group); with more waves that ring would not fit three workgroups per
  // compute unit, and a second barrier separates emit from the next process.
  constexpr bool ONE_BARRIER = WAVES <= 4;
  constexpr int RS = 2 * R + (ONE_BARRIER ? 2 : 1) * GW;
  constexpr int TAPS = 2 * R + 1;
  // ring lane pitch (floats): an odd number of 16-byte units, so the 64
  // lanes' 16-byte accesses fall on distinct banks in every pass
  constexpr int LP = (TY / 4) % 2 == 1 ? TY : TY + 4;
  constexpr int EB = Elt<T>::BYTES;
  static_assert(TY % 4 == 0, "rows per strip must be a multiple of 4");
  static_assert(NBUF == 1 || NBUF == 2, "one or two source-slice buffers");
  static_assert(sizeof(float) * RS * 64 * LP >= NT * (sizeof(double) + sizeof(float)), "reduction fits the ring");

  __shared__ __attribute__((aligned(16))) float ring[RS][64][LP];
  // per-channel shift table, sized by the launch to the job's heading count
  // (4 x 4 bytes per channel) so that small heading counts leave LDS for
  // more resident workgroups
  extern __shared__ int shift_table[];
  int* pnx = shift_table;
  int* pny = shift_table + a.n_theta;
  float* pfx = reinterpret_cast<float*>(shift_table + 2 * a.n_theta);
  float* pfy = reinterpret_cast<float*>(shift_table + 3 * a.n_theta);
  __shared__ int last_flag;
  // the block reduction reuses the ring once every wave has left the loop
  double* red_s = reinterpret_cast<double*>(&ring[0][0][0]);
  float* red_m = reinterpret_cast<float*>(red_s + NT);

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);  // wave index, uniform per wave
  const int H = a.H, pitch = a.pitch, nth = a.n_theta;
  const int64_t sstride = a.sstride;
  const uint32_t row_bytes = static_cast<uint32_t>(pitch) * EB;
  const uint32_t plane_bytes = static_cast<uint32_t>(sstride) * EB;  // < 2^30 (host-checked)
  const int tiles_x = a.tiles_x;
  const int ntile = tiles_x * a.tiles_y;
  const int chunk = blk / ntile, tile = blk % ntile;
  const int strip = a.strip;
  const int xb = (tile % tiles_x) * strip - (R + 1);
  const int y0 = (tile / tiles_x) * TY;
  const int x = xb + lane;
  const int kbeg = chunk * a.chunk_len;
  const int kend = min(nth, kbeg + a.chunk_len);
  const int nk = kend - kbeg;
  const int count = nk + 2 * R;
  const int jbeg = kbeg - R;
  FilterDev* dev = a.dev;
  const int cur = dev->cur;
  const float scale = dev->scale;
  const T* __restrict__ bin = static_cast<const T*>(a.buf[cur]);
  T* __restrict__ bout = static_cast<T*>(a.buf[cur ^ 1]);
  // the host's per-channel shift table (FP64 displacement split into whole
  // cells and a bilinear fraction), copied to LDS
  for (int k = t; k < nth; k += NT) {
    const ShiftEntry e = tab[k];
    pnx[k] = e.nx;
    pny[k] = e.ny;
    pfx[k] = e.fx;
    pfy[k] = e.fy;
  }
  // 16-bit storage is bound by vector issue at this kernel's shapes: its
  // three blurs run with the centre tap scaled to one (one multiply fewer
  // per blur and row), and the product of the three centre taps moves into
  // the post-blur weights
  constexpr bool kUnitCentre = sizeof(T) == 2;
  float gx[TAPS], gt[TAPS];
#pragma unroll
  for (int l = 0; l < TAPS; ++l) {
    gx[l] = a.gxy[l];
    gt[l] = a.gth[l];
  }
  float centre = 1.f;
  if constexpr (kUnitCentre) {
    const float cx = gx[R], ct = gt[R];
    centre = cx * cx * ct;
#pragma unroll
    for (int l = 0; l < TAPS; ++l) {
      // uniform values: kept in scalar registers
      gx[l] = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, gx[l] / cx)));
      gt[l] = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, gt[l] / ct)));
    }
  }
  const bool xin = x >= 0 && x < pitch;
  float mreg[NS];
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    const int y = y0 - R + r;
    mreg[r] = (xin && y >= 0 && y < H) ? a.mpre[static_cast<int64_t>(y) * pitch + x] : 0.f;
  }
  const bool out_lane = lane >= R + 1 && lane <= R + strip && xin;
  float wreg[TY];
#pragma unroll
  for (int o = 0; o < TY; ++o) {
    const int y = y0 + o;
    wreg[o] = (out_lane && y < H) ? a.wt[static_cast<int64_t>(y) * pitch + x] * scale * centre : 0.f;
  }
  // store offset of this lane (out of range for lanes that hold no output)
  const uint32_t soff = out_lane ? static_cast<uint32_t>(x) * EB : kColOut;
  auto phys = [nth](int j) {
    int k = j % nth;
    return k < 0 ? k + nth : k;
  };
  __syncthreads();  // shift table ready

  // Row offsets from a slice's first row, the interior-strip test and the
  // load cursor, as in the variant-1 kernel below: strips whose slices all
  // start at or below row 0 address rows from each slice's first row through
  // the buffer instructions' scalar offset, without per-row checks.
  uint32_t rowoff[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) rowoff[r] = static_cast<uint32_t>(r) * row_bytes;
  const bool interior = y0 - R - 1 - a.ny_max >= 0;
  int kp_cur = phys(jbeg + w);
  const int gstep = GW % nth;
  int pslot = w;
  const uint32_t out_bytes = static_cast<uint32_t>(min(H - y0, TY)) * row_bytes;

  // Source rows of channel jrel and its fractional shift (read here, one
  // group ahead, so that process() starts without an LDS round trip).
  //
  // The loop below has no data-dependent branch around a memory operation:
  // channels past the end of the chunk load through empty descriptors (the
  // hardware returns zeros without a memory access) and outputs outside the
  // chunk store through empty descriptors.  With straight-line control flow
  // the compiler's wait-counter tracking stays exact across iterations, so
  // the next group's loads stay in flight while the current group computes
  // (a branch here makes it wait for every outstanding load and store).
  struct Slice {
    float v[NR];
    float fx, fy;
  };
  auto load_slice = [&](auto mode, int jrel, Slice& sl) {
    const bool live = jrel < count;
    const int kp = kp_cur;
    kp_cur += gstep;
    if (kp_cur >= nth) kp_cur -= nth;
    const int nx = __builtin_amdgcn_readfirstlane(pnx[kp]);
    const int ny = __builtin_amdgcn_readfirstlane(pny[kp]);
    sl.fx = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, pfx[kp])));
    sl.fy = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, pfy[kp])));
    const int c = x - nx;
    const uint32_t loff = static_cast<unsigned>(c) < static_cast<unsigned>(pitch) ? static_cast<uint32_t>(c) * EB
                                                                                   : kColOut;
    const int sy0 = y0 - R - ny - 1;
    const T* plane = bin + static_cast<int64_t>(kp) * sstride;
    if constexpr (decltype(mode)::interior) {
      const uint32_t rows_in = static_cast<uint32_t>(max(H - sy0, 0));
      const __amdgpu_buffer_rsrc_t rs =
          buf_rsrc(plane + static_cast<int64_t>(sy0) * pitch, live ? rows_in * row_bytes : 0u);
#pragma unroll
      for (int r = 0; r < NR; ++r) sl.v[r] = load_row<T>(rs, loff, rowoff[r]);
    } else {
      const __amdgpu_buffer_rsrc_t rs = buf_rsrc(plane, live ? plane_bytes : 0u);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int sy = sy0 + r;
        const uint32_t roff = static_cast<unsigned>(sy) < static_cast<unsigned>(H)
                                  ? static_cast<uint32_t>(sy) * row_bytes
                                  : kRowOut;
        sl.v[r] = load_row<T>(rs, loff, roff);
      }
    }
  };
  auto process = [&](Slice& sl) {
    float(&vv)[NR] = sl.v;
    const float fx = sl.fx, fy = sl.fy;
#pragma unroll
    for (int r = 0; r < NR; ++r) vv[r] = fmaf(fx, from_left(vv[r]) - vv[r], vv[r]);
#pragma unroll
    for (int r = 0; r < NS; ++r) vv[r] = fmaf(fy, vv[r] - vv[r + 1], vv[r + 1]) * mreg[r];
    float* slot = &ring[pslot][lane][0];
    pslot += GW;
    if (pslot >= RS) pslot -= RS;
#pragma unroll
    for (int o4 = 0; o4 < TY; o4 += 4) {
      float p4[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int o = o4 + q;
        float yv;
        if constexpr (kUnitCentre) {
          yv = vv[o + R];
#pragma unroll
          for (int l = 0; l < TAPS; ++l)
            if (l != R) yv = fmaf(gx[l], vv[o + l], yv);
        } else {
          yv = gx[0] * vv[o];
#pragma unroll
          for (int l = 1; l < TAPS; ++l) yv = fmaf(gx[l], vv[o + l], yv);
        }
        // 16-bit storage is bound by vector issue at this shape: the form
        // without lane moves saves 5 % of its VALU work (FP32, closer to its
        // memory limit, runs no faster with it and keeps the fused form)
        float p;
        if constexpr (sizeof(T) == 2) {
          p = x_blur_shifted_sums<R, kUnitCentre>(yv, gx);
        } else {
          p = gx[R] * yv;
          float dl = yv, dr = yv;
#pragma unroll
          for (int m = 1; m <= R; ++m) {
            dl = from_left(dl);
            dr = from_right(dr);
            p = fmaf(gx[R + m], dl + dr, p);
          }
        }
        p4[q] = p;
      }
      *reinterpret_cast<float4*>(slot + o4) = make_float4(p4[0], p4[1], p4[2], p4[3]);
    }
  };
  float psum = 0.f, pmax = 0.f;
  // Theta blur of one channel.  All ring reads of a batch of rows are issued
  // before the first use (the scheduling barrier keeps the compiler from
  // interleaving them with the dependent FMAs), so a batch costs one LDS
  // round trip instead of one per tap.
  constexpr int RB = 4;
  auto emit = [&](int g) {
    const int krel = GW * g - 2 * R + w;
    const bool live = krel >= 0 && krel < nk;
    const int ko = kbeg + (live ? krel : 0);
    // the descriptor covers the strip's rows inside the grid
    const __amdgpu_buffer_rsrc_t rs =
        buf_rsrc(bout + static_cast<int64_t>(ko) * sstride + static_cast<int64_t>(y0) * pitch, live ? out_bytes : 0u);
    // ring slots of channels krel .. krel + 2R; krel >= -(2R + GW) (padding
    // emits), so a multiple of RS keeps the modulus non-negative
    constexpr int OFF = ((2 * R + GW + RS - 1) / RS) * RS;
    int slot[TAPS];
    slot[0] = (krel + OFF) % RS;
#pragma unroll
    for (int l = 1; l < TAPS; ++l) slot[l] = slot[l - 1] + 1 == RS ? 0 : slot[l - 1] + 1;
#pragma unroll
    for (int ob = 0; ob < TY; ob += RB) {
      float4 rv[RB / 4][TAPS];
#pragma unroll
      for (int q = 0; q < RB / 4; ++q)
#pragma unroll
        for (int l = 0; l < TAPS; ++l)
          rv[q][l] = *reinterpret_cast<const float4*>(&ring[slot[l]][lane][ob + 4 * q]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int q = 0; q < RB / 4; ++q) {
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        if constexpr (kUnitCentre) {
          acc[0] = rv[q][R].x;
          acc[1] = rv[q][R].y;
          acc[2] = rv[q][R].z;
          acc[3] = rv[q][R].w;
        }
#pragma unroll
        for (int l = 0; l < TAPS; ++l) {
          if (kUnitCentre && l == R) continue;
          acc[0] = fmaf(gt[l], rv[q][l].x, acc[0]);
          acc[1] = fmaf(gt[l], rv[q][l].y, acc[1]);
          acc[2] = fmaf(gt[l], rv[q][l].z, acc[2]);
          acc[3] = fmaf(gt[l], rv[q][l].w, acc[3]);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int o = ob + 4 * q + e;
          const float ov = acc[e] * wreg[o];
          const float ovk = live ? ov : 0.f;
          psum += ovk;
          pmax = fmaxf(pmax, ovk);
          store_row<T>(ov, rs, soff, rowoff[o]);
        }
      }
    }
  };

  // Software pipeline over the groups.  The prologue runs a padding emit
  // (its stores are dropped) so that the loop is entered with the same
  // sequence of outstanding memory operations as every later iteration: the
  // wait for a slice then never includes the stores issued after it.
  // NBUF = 2: slice A is carried across iterations and slice B lives within
  // one, so each slice's loads are issued a whole group ahead.  NBUF = 1: the
  // next slice is loaded into the registers the current one just left, one
  // emit ahead (fewer registers, for more waves per SIMD).
  auto ch = [&](int g) { return GW * g + w; };
  auto pipeline = [&](auto mode) {
    if constexpr (NBUF == 2) {
      const int G = (((count + GW - 1) / GW) + 1) & ~1;  // even: the last may be padding
      Slice sA, sB;
      load_slice(mode, ch(0), sA);
      emit(-1);
      for (int g = 0; g < G; g += 2) {
        load_slice(mode, ch(g + 1), sB);
        process(sA);
        __syncthreads();
        emit(g);
        if (!ONE_BARRIER) __syncthreads();
        load_slice(mode, ch(g + 2), sA);
        process(sB);
        __syncthreads();
        emit(g + 1);
        if (!ONE_BARRIER) __syncthreads();
      }
    } else {
      const int G = (count + GW - 1) / GW;
      Slice sA;
      load_slice(mode, ch(0), sA);
      emit(-1);
      for (int g = 0; g < G; ++g) {
        process(sA);
        load_slice(mode, ch(g + 1), sA);
        __syncthreads();
        emit(g);
        if (!ONE_BARRIER) __syncthreads();
      }
    }
  };
  if (interior)
    pipeline(RowMode<true>{});
  else
    pipeline(RowMode<false>{});
  __syncthreads();  // the ring becomes the reduction buffer

  red_s[t] = static_cast<double>(psum);
  red_m[t] = pmax;
  __syncthreads();
  static_assert((NT & (NT - 1)) == 0, "the tree reduction needs a power-of-two workgroup");
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (t < s) {
      red_s[t] += red_s[t + s];
      red_m[t] = fmaxf(red_m[t], red_m[t + s]);
    }
    __syncthreads();
  }
  if (t == 0) {
    publish(&a.partials[2 * blk], red_s[0]);
    publish(&a.partials[2 * blk + 1], static_cast<double>(red_m[0]));
    last_flag = arrive_last(dev, static_cast<uint32_t>(blk), static_cast<uint32_t>(nblk));
  }
  __syncthreads();
  if (!last_flag) return;
  finalize_step<NT>(a, dev, nblk, scale, cur, red_s, red_m);
}

// ---- streaming variant with the mask in the y taps and the x blur last --------------
// Same strips, waves and theta ring as stream_body, with three changes that
// take VALU work off every channel:
//  * the pre-blur mask is folded into the y taps: each lane holds, per output
//    row o, the taps g_y[l] M(y0 - R + o + l), so the masked S rows are never
//    formed (M is 0 or 1, so the products are exact);
//  * the ring holds y-blurred rows; the emit blurs over theta first and then
//    along x (the two blurs commute: no mask sits between them), reading the
//    neighbouring lanes' theta-blurred values from a per-wave LDS row instead
//    of chaining lane shifts;
// The shift table (whole-cell offsets and bilinear fractions per channel) is
// computed on the host and read with scalar loads; row offsets go in the
// buffer instructions' scalar offset, which the range check includes.
// The shift table as constant memory: loads at a uniform index become scalar
// loads (the table is not written while a step runs).
typedef const __attribute__((address_space(4))) ShiftEntry* ConstTable;
__device__ inline ConstTable const_table(const ShiftEntry* p) { return (ConstTable)p; }

template <typename T, int R, int TY, int WAVES, int NBUF, typename Args = const StepArgs>
__device__ __forceinline__ void stream2_body(Args& a, const ShiftEntry* __restrict__ tab, const int blk,
                                             const int nblk) {
  constexpr int NT = 64 * WAVES;
  constexpr int NS = TY + 2 * R;   // S rows
  constexpr int NR = NS + 1;       // source rows
  constexpr int GW = WAVES;        // channels per group (one per wave)
  // ring slots: between two barriers a wave emits one group (2R + GW
  // channels) while the group after it is written
  constexpr int RS = 2 * R + 2 * GW;
  constexpr int TAPS = 2 * R + 1;
  constexpr int LP = (TY / 4) % 2 == 1 ? TY : TY + 4;      // odd number of 16-byte units per lane
  constexpr int ZL = 64 + 2 * R;                           // x-blur row: R zero lanes on each side
  constexpr int EB = Elt<T>::BYTES;
  static_assert(TY % 4 == 0, "rows per strip must be a multiple of 4");
  static_assert(NBUF == 1 || NBUF == 2, "one or two source-slice buffers");
  static_assert(sizeof(float) * RS * 64 * LP >= NT * (sizeof(double) + sizeof(float)), "reduction fits the ring");
  // Full-circle schedule, for a workgroup that holds every heading: each
  // channel is warped once, in order, and the emits lag the warps by LW
  // groups, so that no group is padding.  The outputs next to the end of the
  // circle read the first 2R channels' y-blurred rows from RSW + 0 .. 2R - 1,
  // which nothing overwrites; the other channels rotate through RSW slots.
  constexpr bool kCircle = NBUF == 2 && TY == 4;
  constexpr int LW = 1 + (2 * R + GW - 1) / GW;
  constexpr int RSW = (LW + 1) * GW <= 16 ? 16 : 32;
  static_assert((LW + 1) * GW <= RSW, "the circle's live channels fit its slots");
  constexpr int RSA = kCircle ? (RS > RSW + 2 * R ? RS : RSW + 2 * R) : RS;

  __shared__ __attribute__((aligned(16))) float ring[RSA][64][LP];
  __shared__ __attribute__((aligned(16))) float zrow[WAVES][ZL][LP];
  __shared__ int last_flag;
  double* red_s = reinterpret_cast<double*>(&ring[0][0][0]);
  float* red_m = reinterpret_cast<float*>(red_s + NT);

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int H = a.H, pitch = a.pitch, nth = a.n_theta;
  const int64_t sstride = a.sstride;
  const uint32_t row_bytes = static_cast<uint32_t>(pitch) * EB;
  const uint32_t plane_bytes = static_cast<uint32_t>(sstride) * EB;  // < 2^30 (host-checked)
  const int tiles_x = a.tiles_x;
  const int ntile = tiles_x * a.tiles_y;
  const int chunk = blk / ntile, tile = blk % ntile;
  const int strip = a.strip;
  const int xb = (tile % tiles_x) * strip - (R + 1);
  const int y0 = (tile / tiles_x) * TY;
  const int x = xb + lane;
  const int kbeg = chunk * a.chunk_len;
  const int kend = min(nth, kbeg + a.chunk_len);
  const int nk = kend - kbeg;
  const int count = nk + 2 * R;  // relative channels warped: the chunk and R on each side
  const int jbeg = kbeg - R;
  FilterDev* dev = a.dev;
  const int cur = dev->cur;
  const float scale = dev->scale;
  const T* __restrict__ bin = static_cast<const T*>(a.buf[cur]);
  T* __restrict__ bout = static_cast<T*>(a.buf[cur ^ 1]);

  // zero lanes on both sides of every wave's x-blur row
  for (int i = t; i < WAVES * 2 * R * LP; i += NT) {
    const int wv = i / (2 * R * LP), rem = i % (2 * R * LP);
    const int ln = rem / LP, e = rem % LP;
    zrow[wv][ln < R ? ln : 64 + ln][e] = 0.f;
  }
  float gt[TAPS], gx[TAPS];
#pragma unroll
  for (int l = 0; l < TAPS; ++l) {
    gt[l] = a.gth[l];
    gx[l] = a.gxy[l];
  }
  const bool xin = x >= 0 && x < pitch;
  // masked y taps: gm[o][l] = g_y[l] M(row y0 - R + o + l)
  float gm[TY][TAPS];
  {
    float mreg[NS];
#pragma unroll
    for (int r = 0; r < NS; ++r) {
      const int y = y0 - R + r;
      mreg[r] = (xin && y >= 0 && y < H) ? a.mpre[static_cast<int64_t>(y) * pitch + x] : 0.f;
    }
#pragma unroll
    for (int o = 0; o < TY; ++o)
#pragma unroll
      for (int l = 0; l < TAPS; ++l) gm[o][l] = gx[l] * mreg[o + l];
  }
  const bool out_lane = lane >= R + 1 && lane <= R + strip && xin;
  float wreg[TY];
#pragma unroll
  for (int o = 0; o < TY; ++o) {
    const int y = y0 + o;
    wreg[o] = (out_lane && y < H) ? a.wt[static_cast<int64_t>(y) * pitch + x] * scale : 0.f;
  }
  const uint32_t soff = out_lane ? static_cast<uint32_t>(x) * EB : kColOut;
  auto phys = [nth](int j) {
    int k = j % nth;
    return k < 0 ? k + nth : k;
  };
  __syncthreads();  // zero lanes written

  // Byte offsets of a slice's rows from its first row (loop-invariant).  In
  // strips whose slices all start at or below row 0 (no channel shifts its
  // source rows past the grid's top edge) the load descriptor starts at the
  // slice's first row and ends with the plane, so rows past the bottom read 0
  // without per-row checks; the other strips check every row.
  uint32_t rowoff[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) rowoff[r] = static_cast<uint32_t>(r) * row_bytes;
  const bool interior = y0 - R - 1 - a.ny_max >= 0;
  // Cursors: a wave loads and warps relative channels w, w + GW, ... and
  // emits w - 2R, w - 2R + GW, ... in order, so the physical channel, the ring
  // slots and the output plane advance by GW per group.
  int kp_cur = phys(jbeg + w);
  const int gstep = GW % nth;
  int pslot = w;
  int eslot = (w - 2 * R + ((2 * R + GW + RS - 1) / RS) * RS) % RS;
  const uint32_t out_bytes = static_cast<uint32_t>(min(H - y0, TY)) * row_bytes;
  const bool circle = kCircle && a.chunks == 1 && nth >= 2 * R + 2 * GW;
  int lim = count;  // relative channels below lim are warped

  struct Slice {
    float v[NR];
    float fx, fy;
  };
  // Source rows of relative channel c, one group ahead (no branch around the
  // loads: channels past the end read through an empty descriptor).
  auto load_slice = [&](auto mode, int c, Slice& sl) {
    const bool live = c < lim;
    const int kp = kp_cur;
    kp_cur += gstep;
    if (kp_cur >= nth) kp_cur -= nth;
    // uniform index into a table that no workgroup writes: scalar loads
    const ConstTable e = const_table(tab) + kp;
    const int nx = __builtin_amdgcn_readfirstlane(e->nx);
    const int ny = __builtin_amdgcn_readfirstlane(e->ny);
    sl.fx = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, e->fx)));
    sl.fy = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, e->fy)));
    const int cx = x - nx;
    const uint32_t loff = static_cast<unsigned>(cx) < static_cast<unsigned>(pitch) ? static_cast<uint32_t>(cx) * EB
                                                                                    : kColOut;
    const int sy0 = y0 - R - ny - 1;
    const T* plane = bin + static_cast<int64_t>(kp) * sstride;
    if constexpr (decltype(mode)::interior) {
      const uint32_t rows_in = static_cast<uint32_t>(max(H - sy0, 0));
      const __amdgpu_buffer_rsrc_t rs =
          buf_rsrc(plane + static_cast<int64_t>(sy0) * pitch, live ? rows_in * row_bytes : 0u);
#pragma unroll
      for (int r = 0; r < NR; ++r) sl.v[r] = load_row<T>(rs, loff, rowoff[r]);
    } else {
      const __amdgpu_buffer_rsrc_t rs = buf_rsrc(plane, live ? plane_bytes : 0u);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int sy = sy0 + r;
        const uint32_t roff = static_cast<unsigned>(sy) < static_cast<unsigned>(H)
                                  ? static_cast<uint32_t>(sy) * row_bytes
                                  : kRowOut;
        sl.v[r] = load_row<T>(rs, loff, roff);
      }
    }
  };
  // bilinear warp and masked y blur of a slice into a ring slot (and, when
  // keep is set, into a reserved slot as well)
  auto process_into = [&](Slice& sl, float* slot, float* keep) {
    float(&vv)[NR] = sl.v;
    const float fx = sl.fx, fy = sl.fy;
#pragma unroll
    for (int r = 0; r < NR; ++r) vv[r] = fmaf(fx, from_left(vv[r]) - vv[r], vv[r]);
#pragma unroll
    for (int r = 0; r < NS; ++r) vv[r] = fmaf(fy, vv[r] - vv[r + 1], vv[r + 1]);
#pragma unroll
    for (int o4 = 0; o4 < TY; o4 += 4) {
      float p4[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int o = o4 + q;
        float yv = gm[o][0] * vv[o];
#pragma unroll
        for (int l = 1; l < TAPS; ++l) yv = fmaf(gm[o][l], vv[o + l], yv);
        p4[q] = yv;
      }
      *reinterpret_cast<float4*>(slot + o4) = make_float4(p4[0], p4[1], p4[2], p4[3]);
      if (keep) *reinterpret_cast<float4*>(keep + o4) = make_float4(p4[0], p4[1], p4[2], p4[3]);
    }
  };
  // the wave's next channel of the chunk schedule
  auto process = [&](Slice& sl) {
    float* slot = &ring[pslot][lane][0];
    pslot += GW;
    if (pslot >= RS) pslot -= RS;
    process_into(sl, slot, nullptr);
  };
  float psum = 0.f, pmax = 0.f;
  float* zmine = &zrow[w][lane + R][0];
  // Output channel of group g for this wave, in two parts so that the ring
  // reads are in flight while the next group is warped: emit_read issues the
  // theta ring reads; emit_finish blurs over theta into the wave's x-blur row,
  // blurs along x from the neighbouring lanes, applies the post-blur weights,
  // stores and reduces.
  typedef float4 RingRead[TY / 4][TAPS];
  auto emit_read = [&](RingRead& rv) {
    // ring slots of channels krel .. krel + 2R, krel = GW g - 2R + w
    int slot = eslot;
    eslot += GW;
    if (eslot >= RS) eslot -= RS;
#pragma unroll
    for (int l = 0; l < TAPS; ++l) {
#pragma unroll
      for (int b = 0; b < TY / 4; ++b) rv[b][l] = *reinterpret_cast<const float4*>(&ring[slot][lane][4 * b]);
      slot = slot + 1 == RS ? 0 : slot + 1;
    }
  };
  // theta blur of the group's ring rows into the wave's x-blur row
  auto emit_theta = [&](RingRead& rv) {
#pragma unroll
    for (int b = 0; b < TY / 4; ++b) {
      float z[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int l = 0; l < TAPS; ++l) {
        z[0] = fmaf(gt[l], rv[b][l].x, z[0]);
        z[1] = fmaf(gt[l], rv[b][l].y, z[1]);
        z[2] = fmaf(gt[l], rv[b][l].z, z[2]);
        z[3] = fmaf(gt[l], rv[b][l].w, z[3]);
      }
      *reinterpret_cast<float4*>(zmine + 4 * b) = make_float4(z[0], z[1], z[2], z[3]);
    }
  };
  // the neighbouring lanes' theta-blurred values of rows ob .. ob + 3
  auto emit_x_read = [&](int ob, float4 (&zv)[TAPS]) {
#pragma unroll
    for (int l = 0; l < TAPS; ++l) zv[l] = *reinterpret_cast<const float4*>(zmine + (l - R) * LP + ob);
  };
  // output channel krel (relative to the chunk; stores and sums nothing
  // outside it): the descriptor covers the strip's rows inside the grid
  auto out_rsrc = [&](const int krel) {
    const bool live = krel >= 0 && krel < nk;
    const int ko = kbeg + (live ? krel : 0);
    return buf_rsrc(bout + static_cast<int64_t>(ko) * sstride + static_cast<int64_t>(y0) * pitch,
                    live ? out_bytes : 0u);
  };
  // x blur of rows ob .. ob + 3, post-blur weights, stores and the sums
  auto emit_x_finish = [&](int ob, const __amdgpu_buffer_rsrc_t rs, float4 (&zv)[TAPS], float& es, float& em) {
    float o4[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int l = 0; l < TAPS; ++l) {
      o4[0] = fmaf(gx[l], zv[l].x, o4[0]);
      o4[1] = fmaf(gx[l], zv[l].y, o4[1]);
      o4[2] = fmaf(gx[l], zv[l].z, o4[2]);
      o4[3] = fmaf(gx[l], zv[l].w, o4[3]);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int o = ob + e;
      const float ov = o4[e] * wreg[o];
      es += ov;
      em = fmaxf(em, ov);
      store_row<T>(ov, rs, soff, rowoff[o]);
    }
  };
  auto emit_sum = [&](const int krel, float es, float em) {
    if (krel >= 0 && krel < nk) {
      psum += es;
      pmax = fmaxf(pmax, em);
    }
  };
  auto emit_finish_k = [&](const int krel, RingRead& rv) {
    const __amdgpu_buffer_rsrc_t rs = out_rsrc(krel);
    emit_theta(rv);
    // the x-blur row is written and read by this wave only: LDS operations
    // of one wave complete in order, so a wave-scope fence suffices
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float es = 0.f, em = 0.f;
#pragma unroll
    for (int ob = 0; ob < TY; ob += 4) {
      float4 zv[TAPS];
      emit_x_read(ob, zv);
      emit_x_finish(ob, rs, zv, es, em);
    }
    emit_sum(krel, es, em);
  };

  auto emit_finish = [&](int g, RingRead& rv) { emit_finish_k(GW * g - 2 * R + w, rv); };
  // Full-circle schedule: relative channel c (physical c - R) lives in slot
  // c mod RSW, the first 2R also in RSW + c; output k reads relative k .. k + 2R.
  auto process_circle = [&](int h, Slice& sl) {
    const int c = GW * h + w;
    process_into(sl, &ring[c & (RSW - 1)][lane][0], c < 2 * R ? &ring[RSW + c][lane][0] : nullptr);
  };
  auto emit_read_circle = [&](int e, RingRead& rv) {
    // outputs past the last heading store nothing; clamping their first
    // channel keeps every slot index below RSW + 2R
    const int c0 = min(GW * e + w, nth - 1);
#pragma unroll
    for (int l = 0; l < TAPS; ++l) {
      const int c = c0 + l;
      const int slot = c < nth ? (c & (RSW - 1)) : RSW + (c - nth);
#pragma unroll
      for (int b = 0; b < TY / 4; ++b) rv[b][l] = *reinterpret_cast<const float4*>(&ring[slot][lane][4 * b]);
    }
  };

  auto ch = [&](int g) { return GW * g + w; };
  auto pipeline_circle = [&](auto mode) {
    if constexpr (kCircle) {
      lim = nth;
      const int GP = (nth + GW - 1) / GW;  // warp groups; emit group e runs with warp group e + LW
      const ProgressPriority prio(GP + LW);
      Slice sA, sB;
      RingRead rv;
      // group h's slice is sA for even h, sB for odd h; it is loaded while
      // group h - 1 is warped
      // stage h: load group h + 1, warp group h, emit group h - LW
      auto step = [&](int h, Slice& cur_sl, Slice& next_sl, bool emit, bool warp) {
        if (warp) load_slice(mode, ch(h + 1), next_sl);
        if (emit) emit_read_circle(h - LW, rv);
        if (warp) process_circle(h, cur_sl);
        if (emit) emit_finish_k(GW * (h - LW) + w, rv);
        __syncthreads();
      };
      load_slice(mode, ch(0), sA);
      load_slice(mode, ch(1), sB);
      process_circle(0, sA);
      __syncthreads();
#pragma unroll
      for (int h = 1; h < LW; ++h) {
        if (h & 1)
          step(h, sB, sA, false, true);
        else
          step(h, sA, sB, false, true);
      }
      int h = LW;
      for (; h + 1 < GP; h += 2) {
        prio.at(h);
        if constexpr (LW & 1) {
          step(h, sB, sA, true, true);
          step(h + 1, sA, sB, true, true);
        } else {
          step(h, sA, sB, true, true);
          step(h + 1, sB, sA, true, true);
        }
      }
      if (h < GP) {
        if constexpr (LW & 1)
          step(h, sB, sA, true, true);
        else
          step(h, sA, sB, true, true);
        ++h;
      }
#pragma unroll
      for (int i = 0; i < LW; ++i) {
        prio.at(GP + i);
        step(GP + i, sA, sB, true, false);
      }
    }
  };
  auto pipeline = [&](auto mode) {
    // Software pipeline: between two barriers a wave emits group g - 1 and
    // warps group g (their ring slots are distinct), so the emit's LDS reads
    // are in flight during the warp.  Channels past the end (the last groups)
    // load through empty descriptors and their emits store nothing.
    if constexpr (NBUF == 2) {
      const int G = (((count + GW - 1) / GW) + 1) & ~1;  // even: the last may be padding
      const ProgressPriority prio(G);
      Slice sA, sB;
      RingRead rv;
      load_slice(mode, ch(0), sA);
      load_slice(mode, ch(1), sB);
      process(sA);
      __syncthreads();
      for (int g = 1; g <= G; g += 2) {
        prio.at(g);
        load_slice(mode, ch(g + 1), sA);
        emit_read(rv);
        process(sB);
        emit_finish(g - 1, rv);
        __syncthreads();
        load_slice(mode, ch(g + 2), sB);
        emit_read(rv);
        process(sA);
        emit_finish(g, rv);
        __syncthreads();
      }
    } else {
      const int G = (count + GW - 1) / GW;
      const ProgressPriority prio(G);
      Slice sA;
      RingRead rv;
      load_slice(mode, ch(0), sA);
      process(sA);
      load_slice(mode, ch(1), sA);
      __syncthreads();
      for (int g = 1; g <= G; ++g) {
        prio.at(g);
        emit_read(rv);
        process(sA);
        load_slice(mode, ch(g + 1), sA);
        emit_finish(g - 1, rv);
        __syncthreads();
      }
    }
  };
  if (circle) {
    if (interior)
      pipeline_circle(RowMode<true>{});
    else
      pipeline_circle(RowMode<false>{});
  } else {
    if (interior)
      pipeline(RowMode<true>{});
    else
      pipeline(RowMode<false>{});
  }
  __syncthreads();  // the ring becomes the reduction buffer

  red_s[t] = static_cast<double>(psum);
  red_m[t] = pmax;
  __syncthreads();
  static_assert((NT & (NT - 1)) == 0, "the tree reduction needs a power-of-two workgroup");
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (t < s) {
      red_s[t] += red_s[t + s];
      red_m[t] = fmaxf(red_m[t], red_m[t + s]);
    }
    __syncthreads();
  }
  if (t == 0) {
    publish(&a.partials[2 * blk], red_s[0]);
    publish(&a.partials[2 * blk + 1], static_cast<double>(red_m[0]));
    last_flag = arrive_last(dev, static_cast<uint32_t>(blk), static_cast<uint32_t>(nblk));
  }
  __syncthreads();
  if (!last_flag) return;
  finalize_step<NT>(a, dev, nblk, scale, cur, red_s, red_m);
}

// ---- streaming variant with the emit split by rows ----------------------------------
// As stream2_body (mask in the y taps, theta blur before the x blur, host
// shift table), but after each group's barrier wave w emits output row(s)
// w RW .. (w + 1) RW - 1 of all GW channels of the group instead of every row
// of one channel.  The theta blur of GW channels reads the 2R + GW ring slots
// once per row (ring layout [slot][row][lane]), so the ring is read
// (2R + GW) / (GW (2R + 1)) as often as with one channel per wave.  The post-
// blur weights are folded into the x taps of the wave's rows.
template <typename T, int R, int TY, int WAVES, int NBUF, typename Args = const StepArgs>
__device__ __forceinline__ void stream3_body(Args& a, const ShiftEntry* __restrict__ tab, const int blk,
                                             const int nblk) {
  constexpr int NT = 64 * WAVES;
  constexpr int NS = TY + 2 * R;   // S rows
  constexpr int NR = NS + 1;       // source rows
  constexpr int GW = WAVES;        // channels per group (one per wave)
  constexpr int RW = TY / GW;      // output rows each wave emits
  constexpr bool ONE_BARRIER = WAVES <= 4;
  constexpr int RS = 2 * R + (ONE_BARRIER ? 2 : 1) * GW;  // ring slots (as stream_body)
  constexpr int TAPS = 2 * R + 1;
  constexpr int NSL = GW + 2 * R;                         // ring slots one emit reads
  constexpr int ZV = GW * RW;                             // theta-blurred values per lane and emit
  constexpr int ZP = (ZV / 4) % 2 == 1 ? ZV : ZV + 4;     // odd number of 16-byte units per lane
  constexpr int ZL = 64 + 2 * R;                          // x-blur row: R zero lanes on each side
  constexpr int EB = Elt<T>::BYTES;
  static_assert(TY % GW == 0 && RW >= 1, "rows per strip must be a multiple of the waves");
  static_assert(ZV % 4 == 0, "four theta-blurred values per 16-byte word");
  static_assert(NBUF == 1 || NBUF == 2, "one or two source-slice buffers");
  static_assert(sizeof(float) * RS * TY * 64 >= NT * (sizeof(double) + sizeof(float)), "reduction fits the ring");

  __shared__ __attribute__((aligned(16))) float ring[RS][TY][64];
  __shared__ __attribute__((aligned(16))) float zrow[WAVES][ZL][ZP];
  __shared__ int last_flag;
  double* red_s = reinterpret_cast<double*>(&ring[0][0][0]);
  float* red_m = reinterpret_cast<float*>(red_s + NT);

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int H = a.H, pitch = a.pitch, nth = a.n_theta;
  const int64_t sstride = a.sstride;
  const uint32_t row_bytes = static_cast<uint32_t>(pitch) * EB;
  const uint32_t plane_bytes = static_cast<uint32_t>(sstride) * EB;  // < 2^30 (host-checked)
  const int tiles_x = a.tiles_x;
  const int ntile = tiles_x * a.tiles_y;
  const int chunk = blk / ntile, tile = blk % ntile;
  const int strip = a.strip;
  const int xb = (tile % tiles_x) * strip - (R + 1);
  const int y0 = (tile / tiles_x) * TY;
  const int x = xb + lane;
  const int kbeg = chunk * a.chunk_len;
  const int kend = min(nth, kbeg + a.chunk_len);
  const int nk = kend - kbeg;
  const int count = nk + 2 * R;  // relative channels warped: the chunk and R on each side
  const int jbeg = kbeg - R;
  FilterDev* dev = a.dev;
  const int cur = dev->cur;
  const float scale = dev->scale;
  const T* __restrict__ bin = static_cast<const T*>(a.buf[cur]);
  T* __restrict__ bout = static_cast<T*>(a.buf[cur ^ 1]);

  // zero lanes on both sides of every wave's x-blur row
  for (int i = t; i < WAVES * 2 * R * ZP; i += NT) {
    const int wv = i / (2 * R * ZP), rem = i % (2 * R * ZP);
    const int ln = rem / ZP, e = rem % ZP;
    zrow[wv][ln < R ? ln : 64 + ln][e] = 0.f;
  }
  float gt[TAPS], gx[TAPS];
#pragma unroll
  for (int l = 0; l < TAPS; ++l) {
    gt[l] = a.gth[l];
    gx[l] = a.gxy[l];
  }
  const bool xin = x >= 0 && x < pitch;
  // masked y taps: gm[o][l] = g_y[l] M(row y0 - R + o + l)
  float gm[TY][TAPS];
  {
    float mreg[NS];
#pragma unroll
    for (int r = 0; r < NS; ++r) {
      const int y = y0 - R + r;
      mreg[r] = (xin && y >= 0 && y < H) ? a.mpre[static_cast<int64_t>(y) * pitch + x] : 0.f;
    }
#pragma unroll
    for (int o = 0; o < TY; ++o)
#pragma unroll
      for (int l = 0; l < TAPS; ++l) gm[o][l] = gx[l] * mreg[o + l];
  }
  // x taps weighted by the post-blur weights of this wave's output rows
  const bool out_lane = lane >= R + 1 && lane <= R + strip && xin;
  float wx[RW][TAPS];
#pragma unroll
  for (int rr = 0; rr < RW; ++rr) {
    const int y = y0 + w * RW + rr;
    const float wv = (out_lane && y < H) ? a.wt[static_cast<int64_t>(y) * pitch + x] * scale : 0.f;
#pragma unroll
    for (int l = 0; l < TAPS; ++l) wx[rr][l] = gx[l] * wv;
  }
  const uint32_t soff = out_lane ? static_cast<uint32_t>(x) * EB : kColOut;
  auto phys = [nth](int j) {
    int k = j % nth;
    return k < 0 ? k + nth : k;
  };
  __syncthreads();  // zero lanes written

  struct Slice {
    float v[NR];
    float fx, fy;
  };
  // Source rows of relative channel c, one group ahead (no branch around the
  // loads: channels past the end read through an empty descriptor).
  auto load_slice = [&](int c, Slice& sl) {
    const bool live = c < count;
    const int kp = phys(jbeg + (live ? c : 0));
    // uniform index into a table that no workgroup writes: scalar loads
    const ConstTable e = const_table(tab) + kp;
    const int nx = __builtin_amdgcn_readfirstlane(e->nx);
    const int ny = __builtin_amdgcn_readfirstlane(e->ny);
    sl.fx = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, e->fx)));
    sl.fy = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, e->fy)));
    const int cx = x - nx;
    const uint32_t loff = static_cast<unsigned>(cx) < static_cast<unsigned>(pitch) ? static_cast<uint32_t>(cx) * EB
                                                                                    : kColOut;
    const int sy0 = y0 - R - ny - 1;
    const __amdgpu_buffer_rsrc_t rs = buf_rsrc(bin + static_cast<int64_t>(kp) * sstride, live ? plane_bytes : 0u);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int sy = sy0 + r;
      const uint32_t roff = static_cast<unsigned>(sy) < static_cast<unsigned>(H) ? static_cast<uint32_t>(sy) * row_bytes
                                                                                 : kRowOut;
      sl.v[r] = load_row<T>(rs, loff, roff);
    }
  };
  // bilinear warp (y, then x) and masked y blur of relative channel c into its ring slot
  auto process = [&](int c, Slice& sl) {
    float(&vv)[NR] = sl.v;
    const float fx = sl.fx, fy = sl.fy;
#pragma unroll
    for (int r = 0; r < NS; ++r) vv[r] = fmaf(fy, vv[r] - vv[r + 1], vv[r + 1]);
#pragma unroll
    for (int r = 0; r < NS; ++r) vv[r] = fmaf(fx, from_left(vv[r]) - vv[r], vv[r]);
    const int sl_ = c % RS;
#pragma unroll
    for (int o = 0; o < TY; ++o) {
      float yv = gm[o][0] * vv[o];
#pragma unroll
      for (int l = 1; l < TAPS; ++l) yv = fmaf(gm[o][l], vv[o + l], yv);
      ring[sl_][o][lane] = yv;
    }
  };
  float psum = 0.f, pmax = 0.f;
  float* zmine = &zrow[w][lane + R][0];
  // Group g's output channels GW g - 2R .. GW g - 2R + GW - 1, rows of this
  // wave: theta blur from the ring into the wave's x-blur row, x blur (with
  // the post-blur weights) from the neighbouring lanes, store, reduce.
  auto emit = [&](int g) {
    const int k0 = GW * g - 2 * R;
    // ring slots of channels k0 .. k0 + GW - 1 + 2R; k0 >= -(2R + GW)
    // (padding emits), so a multiple of RS keeps the modulus non-negative
    constexpr int OFF = ((2 * R + GW + RS - 1) / RS) * RS;
    int slot[NSL];
    slot[0] = (k0 + OFF) % RS;
#pragma unroll
    for (int i = 1; i < NSL; ++i) slot[i] = slot[i - 1] + 1 == RS ? 0 : slot[i - 1] + 1;
    float z[ZV];
#pragma unroll
    for (int rr = 0; rr < RW; ++rr) {
      const int o = w * RW + rr;
      float rv[NSL];
#pragma unroll
      for (int i = 0; i < NSL; ++i) rv[i] = ring[slot[i]][o][lane];
#pragma unroll
      for (int q = 0; q < GW; ++q) {
        float acc = gt[0] * rv[q];
#pragma unroll
        for (int l = 1; l < TAPS; ++l) acc = fmaf(gt[l], rv[q + l], acc);
        z[q * RW + rr] = acc;
      }
    }
#pragma unroll
    for (int i = 0; i < ZV; i += 4) *reinterpret_cast<float4*>(zmine + i) = make_float4(z[i], z[i + 1], z[i + 2], z[i + 3]);
    // the x-blur row is written and read by this wave only: LDS operations
    // of one wave complete in order, so a wave-scope fence suffices
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float acc[ZV];
#pragma unroll
    for (int i = 0; i < ZV; ++i) acc[i] = wx[i % RW][R] * z[i];
#pragma unroll
    for (int l = 0; l < TAPS; ++l) {
      if (l == R) continue;
#pragma unroll
      for (int i = 0; i < ZV; i += 4) {
        const float4 nv = *reinterpret_cast<const float4*>(zmine + (l - R) * ZP + i);
        acc[i] = fmaf(wx[i % RW][l], nv.x, acc[i]);
        acc[i + 1] = fmaf(wx[(i + 1) % RW][l], nv.y, acc[i + 1]);
        acc[i + 2] = fmaf(wx[(i + 2) % RW][l], nv.z, acc[i + 2]);
        acc[i + 3] = fmaf(wx[(i + 3) % RW][l], nv.w, acc[i + 3]);
      }
    }
#pragma unroll
    for (int q = 0; q < GW; ++q) {
      const int kr = k0 + q;
      const bool live = kr >= 0 && kr < nk;
      const int ko = kbeg + (live ? kr : 0);
      const __amdgpu_buffer_rsrc_t rs = buf_rsrc(bout + static_cast<int64_t>(ko) * sstride, live ? plane_bytes : 0u);
      float es = 0.f, em = 0.f;
#pragma unroll
      for (int rr = 0; rr < RW; ++rr) {
        const float ov = acc[q * RW + rr];
        es += ov;
        em = fmaxf(em, ov);
        const int y = y0 + w * RW + rr;
        const uint32_t roff = y < H ? static_cast<uint32_t>(y) * row_bytes : kRowOut;
        store_row<T>(ov, rs, soff, roff);
      }
      if (live) {
        psum += es;
        pmax = fmaxf(pmax, em);
      }
    }
  };

  auto ch = [&](int g) { return GW * g + w; };
  if constexpr (NBUF == 2) {
    const int G = (((count + GW - 1) / GW) + 1) & ~1;
    Slice sA, sB;
    load_slice(ch(0), sA);
    emit(-1);
    for (int g = 0; g < G; g += 2) {
      load_slice(ch(g + 1), sB);
      process(ch(g), sA);
      __syncthreads();
      emit(g);
      if (!ONE_BARRIER) __syncthreads();
      load_slice(ch(g + 2), sA);
      process(ch(g + 1), sB);
      __syncthreads();
      emit(g + 1);
      if (!ONE_BARRIER) __syncthreads();
    }
  } else {
    const int G = (count + GW - 1) / GW;
    Slice sA;
    load_slice(ch(0), sA);
    emit(-1);
    for (int g = 0; g < G; ++g) {
      process(ch(g), sA);
      load_slice(ch(g + 1), sA);
      __syncthreads();
      emit(g);
      if (!ONE_BARRIER) __syncthreads();
    }
  }
  __syncthreads();  // the ring becomes the reduction buffer

  red_s[t] = static_cast<double>(psum);
  red_m[t] = pmax;
  __syncthreads();
  static_assert((NT & (NT - 1)) == 0, "the tree reduction needs a power-of-two workgroup");
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (t < s) {
      red_s[t] += red_s[t + s];
      red_m[t] = fmaxf(red_m[t], red_m[t + s]);
    }
    __syncthreads();
  }
  if (t == 0) {
    publish(&a.partials[2 * blk], red_s[0]);
    publish(&a.partials[2 * blk + 1], static_cast<double>(red_m[0]));
    last_flag = arrive_last(dev, static_cast<uint32_t>(blk), static_cast<uint32_t>(nblk));
  }
  __syncthreads();
  if (!last_flag) return;
  finalize_step<NT>(a, dev, nblk, scale, cur, red_s, red_m);
}

template <typename T, int R, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void step_single(StepArgs a) {
  const int n = a.tiles_x * a.tiles_y * a.chunks;
  step_body<T, R, TX, TY, NT>(a, xcd_remap(blockIdx.x, n), n);
}

template <typename T, int R, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void step_batch(const StepArgs* __restrict__ jobs,
                                                 const int32_t* __restrict__ first, int njobs, int total) {
  const int g = xcd_remap(blockIdx.x, total);
  const int j = find_job(first, njobs, g);
  int blk = 0;
  const auto& a = job_args(jobs, first, j, g, blk);
  const int n = a.tiles_x * a.tiles_y * a.chunks;
  step_body<T, R, TX, TY, NT>(a, blk, n);
}

// Eight-wave workgroups aim at six waves per SIMD (three workgroups per
// compute unit), which caps the register budget.
template <int WAVES>
constexpr int stream_waves_per_eu() {
  return WAVES >= 8 ? 6 : 1;
}
// The variant-1 kernel's 4-row, 4-wave shape is launched with five waves per
// SIMD at 512 x 512 (1280 workgroups); at four it ran 56.5 against 41.4 us.
template <int TY, int WAVES>
constexpr int stream2_waves_per_eu() {
  return TY == 4 && WAVES == 4 ? 5 : stream_waves_per_eu<WAVES>();
}

template <typename T, int R, int TY, int WAVES, int NBUF>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(stream_waves_per_eu<WAVES>())))
void stream_single(StepArgs a, ShiftArgs tab) {
  const int n = a.tiles_x * a.tiles_y * a.chunks;
  stream_body<T, R, TY, WAVES, NBUF>(a, a.table ? a.table : tab.e, xcd_remap(blockIdx.x, n), n);
}

template <typename T, int R, int TY, int WAVES, int NBUF>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(stream_waves_per_eu<WAVES>())))
void stream_batch(const StepArgs* __restrict__ jobs,
                                                           const int32_t* __restrict__ first, int njobs, int total) {
  const int g = xcd_remap(blockIdx.x, total);
  const int j = find_job(first, njobs, g);
  int blk = 0;
  const auto& a = job_args(jobs, first, j, g, blk);
  const int n = a.tiles_x * a.tiles_y * a.chunks;
  stream_body<T, R, TY, WAVES, NBUF>(a, a.table, blk, n);
}

template <typename T, int R, int TY, int WAVES, int NBUF>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(stream2_waves_per_eu<TY, WAVES>())))
void stream2_single(StepArgs a, ShiftArgs tab) {
  const int n = a.tiles_x * a.tiles_y * a.chunks;
  stream2_body<T, R, TY, WAVES, NBUF>(a, a.table ? a.table : tab.e, xcd_remap(blockIdx.x, n), n);
}

template <typename T, int R, int TY, int WAVES, int NBUF>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(stream2_waves_per_eu<TY, WAVES>())))
void stream2_batch(const StepArgs* __restrict__ jobs, const int32_t* __restrict__ first, int njobs, int total) {
  const int g = xcd_remap(blockIdx.x, total);
  const int j = find_job(first, njobs, g);
  int blk = 0;
  const auto& a = job_args(jobs, first, j, g, blk);
  const int n = a.tiles_x * a.tiles_y * a.chunks;
  stream2_body<T, R, TY, WAVES, NBUF>(a, a.table, blk, n);
}

template <typename T, int R, int TY, int WAVES, int NBUF>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(stream_waves_per_eu<WAVES>())))
void stream3_single(StepArgs a, ShiftArgs tab) {
  const int n = a.tiles_x * a.tiles_y * a.chunks;
  stream3_body<T, R, TY, WAVES, NBUF>(a, a.table ? a.table : tab.e, xcd_remap(blockIdx.x, n), n);
}

template <typename T, int R, int TY, int WAVES, int NBUF>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(stream_waves_per_eu<WAVES>())))
void stream3_batch(const StepArgs* __restrict__ jobs, const int32_t* __restrict__ first, int njobs, int total) {
  const int g = xcd_remap(blockIdx.x, total);
  const int j = find_job(first, njobs, g);
  int blk = 0;
  const auto& a = job_args(jobs, first, j, g, blk);
  const int n = a.tiles_x * a.tiles_y * a.chunks;
  stream3_body<T, R, TY, WAVES, NBUF>(a, a.table, blk, n);
}

template <typename T, int R, int TX, int TY, int NT>
hipError_t launch_tiled(const StepArgs* single, const StepArgs* jobs, const int32_t* first, int njobs, int total,
                        hipStream_t s) {
  if (single) {
    const int n = single->tiles_x * single->tiles_y * single->chunks;
    hipLaunchKernelGGL((step_single<T, R, TX, TY, NT>), dim3(n), dim3(NT), 0, s, *single);
  } else {
    hipLaunchKernelGGL((step_batch<T, R, TX, TY, NT>), dim3(total), dim3(NT), 0, s, jobs, first, njobs, total);
  }
  return hipGetLastError();
}

template <typename T, int R, int TY, int WAVES, int NBUF>
hipError_t launch_stream(const StepArgs* single, const ShiftArgs* tab, const StepArgs* jobs, const int32_t* first,
                         int njobs, int total, int max_theta, hipStream_t s) {
  const size_t table = static_cast<size_t>(max_theta) * 4 * sizeof(int);
  if (single) {
    const int n = single->tiles_x * single->tiles_y * single->chunks;
    if (!single->table && !tab) return hipErrorInvalidValue;
    static const ShiftArgs kNone = {};
    hipLaunchKernelGGL((stream_single<T, R, TY, WAVES, NBUF>), dim3(n), dim3(64 * WAVES), table, s, *single,
                       single->table ? kNone : *tab);
  } else {
    hipLaunchKernelGGL((stream_batch<T, R, TY, WAVES, NBUF>), dim3(total), dim3(64 * WAVES), table, s, jobs, first,
                       njobs, total);
  }
  return hipGetLastError();
}

template <typename T, int R, int TY, int WAVES, int NBUF>
hipError_t launch_stream2(const StepArgs* single, const ShiftArgs* tab, const StepArgs* jobs, const int32_t* first,
                          int njobs, int total, hipStream_t s) {
  if (single) {
    const int n = single->tiles_x * single->tiles_y * single->chunks;
    if (!single->table && !tab) return hipErrorInvalidValue;
    static const ShiftArgs kNone = {};
    hipLaunchKernelGGL((stream2_single<T, R, TY, WAVES, NBUF>), dim3(n), dim3(64 * WAVES), 0, s, *single,
                       single->table ? kNone : *tab);
  } else {
    hipLaunchKernelGGL((stream2_batch<T, R, TY, WAVES, NBUF>), dim3(total), dim3(64 * WAVES), 0, s, jobs, first, njobs,
                       total);
  }
  return hipGetLastError();
}

template <typename T, int R, int TY, int WAVES, int NBUF>
hipError_t launch_stream3(const StepArgs* single, const ShiftArgs* tab, const StepArgs* jobs, const int32_t* first,
                          int njobs, int total, hipStream_t s) {
  if (single) {
    const int n = single->tiles_x * single->tiles_y * single->chunks;
    if (!single->table && !tab) return hipErrorInvalidValue;
    static const ShiftArgs kNone = {};
    hipLaunchKernelGGL((stream3_single<T, R, TY, WAVES, NBUF>), dim3(n), dim3(64 * WAVES), 0, s, *single,
                       single->table ? kNone : *tab);
  } else {
    hipLaunchKernelGGL((stream3_batch<T, R, TY, WAVES, NBUF>), dim3(total), dim3(64 * WAVES), 0, s, jobs, first, njobs,
                       total);
  }
  return hipGetLastError();
}

// Instantiated launch shapes.  Tiled kernel: (TX, TY, NT).  Streaming
// kernel: (TY rows per strip, waves, source-slice buffers).
#define MCL_SHAPES(X) X(64, 16, 256) X(32, 16, 128)
#define MCL_STREAM_SHAPES(X) X(4, 4, 2) X(8, 4, 2) X(12, 4, 2) X(16, 4, 2) X(4, 8, 1) X(8, 8, 1) X(16, 8, 1)
// Variant-1 streaming kernel: (TY rows per strip, waves, source-slice buffers).
#define MCL_STREAM2_SHAPES(X) X(4, 4, 2) X(8, 4, 2) X(4, 8, 1) X(8, 8, 1) X(4, 4, 1) X(8, 4, 1)
// Variant-2 streaming kernel (rows per strip a multiple of the waves).
#define MCL_STREAM3_SHAPES(X) X(4, 4, 2) X(8, 4, 2) X(4, 4, 1) X(8, 4, 1) X(8, 8, 1)

template <typename T, int R>
hipError_t dispatch_shape(const KernelShape& k, const StepArgs* single, const ShiftArgs* tab, const StepArgs* jobs,
                          const int32_t* bj, int nj, int total, int max_theta, hipStream_t s) {
#define MCL_TRY_STREAM2(TY_, WV_, NB_)                                                     \
  if (k.tx == 0 && k.variant == 1 && k.ty == TY_ && k.nt == 64 * WV_ && k.nbuf == NB_) \
    return launch_stream2<T, R, TY_, WV_, NB_>(single, tab, jobs, bj, nj, total, s);
  MCL_STREAM2_SHAPES(MCL_TRY_STREAM2)
#undef MCL_TRY_STREAM2
#define MCL_TRY_STREAM3(TY_, WV_, NB_)                                                     \
  if (k.tx == 0 && k.variant == 2 && k.ty == TY_ && k.nt == 64 * WV_ && k.nbuf == NB_) \
    return launch_stream3<T, R, TY_, WV_, NB_>(single, tab, jobs, bj, nj, total, s);
  MCL_STREAM3_SHAPES(MCL_TRY_STREAM3)
#undef MCL_TRY_STREAM3
  if (k.variant != 0) return hipErrorInvalidValue;
#define MCL_TRY_STREAM(TY_, WV_, NB_)                                     \
  if (k.tx == 0 && k.ty == TY_ && k.nt == 64 * WV_ && k.nbuf == NB_) \
    return launch_stream<T, R, TY_, WV_, NB_>(single, tab, jobs, bj, nj, total, max_theta, s);
  MCL_STREAM_SHAPES(MCL_TRY_STREAM)
#undef MCL_TRY_STREAM
#define MCL_TRY(TX_, TY_, NT_)                        \
  if (k.tx == TX_ && k.ty == TY_ && k.nt == NT_) \
    return launch_tiled<T, R, TX_, TY_, NT_>(single, jobs, bj, nj, total, s);
  MCL_SHAPES(MCL_TRY)
#undef MCL_TRY
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t dispatch_radius(int radius, const KernelShape& k, const StepArgs* single, const ShiftArgs* tab,
                           const StepArgs* jobs, const int32_t* bj, int nj, int total, int max_theta, hipStream_t s) {
  switch (radius) {
    case 1: return dispatch_shape<T, 1>(k, single, tab, jobs, bj, nj, total, max_theta, s);
    case 2: return dispatch_shape<T, 2>(k, single, tab, jobs, bj, nj, total, max_theta, s);
    case 3: return dispatch_shape<T, 3>(k, single, tab, jobs, bj, nj, total, max_theta, s);
    case 4: return dispatch_shape<T, 4>(k, single, tab, jobs, bj, nj, total, max_theta, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t dispatch(int dtype, int radius, const KernelShape& k, const StepArgs* single, const ShiftArgs* tab,
                    const StepArgs* jobs, const int32_t* bj, int nj, int total, int max_theta, hipStream_t s) {
  switch (dtype) {
    case 0: return dispatch_radius<float>(radius, k, single, tab, jobs, bj, nj, total, max_theta, s);
    case 1: return dispatch_radius<__bf16>(radius, k, single, tab, jobs, bj, nj, total, max_theta, s);
    case 2: return dispatch_radius<_Float16>(radius, k, single, tab, jobs, bj, nj, total, max_theta, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool step_config_supported(int dtype, int radius, const KernelShape& k) {
  if (dtype < 0 || dtype > 2 || radius < 1 || radius > kMaxRadius) return false;
#define MCL_HAS(TX_, TY_, NT_) \
  if (k.tx == TX_ && k.ty == TY_ && k.nt == NT_ && k.variant == 0) return true;
  MCL_SHAPES(MCL_HAS)
#undef MCL_HAS
#define MCL_HAS_STREAM2(TY_, WV_, NB_) \
  if (k.tx == 0 && k.variant == 1 && k.ty == TY_ && k.nt == 64 * WV_ && k.nbuf == NB_) return true;
  MCL_STREAM2_SHAPES(MCL_HAS_STREAM2)
#undef MCL_HAS_STREAM2
#define MCL_HAS_STREAM3(TY_, WV_, NB_) \
  if (k.tx == 0 && k.variant == 2 && k.ty == TY_ && k.nt == 64 * WV_ && k.nbuf == NB_) return true;
  MCL_STREAM3_SHAPES(MCL_HAS_STREAM3)
#undef MCL_HAS_STREAM3
  if (k.variant != 0) return false;
#define MCL_HAS_STREAM(TY_, WV_, NB_) \
  if (k.tx == 0 && k.ty == TY_ && k.nt == 64 * WV_ && k.nbuf == NB_) return true;
  MCL_STREAM_SHAPES(MCL_HAS_STREAM)
#undef MCL_HAS_STREAM
  return false;
}

hipError_t launch_step(int dtype, int radius, const KernelShape& k, const StepArgs& a, const ShiftArgs* tab,
                       hipStream_t s) {
  return dispatch(dtype, radius, k, &a, tab, nullptr, nullptr, 0, 0, a.n_theta, s);
}

hipError_t launch_step_batch(int dtype, int radius, const KernelShape& k, const StepArgs* jobs_dev,
                             const int32_t* first_dev, int32_t njobs, int32_t total_blocks, int32_t max_theta,
                             hipStream_t s) {
  return dispatch(dtype, radius, k, nullptr, nullptr, jobs_dev, first_dev, njobs, total_blocks, max_theta, s);
}

}  // namespace mcl
