// Device-side building blocks shared by the dynamic-screening kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ds {

constexpr int WAVE = 64;

typedef uint16_t bf16_t;  // bfloat16 bit pattern

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

// Storage traits.  VEC = elements per 16-byte load; V = vector (y, x, theta) type;
// A = accumulation type of the streaming GEMVs.  Products of float (or bfloat16) values
// are exact in FP64, so FP64 accumulation leaves only the summation rounding (~N 2^-53):
// the rounding slack of the dual scaling becomes negligible, and the extra FP64 FMA per
// element is far below the FP64 rate of the chip at HBM speed.
template <typename T> struct Store;
template <> struct Store<double> { using V = double; using A = double; static constexpr int VEC = 2; };
template <> struct Store<float>  { using V = float;  using A = double; static constexpr int VEC = 4; };
template <> struct Store<bf16_t> { using V = float;  using A = double; static constexpr int VEC = 8; };

// 16-byte load of VEC consecutive stored elements, widened to A.
template <typename T, typename A>
__device__ __forceinline__ void load_vec(const T* __restrict__ p, A (&out)[Store<T>::VEC]);

template <>
__device__ __forceinline__ void load_vec<double, double>(const double* __restrict__ p, double (&o)[2]) {
  const double2 v = *reinterpret_cast<const double2*>(p);
  o[0] = v.x; o[1] = v.y;
}
template <>
__device__ __forceinline__ void load_vec<float, float>(const float* __restrict__ p, float (&o)[4]) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
template <>
__device__ __forceinline__ void load_vec<bf16_t, float>(const bf16_t* __restrict__ p, float (&o)[8]) {
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  o[0] = __uint_as_float(v.x << 16); o[1] = __uint_as_float(v.x & 0xffff0000u);
  o[2] = __uint_as_float(v.y << 16); o[3] = __uint_as_float(v.y & 0xffff0000u);
  o[4] = __uint_as_float(v.z << 16); o[5] = __uint_as_float(v.z & 0xffff0000u);
  o[6] = __uint_as_float(v.w << 16); o[7] = __uint_as_float(v.w & 0xffff0000u);
}
// Same widths, double accumulation (setup passes: products of stored values are exact
// in FP64 for float and bfloat16 storage).
template <>
__device__ __forceinline__ void load_vec<float, double>(const float* __restrict__ p, double (&o)[4]) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
template <>
__device__ __forceinline__ void load_vec<bf16_t, double>(const bf16_t* __restrict__ p, double (&o)[8]) {
  float f[8];
  load_vec<bf16_t, float>(p, f);
#pragma unroll
  for (int k = 0; k < 8; ++k) o[k] = f[k];
}

template <typename T> __device__ __forceinline__ double to_double(T v);
template <> __device__ __forceinline__ double to_double<double>(double v) { return v; }
template <> __device__ __forceinline__ double to_double<float>(float v) { return v; }
template <> __device__ __forceinline__ double to_double<bf16_t>(bf16_t v) { return bf16_to_f32(v); }


// ---------------------------------------------------------------- reductions ------
// Wave reductions on the data-parallel primitives of the vector ALU: two quad
// permutations and the half-row and row mirrors leave the sum (max, min) of each row of
// 16 lanes in every lane of the row, then the four row results are combined with lane
// reads in row order.  The combination tree is fixed, so the result is deterministic and
// the same in every lane.  All 64 lanes must be active.
namespace dpp {
constexpr int QUAD_1032 = 0xB1;    // quad_perm [1, 0, 3, 2]
constexpr int QUAD_2301 = 0x4E;    // quad_perm [2, 3, 0, 1]
constexpr int HALF_MIRROR = 0x141;  // lane j of 8 reads lane 7 - j
constexpr int ROW_MIRROR = 0x140;   // lane j of 16 reads lane 15 - j

template <int C> __device__ __forceinline__ int mov(int v) {
  return __builtin_amdgcn_update_dpp(0, v, C, 0xf, 0xf, false);
}
template <int C> __device__ __forceinline__ int64_t mov(int64_t v) {
  const int lo = mov<C>(static_cast<int>(v)), hi = mov<C>(static_cast<int>(v >> 32));
  return static_cast<int64_t>((static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                              static_cast<uint32_t>(lo));
}
template <int C> __device__ __forceinline__ uint64_t mov(uint64_t v) {
  return static_cast<uint64_t>(mov<C>(static_cast<int64_t>(v)));
}
template <int C> __device__ __forceinline__ unsigned mov(unsigned v) {
  return static_cast<unsigned>(mov<C>(static_cast<int>(v)));
}
template <int C> __device__ __forceinline__ float mov(float v) {
  return __int_as_float(mov<C>(__float_as_int(v)));
}
template <int C> __device__ __forceinline__ double mov(double v) {
  return __hiloint2double(mov<C>(__double2hiint(v)), mov<C>(__double2loint(v)));
}
__device__ __forceinline__ int lane_read(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ unsigned lane_read(unsigned v, int l) {
  return static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(v), l));
}
__device__ __forceinline__ int64_t lane_read(int64_t v, int l) {
  const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), l));
  const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v >> 32), l));
  return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}
__device__ __forceinline__ uint64_t lane_read(uint64_t v, int l) {
  return static_cast<uint64_t>(lane_read(static_cast<int64_t>(v), l));
}
__device__ __forceinline__ float lane_read(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_read(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
template <typename X, typename Op>
__device__ __forceinline__ X reduce(X v, Op op) {
  v = op(v, mov<QUAD_1032>(v));
  v = op(v, mov<QUAD_2301>(v));
  v = op(v, mov<HALF_MIRROR>(v));
  v = op(v, mov<ROW_MIRROR>(v));
  return op(op(op(lane_read(v, 0), lane_read(v, 16)), lane_read(v, 32)), lane_read(v, 48));
}
}  // namespace dpp

template <typename X>
__device__ __forceinline__ X wave_sum(X v) {
  return dpp::reduce(v, [](X p, X q) { return p + q; });
}
template <typename X>
__device__ __forceinline__ X wave_max(X v) {
  return dpp::reduce(v, [](X p, X q) { return q > p ? q : p; });
}
template <typename X>
__device__ __forceinline__ X wave_min(X v) {
  return dpp::reduce(v, [](X p, X q) { return q < p ? q : p; });
}

// Block-wide reductions with a fixed combination order (deterministic).  `scratch`
// must hold one X per wave; the result is returned to every thread.
template <typename X, int NWAVES>
__device__ __forceinline__ X block_sum(X v, X* scratch) {
  v = wave_sum(v);
  const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
  __syncthreads();
  if (l == 0) scratch[w] = v;
  __syncthreads();
  X s = scratch[0];
#pragma unroll
  for (int k = 1; k < NWAVES; ++k) s += scratch[k];
  return s;
}
template <typename X, int NWAVES>
__device__ __forceinline__ X block_max(X v, X* scratch) {
  v = wave_max(v);
  const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
  __syncthreads();
  if (l == 0) scratch[w] = v;
  __syncthreads();
  X s = scratch[0];
#pragma unroll
  for (int k = 1; k < NWAVES; ++k) s = scratch[k] > s ? scratch[k] : s;
  return s;
}
template <typename X, int NWAVES>
__device__ __forceinline__ X block_min(X v, X* scratch) {
  v = wave_min(v);
  const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
  __syncthreads();
  if (l == 0) scratch[w] = v;
  __syncthreads();
  X s = scratch[0];
#pragma unroll
  for (int k = 1; k < NWAVES; ++k) s = scratch[k] < s ? scratch[k] : s;
  return s;
}

// Exclusive block scan of one int per thread (any NWAVES <= 16).  Returns the exclusive
// prefix; *total receives the block sum.
template <int NWAVES>
__device__ __forceinline__ int block_exclusive_scan(int v, int* scratch, int* total) {
  const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
  int incl = v;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    int t = __shfl_up(incl, o, WAVE);
    if (l >= o) incl += t;
  }
  __syncthreads();
  if (l == WAVE - 1) scratch[w] = incl;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < NWAVES; ++k) {
    const int s = scratch[k];
    if (k < w) base += s;
    tot += s;
  }
  *total = tot;
  return base + incl - v;
}

// Execution span of one launch from per-workgroup wall-clock stamps (start, end pairs):
// last end minus first start.  One block of up to 256 threads.
template <int UNUSED = 0>
__global__ void k_clock_span(const uint64_t* __restrict__ clk, int nblk, uint64_t* __restrict__ out) {
  __shared__ uint64_t s_lo[4], s_hi[4];
  uint64_t lo = ~0ull, hi = 0ull;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
    lo = min(lo, clk[2 * b]);
    hi = max(hi, clk[2 * b + 1]);
  }
  lo = wave_min(lo);
  hi = wave_max(hi);
  if (threadIdx.x % WAVE == 0) {
    s_lo[threadIdx.x / WAVE] = lo;
    s_hi[threadIdx.x / WAVE] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < static_cast<int>(blockDim.x) / WAVE; ++w) {
      lo = min(lo, s_lo[w]);
      hi = max(hi, s_hi[w]);
    }
    *out = hi > lo ? hi - lo : 0ull;
  }
}

__device__ __forceinline__ double dinf() { return __builtin_huge_val(); }

// Dynamic Dome test: the largest radius R at which max |d_i^T theta| < 1 over the dome,
// the ball B(y/lambda, R) cut by the half-space n^T theta <= 1 (n = d_*, signed so that
// n^T y = lambda_*); the test screens atom i when the SAFE radius is below it.  With
// nh = n/||n||, the plane lies at distance delta = (n^T y/lambda - 1)/||n|| from the centre
// and cuts from the ball a disc of centre c' = y/lambda - delta nh and radius
// sqrt(R^2 - delta^2).  For u = +-d_i, s = u^T nh/||u||: while the ball's own maximiser is
// outside the half-space (delta + R s > 0) the maximum is u^T c' + sqrt(R^2 - delta^2)
// ||u - (u^T nh) nh||, else it is the ball's, u^T y/lambda + R ||u|| (the SAFE bound).  The
// two meet with equal slope at R = delta/(-s), and the threshold solves the branch in force:
// ra = sqrt(delta^2 + (a / ||u_perp||)^2), a = 1 - u^T c', or the SAFE margin.
// Returned as a lower bound that covers the FP64 rounding of the inputs (z = d_i^T y,
// g = d_i^T n, nu = ||d_i||, ||n||, n^T y, each with relative error at most gam, the
// rounding unit times N + 16): the disc branch is taken only when it is certainly in force
// at its (upper-bounded) threshold, and then with pessimistic inputs; otherwise the SAFE
// margin (never above the threshold), whose own rounding the global slack covers.  An
// atom whose bound can reach 1 at the smallest radius (d_* itself) gets -inf.
__device__ inline double dome_margin(double z, double g, double nu, double lam, double nrm_n,
                                     double delta, double ry, double gam) {
  const double ed = 2.0 * gam * (ry + delta);          // error bound of delta
  const double d_lo = fmax(delta - ed, 0.0), d_hi = delta + ed;
  double m = dinf();
  for (int k = 0; k < 2; ++k) {
    const double sg = k == 0 ? 1.0 : -1.0;
    const double un = sg * g / nrm_n;                    // u^T nh
    const double a = 1.0 - (sg * z / lam - delta * un);  // 1 - u^T c'
    const double ea = 5.0 * gam * nu * (ry + delta + 1.0);
    const double rb = (1.0 - sg * z / lam) / nu;         // the SAFE branch
    double r;
    if (!(a - ea > 0.0)) {
      r = -dinf();
    } else {
      const double p2 = fma(nu, nu, -un * un), ep2 = 8.0 * gam * nu * nu;
      const double p_hi = sqrt(fmax(p2, 0.0) + ep2), p_lo = sqrt(fmax(p2 - ep2, 0.0));
      const double q_lo = (a - ea) / p_hi;
      const double ra_lo = sqrt(fma(d_lo, d_lo, q_lo * q_lo)) * (1.0 - 0x1p-49);
      const double q_hi = p_lo > 0.0 ? (a + ea) / p_lo : dinf();
      const double ra_hi = sqrt(fma(d_hi, d_hi, q_hi * q_hi)) * (1.0 + 0x1p-49);
      const double s = un / nu;
      const double rs_lo = d_lo / (fmax(-s, 0.0) + 4.0 * gam);  // switch radius, lower bound
      r = ra_hi < rs_lo ? ra_lo : rb;
    }
    m = fmin(m, r);
  }
  return m;
}

}  // namespace ds
