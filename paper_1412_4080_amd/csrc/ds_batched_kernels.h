// Batched path: B signals sharing one bfloat16 dictionary, Algorithm 3 with the ISTA /
// FISTA update of Table 1 and the SAFE / DST3 sphere tests (Lemmas 1, 2) or the dynamic
// Dome test, or for the
// Group-Lasso the group soft thresholding and the GSAFE / DGST3 tests (Lemmas 4, 5).
// Every signal keeps its own penalty, dual point, radius and active set.
//
// Per iteration:
//   theta = D_S p - y   sparse: each signal gathers the columns of its support S (the
//                       non-zeros of p), FP64 accumulation of exact bfloat16 x FP32
//                       products, so theta is exact up to FP64 rounding;
//   Z = D^T Theta       dense GEMM on the matrix cores (v_mfma_f32_32x32x16_bf16, FP32
//                       accumulation) over the 32 x 32 (atom, signal) tiles that hold an
//                       active pair.  theta enters as THP bfloat16 parts (hi + mid agrees
//                       with its FP32 rounding to 2^-16 relative; a third part would make
//                       it exact), and every product of parts is exact;
//   the update of Table 1 in the GEMM epilogue (groups: in a pass of its own, one thread
//   per (group, signal), since a group's norm spans tiles), the FP64 scalars per signal,
//   and the screening of the pairs whose margin passed the new radius.  A group's margin
//   is stored on each of its atoms, so the tile masks and the screening work per atom.
//
// Precision.  ||theta||^2, theta^T y and Omega(p) are exact FP64 sums, so the primal
// value is exact.  max|z| comes from the MFMA correlations of the FP32 rounding of theta;
// with e a bound on their distance to the exact correlations, the dual point
// v = mu theta is within eps = e / max|z| (relative) of a feasible point, and the sphere
// radius grows by eps ||v||: screening stays safe.  The gap that ends a solve is
// recomputed once its estimate meets tolerance, from ||D_A^T theta||_inf evaluated in
// FP64, which gives a feasible dual point and the gap in FP64.
#pragma once
#include <cmath>

#include "ds_device.h"

namespace ds {
namespace batch {

constexpr int BW = 64;   // wave size
constexpr int TB = 256;  // threads per block
constexpr int NWB = TB / BW;
constexpr int MT = 32;   // MFMA tile edge (32 x 32 x 16)

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

__device__ __forceinline__ bf16x8 as_bf16x8(const uint4& r) { return __builtin_bit_cast(bf16x8, r); }
__device__ __forceinline__ uint4 ldg16(const uint16_t* p) { return *reinterpret_cast<const uint4*>(p); }

// Round-to-nearest-even float -> bfloat16 bits (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t lsb = (u >> 16) & 1u;
  return static_cast<uint16_t>((u + 0x7fffu + lsb) >> 16);
}
__device__ __forceinline__ float bf16f(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }
// Parts of theta that enter the GEMM.  The split v = hi + mid + lo is exact for normal
// FP32 values (each remainder is a multiple of ulp(v) and needs at most 8 significant bits
// by the third part); with two parts |v - hi - mid| <= 2^-8 |v - hi| <= 2^-16 |v| (round to
// nearest in 8-bit precision, twice), a term the correlation slack carries.  Two parts
// cost two thirds of the matrix-core work and of the LDS traffic of three.
constexpr int THP = 2;
__device__ __forceinline__ void split_parts(float v, uint16_t (&part)[THP]) {
  float r = v;
#pragma unroll
  for (int k = 0; k < THP; ++k) {
    part[k] = f32_to_bf16(r);
    r -= bf16f(part[k]);
  }
}

// done: 0 running, 2 finished in the iteration in flight, 1 finished earlier.
struct alignas(16) Inst {
  double lam, lam_max, yy, rho2, alpha, nn, ny, marg_slack, gap_tol_abs;
  double tt, ty, omega, zmax, mu, gap, primal, dual;
  double r_min, r_scr, r_keep, r_prev, r_slack, l_prev;
  double act_sum, sup_sum;  // sums over iterations of |A_t| and |S_t| (work accounting)
  int32_t iter, done, status, verify, nnz, n_active, i_star, converged;
};

struct BArgs {
  int N, K, B, Np, Kp, Bp, nrb;
  int test, rule, max_iter, screen_static;
  int G;                // 0: Lasso; > 0: groups (contiguous, at most 128 atoms each)
  const int64_t* gptr;  // G + 1 group offsets
  const int* agrp;      // Kp: group of each atom (-1 past K)
  const double* gw;     // G weights w_g
  const double* gspec;  // G spectral norms ||D_g||_2 (FP64, of the stored values)
  const double* gfro;   // G Frobenius norms ||D_g||_F
  double L, gamma_acc, gamma64;
  const uint16_t* dcm;  // Kp x Np, atom (column) major, zero padded
  const double* dsc;    // dictionary scalars: [0] correlation slack scale (max nu_i; groups
                        // max ||D_g||_F / w_g), [1] margin slack scale (max (1 + 1/nu_i);
                        // groups max (||D_g||_F + w_g) / ||D_g||_2)
  const double* nu;     // Kp atom norms
  const float* Y;       // Bp x Np observations (slot order, zero padded)
  float* X;             // Bp x Kp
  float* U0;            // Bp x Kp: u_{t-1} on odd t
  float* U1;            // Bp x Kp: u_{t-1} on even t
  uint32_t* umask;      // (Kp/32) x Bp non-zero bits of u_t per 32-atom tile
  uint16_t* Ths;        // THP x Bp x Np bfloat16 parts of theta
  double* th64;         // Bp x Np theta in FP64
  double* ptt;          // nrb x Bp partial ||theta||^2
  double* pty;          // nrb x Bp partial theta^T y
  const float* marg;    // Bp x Kp margins, rounded towards -inf
  const float* tminm;   // (Kp/32) x Bp smallest margin of each 32-atom tile
  double* pz;           // (Kp/32) x Bp partial max |z| over active pairs
  double* pom;          // (Kp/32) x Bp partial Omega(p)
  int* pact;            // (Kp/32) x Bp active pairs | (non-zeros of p << 8); groups: per
                        // 64-group chunk, atoms active | (non-zeros of p << 16)
  float* Z;             // Bp x Kp correlations of the pairs computed this iteration
  int* ccount;          // Bp x (K/1024 rounded up) candidates per flagged signal and range
  int* cidx;            // Bp x Kp candidate atoms
  double* cval;         // Bp x Kp their exact |d_i^T theta|
  Inst* inst;           // Bp
  int* ndone;           // signals finished
  int* vcount;          // number of signals flagged for verification this iteration
  int* vlist;           // Bp flagged slots
  uint64_t* kclk;       // NULL, or 2 wall-clock stamps per Z-GEMM wave (start, end)
};

constexpr double VWIN = 1.25;   // estimate / tolerance ratio below which the gap is checked

// ============================================================== setup kernels
// Padded atom-major copy of D: dcm[a][n] (zeros beyond N and K).
__global__ __launch_bounds__(TB) void k_b_prep(const uint16_t* __restrict__ D, int64_t ldd, int N,
                                               int K, int Np, uint16_t* __restrict__ dcm) {
  const int a = blockIdx.x;
  const int n = blockIdx.y * TB + threadIdx.x;
  if (n >= Np) return;
  dcm[static_cast<int64_t>(a) * Np + n] = (a < K && n < N) ? D[static_cast<int64_t>(a) * ldd + n] : uint16_t(0);
}

// FP64 atom norms nu_i (one wave per atom).
__global__ __launch_bounds__(TB) void k_b_norms(const uint16_t* __restrict__ dcm, int Np, int Kp,
                                                double* __restrict__ nu) {
  const int lane = threadIdx.x % BW;
  const int a = blockIdx.x * NWB + threadIdx.x / BW;
  if (a >= Kp) return;
  double s = 0.0;
  for (int n = lane; n < Np; n += BW) {
    const double d = bf16f(dcm[static_cast<int64_t>(a) * Np + n]);
    s = fma(d, d, s);
  }
  s = wave_sum(s);
  if (lane == 0) nu[a] = sqrt(s);
}

// Dictionary scalars: max nu_i and max (1 + 1/nu_i) over non-zero atoms (one block).
__global__ __launch_bounds__(TB) void k_b_dict_scalars(const double* __restrict__ nu, int K,
                                                       double* __restrict__ dsc) {
  __shared__ double sd[NWB];
  double m = 0.0, kap = 0.0;
  for (int a = threadIdx.x; a < K; a += TB) {
    m = fmax(m, nu[a]);
    if (nu[a] > 0.0) kap = fmax(kap, 1.0 + 1.0 / nu[a]);
  }
  m = block_max<double, NWB>(m, sd);
  kap = block_max<double, NWB>(kap, sd);
  if (threadIdx.x == 0) {
    dsc[0] = m;
    dsc[1] = kap;
  }
}

// The set-up and output kernels work on a list of slots (blockIdx.y or blockIdx.x indexes
// `slots`): the whole batch at the start, the refilled or finished slots later.
// perm[s] is the signal held by slot s, or -1 for an idle slot.

// Observations of the listed slots: Yp[s][n] = Y[perm[s] * ldy + n] (zero padded; zero
// for an idle slot); x, both u buffers and the non-zero masks of the slot are cleared.
__global__ __launch_bounds__(TB) void k_b_load_slots(BArgs a, const float* __restrict__ Yin,
                                                     int64_t ldy, const int* __restrict__ perm,
                                                     const int* __restrict__ slots,
                                                     float* __restrict__ Yp) {
  const int s = slots[blockIdx.y];
  const int sig = perm[s];
  for (int n = blockIdx.x * TB + threadIdx.x; n < a.Np; n += gridDim.x * TB) {
    float v = 0.f;
    if (sig >= 0 && n < a.N) v = Yin[static_cast<int64_t>(sig) * ldy + n];
    Yp[static_cast<int64_t>(s) * a.Np + n] = v;
  }
  const int64_t row = static_cast<int64_t>(s) * a.Kp;
  for (int i = blockIdx.x * TB + threadIdx.x; i < a.Kp; i += gridDim.x * TB) {
    a.X[row + i] = 0.f;
    a.U0[row + i] = 0.f;
    a.U1[row + i] = 0.f;
    if (i < a.Kp / MT) a.umask[static_cast<int64_t>(i) * a.Bp + s] = 0u;
  }
}

// FP64 batched products out[b][a] = d_a^T v_b for the listed slots b = slots[j], j < nsl
// (exact bfloat16 x FP32 / FP64 products, FP64 accumulation on the matrix cores,
// v_mfma_f64_16x16x4_f64).  The summation order is fixed by Np alone, so a value depends
// neither on the grid nor on which or how many slots are listed: with Q = Np / 4 the rows
// form Q groups {s, Q + s, 2Q + s, 3Q + s}; a group is one k-step of the instruction (its
// four products added to the accumulator); wave w of a block chains the groups
// s = wQ/4 .. (w + 1)Q/4 - 1 in order, and the block adds the four waves' sums in wave order.
// Block: a tile of 16 atoms x 16 list entries (entries past nsl repeat the last slot and
// are not stored).  Operands: lane l holds A[i][k] = d_{a0+i}[kQ + s] and B[k][j] =
// v_{b0+j}[kQ + s] (i = j = l % 16, k = l / 16); the accumulator's element r of lane l is
// C[4r + l / 16][l % 16].  A wave's operand rows form 64 segments of A (atom, k) and 64 of
// B (entry, k); per batch of GB groups the wave loads each segment whole (8-byte pieces,
// consecutive lanes on consecutive pieces) into its own LDS area, padded so that the 64
// lanes' operand reads fall in different banks, and the next batch's loads are in flight
// while the matrix cores consume one.
typedef double dtv_acc __attribute__((ext_vector_type(4)));
template <typename VT>
__global__ __launch_bounds__(TB) void k_b_dtv(const uint16_t* __restrict__ dcm,
                                              const VT* __restrict__ V, int Np, int Kp,
                                              double* __restrict__ out,
                                              const int* __restrict__ slots, int nsl) {
  constexpr int VB = static_cast<int>(sizeof(VT));
  constexpr int GB = 128 / VB;          // groups per batch (a B segment is 128 bytes)
  constexpr int SA = GB * 2 + 4;        // LDS bytes per A segment (bfloat16, padded)
  constexpr int SB = GB * VB + (VB == 4 ? 4 : 8);  // LDS bytes per B segment (padded, VT-aligned)
  constexpr int RA = 4, RB = 8 / VB;    // rows per 8-byte piece of A and of B
  constexpr int PA = GB / RA, PB = GB / RB;  // pieces per segment (= pieces per lane)
  constexpr int WL = 64 * (SA + SB);    // LDS bytes per wave
  __shared__ __align__(16) unsigned char lds[NWB * WL];
  __shared__ dtv_acc part[NWB - 1][BW];
  const int tid = threadIdx.x, lane = tid % BW, wave = tid / BW;
  const int a0 = blockIdx.x * 16, b0 = blockIdx.y * 16;
  const int q16 = lane % 16, k = lane / 16;
  const int Q = Np / 4, S = Q / NWB;  // groups per wave (a multiple of 4: Np % 64 == 0)
  const int s0 = wave * S;
  unsigned char* la = lds + wave * WL;
  unsigned char* lb = la + 64 * SA;
  // piece q of this lane: p = q * 64 + lane, segment p / P (atom or entry seg / 4, k =
  // seg % 4), rows (p % P) * R .. + R - 1 of the batch
  const uint16_t* ga[PA];
  const VT* gb[PB];
#pragma unroll
  for (int q = 0; q < PA; ++q) {
    const int seg = (q * BW + lane) / PA;
    ga[q] = dcm + static_cast<int64_t>(a0 + seg / 4) * Np + (seg % 4) * Q + s0;
  }
#pragma unroll
  for (int q = 0; q < PB; ++q) {
    const int seg = (q * BW + lane) / PB;
    const int slot = slots[min(b0 + seg / 4, nsl - 1)];
    gb[q] = V + static_cast<int64_t>(slot) * Np + (seg % 4) * Q + s0;
  }
  uint2 ra[PA], rb[PB];
  // the pieces of the batch starting at group s; a piece past the wave's range re-reads its
  // last rows (staged but never multiplied), so every load stays inside the range
  auto load = [&](int s) {
#pragma unroll
    for (int q = 0; q < PA; ++q) {
      const int r = min(s + ((q * BW + lane) % PA) * RA, S - RA);
      ra[q] = *reinterpret_cast<const uint2*>(ga[q] + r);
    }
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      const int r = min(s + ((q * BW + lane) % PB) * RB, S - RB);
      rb[q] = *reinterpret_cast<const uint2*>(gb[q] + r);
    }
  };
  dtv_acc acc = {0.0, 0.0, 0.0, 0.0};
  load(0);
  for (int s = 0; s < S; s += GB) {
    __syncthreads();  // the previous batch has been consumed
#pragma unroll
    for (int q = 0; q < PA; ++q) {
      const int p = q * BW + lane;
      uint32_t* d = reinterpret_cast<uint32_t*>(la + (p / PA) * SA + (p % PA) * 8);
      d[0] = ra[q].x;
      d[1] = ra[q].y;
    }
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      const int p = q * BW + lane;
      uint32_t* d = reinterpret_cast<uint32_t*>(lb + (p / PB) * SB + (p % PB) * 8);
      d[0] = rb[q].x;
      d[1] = rb[q].y;
    }
    __syncthreads();
    if (s + GB < S) load(s + GB);
    const unsigned char* pa = la + (q16 * 4 + k) * SA;
    const unsigned char* pb = lb + (q16 * 4 + k) * SB;
    const int n = min(GB, S - s);  // a multiple of 4
    for (int g = 0; g < n; g += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint16_t av = *reinterpret_cast<const uint16_t*>(pa + (g + u) * 2);
        const VT bv = *reinterpret_cast<const VT*>(pb + (g + u) * VB);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(
            static_cast<double>(__uint_as_float(static_cast<uint32_t>(av) << 16)),
            static_cast<double>(bv), acc, 0, 0, 0);
      }
    }
  }
  if (wave > 0) part[wave - 1][lane] = acc;
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int w = 0; w < NWB - 1; ++w) acc += part[w][lane];
  const int e = b0 + q16;
  if (e >= nsl) return;
  const int64_t row = static_cast<int64_t>(slots[e]) * Kp + a0 + k;
#pragma unroll
  for (int r = 0; r < 4; ++r) out[row + 4 * r] = acc[r];
}

// Per-signal setup (one block per slot): ||y||^2, finiteness, lambda_* = max_i |z0_i|
// with the smallest-index tie break, lambda, the trivial case lambda >= lambda_*, and the
// DST3 hyperplane n = sign(z0_i*) d_i* (Lemma 2; general atom norms): ||n||^2, n^T y,
// alpha = (n^T y / lambda - 1) / ||n||^2, rho^2 = alpha^2 ||n||^2.  Writes the column
// Vn[s] = n used to form D^T n.
__global__ __launch_bounds__(TB) void k_b_inst_init(BArgs a, const double* __restrict__ z0,
                                                    const double* __restrict__ lam_in,
                                                    int lam_relative, double gap_tol,
                                                    float* __restrict__ Vn,
                                                    const int* __restrict__ perm,
                                                    const int* __restrict__ slots) {
  __shared__ double sd[NWB];
  __shared__ int si[NWB];
  __shared__ double s_best;
  __shared__ int s_arg;
  const int s = slots[blockIdx.x], tid = threadIdx.x;
  Inst* st = a.inst + s;
  const float* y = a.Y + static_cast<int64_t>(s) * a.Np;
  if (perm[s] < 0) {  // idle slot
    for (int n = tid; n < a.Np; n += TB) Vn[static_cast<int64_t>(s) * a.Np + n] = 0.f;
    if (tid == 0) {
      Inst z = {};
      z.done = 1;
      z.status = 1;
      *st = z;
    }
    return;
  }
  double yy = 0.0;
  int bad = 0;
  for (int n = tid; n < a.N; n += TB) {
    const double v = y[n];
    if (!isfinite(v)) bad = 1;
    yy = fma(v, v, yy);
  }
  yy = block_sum<double, NWB>(yy, sd);
  bad = block_sum<int, NWB>(bad, si);
  const double* z = z0 + static_cast<int64_t>(s) * a.Kp;
  double best = -1.0;
  int barg = 0x7fffffff;
  constexpr int IU = 8;  // loads issued before the first comparison (same order of i)
  for (int i0 = tid; i0 < a.K; i0 += TB * IU) {
    double v[IU];
#pragma unroll
    for (int u = 0; u < IU; ++u) v[u] = fabs(z[min(i0 + u * TB, a.K - 1)]);
#pragma unroll
    for (int u = 0; u < IU; ++u)
      if (i0 + u * TB < a.K && v[u] > best) { best = v[u]; barg = i0 + u * TB; }
  }
  for (int o = BW / 2; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o, BW);
    const int oa = __shfl_xor(barg, o, BW);
    if (ob > best || (ob == best && oa < barg)) { best = ob; barg = oa; }
  }
  __syncthreads();
  if (tid % BW == 0) { sd[tid / BW] = best; si[tid / BW] = barg; }
  __syncthreads();
  if (tid == 0) {
    double b = sd[0];
    int ba = si[0];
    for (int k = 1; k < NWB; ++k)
      if (sd[k] > b || (sd[k] == b && si[k] < ba)) { b = sd[k]; ba = si[k]; }
    s_best = b;
    s_arg = ba;
  }
  __syncthreads();
  const double lam_max = s_best;
  const int arg = s_arg;
  if (!(arg >= 0 && arg < a.K) || !isfinite(lam_max)) bad = 1;
  const double lam = lam_relative ? lam_in[s] * lam_max : lam_in[s];
  const bool trivial = !(lam < lam_max);
  // the hyperplane n = sign(z0_i*) d_i* of DST3, and of the Dome test's half-space
  const bool hyp = (a.test == 2 || a.test == 3) && !trivial && !bad;
  const bool dst3 = a.test == 2 && hyp;
  const double sgn = (!bad && z[arg] < 0.0) ? -1.0 : 1.0;
  double nn = 0.0, ny = 0.0;
  for (int n = tid; n < a.Np; n += TB) {
    float v = 0.f;
    if (hyp) {
      v = static_cast<float>(sgn * bf16f(a.dcm[static_cast<int64_t>(arg) * a.Np + n]));
      nn = fma(static_cast<double>(v), static_cast<double>(v), nn);
      ny = fma(static_cast<double>(v), static_cast<double>(y[n]), ny);
    }
    Vn[static_cast<int64_t>(s) * a.Np + n] = v;
  }
  nn = block_sum<double, NWB>(nn, sd);
  ny = block_sum<double, NWB>(ny, sd);
  if (tid == 0) {
    Inst t = {};
    const double alpha = (dst3 && nn > 0.0) ? (ny / lam - 1.0) / nn : 0.0;
    t.lam = lam;
    t.lam_max = lam_max;
    t.yy = yy;
    t.alpha = alpha;
    t.nn = nn;
    t.ny = ny;
    t.rho2 = alpha * alpha * nn;
    t.gap_tol_abs = gap_tol * yy;
    t.r_min = 1e300;
    t.r_scr = 1e300;
    t.r_keep = 1e300;
    t.r_prev = 1e300;
    t.l_prev = 1.0;
    t.i_star = bad ? 0 : arg;
    t.status = bad ? -1 : (trivial ? 1 : 0);
    t.done = (bad || trivial) ? 1 : 0;
    t.converged = t.done;
    // rounding slack of the FP64 margins (products exact, N-term FP64 sums)
    const double eps = (a.N + 16) * 0x1p-53;
    t.marg_slack = eps * a.dsc[1] * (sqrt(yy) / lam + fabs(alpha) * sqrt(nn) + 1.0);
    *st = t;
    if (t.done) atomicAdd(a.ndone, 1);
  }
}

// Margins m_i = (1 - |d_i^T c|) / nu_i with d_i^T c = z0_i / lambda - alpha d_i^T n
// (SAFE: alpha = 0), stored in FP32 rounded towards -inf so that m32 > r implies m > r.
// Zero atoms and padding: +inf (screened from the start); no test: -inf.
__global__ __launch_bounds__(TB) void k_b_margins(BArgs a, const double* __restrict__ z0,
                                                  const double* __restrict__ gn,
                                                  float* __restrict__ marg,
                                                  const int* __restrict__ perm,
                                                  const int* __restrict__ slots) {
  const int s = slots[blockIdx.y];
  const int i = blockIdx.x * TB + threadIdx.x;
  if (i >= a.Kp) return;
  const Inst& st = a.inst[s];
  const int64_t o = static_cast<int64_t>(s) * a.Kp + i;
  float m;
  if (i >= a.K || perm[s] < 0 || st.done) {
    m = INFINITY;
  } else if (a.test == 0) {
    m = -INFINITY;
  } else if (a.test == 3) {
    // the dynamic Dome test: the largest SAFE radius at which the dome still screens the
    // atom (a lower bound, covering the rounding of its FP64 inputs)
    const double nu = a.nu[i], nrm_n = sqrt(st.nn);
    const double delta = (st.ny / st.lam - 1.0) / nrm_n;
    const double gam = (a.N + 16) * 0x1p-53;
    m = nu > 0.0 ? __double2float_rd(dome_margin(z0[o], gn[o], nu, st.lam, nrm_n, delta,
                                                 sqrt(st.yy) / st.lam, gam))
                 : INFINITY;
  } else {
    const double nu = a.nu[i];
    const double ci = z0[o] / st.lam - (a.test == 2 ? st.alpha * gn[o] : 0.0);
    m = nu > 0.0 ? __double2float_rd((1.0 - fabs(ci)) / nu) : INFINITY;
  }
  marg[o] = m;
}

// Smallest margin of each 32-atom tile: tminm[tile][s].
__global__ __launch_bounds__(TB) void k_b_tile_min(BArgs a, float* __restrict__ tminm,
                                                   const int* __restrict__ slots) {
  const int s = slots[blockIdx.y];
  const int tile = blockIdx.x * TB + threadIdx.x;
  if (tile >= a.Kp / MT) return;
  const float* m = a.marg + static_cast<int64_t>(s) * a.Kp + tile * MT;
  float v = INFINITY;
  for (int k = 0; k < MT; ++k) v = fminf(v, m[k]);
  tminm[static_cast<int64_t>(tile) * a.Bp + s] = v;
}

// ------------------------------------------------------------- groups: set-up
// Dictionary scalars of a grouped dictionary (one block): max ||D_g||_F / w_g, the scale of
// the correlation rounding slack, and max (||D_g||_F + w_g) / ||D_g||_2 over groups with
// ||D_g||_2 > 0, the scale of the margins' rounding slack.
__global__ __launch_bounds__(TB) void k_b_gdict_scalars(BArgs a, double* __restrict__ dsc) {
  __shared__ double sd[NWB];
  double m = 0.0, kap = 0.0;
  for (int g = threadIdx.x; g < a.G; g += TB) {
    m = fmax(m, a.gfro[g] / a.gw[g]);
    if (a.gspec[g] > 0.0) kap = fmax(kap, (a.gfro[g] + a.gw[g]) / a.gspec[g]);
  }
  m = block_max<double, NWB>(m, sd);
  kap = block_max<double, NWB>(kap, sd);
  if (threadIdx.x == 0) {
    dsc[0] = m;
    dsc[1] = kap;
  }
}

// Per-signal setup for groups (one block per listed slot): ||y||^2, finiteness,
// lambda_* = max_g ||z0_g|| / w_g with the smallest-index tie break (eq. gstar), lambda,
// the trivial case, and the DGST3 hyperplane of Lemma 5: n = D_g* D_g*^T y / lambda_*
// (FP64, written to Vd for D^T n), ||n||^2, n^T y, alpha = (n^T y / lambda - w_g*^2) /
// ||n||^2, rho^2 = alpha^2 ||n||^2.
__global__ __launch_bounds__(TB) void k_b_ginst_init(BArgs a, const double* __restrict__ z0,
                                                     const double* __restrict__ lam_in,
                                                     int lam_relative, double gap_tol,
                                                     double* __restrict__ Vd,
                                                     const int* __restrict__ perm,
                                                     const int* __restrict__ slots) {
  __shared__ double sd[NWB];
  __shared__ int si[NWB];
  __shared__ double s_best;
  __shared__ int s_arg;
  const int s = slots[blockIdx.x], tid = threadIdx.x;
  Inst* st = a.inst + s;
  const float* y = a.Y + static_cast<int64_t>(s) * a.Np;
  double* vd = Vd + static_cast<int64_t>(s) * a.Np;
  if (perm[s] < 0) {  // idle slot
    for (int n = tid; n < a.Np; n += TB) vd[n] = 0.0;
    if (tid == 0) {
      Inst z = {};
      z.done = 1;
      z.status = 1;
      *st = z;
    }
    return;
  }
  double yy = 0.0;
  int bad = 0;
  for (int n = tid; n < a.N; n += TB) {
    const double v = y[n];
    if (!isfinite(v)) bad = 1;
    yy = fma(v, v, yy);
  }
  yy = block_sum<double, NWB>(yy, sd);
  bad = block_sum<int, NWB>(bad, si);
  const double* z = z0 + static_cast<int64_t>(s) * a.Kp;
  double best = -1.0;
  int barg = 0x7fffffff;
  for (int g = tid; g < a.G; g += TB) {  // increasing g per thread: strict > keeps the first
    double s2 = 0.0;
    for (int64_t k = a.gptr[g]; k < a.gptr[g + 1]; ++k) s2 = fma(z[k], z[k], s2);
    const double v = sqrt(s2) / a.gw[g];
    if (v > best) { best = v; barg = g; }
  }
  for (int o = BW / 2; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o, BW);
    const int oa = __shfl_xor(barg, o, BW);
    if (ob > best || (ob == best && oa < barg)) { best = ob; barg = oa; }
  }
  __syncthreads();
  if (tid % BW == 0) { sd[tid / BW] = best; si[tid / BW] = barg; }
  __syncthreads();
  if (tid == 0) {
    double b = sd[0];
    int ba = si[0];
    for (int k = 1; k < NWB; ++k)
      if (sd[k] > b || (sd[k] == b && si[k] < ba)) { b = sd[k]; ba = si[k]; }
    s_best = b;
    s_arg = ba;
  }
  __syncthreads();
  const double lam_max = s_best;
  const int arg = s_arg;
  if (!(arg >= 0 && arg < a.G) || !isfinite(lam_max)) bad = 1;
  const double lam = lam_relative ? lam_in[s] * lam_max : lam_in[s];
  const bool trivial = !(lam < lam_max);
  const bool dst3 = a.test == 2 && !trivial && !bad;
  double nn = 0.0, ny = 0.0;
  const int64_t g0 = dst3 ? a.gptr[arg] : 0, g1 = dst3 ? a.gptr[arg + 1] : 0;
  for (int n = tid; n < a.Np; n += TB) {
    double v = 0.0;
    if (dst3) {
      for (int64_t k = g0; k < g1; ++k) v = fma(bf16f(a.dcm[k * a.Np + n]), z[k], v);
      v /= lam_max;
      nn = fma(v, v, nn);
      ny = fma(v, static_cast<double>(y[n]), ny);
    }
    vd[n] = v;
  }
  nn = block_sum<double, NWB>(nn, sd);
  ny = block_sum<double, NWB>(ny, sd);
  if (tid == 0) {
    Inst t = {};
    const double ws2 = dst3 ? a.gw[arg] * a.gw[arg] : 1.0;
    const double alpha = (dst3 && nn > 0.0) ? (ny / lam - ws2) / nn : 0.0;
    t.lam = lam;
    t.lam_max = lam_max;
    t.yy = yy;
    t.alpha = alpha;
    t.nn = nn;
    t.rho2 = alpha * alpha * nn;
    t.gap_tol_abs = gap_tol * yy;
    t.r_min = 1e300;
    t.r_scr = 1e300;
    t.r_keep = 1e300;
    t.r_prev = 1e300;
    t.l_prev = 1.0;
    t.i_star = bad ? 0 : arg;
    t.status = bad ? -1 : (trivial ? 1 : 0);
    t.done = (bad || trivial) ? 1 : 0;
    t.converged = t.done;
    const double eps = (a.N + 16) * 0x1p-53;
    t.marg_slack = eps * a.dsc[1] * (sqrt(yy) / lam + fabs(alpha) * sqrt(nn) + 1.0);
    *st = t;
    if (t.done) atomicAdd(a.ndone, 1);
  }
}

// Group margins m_g = (w_g - ||D_g^T c||) / ||D_g||_2 (Lemmas 4, 5 through the sphere bound
// of Lemma 6) with D_g^T c = z0_g / lambda - alpha D_g^T n (GSAFE: alpha = 0), rounded
// towards -inf and stored on every atom of the group.  Padding atoms, idle and finished
// slots, groups with ||D_g||_2 = 0: +inf; no test: -inf.  Thread: one group (and one
// padding atom) of one listed slot.
__global__ __launch_bounds__(TB) void k_b_gmargins(BArgs a, const double* __restrict__ z0,
                                                   const double* __restrict__ gn,
                                                   float* __restrict__ marg,
                                                   const int* __restrict__ perm,
                                                   const int* __restrict__ slots) {
  const int s = slots[blockIdx.y];
  const int j = blockIdx.x * TB + threadIdx.x;
  const int64_t row = static_cast<int64_t>(s) * a.Kp;
  if (j >= a.K && j < a.Kp) marg[row + j] = INFINITY;
  if (j >= a.G) return;
  const Inst& st = a.inst[s];
  const int64_t g0 = a.gptr[j], g1 = a.gptr[j + 1];
  float m;
  if (perm[s] < 0 || st.done) {
    m = INFINITY;
  } else if (a.test == 0) {
    m = -INFINITY;
  } else {
    double s2 = 0.0;
    for (int64_t k = g0; k < g1; ++k) {
      const double ck = z0[row + k] / st.lam - (a.test == 2 ? st.alpha * gn[row + k] : 0.0);
      s2 = fma(ck, ck, s2);
    }
    const double sp = a.gspec[j];
    m = sp > 0.0 ? __double2float_rd((a.gw[j] - sqrt(s2)) / sp) : INFINITY;
  }
  for (int64_t k = g0; k < g1; ++k) marg[row + k] = m;
}

// ============================================================== iteration kernels
constexpr int TR = 512;  // rows of theta per block (64 lanes x 8 rows)
constexpr int TW = 128;  // mask words (32 atoms each) per support-list round

// theta = D_S p - y for every running signal, S the support of p = u_{t-1} (from the
// non-zero bits the previous update left), FP64 accumulation; writes theta in FP64, the
// bfloat16 parts of its FP32 rounding, and per-block FP64 ||theta||^2 and theta^T y.
// Block: 512 rows of one signal.  The support list (atom indices) is built through LDS
// 4096 atoms at a time by the whole block; the four waves split it, each lane
// accumulating 8 rows, and the waves are summed in a fixed order.  Also retires the
// signals finished in the previous iteration and clears the verification list.
__global__ __launch_bounds__(TB) void k_b_theta(BArgs a, const float* __restrict__ Uin) {
  __shared__ int sidx[TW * MT];
  __shared__ int scan[NWB];
  __shared__ double red[NWB][TR + 8];
  __shared__ double sd[NWB];
  const int s = blockIdx.y;
  if (blockIdx.x == 0 && s == 0 && threadIdx.x == 0) *a.vcount = 0;
  Inst& st = a.inst[s];
  const int done = st.done;
  if (done != 0) {
    if (done == 2 && blockIdx.x == 0 && threadIdx.x == 0) st.done = 1;
    return;
  }
  const int lane = threadIdx.x % BW, wave = threadIdx.x / BW;
  const int nl = blockIdx.x * TR + lane * 8;  // this lane's 8 rows
  const bool rows_ok = nl < a.Np;
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const int nw = a.Kp / MT;
  const float* u = Uin + static_cast<int64_t>(s) * a.Kp;
  // Stream the `total` entries of the support list in sidx: wave w takes entries w, w + 4,
  // w + 8, ... in increasing order, GB of them per batch, every load of a batch issued before
  // its first FMA and the next batch's loads in flight while a batch is multiplied.
  // Entries past the end re-read the last one with weight zero: the accumulators start at
  // +0 and a sum never rounds to -0, so adding a zero product leaves them bit for bit
  // unchanged.
  constexpr int GB = 8;
  struct Batch {
    float uv[GB];
    uint4 d[GB];
  };
  auto stream = [&](int total) {
    if (!rows_ok || total == 0) return;
    const int nb = (total + NWB * GB - 1) / (NWB * GB);
    auto issue = [&](Batch& X, int b) {
      const int j0 = b * NWB * GB;
      int at[GB];
#pragma unroll
      for (int g = 0; g < GB; ++g) at[g] = sidx[min(j0 + wave + NWB * g, total - 1)];
#pragma unroll
      for (int g = 0; g < GB; ++g) X.uv[g] = u[at[g]];
#pragma unroll
      for (int g = 0; g < GB; ++g) X.d[g] = ldg16(a.dcm + static_cast<int64_t>(at[g]) * a.Np + nl);
    };
    auto compute = [&](const Batch& X, int b) {
      const int j0 = b * NWB * GB;
#pragma unroll
      for (int g = 0; g < GB; ++g) {
        const double ug = j0 + wave + NWB * g < total ? static_cast<double>(X.uv[g]) : 0.0;
        const uint32_t wd[4] = {X.d[g].x, X.d[g].y, X.d[g].z, X.d[g].w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          acc[2 * e] = fma(static_cast<double>(__uint_as_float(wd[e] << 16)), ug, acc[2 * e]);
          acc[2 * e + 1] = fma(static_cast<double>(__uint_as_float(wd[e] & 0xffff0000u)), ug, acc[2 * e + 1]);
        }
      }
    };
    Batch A, Bt;
    issue(A, 0);
    for (int b = 0; b < nb; b += 2) {
      if (b + 1 < nb) issue(Bt, b + 1);
      __builtin_amdgcn_sched_barrier(0);
      compute(A, b);
      if (b + 1 >= nb) break;
      if (b + 2 < nb) issue(A, b + 2);
      __builtin_amdgcn_sched_barrier(0);
      compute(Bt, b + 1);
    }
  };
  // The whole support list in one pass when the mask words fit four per thread and the
  // support fits sidx (the usual case): thread t scans words t*wpt .. t*wpt + wpt - 1, so
  // the block scan of the counts places the atoms in increasing order.
  bool listed = false;
  constexpr int WPT = 4;
  if (nw <= TB * WPT) {
    const int wpt = (nw + TB - 1) / TB;
    uint32_t mw[WPT];
#pragma unroll
    for (int q = 0; q < WPT; ++q) {
      const int w = threadIdx.x * wpt + q;
      const uint32_t v = a.umask[static_cast<int64_t>(min(w, nw - 1)) * a.Bp + s];
      mw[q] = (q < wpt && w < nw) ? v : 0u;
    }
    int cnt = 0;
#pragma unroll
    for (int q = 0; q < WPT; ++q) cnt += __popc(mw[q]);
    int total;
    int pos = block_exclusive_scan<NWB>(cnt, scan, &total);
    if (total <= TW * MT) {
#pragma unroll
      for (int q = 0; q < WPT; ++q) {
        uint32_t m = mw[q];
        const int w = threadIdx.x * wpt + q;
        while (m != 0u) {
          sidx[pos++] = w * MT + __ffs(m) - 1;
          m &= m - 1u;
        }
      }
      __syncthreads();
      stream(total);
      listed = true;
    }
    __syncthreads();
  }
  if (!listed) {
    // rounds of TW mask words; each later round's words are fetched while a round streams
    uint32_t m_next =
        (threadIdx.x < TW && threadIdx.x < nw) ? a.umask[static_cast<int64_t>(threadIdx.x) * a.Bp + s] : 0u;
    for (int w0 = 0; w0 < nw; w0 += TW) {
      const int w = w0 + threadIdx.x;
      uint32_t m = m_next;
      int total;
      int pos = block_exclusive_scan<NWB>(__popc(m), scan, &total);
      while (m != 0u) {
        sidx[pos++] = w * MT + __ffs(m) - 1;
        m &= m - 1u;
      }
      __syncthreads();
      const int wn = w + TW;
      m_next = (threadIdx.x < TW && wn < nw) ? a.umask[static_cast<int64_t>(wn) * a.Bp + s] : 0u;
      stream(total);
      __syncthreads();
    }
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) red[wave][lane * 8 + k] = acc[k];
  __syncthreads();
  const int64_t plane = static_cast<int64_t>(a.Bp) * a.Np;
  double tt = 0.0, ty = 0.0;
  for (int r = threadIdx.x; r < TR; r += TB) {
    const int n = blockIdx.x * TR + r;
    if (n >= a.Np) break;
    const int64_t o = static_cast<int64_t>(s) * a.Np + n;
    const double v = ((red[0][r] + red[1][r]) + red[2][r]) + red[3][r];
    const double yv = a.Y[o];
    const double th = n < a.N ? v - yv : 0.0;
    a.th64[o] = th;
    uint16_t part[THP];
    split_parts(static_cast<float>(th), part);
#pragma unroll
    for (int k = 0; k < THP; ++k) a.Ths[k * plane + o] = part[k];
    tt = fma(th, th, tt);
    ty = fma(th, yv, ty);
  }
  tt = block_sum<double, NWB>(tt, sd);
  ty = block_sum<double, NWB>(ty, sd);
  if (threadIdx.x == 0) {
    a.ptt[static_cast<int64_t>(blockIdx.x) * a.Bp + s] = tt;
    a.pty[static_cast<int64_t>(blockIdx.x) * a.Bp + s] = ty;
  }
}

constexpr int ZR = 64;       // rows of D and Theta staged in LDS per step
constexpr int ZP = ZR + 8;   // padded LDS row (144 bytes: fragment reads free of bank conflicts)
constexpr int RP = ZR / 8;   // 16-byte pieces of a staged row

// Z = D^T Theta with the update of Table 1 in the epilogue.  Block shapes: RA x RB waves
// (atoms x signals), each computing WA x WB output tiles of 32 atoms x 32 signals, so a
// block covers TA = 32 RA WA atoms and TS = 32 RB WB signals.  Every 32 x 32
// output tile is accumulated by the same instruction sequence whatever the shape (64-row
// chunks in order, the parts of theta, four k steps of 16 per chunk), so the results
// are the same bit for bit; the shape only changes how often each piece of D and Theta is
// staged (D once per block of signals, Theta once per block of atoms) and the parallelism.
// The block stages 64-row chunks of its atoms and of the parts of its signals' theta
// through LDS with 16-byte loads while the next chunk is fetched into registers.  Each
// chunk is accumulated in FP32 on the matrix cores from zero and then added to FP64
// registers, so an FP32 rounding chain spans THP x 64 products.  Output tiles without an
// active pair are skipped; a block without any returns at once.
template <int RA, int RB, int WA, int WB>
__global__ __launch_bounds__(BW * RA * RB) __attribute__((amdgpu_waves_per_eu(WA * WB > 1 ? 2 : 1))) void k_b_zgemm(BArgs a, const float* __restrict__ Uin,
                                                          float* __restrict__ Uout) {
  constexpr int NWV = RA * RB, NT = BW * NWV;  // waves and threads of a block
  constexpr int TA = MT * RA * WA, TS = MT * RB * WB;
  constexpr int PA = TA * RP / NT;       // 16-byte pieces of a D chunk per thread
  constexpr int PB = THP * TS * RP / NT;   // 16-byte pieces of a Theta chunk per thread
  static_assert(PA * NT == TA * RP && PB * NT == THP * TS * RP, "pieces tile the block");
  __shared__ __align__(16) uint16_t sA[TA][ZP];     // TA atoms x 64 rows
  __shared__ __align__(16) uint16_t sB[THP][TS][ZP];  // THP parts x TS signals x 64 rows
  __shared__ int s_on[NWV];
  const int lane = threadIdx.x % BW, wave = threadIdx.x / BW;
  const int64_t gw = (static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x) * NWV + wave;
  if (a.kclk != nullptr && lane == 0) a.kclk[2 * gw] = wall_clock64();
  const int a0b = blockIdx.x * TA, b0b = blockIdx.y * TS;
  const int wal = (wave / RB) * (MT * WA), wbl = (wave % RB) * (MT * WB);  // in the block
  // this lane's signal in output tile column ib, and the tiles' activity
  const Inst* sl[WB];
  bool alive[WB];
  double r_act[WB];
#pragma unroll
  for (int ib = 0; ib < WB; ++ib) {
    sl[ib] = a.inst + (b0b + wbl + MT * ib + lane % MT);
    alive[ib] = sl[ib]->done == 0;
    r_act[ib] = sl[ib]->r_keep;  // active pairs: margin <= r_act
  }
  bool tile_on[WA][WB], sub_on[WA][WB];
  bool wave_on = false;
#pragma unroll
  for (int ia = 0; ia < WA; ++ia)
#pragma unroll
    for (int ib = 0; ib < WB; ++ib) {
      const int at = (a0b + wal + MT * ia) / MT;
      const int64_t tix = static_cast<int64_t>(at) * a.Bp + (b0b + wbl + MT * ib + lane % MT);
      tile_on[ia][ib] = alive[ib] && static_cast<double>(a.tminm[tix]) <= r_act[ib];
      sub_on[ia][ib] = __ballot(tile_on[ia][ib]) != 0;
      wave_on |= sub_on[ia][ib];
      if (!sub_on[ia][ib] && lane < MT) {
        a.pz[tix] = 0.0;
        a.pom[tix] = 0.0;
        a.pact[tix] = 0;
        a.umask[tix] = 0u;
      }
    }
  if (lane == 0) s_on[wave] = wave_on ? 1 : 0;
  __syncthreads();
  bool block_on = false;
#pragma unroll
  for (int w = 0; w < NWV; ++w) block_on |= s_on[w] != 0;
  if (!block_on) {
    if (a.kclk != nullptr && lane == 0) a.kclk[2 * gw + 1] = wall_clock64();
    return;
  }
  const int64_t plane = static_cast<int64_t>(a.Bp) * a.Np;
  const int kk = (lane / MT) * 8;
  double zacc[WA][WB][16];
#pragma unroll
  for (int ia = 0; ia < WA; ++ia)
#pragma unroll
    for (int ib = 0; ib < WB; ++ib)
#pragma unroll
      for (int i = 0; i < 16; ++i) zacc[ia][ib][i] = 0.0;
  // chunk n0 + ZR is fetched into registers while chunk n0 is multiplied
  uint4 pa[PA], pb[PB];
  auto fetch = [&](int n0) {
#pragma unroll
    for (int r = 0; r < PA; ++r) {  // TA rows x 128 bytes of D
      const int e = threadIdx.x + r * NT;
      pa[r] = ldg16(a.dcm + static_cast<int64_t>(a0b + e / RP) * a.Np + n0 + (e % RP) * 8);
    }
#pragma unroll
    for (int r = 0; r < PB; ++r) {  // THP x TS rows x 128 bytes of theta
      const int e = threadIdx.x + r * NT;
      pb[r] = ldg16(a.Ths + (e / (TS * RP)) * plane +
                    static_cast<int64_t>(b0b + (e % (TS * RP)) / RP) * a.Np + n0 + (e % RP) * 8);
    }
  };
  fetch(0);
  for (int n0 = 0; n0 < a.Np; n0 += ZR) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PA; ++r) {
      const int e = threadIdx.x + r * NT;
      *reinterpret_cast<uint4*>(&sA[e / RP][(e % RP) * 8]) = pa[r];
    }
#pragma unroll
    for (int r = 0; r < PB; ++r) {
      const int e = threadIdx.x + r * NT;
      *reinterpret_cast<uint4*>(&sB[e / (TS * RP)][(e % (TS * RP)) / RP][(e % RP) * 8]) = pb[r];
    }
    __syncthreads();
    if (n0 + ZR < a.Np) fetch(n0 + ZR);
    if (wave_on) {
      f32x16 c[WA][WB];
#pragma unroll
      for (int ia = 0; ia < WA; ++ia)
#pragma unroll
        for (int ib = 0; ib < WB; ++ib)
#pragma unroll
          for (int i = 0; i < 16; ++i) c[ia][ib][i] = 0.f;
      // raised wave priority while the chunk's MFMAs issue: the waves staging the next
      // chunk through LDS then yield to the ones that keep the matrix cores busy
      __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int s16 = 0; s16 < ZR; s16 += 16) {
        bf16x8 ad[WA], bp[THP][WB];
#pragma unroll
        for (int ia = 0; ia < WA; ++ia)
          ad[ia] = as_bf16x8(*reinterpret_cast<const uint4*>(&sA[wal + MT * ia + lane % MT][s16 + kk]));
#pragma unroll
        for (int ib = 0; ib < WB; ++ib) {
          const int sr = wbl + MT * ib + lane % MT;
#pragma unroll
          for (int k = 0; k < THP; ++k)
            bp[k][ib] = as_bf16x8(*reinterpret_cast<const uint4*>(&sB[k][sr][s16 + kk]));
        }
#pragma unroll
        for (int ia = 0; ia < WA; ++ia)
#pragma unroll
          for (int ib = 0; ib < WB; ++ib) {
            if (!sub_on[ia][ib]) continue;
#pragma unroll
            for (int k = 0; k < THP; ++k)
              c[ia][ib] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ad[ia], bp[k][ib], c[ia][ib], 0, 0, 0);
          }
      }
      __builtin_amdgcn_s_setprio(0);
#pragma unroll
      for (int ia = 0; ia < WA; ++ia)
#pragma unroll
        for (int ib = 0; ib < WB; ++ib)
#pragma unroll
          for (int i = 0; i < 16; ++i) zacc[ia][ib][i] += static_cast<double>(c[ia][ib][i]);
    }
  }
  if (!wave_on) {
    if (a.kclk != nullptr && lane == 0) a.kclk[2 * gw + 1] = wall_clock64();
    return;
  }
  if (a.G > 0) {
    // groups: z of the active atoms for the group update; the tile masks are cleared for
    // k_b_gprox to OR the new non-zero bits into
#pragma unroll
    for (int ib = 0; ib < WB; ++ib) {
      const int bl = b0b + wbl + MT * ib + lane % MT;
#pragma unroll
      for (int ia = 0; ia < WA; ++ia) {
        if (!sub_on[ia][ib]) continue;
        const int a0 = a0b + wal + MT * ia;
        if (tile_on[ia][ib]) {
          float4 m4q[4];  // the lane's margins in one round trip
#pragma unroll
          for (int q = 0; q < 4; ++q)
            m4q[q] = *reinterpret_cast<const float4*>(
                a.marg + static_cast<int64_t>(bl) * a.Kp + a0 + 8 * q + (lane / MT) * 4);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int64_t o = static_cast<int64_t>(bl) * a.Kp + a0 + 8 * q + (lane / MT) * 4;
            const float4 m4 = m4q[q];
            if (!(static_cast<double>(m4.x) <= r_act[ib] || static_cast<double>(m4.y) <= r_act[ib] ||
                  static_cast<double>(m4.z) <= r_act[ib] || static_cast<double>(m4.w) <= r_act[ib]))
              continue;
            const double* zq = &zacc[ia][ib][4 * q];
            *reinterpret_cast<float4*>(a.Z + o) =
                make_float4(static_cast<float>(zq[0]), static_cast<float>(zq[1]),
                            static_cast<float>(zq[2]), static_cast<float>(zq[3]));
          }
        }
        if (lane < MT) a.umask[static_cast<int64_t>(a0 / MT) * a.Bp + bl] = 0u;
      }
    }
    if (a.kclk != nullptr && lane == 0) a.kclk[2 * gw + 1] = wall_clock64();
    return;
  }
  // epilogue per output tile: lane holds signal bl, atoms a0 + 8 q + (lane / 32) * 4 + e
#pragma unroll
  for (int ib = 0; ib < WB; ++ib) {
    const int bl = b0b + wbl + MT * ib + lane % MT;
    const Inst& st = *sl[ib];
    const double invL = 1.0 / a.L, thr = st.lam / a.L;
    double beta = 0.0;
    if (a.rule == 1) {
      const double lp = st.l_prev;
      beta = (lp - 1.0) / (0.5 * (1.0 + sqrt(1.0 + 4.0 * lp * lp)));
    }
#pragma unroll
    for (int ia = 0; ia < WA; ++ia) {
      if (!sub_on[ia][ib]) continue;
      const int a0 = a0b + wal + MT * ia;
      const int64_t tix = static_cast<int64_t>(a0 / MT) * a.Bp + bl;
      double zm = 0.0;
      double om = 0.0;
      int nact = 0, nsup = 0;
      uint32_t bits = 0u;
      if (tile_on[ia][ib]) {
        // margins, momentum point and iterate of the lane's 16 atoms in one round trip
        // (loaded whether or not an atom is active; a branch before them would let each
        // wait for the previous group's)
        float4 m4q[4], u4q[4], x4q[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t o = static_cast<int64_t>(bl) * a.Kp + a0 + 8 * q + (lane / MT) * 4;
          m4q[q] = *reinterpret_cast<const float4*>(a.marg + o);
          u4q[q] = *reinterpret_cast<const float4*>(Uin + o);
          x4q[q] = *reinterpret_cast<const float4*>(a.X + o);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int ab = a0 + 8 * q + (lane / MT) * 4;
          const int64_t o = static_cast<int64_t>(bl) * a.Kp + ab;
          const float4 m4 = m4q[q];
          const float mm[4] = {m4.x, m4.y, m4.z, m4.w};
          bool any = false;
#pragma unroll
          for (int e = 0; e < 4; ++e) any |= static_cast<double>(mm[e]) <= r_act[ib];
          if (!any) continue;
          const double* zq = &zacc[ia][ib][4 * q];
          *reinterpret_cast<float4*>(a.Z + o) =
              make_float4(static_cast<float>(zq[0]), static_cast<float>(zq[1]),
                          static_cast<float>(zq[2]), static_cast<float>(zq[3]));
          const float4 u4 = u4q[q];
          const float4 x4 = x4q[q];
          float uu[4] = {u4.x, u4.y, u4.z, u4.w};
          float xx[4] = {x4.x, x4.y, x4.z, x4.w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            if (!(static_cast<double>(mm[e]) <= r_act[ib])) continue;
            const double z = zq[e];
            zm = fmax(zm, fabs(z));
            const double p = uu[e];
            om += fabs(p);
            ++nact;
            nsup += uu[e] != 0.f;
            const double v = p - z * invL;
            const double mag = fabs(v) - thr;
            const double xn = mag > 0.0 ? copysign(mag, v) : 0.0;
            const double un = xn + beta * (xn - static_cast<double>(xx[e]));
            xx[e] = static_cast<float>(xn);
            uu[e] = static_cast<float>(un);
          }
          *reinterpret_cast<float4*>(a.X + o) = make_float4(xx[0], xx[1], xx[2], xx[3]);
          *reinterpret_cast<float4*>(Uout + o) = make_float4(uu[0], uu[1], uu[2], uu[3]);
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (uu[e] != 0.f) bits |= 1u << (8 * q + (lane / MT) * 4 + e);
        }
      }
      // the two half-waves hold the same signals on different atoms of the tile
      zm = fmax(zm, __shfl_xor(zm, 32, BW));
      om += __shfl_xor(om, 32, BW);
      int cnt = nact | (nsup << 8);
      cnt += __shfl_xor(cnt, 32, BW);
      bits |= __shfl_xor(bits, 32, BW);
      if (lane < MT) {
        a.pz[tix] = zm;
        a.pom[tix] = om;
        a.pact[tix] = cnt;
        a.umask[tix] = bits;
      }
    }
  }
  if (a.kclk != nullptr && lane == 0) a.kclk[2 * gw + 1] = wall_clock64();
}

// The block shapes the autotuner chooses from: {RA, RB, WA, WB} (RA x RB waves, each
// WA x WB output tiles of 32 x 32).
struct ZShapeDesc { int ra, rb, wa, wb; };
constexpr ZShapeDesc ZSHAPES[] = {{2, 2, 1, 1}, {4, 2, 1, 1}, {4, 1, 1, 1}, {2, 4, 1, 1},
                                  {1, 4, 1, 1}, {2, 2, 2, 1}, {4, 1, 2, 1}};
constexpr int NZSHAPE = sizeof(ZSHAPES) / sizeof(ZSHAPES[0]);
constexpr int KP_ALIGN = 128;  // Kp is a multiple of it; larger atom extents need Kp % TA == 0

constexpr int GCH = BW;  // groups per partial entry (one wave)

// The update of Table 1 for the Group-Lasso (one thread per (group, signal), for the groups
// active in this iteration): v_g = p_g - z_g / L, x_g = max(0, 1 - (lambda / L) w_g /
// ||v_g||) v_g (eq. gr_softTh, FP64), FISTA momentum u_g = x_g + beta (x_g - x_{t-1,g}).
// Per 64-group chunk (one wave): max ||z_g|| / w_g, Omega(p) = sum w_g ||p_g||, the active
// atoms and the non-zeros of p.  The new non-zero bits of u are OR-ed into the tile masks,
// which the GEMM cleared (a group can span tiles).
__global__ __launch_bounds__(TB) void k_b_gprox(BArgs a, const float* __restrict__ Uin,
                                                float* __restrict__ Uout) {
  const int s = blockIdx.y, g = blockIdx.x * TB + threadIdx.x, lane = threadIdx.x % BW;
  const Inst& st = a.inst[s];
  if (st.done != 0) return;  // the whole block: one signal
  const double invL = 1.0 / a.L, thr = st.lam / a.L, r_act = st.r_keep;
  double beta = 0.0;
  if (a.rule == 1) {
    const double lp = st.l_prev;
    beta = (lp - 1.0) / (0.5 * (1.0 + sqrt(1.0 + 4.0 * lp * lp)));
  }
  const int64_t row = static_cast<int64_t>(s) * a.Kp;
  double zs = 0.0, om = 0.0;
  int nact = 0, nsup = 0;
  if (g < a.G) {
    const int64_t g0 = a.gptr[g], g1 = a.gptr[g + 1];
    const int m = static_cast<int>(g1 - g0);
    constexpr int GS = 16;  // groups up to this size: all loads issued before the first use
    if (m > 0 && m <= GS && static_cast<double>(a.marg[row + g0]) <= r_act) {
      // the same arithmetic, in the same order, as the loops below
      float zl[GS], pl[GS], xl[GS];
#pragma unroll
      for (int k = 0; k < GS; ++k) {
        const int64_t o = row + g0 + min(k, m - 1);
        zl[k] = a.Z[o];
        pl[k] = Uin[o];
        xl[k] = a.X[o];
      }
      double zz = 0.0, vv = 0.0, pp = 0.0;
#pragma unroll
      for (int k = 0; k < GS; ++k) {
        if (k < m) {
          const double z = zl[k], p = pl[k];
          const double v = p - z * invL;
          zz = fma(z, z, zz);
          vv = fma(v, v, vv);
          pp = fma(p, p, pp);
          nsup += p != 0.0;
        }
      }
      const double w = a.gw[g];
      nact = m;
      zs = sqrt(zz) / w;
      om = w * sqrt(pp);
      const double nv = sqrt(vv);
      const double sc = nv > 0.0 ? fmax(0.0, 1.0 - thr * w / nv) : 0.0;
      uint32_t bits = 0u;
      int64_t tile = g0 / MT;
#pragma unroll
      for (int k = 0; k < GS; ++k) {
        if (k < m) {
          const int64_t ka = g0 + k;
          if (ka / MT != tile) {
            if (bits != 0u) atomicOr(&a.umask[tile * a.Bp + s], bits);
            bits = 0u;
            tile = ka / MT;
          }
          const double z = zl[k], p = pl[k];
          const double xn = sc * (p - z * invL);
          const double un = xn + beta * (xn - static_cast<double>(xl[k]));
          const float uf = static_cast<float>(un);
          a.X[row + ka] = static_cast<float>(xn);
          Uout[row + ka] = uf;
          if (uf != 0.f) bits |= 1u << (ka % MT);
        }
      }
      if (bits != 0u) atomicOr(&a.umask[tile * a.Bp + s], bits);
    } else if (m > GS && static_cast<double>(a.marg[row + g0]) <= r_act) {
      double zz = 0.0, vv = 0.0, pp = 0.0;
      for (int64_t k = g0; k < g1; ++k) {
        const double z = a.Z[row + k], p = Uin[row + k];
        const double v = p - z * invL;
        zz = fma(z, z, zz);
        vv = fma(v, v, vv);
        pp = fma(p, p, pp);
        nsup += p != 0.0;
      }
      const double w = a.gw[g];
      nact = static_cast<int>(g1 - g0);
      zs = sqrt(zz) / w;
      om = w * sqrt(pp);
      const double nv = sqrt(vv);
      const double sc = nv > 0.0 ? fmax(0.0, 1.0 - thr * w / nv) : 0.0;
      uint32_t bits = 0u;
      int64_t tile = g0 / MT;
      for (int64_t k = g0; k < g1; ++k) {
        if (k / MT != tile) {
          if (bits != 0u) atomicOr(&a.umask[tile * a.Bp + s], bits);
          bits = 0u;
          tile = k / MT;
        }
        const double z = a.Z[row + k], p = Uin[row + k];
        const double xn = sc * (p - z * invL);
        const double un = xn + beta * (xn - static_cast<double>(a.X[row + k]));
        const float uf = static_cast<float>(un);
        a.X[row + k] = static_cast<float>(xn);
        Uout[row + k] = uf;
        if (uf != 0.f) bits |= 1u << (k % MT);
      }
      if (bits != 0u) atomicOr(&a.umask[tile * a.Bp + s], bits);
    }
  }
  zs = wave_max(zs);
  om = wave_sum(om);
  nact = wave_sum(nact);
  nsup = wave_sum(nsup);
  const int ch = g / GCH;
  if (lane == 0 && ch * GCH < a.G) {
    const int64_t o = static_cast<int64_t>(ch) * a.Bp + s;
    a.pz[o] = zs;
    a.pom[o] = om;
    a.pact[o] = nact | (nsup << 16);
  }
}

// FP64 scalars of iteration t, one wave per slot: dual scaling (Lemma 7) from the MFMA
// correlations, gap estimate, sphere radius (SAFE: R; DST3: sqrt(R^2 - rho^2)) grown by
// the accumulation slack, screening threshold for the next iteration.  Flags the signal
// for the exact gap when the estimate meets tolerance or the budget is spent.
__global__ __launch_bounds__(TB) void k_b_scalars(BArgs a) {
  // Block: SPB consecutive signals x TG tile groups.  Thread (tg, sl) sums the partial
  // entries tg, tg + TG, ... of signal s0 + sl in that order (a wave reads SPB consecutive
  // signals of four entries per load: whole cache lines), then the TG sums of a signal are
  // combined in group order and one thread per signal forms its scalars.
  constexpr int SPB = 16, TG = TB / SPB;
  __shared__ double r_z[TG][SPB], r_o[TG][SPB], r_t[TG][SPB], r_y[TG][SPB];
  __shared__ int r_a[TG][SPB], r_s[TG][SPB];
  const int sl = threadIdx.x % SPB, tg = threadIdx.x / SPB;
  const int s = blockIdx.x * SPB + sl;  // Bp is a multiple of 64
  // partial entries: 32-atom tiles (Lasso) or 64-group chunks, whose counts pack the
  // active atoms and the non-zeros of p in 8- or 16-bit fields
  const int ntile = a.G > 0 ? (a.G + GCH - 1) / GCH : a.Kp / MT;
  const int cb = a.G > 0 ? 16 : 8;
  const int cm = (1 << cb) - 1;
  // Every load is issued before the first wait, at clamped indices: the signal's state
  // (each of its TG threads reads the same words), the first row-block partials of theta
  // and the first QT tile entries of this thread (all of them while ntile <= TG * QT).
  // The sums then run in the same order as one entry at a time.
  Inst& st = a.inst[s];
  const int t_done = st.done, t_iter = st.iter;
  const double lam = st.lam, yy = st.yy, rho2 = st.rho2;
  const double act_sum = st.act_sum, sup_sum = st.sup_sum, r_min = st.r_min;
  const double r_keep_old = st.r_keep, l_prev = st.l_prev, r_scr_old = st.r_scr;
  const double marg_slack = st.marg_slack, gap_tol_abs = st.gap_tol_abs;
  const int64_t oc = static_cast<int64_t>(min(tg, a.nrb - 1)) * a.Bp + s;
  const double tt0 = a.ptt[oc], ty0 = a.pty[oc];
  double zm = 0.0, om = 0.0;
  int nact = 0, nsup = 0;
  constexpr int QT = 24;
  for (int t0 = tg; t0 < ntile; t0 += TG * QT) {
    double qz[QT], qo[QT];
    int qa[QT];
#pragma unroll
    for (int q = 0; q < QT; ++q) {
      const int64_t o = static_cast<int64_t>(min(t0 + q * TG, ntile - 1)) * a.Bp + s;
      qz[q] = a.pz[o];
      qo[q] = a.pom[o];
      qa[q] = a.pact[o];
    }
#pragma unroll
    for (int q = 0; q < QT; ++q) {
      if (t0 + q * TG < ntile) {
        zm = fmax(zm, qz[q]);
        om += qo[q];
        nact += qa[q] & cm;
        nsup += qa[q] >> cb;
      }
    }
  }
  double tt = tg < a.nrb ? tt0 : 0.0, ty = tg < a.nrb ? ty0 : 0.0;
  for (int c = tg + TG; c < a.nrb; c += TG) {
    tt += a.ptt[static_cast<int64_t>(c) * a.Bp + s];
    ty += a.pty[static_cast<int64_t>(c) * a.Bp + s];
  }
  r_z[tg][sl] = zm;
  r_o[tg][sl] = om;
  r_t[tg][sl] = tt;
  r_y[tg][sl] = ty;
  r_a[tg][sl] = nact;
  r_s[tg][sl] = nsup;
  __syncthreads();
  if (tg != 0) return;
#pragma unroll
  for (int k = 1; k < TG; ++k) {
    zm = fmax(zm, r_z[k][sl]);
    om += r_o[k][sl];
    tt += r_t[k][sl];
    ty += r_y[k][sl];
    nact += r_a[k][sl];
    nsup += r_s[k][sl];
  }
  if (t_done != 0) return;
  const int t = t_iter + 1;
  const double sb = zm > 0.0 ? 1.0 / zm : 1e300;
  double mu = 0.0;
  if (tt > 0.0) mu = fmin(fmax(ty / (lam * tt), -sb), sb);
  const double primal = 0.5 * tt + lam * om;
  const double dual = lam * mu * ty - 0.5 * lam * lam * mu * mu * tt;
  // R^2 = ||y/lambda - v||^2 expanded; E bounds its FP64 rounding, eps |mu| ||theta|| the
  // distance from v to the feasible point of the exact correlations
  const double a1 = yy / (lam * lam), a2 = 2.0 * mu * ty / lam, a3 = mu * mu * tt;
  const double rr = a.test == 2 ? rho2 : 0.0;
  const double R2 = a1 - a2 + a3;
  const double E = (a.N + 16) * 0x1p-53 * (a1 + fabs(a2) + a3 + rr);
  const double nth = sqrt(tt);
  // relative error of max|z| (groups: of max ||z_g|| / w_g, from the stored FP32 z)
  const double eps = zm > 0.0 ? a.gamma_acc * a.dsc[0] * nth / zm + (a.G > 0 ? 0x1p-23 : 0.0) : 0.0;
  const double Rup = sqrt(fmax(R2 + E, 0.0)) + eps * fabs(mu) * nth;
  double r = 1e300, r_safe = 1e300;
  if (a.test != 0) {
    r = sqrt(fmax(R2 - rr, 0.0));
    r_safe = sqrt(fmax(Rup * Rup - rr + E, 0.0));
  }
  st.iter = t;
  st.tt = tt;
  st.ty = ty;
  st.act_sum = act_sum + nact;
  st.sup_sum = sup_sum + nsup;
  st.zmax = zm;
  st.omega = om;
  st.mu = mu;
  st.gap = primal - dual;
  st.primal = primal;
  st.dual = dual;
  st.r_min = fmin(r_min, r);
  st.r_prev = r_keep_old;
  if (a.rule == 1) st.l_prev = 0.5 * (1.0 + sqrt(1.0 + 4.0 * l_prev * l_prev));
  double r_scr = r_scr_old;
  if (r_safe < r_scr && (!a.screen_static || t == 1)) {  // static: first radius only
    r_scr = r_safe;
    st.r_scr = r_safe;
    st.r_slack = r_safe - r;
  }
  st.r_keep = fmin(r_keep_old, r_scr + marg_slack);
  // the estimate differs from the exact gap only through max|z|: every iteration whose
  // estimate is within VWIN of tolerance is checked, so the solve ends at the first
  // iteration whose exact gap meets it
  const bool flag = (gap_tol_abs > 0.0 && primal - dual <= VWIN * gap_tol_abs) || t >= a.max_iter;
  st.verify = flag ? 1 : 0;
  if (flag) a.vlist[atomicAdd(a.vcount, 1)] = s;
}

constexpr int VC = TB * 4;  // atoms per candidate block
constexpr int VG = 16;      // groups of flagged signals compacted at once (grid y)

// Verification, step 1: candidates for the FP64 maximum over the atoms active in this
// iteration of |d_i^T theta|, for the flagged signals.  With e a bound on
// |z_hat_i - d_i^T theta| for every atom (the accumulation bound plus the FP32 rounding of
// the stored z_hat), an atom with |z_hat_i| < max_k |z_hat_k| - 2 e cannot attain the
// maximum; the others are listed in atom order.  Block: 1024 atoms of one flagged signal.
__global__ __launch_bounds__(TB) void k_b_vcand(BArgs a) {
  __shared__ int scan[NWB];
  const int nflag = *a.vcount;
  const int nch = (a.K + VC - 1) / VC;
  const int i0 = blockIdx.x * VC;
  for (int j = blockIdx.y; j < nflag; j += gridDim.y) {
    const int s = a.vlist[j];
    const Inst& st = a.inst[s];
    const double r_act = st.r_prev;
    const double zmax = st.zmax;
    const double e = a.gamma_acc * a.dsc[0] * sqrt(st.tt) + 0x1p-23 * zmax;
    const double thr = zmax - 2.0 * e;
    const float* z = a.Z + static_cast<int64_t>(s) * a.Kp;
    const float* mg = a.marg + static_cast<int64_t>(s) * a.Kp;
    int* out = a.cidx + static_cast<int64_t>(s) * a.Kp + i0;
    int mine[4], cnt = 0;
    // the thread's four margins and correlations in two 16-byte loads (rows are Kp long,
    // Kp a multiple of 64; the index is clamped into the row and entries past K ignored)
    const int ib = i0 + threadIdx.x * 4;
    const int ic = min(ib, a.Kp - 4);
    const float4 m4 = *reinterpret_cast<const float4*>(mg + ic);
    const float4 z4 = *reinterpret_cast<const float4*>(z + ic);
    const float mv[4] = {m4.x, m4.y, m4.z, m4.w}, zv[4] = {z4.x, z4.y, z4.z, z4.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = ib + k;
      const bool c = i < a.K && static_cast<double>(mv[k]) <= r_act &&
                     fabs(static_cast<double>(zv[k])) >= thr;
      mine[k] = c ? i : -1;
      cnt += c;
    }
    int total;
    int pos = block_exclusive_scan<NWB>(cnt, scan, &total);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (mine[k] >= 0) out[pos++] = mine[k];
    if (threadIdx.x == 0) a.ccount[static_cast<int64_t>(s) * nch + blockIdx.x] = total;
    __syncthreads();
  }
}

// Verification, step 2: exact FP64 |d_i^T theta| of every candidate of every flagged
// signal, one wave per candidate (rows across the lanes), all waves of the grid sharing
// the work in a fixed order.
constexpr int VLDS = 2048;  // (signal, range) pairs staged in LDS per round

__global__ __launch_bounds__(TB) void k_b_vdot(BArgs a) {
  __shared__ int ssig[VLDS];
  __shared__ int scnt[VLDS];
  const int nflag = *a.vcount;
  const int lane = threadIdx.x % BW;
  const int nw = gridDim.x * NWB;
  const int gw = blockIdx.x * NWB + threadIdx.x / BW;
  const int nch = (a.K + VC - 1) / VC;
  const int npair = nflag * nch;
  int off = 0;  // work items before the current pair, in the fixed order of all waves
  for (int p0 = 0; p0 < npair; p0 += VLDS) {
    const int np = min(VLDS, npair - p0);
    __syncthreads();
    for (int e = threadIdx.x; e < np; e += TB) {
      const int jc = p0 + e;
      const int sg = a.vlist[jc / nch];
      ssig[e] = sg;
      scnt[e] = a.ccount[static_cast<int64_t>(sg) * nch + jc % nch];
    }
    __syncthreads();
    for (int e = 0; e < np; ++e) {
      const int s = ssig[e], ch = (p0 + e) % nch, cnt = scnt[e];
      const double* th = a.th64 + static_cast<int64_t>(s) * a.Np;
      for (int c = ((gw - off) % nw + nw) % nw; c < cnt; c += nw) {
        const int64_t slot = static_cast<int64_t>(s) * a.Kp + ch * VC + c;
        const uint16_t* col = a.dcm + static_cast<int64_t>(a.cidx[slot]) * a.Np;
        double acc = 0.0;
        // NB steps of 512 rows per batch, every load issued before the first FMA; steps
        // past the end re-read the last rows with weight zero (acc starts at +0 and never
        // becomes -0, so a zero product leaves it unchanged bit for bit)
        constexpr int NB = 4;
        for (int n0 = lane * 8; n0 < a.Np; n0 += NB * BW * 8) {
          uint4 d[NB];
          double2 t2[NB][4];
#pragma unroll
          for (int k = 0; k < NB; ++k) {
            const int n = min(n0 + k * BW * 8, a.Np - 8);
            d[k] = ldg16(col + n);
#pragma unroll
            for (int q = 0; q < 4; ++q) t2[k][q] = *reinterpret_cast<const double2*>(th + n + 2 * q);
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int k = 0; k < NB; ++k) {
            const bool ok = n0 + k * BW * 8 < a.Np;
            const uint32_t w[4] = {d[k].x, d[k].y, d[k].z, d[k].w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              acc = fma(static_cast<double>(__uint_as_float(w[q] << 16)), ok ? t2[k][q].x : 0.0, acc);
              acc = fma(static_cast<double>(__uint_as_float(w[q] & 0xffff0000u)), ok ? t2[k][q].y : 0.0, acc);
            }
          }
        }
        acc = wave_sum(acc);
        if (lane == 0) a.cval[slot] = fabs(acc);
      }
      off += cnt;
    }
  }
}

// Verification for groups, step 1: candidate groups for the FP64 maximum of
// ||D_g^T theta|| / w_g over the groups active in this iteration.  ||z_hat_g|| / w_g is
// within e = gamma_acc dsc[0] ||theta|| + 2^-23 zmax of the exact value (the accumulation
// bound summed over the group's atoms, and the FP32 rounding of the stored z), so a group
// below zmax - 2 e cannot attain the maximum.  Block: the groups whose first atom lies in
// a 1024-atom range of one flagged signal, listed in group order.
__global__ __launch_bounds__(TB) void k_b_gvcand(BArgs a) {
  __shared__ int scan[NWB];
  const int nflag = *a.vcount;
  const int nch = (a.K + VC - 1) / VC;
  const int i0 = blockIdx.x * VC;
  for (int j = blockIdx.y; j < nflag; j += gridDim.y) {
    const int s = a.vlist[j];
    const Inst& st = a.inst[s];
    const double r_act = st.r_prev;
    const double zmax = st.zmax;
    const double e = a.gamma_acc * a.dsc[0] * sqrt(st.tt) + 0x1p-23 * zmax;
    const double thr = zmax - 2.0 * e;
    const int64_t row = static_cast<int64_t>(s) * a.Kp;
    int* out = a.cidx + row + i0;
    int mine[4], cnt = 0;
    const int ib = i0 + threadIdx.x * 4;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = ib + k;
      mine[k] = -1;
      if (i >= a.K) continue;
      const int g = a.agrp[i];
      const int64_t g0 = a.gptr[g], g1 = a.gptr[g + 1];
      if (g0 != i || !(static_cast<double>(a.marg[row + i]) <= r_act)) continue;
      double zz = 0.0;
      for (int64_t q = g0; q < g1; ++q) {
        const double z = a.Z[row + q];
        zz = fma(z, z, zz);
      }
      if (sqrt(zz) / a.gw[g] >= thr) {
        mine[k] = g;
        ++cnt;
      }
    }
    int total;
    int pos = block_exclusive_scan<NWB>(cnt, scan, &total);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (mine[k] >= 0) out[pos++] = mine[k];
    if (threadIdx.x == 0) a.ccount[static_cast<int64_t>(s) * nch + blockIdx.x] = total;
    __syncthreads();
  }
}

// Verification for groups, step 2: exact FP64 ||D_g^T theta|| / w_g of every candidate
// group, one wave per candidate (each atom's dot product with the rows across the lanes,
// the squares summed in atom order), all waves of the grid sharing the work in a fixed
// order.
__global__ __launch_bounds__(TB) void k_b_gvdot(BArgs a) {
  __shared__ int ssig[VLDS];
  __shared__ int scnt[VLDS];
  const int nflag = *a.vcount;
  const int lane = threadIdx.x % BW;
  const int nw = gridDim.x * NWB;
  const int gw = blockIdx.x * NWB + threadIdx.x / BW;
  const int nch = (a.K + VC - 1) / VC;
  const int npair = nflag * nch;
  int off = 0;
  for (int p0 = 0; p0 < npair; p0 += VLDS) {
    const int np = min(VLDS, npair - p0);
    __syncthreads();
    for (int e = threadIdx.x; e < np; e += TB) {
      const int jc = p0 + e;
      const int sg = a.vlist[jc / nch];
      ssig[e] = sg;
      scnt[e] = a.ccount[static_cast<int64_t>(sg) * nch + jc % nch];
    }
    __syncthreads();
    for (int e = 0; e < np; ++e) {
      const int s = ssig[e], ch = (p0 + e) % nch, cnt = scnt[e];
      const double* th = a.th64 + static_cast<int64_t>(s) * a.Np;
      for (int c = ((gw - off) % nw + nw) % nw; c < cnt; c += nw) {
        const int64_t slot = static_cast<int64_t>(s) * a.Kp + ch * VC + c;
        const int g = a.cidx[slot];
        const int64_t g0 = a.gptr[g], g1 = a.gptr[g + 1];
        double s2 = 0.0;
        // AB atoms of the group at a time, each with its own accumulator (the same FMA
        // sequence per atom as one atom at a time): theta's rows are loaded once for all of
        // them and their column loads are in flight together
        constexpr int AB = 8;
        for (int64_t k0 = g0; k0 < g1; k0 += AB) {
          const int na = static_cast<int>(min(static_cast<int64_t>(AB), g1 - k0));
          double acc[AB];
#pragma unroll
          for (int j = 0; j < AB; ++j) acc[j] = 0.0;
          for (int n0 = lane * 8; n0 < a.Np; n0 += BW * 8) {
            double2 t2[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) t2[q] = *reinterpret_cast<const double2*>(th + n0 + 2 * q);
            uint4 d[AB];
#pragma unroll
            for (int j = 0; j < AB; ++j) d[j] = ldg16(a.dcm + (k0 + min(j, na - 1)) * a.Np + n0);
#pragma unroll
            for (int j = 0; j < AB; ++j) {
              const uint32_t w[4] = {d[j].x, d[j].y, d[j].z, d[j].w};
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                acc[j] = fma(static_cast<double>(__uint_as_float(w[q] << 16)), t2[q].x, acc[j]);
                acc[j] = fma(static_cast<double>(__uint_as_float(w[q] & 0xffff0000u)), t2[q].y, acc[j]);
              }
            }
          }
#pragma unroll
          for (int j = 0; j < AB; ++j) {
            if (j < na) {
              const double v = wave_sum(acc[j]);
              s2 = fma(v, v, s2);
            }
          }
        }
        if (lane == 0) a.cval[slot] = sqrt(s2) / a.gw[g];
      }
      off += cnt;
    }
  }
}

// Exact gap of the flagged signals (one wave per slot) at the feasible dual point
// v = mu theta, mu = clip(theta^T y / (lambda ||theta||^2), +-1/zs) with zs the FP64
// maximum plus the rounding bound of that pass (Lemma 7).  Finishes the signal when the
// gap meets tolerance or the iteration budget is spent.
__global__ __launch_bounds__(TB) void k_b_vfin(BArgs a) {
  const int lane = threadIdx.x % BW;
  const int s = blockIdx.x * NWB + threadIdx.x / BW;
  if (s >= a.Bp) return;
  Inst& st = a.inst[s];
  if (st.done != 0 || !st.verify) return;
  const int nch = (a.K + VC - 1) / VC;
  const int64_t cb = static_cast<int64_t>(s) * nch, vb = static_cast<int64_t>(s) * a.Kp;
  double zm = 0.0;
  // round trip 1: every chunk's candidate count (lane ch holds chunk ch); round trip 2: the
  // first BW candidates of the first QC chunks, unconditional loads at clamped indices
  constexpr int QC = 16;
  const int cnt_l = a.ccount[cb + min(lane, nch - 1)];
  double qv[QC];
  int qc[QC];
#pragma unroll
  for (int q = 0; q < QC; ++q) {
    const int ch = min(q, nch - 1);
    qc[q] = __builtin_amdgcn_readlane(cnt_l, ch);
    qv[q] = a.cval[vb + ch * VC + min(lane, max(qc[q] - 1, 0))];
  }
#pragma unroll
  for (int q = 0; q < QC; ++q)
    if (q < nch && lane < qc[q]) zm = fmax(zm, qv[q]);
  for (int ch = 0; ch < nch; ++ch) {  // the rest: candidates past BW, chunks past QC
    const int cnt = ch < BW ? __builtin_amdgcn_readlane(cnt_l, ch) : a.ccount[cb + ch];
    for (int c = lane + (ch < QC ? BW : 0); c < cnt; c += BW) zm = fmax(zm, a.cval[vb + ch * VC + c]);
  }
  zm = wave_max(zm);
  if (lane != 0) return;
  const double lam = st.lam, tt = st.tt, ty = st.ty;
  const double primal = st.primal, gap_tol_abs = st.gap_tol_abs;  // read before any store
  const int iter = st.iter;
  // groups: the sum of squares, the square root and the division add a few units of
  // rounding to each candidate's value (at most 132 atoms: below 2^-44 relative)
  const double zs = zm * (a.G > 0 ? 1.0 + 0x1p-44 : 1.0) + a.gamma64 * a.dsc[0] * sqrt(tt);
  const double sb = zs > 0.0 ? 1.0 / zs : 1e300;
  double mu = 0.0;
  if (tt > 0.0) mu = fmin(fmax(ty / (lam * tt), -sb), sb);
  const double dual = lam * mu * ty - 0.5 * lam * lam * mu * mu * tt;
  const double gap = primal - dual;
  st.zmax = zm;
  st.mu = mu;
  st.dual = dual;
  st.gap = gap;
  st.verify = 0;
  const bool ok = gap_tol_abs > 0.0 && gap <= gap_tol_abs;
  if (ok || iter >= a.max_iter) {
    st.converged = (ok || gap_tol_abs <= 0.0) ? 1 : 0;
    st.done = 2;
    atomicAdd(a.ndone, 1);
  }
}

// Screening (the test of Algorithm 3 for the sphere tests): the pairs with
// r_keep < margin <= r_prev leave the active set and their x and u (both buffers) are
// cleared; a non-zero bit the update left for such an atom then reads a zero u.  Signals
// that finished this iteration keep x_t.  Thread: 4 consecutive atoms of one signal.
__global__ __launch_bounds__(TB) void k_b_screen(BArgs a) {
  const int s = blockIdx.y;
  const Inst& st = a.inst[s];
  const int i4 = (blockIdx.x * TB + threadIdx.x) * 4;
  // the state and the tile's minimum margin in one round trip (index clamped into the row)
  const float tm = a.tminm[static_cast<int64_t>(min(i4, a.Kp - 4) / MT) * a.Bp + s];
  const int done = st.done;
  const double rk = st.r_keep, rp = st.r_prev;
  if (done != 0 || !(rk < rp) || i4 >= a.Kp) return;
  if (!(static_cast<double>(tm) <= rp)) return;
  const int64_t o = static_cast<int64_t>(s) * a.Kp + i4;
  const float4 m4 = *reinterpret_cast<const float4*>(a.marg + o);
  const float mm[4] = {m4.x, m4.y, m4.z, m4.w};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const double m = mm[e];
    if (m > rk && m <= rp) {
      a.X[o + e] = 0.f;
      a.U0[o + e] = 0.f;
      a.U1[o + e] = 0.f;
    }
  }
}

// A slot assignment: perm[list[j]] = sig[j] (-1: idle) and lam[list[j]] = lamv[j], j < n.
__global__ __launch_bounds__(TB) void k_b_assign(int* __restrict__ perm, double* __restrict__ lam,
                                                 const int* __restrict__ list,
                                                 const int* __restrict__ sig,
                                                 const double* __restrict__ lamv, int n) {
  const int j = blockIdx.x * TB + threadIdx.x;
  if (j >= n) return;
  perm[list[j]] = sig[j];
  lam[list[j]] = lamv[j];
}

// ============================================================== output
// After each run of iterations, one block per slot: a slot that holds a signal (perm[s] >= 0)
// and has finished is harvested: its counts for the report (non-zeros of x, atoms active in
// the last iteration), x_t into column perm[s] of Xout (leading dimension ldx), the optional
// screened mask (1 = screened, leading dimension K); then perm[s] = -1 (the host clears its
// copy when it reads the flag).  flags[s] = 1 for the slots harvested here, else 0.  A
// finished signal's x and state are no longer changed by the iteration kernels.
__global__ __launch_bounds__(TB) void k_b_harvest(BArgs a, int* __restrict__ perm,
                                                  float* __restrict__ Xout, int64_t ldx,
                                                  uint8_t* __restrict__ scr,
                                                  int* __restrict__ flags) {
  __shared__ int si[NWB];
  const int s = blockIdx.x;
  const int b = perm[s];
  Inst& st = a.inst[s];
  const bool fin = b >= 0 && st.done != 0;
  if (threadIdx.x == 0) flags[s] = fin ? 1 : 0;
  if (!fin) return;
  const bool trivial = st.status != 0;
  const double rp = st.r_prev;
  constexpr int HU = 8;  // atoms per thread whose loads are issued before the first store
  int nz = 0, na = 0;
  const int64_t o = static_cast<int64_t>(s) * a.Kp;
  for (int i0 = threadIdx.x; i0 < a.K; i0 += TB * HU) {
    float xv[HU], mv[HU];
#pragma unroll
    for (int u = 0; u < HU; ++u) {
      const int i = min(i0 + u * TB, a.K - 1);
      xv[u] = a.X[o + i];
      mv[u] = a.marg[o + i];
    }
#pragma unroll
    for (int u = 0; u < HU; ++u) {
      const int i = i0 + u * TB;
      if (i >= a.K) break;
      const bool act = static_cast<double>(mv[u]) <= rp;
      nz += xv[u] != 0.f;
      na += act;
      Xout[static_cast<int64_t>(b) * ldx + i] = trivial ? 0.f : xv[u];
      if (scr != nullptr) scr[static_cast<int64_t>(b) * a.K + i] = (trivial || !act) ? 1 : 0;
    }
  }
  nz = block_sum<int, NWB>(nz, si);  // every thread has read perm[s] before this barrier
  na = block_sum<int, NWB>(na, si);
  if (threadIdx.x == 0) {
    st.nnz = trivial ? 0 : nz;
    st.n_active = trivial ? 0 : na;
    perm[s] = -1;
  }
}

}  // namespace batch
}  // namespace ds
