// Single-signal kernels: Algorithm 3 with ISTA / FISTA (Table 1) and the sphere tests of
// Lemmas 1, 2, 4, 5 (through Lemma 6), one signal at a time.
//
// Per iteration two launches on one stream:
//   k_resid  theta = D_S p_S - y over the support S of the primal point p (row tiles x
//            support segments, FP64 accumulation, per-tile FP64 ||theta||^2, theta^T y);
//            every block first recomputes the FP64 scalars of the previous iteration
//            (dual scaling Lemma 7, gap, radius, stopping rule) from published partials.
//   k_corr   z = D_A^T theta over the active list A (the HBM stream), fused with the prox
//            (eq. softTh / gr_softTh), the FISTA momentum, ||z||_inf or the group norms,
//            Omega(p) and nnz; it drops screened entries from A while it reads them and,
//            when enough are stale, rewrites A in order (decoupled look-back), and it
//            publishes the support of the new primal point for the next k_resid.
// Every scalar is in device memory (SolverState); once `done` is set the kernels return
// immediately, so the host may enqueue iterations ahead of the stopping decision.
#pragma once
#include <cmath>

#include "ds_device.h"
#include "ds_state.h"

namespace ds {

constexpr int BLK = 256;         // threads per block of the streaming kernels
constexpr int NW = BLK / WAVE;   // waves per block
constexpr int CPW = 2;           // columns streamed at once by one wave (more slows HBM)
constexpr int RPW = 8;           // support columns one residual wave loads at once
constexpr int CBLK = 1024;       // threads of the single-block kernels
constexpr int CNW = CBLK / WAVE;
constexpr int MAXB = 16384;      // maximum grid of the kernels with block partials
constexpr int MAXRT = 4096;      // maximum row tiles of the residual
constexpr int GMAX = 128;        // largest group (two atoms per lane in the group epilogue)

enum CounterSlot { CNT_FIN = 0, CNT_CORR = 1, CNT_VID = 2, CNT_SUB = 8 };

// Cross-block publication without agent-scope fences: an agent-scope atomic store goes
// to the coherence point directly, and waiting for it before the arrival counter makes
// it visible to whichever block observes the counter (a release fence would also write
// back the whole L2, which doubles the runtime of a streaming kernel).
template <typename X>
__device__ __forceinline__ void publish(X* p, X v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename X>
__device__ __forceinline__ X consume(const X* p) {
  return __hip_atomic_load(const_cast<X*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Arrival counter after the block's publications; true in the block that arrives last.
__device__ __forceinline__ bool arrive_last(unsigned* counter, unsigned expected, int* flag_lds) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *flag_lds = (prev == expected - 1u) ? 1 : 0;
  }
  __syncthreads();
  return *flag_lds != 0;
}


// ---------------------------------------------------------------- vector loads ------
__device__ __forceinline__ uint4 ld16(const void* p) { return *reinterpret_cast<const uint4*>(p); }

// Widen one raw 16-byte load of stored elements to FP64.
template <typename T> __device__ __forceinline__ void widen(const uint4& r, double (&o)[Store<T>::VEC]);
template <> __device__ __forceinline__ void widen<double>(const uint4& r, double (&o)[2]) {
  o[0] = __hiloint2double(static_cast<int>(r.y), static_cast<int>(r.x));
  o[1] = __hiloint2double(static_cast<int>(r.w), static_cast<int>(r.z));
}
template <> __device__ __forceinline__ void widen<float>(const uint4& r, double (&o)[4]) {
  o[0] = __uint_as_float(r.x); o[1] = __uint_as_float(r.y);
  o[2] = __uint_as_float(r.z); o[3] = __uint_as_float(r.w);
}
template <> __device__ __forceinline__ void widen<bf16_t>(const uint4& r, double (&o)[8]) {
  o[0] = __uint_as_float(r.x << 16); o[1] = __uint_as_float(r.x & 0xffff0000u);
  o[2] = __uint_as_float(r.y << 16); o[3] = __uint_as_float(r.y & 0xffff0000u);
  o[4] = __uint_as_float(r.z << 16); o[5] = __uint_as_float(r.z & 0xffff0000u);
  o[6] = __uint_as_float(r.w << 16); o[7] = __uint_as_float(r.w & 0xffff0000u);
}
// FP64 values of TW raw 16-byte loads of a float or double vector.
template <typename VV, int TW, int NV>
__device__ __forceinline__ void widen_raw(const uint4 (&r)[TW], double (&o)[NV]) {
  if constexpr (sizeof(VV) == 4) {
    static_assert(NV == 4 * TW, "four floats per load");
#pragma unroll
    for (int w = 0; w < TW; ++w) {
      o[4 * w] = __uint_as_float(r[w].x); o[4 * w + 1] = __uint_as_float(r[w].y);
      o[4 * w + 2] = __uint_as_float(r[w].z); o[4 * w + 3] = __uint_as_float(r[w].w);
    }
  } else {
    static_assert(NV == 2 * TW, "two doubles per load");
#pragma unroll
    for (int w = 0; w < TW; ++w) {
      o[2 * w] = __hiloint2double(static_cast<int>(r[w].y), static_cast<int>(r[w].x));
      o[2 * w + 1] = __hiloint2double(static_cast<int>(r[w].w), static_cast<int>(r[w].z));
    }
  }
}

// FP64 dot products of NC columns with a vector v, by one wave.  Branch-free: every
// column pointer must be valid (callers repeat a valid column for unused slots).  With
// VECTOR the columns and v are 16-byte aligned and are read in batches of SB steps of
// 64 x VEC elements whose loads are all in flight before the first FMA (a 2000-row FP32
// column pair is one batch of 24 loads per lane); the tail N % VEC is read element-wise.
template <typename T, typename VV, int NC, bool VECTOR>
__device__ __forceinline__ void wave_dots(const T* const (&cols)[NC], const VV* __restrict__ v,
                                          int N, int lane, double (&acc)[NC]) {
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = 0.0;
  if constexpr (VECTOR) {
    constexpr int VEC = Store<T>::VEC;
    // Steps of 64 x VEC elements whose loads are all issued before the first FMA: eight
    // when one step of v is one 16-byte load, else four.  A column of up to SB * 64 * VEC
    // elements is one round trip; steps past the end re-read the last vector and get a
    // zero weight.
    constexpr int TW = VEC * static_cast<int>(sizeof(VV)) / 16;  // 16-byte loads of v per step
    constexpr int SB = TW == 1 ? 8 : 4;
    const int nfull = N / VEC;
    for (int q0 = 0; q0 < nfull; q0 += SB * WAVE) {
      uint4 tr[SB][TW];
      uint4 r[SB][NC];
      // v first: loads complete in issue order, so step k waits only for its own data
#pragma unroll
      for (int k = 0; k < SB; ++k) {
        const int q = min(q0 + lane + k * WAVE, nfull - 1);
#pragma unroll
        for (int w = 0; w < TW; ++w) tr[k][w] = ld16(v + static_cast<int64_t>(q) * VEC + w * (16 / sizeof(VV)));
      }
#pragma unroll
      for (int k = 0; k < SB; ++k) {
        const int q = min(q0 + lane + k * WAVE, nfull - 1);
#pragma unroll
        for (int c = 0; c < NC; ++c) r[k][c] = ld16(cols[c] + static_cast<int64_t>(q) * VEC);
      }
      // keep the scheduler from interleaving the FMAs (and their waits) with the loads
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < SB; ++k) {
        const bool ok = q0 + lane + k * WAVE < nfull;
        double t[VEC];
        widen_raw<VV>(tr[k], t);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          double d[VEC];
          widen<T>(r[k][c], d);
#pragma unroll
          for (int e = 0; e < VEC; ++e) acc[c] = fma(d[e], ok ? t[e] : 0.0, acc[c]);
        }
      }
    }
    const int e = nfull * VEC + lane;
    if (e < N) {
      const double ve = static_cast<double>(v[e]);
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] = fma(to_double(cols[c][e]), ve, acc[c]);
    }
  } else {
    for (int e = lane; e < N; e += WAVE) {
      const double ve = static_cast<double>(v[e]);
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] = fma(to_double(cols[c][e]), ve, acc[c]);
    }
  }
}

template <typename X, int NC>
__device__ __forceinline__ X pick(const X (&a)[NC], int c) {
  X r = a[0];
#pragma unroll
  for (int k = 1; k < NC; ++k)
    if (c == k) r = a[k];
  return r;
}

// Decoupled look-back: exclusive prefix of `agg` over virtual blocks 0..vb-1.  Words are
// [epoch:16 | flag:2 | value:46]; flag 1 = aggregate only, 2 = inclusive prefix.  The
// virtual block ids are handed out by an atomic counter in arrival order, so every
// predecessor has started and will publish: the wait always ends.
__device__ inline int lookback_prefix(uint64_t* status, int vb, int agg, uint32_t epoch) {
  const uint64_t E = static_cast<uint64_t>(epoch) << 48;
  constexpr uint64_t FA = 1ull << 46, FI = 2ull << 46, VMASK = (1ull << 46) - 1ull;
  if (vb == 0) {
    __hip_atomic_store(&status[0], E | FI | static_cast<uint64_t>(agg), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    return 0;
  }
  __hip_atomic_store(&status[vb], E | FA | static_cast<uint64_t>(agg), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
  int64_t prefix = 0;
  int j = vb - 1;
  while (true) {
    const uint64_t w = __hip_atomic_load(&status[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t flag = (w >> 46) & 3ull;
    if ((w >> 48) != epoch || flag == 0) {
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    prefix += static_cast<int64_t>(w & VMASK);
    if (flag == 2) break;
    --j;
  }
  __hip_atomic_store(&status[vb], E | FI | static_cast<uint64_t>(prefix + agg), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
  return static_cast<int>(prefix);
}

// ============================================================== setup kernels =======

// z[i] = d_i^T v in FP64 and (optionally) nu[i] = ||d_i||, one wave per CPW columns.
template <typename T, typename VV, bool VECTOR, bool NORMS>
__global__ __launch_bounds__(BLK) void k_setup_gemv(const T* __restrict__ D, int64_t ldd,
                                                     int N, int K, const VV* __restrict__ v,
                                                     double* __restrict__ z,
                                                     double* __restrict__ nu) {
  const int lane = threadIdx.x % WAVE;
  const int gw = blockIdx.x * NW + threadIdx.x / WAVE;
  const int nwaves = gridDim.x * NW;
  for (int base = gw * CPW; base < K; base += nwaves * CPW) {
    const int nc = min(CPW, K - base);
    const T* cols[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) cols[c] = D + static_cast<int64_t>(base + min(c, nc - 1)) * ldd;
    double acc[CPW];
    wave_dots<T, VV, CPW, VECTOR>(cols, v, N, lane, acc);
    double sq[CPW];
    if constexpr (NORMS) {
      // columns past nc repeat the last one (their sums are never picked), so every load
      // is unconditional and a row step's loads are in flight together
#pragma unroll
      for (int c = 0; c < CPW; ++c) sq[c] = 0.0;
#pragma unroll 4
      for (int e = lane; e < N; e += WAVE) {
        double d[CPW];
#pragma unroll
        for (int c = 0; c < CPW; ++c) d[c] = to_double(cols[c][e]);
#pragma unroll
        for (int c = 0; c < CPW; ++c) sq[c] = fma(d[c], d[c], sq[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      acc[c] = wave_sum(acc[c]);
      if constexpr (NORMS) sq[c] = wave_sum(sq[c]);
    }
    if (lane < nc) {
      z[base + lane] = pick(acc, lane);
      if constexpr (NORMS) nu[base + lane] = sqrt(pick(sq, lane));
    }
  }
}

// Group spectral norms ||D_g||_2 (Lemma 6) and Frobenius norms, one block per group, for
// groups of at most GM atoms:
//  1. the Gram matrix D_g^T D_g in FP64: rows of D_g are staged through LDS in chunks of
//     GRS rows (column-major, padded stride) and thread (ti, tj) of a 16 x 16 grid keeps
//     the TE x TE tile of columns ti*TE.., tj*TE.. in registers (every entry sums its exact
//     products in row order, so the matrix is exactly symmetric);
//  2. Householder reduction to tridiagonal form in LDS (the symmetric rank-2 update of the
//     trailing block evaluates entries (i, j) and (j, i) with the same expression, so the
//     block stays exactly symmetric);
//  3. the largest eigenvalue of the tridiagonal matrix by multisection on one wave: 64
//     trial points per round split the current interval (Gershgorin bounds at the start),
//     each lane counting the eigenvalues below its point with the Sturm recurrence; the
//     first point with every eigenvalue below it becomes the new upper end.  The norm is
//     the square root of the final upper end.
constexpr int GRS = 32;  // rows of D_g per staged chunk

template <int GM>
struct GramLds {
  static constexpr int TE = GM / 16;
  static constexpr int NA = GM * GM > GM * (GRS + 1) ? GM * GM : GM * (GRS + 1);
};

template <typename T, int GM>
__global__ __launch_bounds__(BLK) void k_group_norms(const T* __restrict__ D, int64_t ldd, int N,
                                                      int G, const int64_t* __restrict__ gptr,
                                                      double* __restrict__ gnorm,
                                                      double* __restrict__ fro) {
  constexpr int TE = GramLds<GM>::TE;
  static_assert(GM % 16 == 0 && BLK == 256, "16 x 16 thread grid of TE x TE tiles");
  __shared__ double gram[GramLds<GM>::NA];  // staged rows, then the Gram matrix (row-major)
  __shared__ double s_v[GM], s_w[GM], s_d[GM], s_e[GM], s_e2[GM];
  __shared__ double sd[NW];
  const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
  const int ti = tid / 16, tj = tid % 16;
  for (int g = blockIdx.x; g < G; g += gridDim.x) {
    const int64_t a0 = gptr[g];
    const int m = static_cast<int>(gptr[g + 1] - a0);
    // ---- 1. Gram matrix ----
    double acc[TE][TE];
#pragma unroll
    for (int x = 0; x < TE; ++x)
#pragma unroll
      for (int y = 0; y < TE; ++y) acc[x][y] = 0.0;
    const bool act = ti * TE < m && tj * TE < m;
    // chunk elements of this thread: unconditional loads at clamped indices (all in flight
    // together), the next chunk fetched while the current one is consumed
    constexpr int PER = GM * GRS / BLK;
    static_assert(GM * GRS % BLK == 0, "chunk elements tile the block");
    double vals[PER];
    auto fetch = [&](int r0) {
      const int nr = min(GRS, N - r0);
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = tid + q * BLK, c = min(e / GRS, m - 1), r = min(e % GRS, nr - 1);
        vals[q] = to_double(D[(a0 + c) * ldd + r0 + r]);
      }
    };
    fetch(0);
    for (int r0 = 0; r0 < N; r0 += GRS) {
      const int nr = min(GRS, N - r0);
      __syncthreads();  // the previous chunk has been consumed
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = tid + q * BLK, c = e / GRS, r = e % GRS;
        gram[c * (GRS + 1) + r] = (c < m && r < nr) ? vals[q] : 0.0;
      }
      __syncthreads();
      if (r0 + GRS < N) fetch(r0 + GRS);
      if (act) {
        for (int r = 0; r < nr; ++r) {
          double ca[TE], cb[TE];
#pragma unroll
          for (int x = 0; x < TE; ++x) {
            ca[x] = gram[(ti * TE + x) * (GRS + 1) + r];
            cb[x] = gram[(tj * TE + x) * (GRS + 1) + r];
          }
#pragma unroll
          for (int x = 0; x < TE; ++x)
#pragma unroll
            for (int y = 0; y < TE; ++y) acc[x][y] = fma(ca[x], cb[y], acc[x][y]);
        }
      }
    }
    __syncthreads();  // the staging area becomes the Gram matrix
#pragma unroll
    for (int x = 0; x < TE; ++x)
#pragma unroll
      for (int y = 0; y < TE; ++y) {
        const int i = ti * TE + x, j = tj * TE + y;
        if (i < m && j < m) gram[i * GM + j] = acc[x][y];
      }
    __syncthreads();
    const double f2 = block_sum<double, NW>(tid < m ? gram[tid * GM + tid] : 0.0, sd);
    // ---- 2. Householder tridiagonalisation: step k reflects rows / columns k+1 .. m-1 ----
    for (int k = 0; k + 2 < m; ++k) {
      const int n2 = m - k - 1;
      const double xi = tid < n2 ? gram[(k + 1 + tid) * GM + k] : 0.0;
      const double tail = block_sum<double, NW>(tid > 0 && tid < n2 ? xi * xi : 0.0, sd);
      const double x0 = gram[(k + 1) * GM + k];
      if (tail == 0.0) {  // already tridiagonal in this column
        if (tid == 0) s_e[k] = x0;
        continue;
      }
      const double nx = sqrt(fma(x0, x0, tail));
      const double alpha = x0 > 0.0 ? -nx : nx;
      const double v0 = x0 - alpha;  // |x0| + ||x||: no cancellation
      const double beta = 2.0 / fma(v0, v0, tail);
      if (tid < n2) s_v[tid] = tid == 0 ? v0 : xi;
      if (tid == 0) s_e[k] = alpha;
      __syncthreads();
      double pi = 0.0;  // p = beta A22 v, from column tid of the symmetric trailing block
      if (tid < n2) {
        for (int j = 0; j < n2; ++j) pi = fma(gram[(k + 1 + j) * GM + (k + 1 + tid)], s_v[j], pi);
        pi *= beta;
      }
      const double pv = block_sum<double, NW>(tid < n2 ? pi * s_v[tid] : 0.0, sd);
      if (tid < n2) s_w[tid] = fma(-0.5 * beta * pv, s_v[tid], pi);  // w = p - (beta p.v / 2) v
      __syncthreads();
      for (int e = tid; e < n2 * n2; e += BLK) {  // A22 -= v w^T + w v^T
        const int i = e / n2, j = e % n2;
        const int lo = min(i, j), hi = max(i, j);
        gram[(k + 1 + i) * GM + (k + 1 + j)] -= fma(s_v[lo], s_w[hi], s_w[lo] * s_v[hi]);
      }
      __syncthreads();
    }
    // ---- 3. largest eigenvalue of the tridiagonal matrix (d, e) ----
    for (int i = tid; i < m; i += BLK) {
      s_d[i] = gram[i * GM + i];
      if (i + 1 < m) {
        const double ei = i + 2 < m ? s_e[i] : gram[(i + 1) * GM + i];
        s_e[i] = ei;
        s_e2[i] = ei * ei;
      }
    }
    __syncthreads();
    if (wv == 0) {
      double lo = 0.0, hi = 0.0, e2max = 0.0;
      bool first = true;
      for (int i = lane; i < m; i += WAVE) {
        const double r = (i > 0 ? fabs(s_e[i - 1]) : 0.0) + (i + 1 < m ? fabs(s_e[i]) : 0.0);
        lo = first ? s_d[i] - r : fmin(lo, s_d[i] - r);
        hi = first ? s_d[i] + r : fmax(hi, s_d[i] + r);
        if (i + 1 < m) e2max = fmax(e2max, s_e2[i]);
        first = false;
      }
      // lanes without an index take lane 0's value (m >= 1)
      const double lo0 = __shfl(lo, 0), hi0 = __shfl(hi, 0);
      lo = wave_min(first ? lo0 : lo);
      hi = wave_max(first ? hi0 : hi);
      e2max = wave_max(e2max);
      const double pivmin = 2.2250738585072014e-308 * fmax(1.0, e2max);
      for (int round = 0; round < 12; ++round) {
        const double w = hi - lo;
        const double xq = lo + w * (static_cast<double>(lane + 1) / 65.0);
        int cnt = 0;
        double q = s_d[0] - xq;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0 ? 1 : 0;
        for (int i = 1; i < m; ++i) {
          q = (s_d[i] - xq) - s_e2[i - 1] / q;
          if (fabs(q) < pivmin) q = -pivmin;
          cnt += q < 0.0 ? 1 : 0;
        }
        const unsigned long long above = __ballot(cnt == m);
        if (above == 0ull) {
          lo = lo + w * (64.0 / 65.0);
        } else {
          const int f = __ffsll(static_cast<long long>(above)) - 1;
          const double nlo = f > 0 ? lo + w * (static_cast<double>(f) / 65.0) : lo;
          hi = lo + w * (static_cast<double>(f + 1) / 65.0);
          lo = nlo;
        }
      }
      if (lane == 0) {
        gnorm[g] = sqrt(hi);
        fro[g] = sqrt(f2);
      }
    }
    __syncthreads();
  }
}

// Gram edge of k_group_norms for a largest group of m atoms.
inline int gram_edge(int m) { return m <= 16 ? 16 : m <= 32 ? 32 : m <= 64 ? 64 : 128; }

// One block: ||y||^2, lambda_*, arg-max, lambda, centre data, state initialisation.
// Group problems: lambda_* = max_g ||z0_g|| / w_g (eq. (gstar)).
template <typename T, typename V, typename A>
__global__ __launch_bounds__(CBLK) void k_setup_scalars(SingleArgs<T, V, A> a, double lam_in,
                                                         int lam_relative, double L,
                                                         double gap_tol, int max_iter,
                                                         double gamma_z, double bt_eta,
                                                         int bb_mem, double bb_sigma,
                                                         double cp_tau, double cp_sigma,
                                                         double cp_gamma, int warm,
                                                         double obj_tol) {
  __shared__ double sd[CNW];
  __shared__ int si[CNW];
  __shared__ double s_lmax;
  __shared__ int s_arg;
  SolverState* st = a.st;
  const int tid = threadIdx.x;
  const int N = a.N, K = a.K, G = a.G;
  // ||y||^2 and finiteness
  double yy = 0.0;
  int bad = 0;
  for (int e = tid; e < N; e += CBLK) {
    const double v = static_cast<double>(a.y[e]);
    if (!isfinite(v)) bad = 1;
    yy = fma(v, v, yy);
  }
  yy = block_sum<double, CNW>(yy, sd);
  bad = block_sum<int, CNW>(bad, si);
  // arg-max of |z0_i| (Lasso) or ||z0_g|| / w_g (groups); ties to the smallest index
  const int units = G > 0 ? G : K;
  double best = -1.0;
  int barg = 0x7fffffff;
  for (int u = tid; u < units; u += CBLK) {
    double val;
    if (G > 0) {
      double s = 0.0;
      for (int64_t i = a.gptr[u]; i < a.gptr[u + 1]; ++i) s = fma(a.z0[i], a.z0[i], s);
      val = sqrt(s) / a.w[u];
    } else {
      val = fabs(a.z0[u]);
    }
    if (val > best) { best = val; barg = u; }
  }
  // block arg-max with smallest-index tie break
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o, WAVE);
    const int oa = __shfl_xor(barg, o, WAVE);
    if (ob > best || (ob == best && oa < barg)) { best = ob; barg = oa; }
  }
  __syncthreads();
  if (tid % WAVE == 0) { sd[tid / WAVE] = best; si[tid / WAVE] = barg; }
  __syncthreads();
  if (tid == 0) {
    double b = sd[0];
    int ba = si[0];
    for (int k = 1; k < CNW; ++k)
      if (sd[k] > b || (sd[k] == b && si[k] < ba)) { b = sd[k]; ba = si[k]; }
    s_lmax = b;
    s_arg = ba;
  }
  __syncthreads();
  const double lam_max = s_lmax;
  const int arg = s_arg;
  // a non-finite dictionary entry leaves no valid arg-max: reject the instance
  if (!(arg >= 0 && arg < units) || !isfinite(lam_max)) bad = 1;
  const double lam = lam_relative ? lam_in * lam_max : lam_in;
  const bool trivial = !(lam < lam_max);
  // centre of the DST3 / DGST3 sphere: n = d_* (Lasso) or D_g* D_g*^T y / lambda_* (groups);
  // the Dome test's half-space n^T theta <= 1 uses the same n
  double nn = 0.0, ny = 0.0, wstar2 = 1.0;
  if ((a.test == TEST_DST3 || a.test == TEST_DOME) && !trivial && !bad) {
    if (G > 0) {
      const int64_t g0 = a.gptr[arg], g1 = a.gptr[arg + 1];
      wstar2 = a.w[arg] * a.w[arg];
      for (int e = tid; e < N; e += CBLK) {
        double s = 0.0;
        for (int64_t i = g0; i < g1; ++i) s = fma(to_double(a.D[i * a.ldd + e]), a.z0[i], s);
        const double ne = s / lam_max;
        nn = fma(ne, ne, nn);
        ny = fma(ne, static_cast<double>(a.y[e]), ny);
      }
    } else {
      const double sgn = a.z0[arg] >= 0.0 ? 1.0 : -1.0;
      for (int e = tid; e < N; e += CBLK) {
        const double de = sgn * to_double(a.D[static_cast<int64_t>(arg) * a.ldd + e]);
        nn = fma(de, de, nn);
        ny = fma(de, static_cast<double>(a.y[e]), ny);
      }
    }
    nn = block_sum<double, CNW>(nn, sd);
    ny = block_sum<double, CNW>(ny, sd);
  }
  // backtracking without a caller's L_0: the largest squared atom norm (Lasso) or
  // ||D_g||_2^2 (groups), the curvature of the data term along one unit
  const bool l0_dev = bt_eta > 0.0 && !(L > 0.0);
  double l0 = 0.0;
  if (l0_dev) {
    for (int u = tid; u < units; u += CBLK) {
      const double v = G > 0 ? a.gnorm[u] : a.nu[u];
      l0 = fmax(l0, v * v);
    }
    l0 = block_max<double, CNW>(l0, sd);
    if (!(l0 > 0.0)) l0 = 1.0;
  }
  if (tid == 0) {
    const double alpha = (a.test == TEST_DST3 && nn > 0.0) ? (ny / lam - wstar2) / nn : 0.0;
    st->lam = lam;
    st->lam_ratio = lam_relative ? lam_in : lam / lam_max;
    st->lam_max = lam_max;
    st->L = l0_dev ? l0 : L;
    st->bt_eta = bt_eta;
    st->rejected = 0;
    st->n_reject = 0;
    st->bb_mem = bb_mem;
    st->phi_n = 0;
    st->bb_new = 1;
    st->warm = warm;
    st->stop_obj = 0;
    st->pad_ = 0;
    st->obj_tol = obj_tol;
    st->bb_sigma = bb_sigma;
    for (int j = 0; j <= BB_MEM_MAX; ++j) st->phi_mem[j] = 0.0;
    st->cp_tau = cp_tau;
    st->cp_sigma = cp_sigma;
    st->cp_gamma = cp_gamma;
    st->yy = yy;
    st->alpha = alpha;
    st->nn = nn;
    st->ny = ny;
    st->rho2 = alpha * alpha * nn;
    st->gamma_z = gamma_z;
    st->gap_tol_abs = gap_tol * yy;
    st->tt = 0.0; st->ty = 0.0; st->zsup = 0.0; st->omega = 0.0;
    st->mu = 0.0; st->gap = 0.0; st->primal = 0.0; st->dual = 0.0;
    st->r_last = dinf(); st->r_min = dinf(); st->r_scr = dinf(); st->r_slack = 0.0;
    st->marg_slack = 0.0;
    st->l_prev = 1.0;
    st->n_support = 0;
    st->iter = 0;
    st->cur = 0;
    st->i_star = bad ? 0 : arg;
    st->nnz = 0;
    st->max_iter = max_iter;
    st->status = bad ? -1 : (trivial ? 1 : 0);
    st->done = (bad || trivial) ? 1 : 0;
    st->n_active = (bad || trivial) ? 0 : units;
    st->n_kept = st->n_active;
    st->compact = 0;
    st->pending = 0;
    st->n_omp = 0;
    st->n_active_atoms = (bad || trivial) ? 0 : K;
  }
}

// FP64 copy of the DST3 / DGST3 normal vector n (N doubles in a.nvec viewed as double).
template <typename T, typename V, typename A>
__global__ __launch_bounds__(BLK) void k_setup_normal(SingleArgs<T, V, A> a) {
  double* nvec = a.nvec;
  const SolverState* st = a.st;
  if (st->status != 0) return;
  const int e = blockIdx.x * BLK + threadIdx.x;
  if (e >= a.N) return;
  const int arg = st->i_star;
  if (a.G > 0) {
    double s = 0.0;
    for (int64_t i = a.gptr[arg]; i < a.gptr[arg + 1]; ++i)
      s = fma(to_double(a.D[i * a.ldd + e]), a.z0[i], s);
    nvec[e] = s / st->lam_max;
  } else {
    const double sgn = a.z0[arg] >= 0.0 ? 1.0 : -1.0;
    nvec[e] = sgn * to_double(a.D[static_cast<int64_t>(arg) * a.ldd + e]);
  }
}

// Margins (Lemmas 1, 2, 4, 5 through the sphere bound of Lemma 6), initial active list,
// x = u = 0.  Lasso: m_i = (1 - |d_i^T c|) / ||d_i||; groups: m_g = (w_g - ||D_g^T c||)/||D_g||.
// d_i^T c = z0_i / lambda - alpha * g_i with g = D^T n.  Dome test: dome_margin.
template <typename T, typename V, typename A>
__global__ __launch_bounds__(BLK) void k_setup_margins(SingleArgs<T, V, A> a) {
  const SolverState* st = a.st;
  const int i = blockIdx.x * BLK + threadIdx.x;
  if (i < a.K) { a.x[i] = V(0); a.u[i] = V(0); }
  const int units = a.G > 0 ? a.G : a.K;
  if (i >= units) return;
  a.act[0][i] = i;
  const double lam = st->lam, alpha = st->alpha;
  const bool dst3 = a.test == TEST_DST3;
  double m;
  if (a.test == TEST_NONE) {
    m = -dinf();
  } else if (a.G > 0) {
    double s = 0.0;
    for (int64_t k = a.gptr[i]; k < a.gptr[i + 1]; ++k) {
      const double ck = a.z0[k] / lam - (dst3 ? alpha * a.g[k] : 0.0);
      s = fma(ck, ck, s);
    }
    const double gn = a.gnorm[i];
    m = gn > 0.0 ? (a.w[i] - sqrt(s)) / gn : dinf();
  } else if (a.test == TEST_DOME) {
    const double nu = a.nu[i], nrm_n = sqrt(st->nn);
    const double delta = (st->ny / lam - 1.0) / nrm_n;
    const double gam = (a.N + 16) * 0x1p-53;
    m = nu > 0.0 ? dome_margin(a.z0[i], a.g[i], nu, lam, nrm_n, delta, sqrt(st->yy) / lam, gam)
                 : dinf();
  } else {
    const double ci = a.z0[i] / lam - (dst3 ? alpha * a.g[i] : 0.0);
    const double nu = a.nu[i];
    m = nu > 0.0 ? (1.0 - fabs(ci)) / nu : dinf();
  }
  a.marg[i] = m;
  a.act_m[0][i] = m;
}

// Rounding slack of the margins: a bound on the FP64 error of every m (one block).
template <typename T, typename V, typename A>
__global__ __launch_bounds__(CBLK) void k_setup_slack(SingleArgs<T, V, A> a) {
  __shared__ double sd[CNW];
  SolverState* st = a.st;
  const int units = a.G > 0 ? a.G : a.K;
  double kappa = 0.0;  // max (||D_g||_F + w_g) / ||D_g||_2 over units with a finite margin
  for (int u = threadIdx.x; u < units; u += CBLK) {
    if (a.G > 0) {
      if (a.gnorm[u] > 0.0) kappa = fmax(kappa, (a.fro[u] + a.w[u]) / a.gnorm[u]);
    } else if (a.nu[u] > 0.0) {
      kappa = fmax(kappa, 1.0 + 1.0 / a.nu[u]);
    }
  }
  kappa = block_max<double, CNW>(kappa, sd);
  double kz = 0.0;  // scale of the correlation rounding slack
  for (int u = threadIdx.x; u < units; u += CBLK)
    kz = fmax(kz, a.G > 0 ? a.fro[u] / a.w[u] : a.nu[u]);
  kz = block_max<double, CNW>(kz, sd);
  if (threadIdx.x == 0) {
    st->kappa_z = kz;
    const double eps = (a.N + 16) * 0x1p-53;
    st->marg_slack = eps * kappa * (sqrt(st->yy) / st->lam + fabs(st->alpha) * sqrt(st->nn) + 1.0);
  }
}

// Warm start (the initial point X_0 of Algorithm 3): x = u = x0 on every atom, and the
// support records of the first residual pass written as a correlation pass over the
// initial list (unit i in block i / units-per-block, every unit kept, in order) would
// write them, so that theta_1 = D x0 - y and Omega(x0) come out of the ordinary residual
// pass.  Run after k_setup_margins (which clears x and u).  A non-finite entry marks the
// instance invalid.  One thread per unit.
template <typename T, typename V, typename A>
__global__ __launch_bounds__(BLK) void k_warm_seed(SingleArgs<T, V, A> a, const V* __restrict__ x0);

// ============================================================== iteration kernels ===
//
// Iteration t runs two kernels.  k_resid(t) forms theta_t = D p_{t-1} - y (p = x for
// ISTA, u for FISTA), and at its start every block recomputes, identically, the FP64
// scalars of iteration t-1 from the partials the previous kernels published (dual
// scaling, gap, radius, stopping rule); block 0 records them.  k_corr(t) streams the
// active columns, applies the prox and momentum, and hands k_resid(t+1) a support
// segment per block.  Neither kernel ends with a cross-block handshake except the
// residual's row-tile reduction: long tails of dependent round trips cost more than the
// stream itself on this device.  State and partials that a kernel both reads and
// writes are double-buffered by the iteration parity, which the host passes in.

constexpr int LR = 2;                 // correlation rounds per block (Lasso)
constexpr int CBL = NW * CPW * LR;    // Lasso units per correlation block (16)
constexpr int CBG = NW * 2;           // groups per correlation block (8)
constexpr int SEGCAP_L = CBL;         // support slots per block (Lasso)
constexpr int SEGCAP_G = CBG * GMAX;  // support slots per block (groups)
constexpr int SGL = 32;               // correlation segments per residual item (Lasso)
constexpr int SGG = 32;               // correlation blocks per residual item (groups)
constexpr int LCAP = 512;             // residual list entries streamed per chunk
constexpr int MAXITEM = 8192;         // residual segment groups

template <typename T, typename V, typename A>
__global__ __launch_bounds__(BLK) void k_warm_seed(SingleArgs<T, V, A> a, const V* __restrict__ x0) {
  const int units = a.G > 0 ? a.G : a.K;
  const int i = blockIdx.x * BLK + threadIdx.x;
  if (i >= units) return;
  bool bad = false;
  if (a.G > 0) {
    const int b = i / CBG, j = i % CBG;
    const int64_t g0 = a.gptr[i], g1 = a.gptr[i + 1];
    double s2 = 0.0;
    for (int64_t k = g0; k < g1; ++k) {
      const V v = x0[k];
      const double d = static_cast<double>(v);
      if (!isfinite(d)) bad = true;
      s2 = fma(d, d, s2);
      a.x[k] = v;
      a.u[k] = v;
      const int64_t slot = static_cast<int64_t>(b) * SEGCAP_G + j * GMAX + (k - g0);
      a.seg_atom[slot] = static_cast<int32_t>(k);
      a.seg_val[slot] = v;
    }
    const int64_t rec = static_cast<int64_t>(b) * CBG + j;
    a.urec_marg[rec] = a.marg[i];
    a.urec_om[rec] = a.w[i] * sqrt(s2);
    a.urec_m[rec] = static_cast<int32_t>(g1 - g0);
    if (j == 0) a.seg_cnt[b] = min(CBG, units - b * CBG);
  } else {
    const int b = i / CBL, k = i % CBL;
    const V v = x0[i];
    const double d = static_cast<double>(v);
    if (!isfinite(d)) bad = true;
    a.x[i] = v;
    a.u[i] = v;
    const int64_t slot = static_cast<int64_t>(b) * SEGCAP_L + k;
    a.seg_atom[slot] = i;
    a.seg_val[slot] = v;
    a.urec_marg[slot] = a.marg[i];
    a.urec_om[slot] = fabs(d);
    if (k == 0) a.seg_cnt[b] = min(CBL, units - b * CBL);
  }
  if (bad) {  // every writer stores the same values
    a.st->status = -1;
    a.st->done = 1;
  }
}

// FP64 scalars of one iteration from the reduced partials (same arithmetic in every
// block): dual scaling (Lemma 7), dual point v = mu theta, gap certificate, radius of
// the chosen test with its rounding slack, stopping rule.
struct IterScalars {
  double mu, gap, primal, dual, r, r_safe;
  bool stop;
};
__device__ inline IterScalars iter_scalars(const SolverState& s, int N, int test, int t,
                                           double tt, double ty, double omega, double zsup,
                                           double pp) {
  IterScalars o;
  const double lam = s.lam, yy = s.yy, rho2 = s.rho2;
  const double sb = zsup > 0.0 ? 1.0 / zsup : dinf();
  double mu = 0.0;
  if (tt > 0.0) mu = fmin(fmax(ty / (lam * tt), -sb), sb);
  o.mu = mu;
  o.primal = 0.5 * pp + lam * omega;  // pp = ||D p - y||^2 (= tt unless theta is carried)
  o.dual = lam * mu * ty - 0.5 * lam * lam * mu * mu * tt;
  o.gap = o.primal - o.dual;
  const double a1 = yy / (lam * lam), a2 = 2.0 * mu * ty / lam, a3 = mu * mu * tt;
  const double R2 = a1 - a2 + a3;
  o.r = dinf();
  o.r_safe = dinf();
  if (test != TEST_NONE) {
    const double q = R2 - (test == TEST_DST3 ? rho2 : 0.0);
    const double E = (N + 16) * 0x1p-53 * (a1 + fabs(a2) + a3 + rho2);
    o.r = sqrt(fmax(q, 0.0));
    o.r_safe = sqrt(fmax(q + E, 0.0));
  }
  o.stop = (s.gap_tol_abs > 0.0 && o.gap <= s.gap_tol_abs) || t >= s.max_iter;
  return o;
}

// Row tile rt of the residual: r = D p - y from the items' partials.  theta = r, except for
// Chambolle-Pock (CP), where the dual iterate is carried: theta = (theta_prev + sigma r) /
// (1 + sigma) (theta_prev = 0 at the first pass) and ||r||^2 is published for the primal
// objective.  Publishes ||theta||^2 and theta^T y per row tile.  With `rows` (a single
// item per row tile) the item's row sums are read from its LDS wave sums (NW x RT, summed
// in wave order as the item would have published them) instead of the published partials.
template <typename T, typename V, bool VECTOR, bool CP = false>
__device__ void resid_finish_tile(SingleArgs<T, V, double>& a, int rt, int nitems_rt,
                                  double* sd, double sigma = 0.0, bool first = false,
                                  const double* rows = nullptr) {
  constexpr int VR = VECTOR ? Store<T>::VEC : 1;
  constexpr int RT = WAVE * VR;
  constexpr int FB = 32;  // item partials loaded at once
  double tt = 0.0, ty = 0.0, rr = 0.0;
  const int r_end = min((rt + 1) * RT, a.N);
  for (int r = rt * RT + static_cast<int>(threadIdx.x); r < r_end; r += BLK) {
    const double yv = static_cast<double>(a.y[r]);
    // item partials in item order, FB loads in flight (unconditional loads at clamped
    // indices: a guarded load would wait for its value before the next one is issued)
    double s = 0.0;
    if (rows != nullptr) {
      const int rr = r - rt * RT;
      double v = rows[rr];
#pragma unroll
      for (int w = 1; w < NW; ++w) v += rows[w * RT + rr];
      s += v;
    } else {
      for (int c = 0; c < nitems_rt; c += FB) {
        double v[FB];
#pragma unroll
        for (int k = 0; k < FB; ++k)
          v[k] = consume(&a.partial[static_cast<int64_t>(min(c + k, nitems_rt - 1)) * a.npad + r]);
#pragma unroll
        for (int k = 0; k < FB; ++k) s += c + k < nitems_rt ? v[k] : 0.0;
      }
    }
    double res = s - yv;
    if constexpr (CP) {
      rr = fma(res, res, rr);
      const double prev = first ? 0.0 : static_cast<double>(a.theta[r]);
      res = fma(sigma, res, prev) / (1.0 + sigma);
    }
    const V th = static_cast<V>(res);
    a.theta[r] = th;
    const double thd = static_cast<double>(th);
    tt = fma(thd, thd, tt);
    ty = fma(thd, yv, ty);
  }
  tt = block_sum<double, NW>(tt, sd);
  ty = block_sum<double, NW>(ty, sd);
  if constexpr (CP) rr = block_sum<double, NW>(rr, sd);
  if (threadIdx.x == 0) {
    double* rtn = a.rtn + a.par * (2 * MAXRT);
    rtn[2 * rt] = tt;  // read by the next kernels only
    rtn[2 * rt + 1] = ty;
    if constexpr (CP) a.rtr[a.par * MAXRT + rt] = rr;
    a.rt_cnt[rt] = 0u;  // every item of this tile has arrived: re-arm
  }
}

// Row segment r0 .. r0 + VR of sum_k l_val[k] d_{l_idx[k]} over the first nl list entries
// in LDS, accumulated into acc (FP64); each wave takes RPW columns at a time.
template <typename T, typename V, bool VECTOR>
__device__ __forceinline__ void stream_list(const SingleArgs<T, V, double>& a, const int* l_idx,
                                            const double* l_val, int r0, int nl, int wave,
                                            double (&acc)[VECTOR ? Store<T>::VEC : 1]) {
  constexpr int VR = VECTOR ? Store<T>::VEC : 1;
  for (int k0 = wave * RPW; k0 < nl; k0 += NW * RPW) {
    int idx[RPW];
    double val[RPW];
#pragma unroll
    for (int p = 0; p < RPW; ++p) {
      const bool ok = k0 + p < nl;
      idx[p] = ok ? l_idx[k0 + p] : l_idx[k0];
      val[p] = ok ? l_val[k0 + p] : 0.0;
    }
    if (VECTOR && r0 + VR <= a.N) {
      if constexpr (VECTOR) {
        uint4 cv[RPW];
#pragma unroll
        for (int p = 0; p < RPW; ++p) cv[p] = ld16(a.D + static_cast<int64_t>(idx[p]) * a.ldd + r0);
#pragma unroll
        for (int p = 0; p < RPW; ++p) {
          double d[VR];
          widen<T>(cv[p], d);
#pragma unroll
          for (int e = 0; e < VR; ++e) acc[e] = fma(d[e], val[p], acc[e]);
        }
      }
    } else {
#pragma unroll
      for (int p = 0; p < RPW; ++p) {
        const T* col = a.D + static_cast<int64_t>(idx[p]) * a.ldd;
        for (int e = 0; e < VR; ++e)
          if (r0 + e < a.N) acc[e] = fma(to_double(col[r0 + e]), val[p], acc[e]);
      }
    }
  }
}

// Groups: list positions c0 .. c0 + nl - 1 of the atoms of the item's selected group records
// (record r owns positions [goff[r], goff[r] + its count), its slots start at gbase[r]),
// located by binary search and read from the slot arrays into the LDS list.
template <typename V>
__device__ __forceinline__ void fill_group_list(const int* s_goff, const int* s_gbase, int c0, int nl,
                                                const int32_t* __restrict__ seg_atom,
                                                const V* __restrict__ vals, int* l_idx, double* l_val) {
  constexpr int FPT = LCAP / BLK;  // list positions filled per thread
  const int tid = threadIdx.x;
  int slot[FPT];
#pragma unroll
  for (int q = 0; q < FPT; ++q) {
    const int pp = c0 + min(tid + q * BLK, nl - 1);
    int lo = 0, hi = BLK;  // first record whose offset exceeds pp
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (s_goff[mid] <= pp) lo = mid + 1; else hi = mid;
    }
    slot[q] = s_gbase[lo - 1] + (pp - s_goff[lo - 1]);
  }
  int at[FPT];
  V vv[FPT];
#pragma unroll
  for (int q = 0; q < FPT; ++q) {
    at[q] = seg_atom[slot[q]];
    vv[q] = vals[slot[q]];
  }
#pragma unroll
  for (int q = 0; q < FPT; ++q) {
    if (tid + q * BLK < nl) {
      l_idx[tid + q * BLK] = at[q];
      l_val[tid + q * BLK] = static_cast<double>(vv[q]);
    }
  }
}

// Raw support records of one residual slot, loaded before the kept / non-zero decision.
struct SlotRaw {
  int nk, m, atom;
  double marg, om, val;
  double omo, valo;  // backtracking: the same for p, before the step
};

template <typename T, typename V, bool VECTOR, int RULE, bool GROUP>
__global__ __launch_bounds__(BLK) void k_resid(SingleArgs<T, V, double> a) {
  constexpr int VR = VECTOR ? Store<T>::VEC : 1;
  constexpr int RT = WAVE * VR;
  constexpr int SG = GROUP ? SGG : SGL;           // correlation blocks per item
  // Lasso: one support slot per list entry; groups: one group record per thread
  constexpr int SPI = GROUP ? SGG * CBG : SGL * SEGCAP_L;
  constexpr int SPT = SPI / BLK;                  // slots (records) per thread
  constexpr int PB = 4;                           // block partials per thread per step
  static_assert(SPI % BLK == 0, "slots must tile the block");
  static_assert(GROUP ? SPI == BLK : SPI <= LCAP, "group records: one per thread");
  __shared__ double red[NW][RT];
  __shared__ int l_idx[LCAP];
  __shared__ double l_val[LCAP];
  __shared__ int s_goff[GROUP ? BLK : 1], s_gbase[GROUP ? BLK : 1];
  __shared__ double sd[NW];
  __shared__ int scan[NW];
  __shared__ int s_last;
  __shared__ SolverState S;
  __shared__ double red8[NW][(RULE == RULE_SPARSA || RULE == RULE_CP) ? 11 : 10];
  const int tid = threadIdx.x, lane = tid % WAVE, wave = tid / WAVE;
  const SolverState* sin = a.st + (1 - a.par);
  SolverState* sout = a.st + a.par;
  const int nrt = (a.N + RT - 1) / RT;
  const int nsg = (a.grid_corr + SG - 1) / SG;
  const int nitems = nrt * nsg;

  // The support records a slot of `item` may use (groups: the record of one group, its
  // atoms' slots start at `atom`).  Every address is in bounds whatever the segment counts
  // are (blocks past the grid read the last block's records and are discarded later), so
  // the loads need neither the counts nor the new radius, and none of them is guarded: a
  // guarded load waits for its value before the next is issued.
  auto load_slots = [&](int item, SlotRaw (&raw)[SPT]) {
    const int sg = item / nrt;
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int s = tid + q * BLK;  // slot (record) within the item
      if constexpr (GROUP) {
        const int b = min(sg * SG + s / CBG, a.grid_corr - 1), j = s % CBG;
        const int64_t rec = static_cast<int64_t>(b) * CBG + j;
        raw[q].nk = a.seg_cnt[b];
        raw[q].marg = a.urec_marg[rec];
        raw[q].om = a.urec_om[rec];
        raw[q].m = a.urec_m[rec];
        raw[q].val = 0.0;
        raw[q].atom = b * SEGCAP_G + j * GMAX;
        raw[q].omo = a.urec_omo[rec];
        raw[q].valo = 0.0;
      } else {
        const int b = min(sg * SG + s / SEGCAP_L, a.grid_corr - 1), k = s % SEGCAP_L;
        const int64_t rec = static_cast<int64_t>(b) * CBL + k;
        const int64_t slot = static_cast<int64_t>(b) * SEGCAP_L + k;
        raw[q].nk = a.seg_cnt[b];
        raw[q].marg = a.urec_marg[rec];
        raw[q].om = a.urec_om[rec];
        raw[q].m = 0;
        raw[q].val = static_cast<double>(a.seg_val[slot]);
        raw[q].atom = a.seg_atom[slot];
        raw[q].omo = a.urec_omo[rec];
        raw[q].valo = static_cast<double>(a.seg_po[slot]);
      }
    }
  };

  // ---- one round trip for the state, the previous pass's partials and the first
  // item's support records: all of them are issued before the first wait ----
  constexpr int NWORDS = sizeof(SolverState) / 4;
  static_assert(NWORDS <= BLK, "state fits one word per thread");
  const int32_t sword = reinterpret_cast<const int32_t*>(sin)[min(tid, NWORDS - 1)];
  // zs nz kt ns at tt ty om; backtracking: ||d||^2 ||D d||^2; SpaRSA: the correlation
  // pass's part of phi(x') - phi(p)
  constexpr int NV = (RULE == RULE_SPARSA || RULE == RULE_CP) ? 11 : 10;
  double v[NV] = {};
  const double* rtp = a.rtn + (1 - a.par) * (2 * MAXRT);
  const double* omp = a.omp + (1 - a.par) * MAXITEM;
  double p0[PB], p1[PB], p2[PB], p3[PB], p4[PB], p8[PB];
  double p10[RULE == RULE_SPARSA ? PB : 1];
#pragma unroll
  for (int k = 0; k < PB; ++k) {  // block partials tid, tid + BLK, ... in that order
    const int b = min(k * BLK + tid, a.grid_corr - 1);
    p0[k] = a.bp0[b];
    p1[k] = a.bpi[b];
    p2[k] = a.bpi[MAXB + b];
    p3[k] = a.bpi[2 * MAXB + b];
    p4[k] = a.bpi[3 * MAXB + b];
    p8[k] = a.bpd[b];
    if constexpr (RULE == RULE_SPARSA) p10[k] = a.bpe[b];
  }
  const int kr = min(tid, nrt - 1), ko = min(tid, a.nsg_prev - 1);
  const double q5 = rtp[2 * kr], q6 = rtp[2 * kr + 1], q7 = omp[ko], q9 = a.dtn[kr];
  double q10 = 0.0;  // Chambolle-Pock: ||D u - y||^2 of the row tile
  if constexpr (RULE == RULE_CP) q10 = a.rtr[(1 - a.par) * MAXRT + kr];
  SlotRaw raw[SPT];
  if (static_cast<int>(blockIdx.x) < nitems) load_slots(blockIdx.x, raw);
#pragma unroll
  for (int k = 0; k < PB; ++k) {
    const bool ok = k * BLK + tid < a.grid_corr;
    v[0] = fmax(v[0], ok ? p0[k] : 0.0);
    v[1] += ok ? p1[k] : 0.0;
    v[2] += ok ? p2[k] : 0.0;
    v[3] += ok ? p3[k] : 0.0;
    v[4] += ok ? p4[k] : 0.0;
    v[8] += ok ? p8[k] : 0.0;
    if constexpr (RULE == RULE_SPARSA) v[NV - 1] += ok ? p10[k] : 0.0;
  }
  v[5] += tid < nrt ? q5 : 0.0;
  v[6] += tid < nrt ? q6 : 0.0;
  v[7] += tid < a.nsg_prev ? q7 : 0.0;
  v[9] += tid < nrt ? q9 : 0.0;
  if constexpr (RULE == RULE_CP) v[NV - 1] += tid < nrt ? q10 : 0.0;
  // larger grids: the remaining partials, in the same order
  for (int b = PB * BLK + tid; b < a.grid_corr; b += BLK) {
    v[0] = fmax(v[0], a.bp0[b]);
    v[1] += a.bpi[b];
    v[2] += a.bpi[MAXB + b];
    v[3] += a.bpi[2 * MAXB + b];
    v[4] += a.bpi[3 * MAXB + b];
    v[8] += a.bpd[b];
    if constexpr (RULE == RULE_SPARSA) v[NV - 1] += a.bpe[b];
  }
  for (int k = BLK + tid; k < nrt; k += BLK) {
    v[5] += rtp[2 * k];
    v[6] += rtp[2 * k + 1];
    v[9] += a.dtn[k];
    if constexpr (RULE == RULE_CP) v[NV - 1] += a.rtr[(1 - a.par) * MAXRT + k];
  }
  for (int k = BLK + tid; k < a.nsg_prev; k += BLK) v[7] += omp[k];
  if (tid < NWORDS) reinterpret_cast<int32_t*>(&S)[tid] = sword;
  __syncthreads();
  if (S.done) {
    if (blockIdx.x == 0 && tid == 0) *sout = S;
    return;
  }
  // ---- scalars of the previous iteration, from the published partials ----
  if (S.pending) {
    // one-pass block reduction of the values (fixed order: lanes, then waves)
    const int nv = a.bt ? NV : 8;
    v[0] = wave_max(v[0]);
#pragma unroll
    for (int k = 1; k < NV; ++k)
      if (k < nv) v[k] = wave_sum(v[k]);
    if (lane == 0)
#pragma unroll
      for (int k = 0; k < NV; ++k) red8[wave][k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double acc = red8[0][k];
#pragma unroll
      for (int w = 1; w < NW; ++w) acc = k == 0 ? fmax(acc, red8[w][k]) : acc + red8[w][k];
      v[k] = acc;
    }
    const double tt = v[5], ty = v[6], om = v[7];
    const int nz = static_cast<int>(v[1]), kt = static_cast<int>(v[2]);
    const int ns = static_cast<int>(v[3]), at = static_cast<int>(v[4]);
    // rounding-safe bound of the largest correlation (FP64 accumulation of exact products)
    const double zs = v[0] + S.gamma_z * sqrt(tt) * S.kappa_z;
    const int t = S.iter + 1;
    // the primal objective's data term: ||theta||^2, or for Chambolle-Pock ||D u - y||^2
    const IterScalars o = iter_scalars(S, a.N, a.test, t, tt, ty, om, zs,
                                       RULE == RULE_CP ? v[NV - 1] : tt);
    // backtracking: the step of this iteration is kept when ||D d||^2 <= L ||d||^2 (the
    // descent condition F(x') <= Q_L(x', p) for the quadratic data term); the stop needs
    // an accepted step, except at the iteration limit
    bool rej = a.bt && RULE != RULE_CP && !(v[9] <= S.L * v[8]);
    if constexpr (RULE == RULE_SPARSA) {
      // SpaRSA: the memory takes phi(p) (a new entry when p is a new iterate, else it
      // replaces the newest); the step is kept when phi(x') - phi(p) = z^T d + ||D d||^2 / 2
      // + lambda (Omega(x') - Omega(p)) satisfies phi(x') <= max(memory) - sigma/2 L ||d||^2
      const int keep0 = S.bb_new ? max(0, S.phi_n - S.bb_mem) : 0;  // first entry kept
      const int keep1 = S.bb_new ? S.phi_n : S.phi_n - 1;            // one past the last
      double phi_ref = o.primal;
      for (int j = keep0; j < keep1; ++j) phi_ref = fmax(phi_ref, S.phi_mem[j]);
      const double dphi = v[NV - 1] + 0.5 * v[9];
      rej = !(dphi + (o.primal - phi_ref) <= -0.5 * S.bb_sigma * S.L * v[8]);
    }
    // the experiments section's rule, optionally: the relative change of the objective
    // between the primal points of two consecutive accepted passes, once both are non-zero
    // (a method whose first steps leave x at 0, such as Chambolle-Pock from a zero dual
    // iterate, would otherwise stop before it starts)
    const bool obj_stop = !rej && !S.rejected && S.obj_tol > 0.0 && t > 1 && om > 0.0 &&
                          S.omega > 0.0 && fabs(o.primal - S.primal) <= S.obj_tol * o.primal;
    const bool stop = (!rej && S.gap_tol_abs > 0.0 && o.gap <= S.gap_tol_abs) || obj_stop ||
                      t >= S.max_iter;
    __syncthreads();
    if (tid == 0) {
      const int n_old = S.n_active;
      if (S.compact) {
        S.n_active = kt;
        S.cur = 1 - S.cur;
      }
      S.compact = (!S.compact && (n_old - kt) * 4 > n_old && (n_old - kt) >= CBL) ? 1 : 0;
      S.iter = t;
      S.tt = tt;
      S.ty = ty;
      S.omega = om;
      S.zsup = zs;
      S.mu = o.mu;
      S.gap = o.gap;
      S.primal = o.primal;
      S.dual = o.dual;
      S.nnz = nz;
      S.n_kept = kt;
      S.n_support = ns;
      S.n_active_atoms = at;
      S.r_last = o.r;
      S.r_min = fmin(S.r_min, o.r);
      if (RULE == RULE_FISTA && !rej) S.l_prev = 0.5 * (1.0 + sqrt(1.0 + 4.0 * S.l_prev * S.l_prev));
      S.rejected = rej ? 1 : 0;
      if constexpr (RULE == RULE_SPARSA) {
        // memory update (oldest first), then the Barzilai-Borwein step after an accepted one
        if (S.bb_new) {
          if (S.phi_n > S.bb_mem) {
            for (int j = 1; j < S.phi_n; ++j) S.phi_mem[j - 1] = S.phi_mem[j];
            --S.phi_n;
          }
          S.phi_mem[S.phi_n++] = o.primal;
        } else {
          S.phi_mem[S.phi_n - 1] = o.primal;
        }
        S.bb_new = rej ? 0 : 1;
        if (!rej && !stop && v[8] > 0.0) S.L = fmin(fmax(v[9] / v[8], 1e-30), 1e30);
      }
      if (rej) {
        ++S.n_reject;
        if (!stop) S.L *= S.bt_eta;
      }
      if constexpr (RULE == RULE_CP) {
        // the certified point is u_{t-1}: at the stop the update of this iteration is undone
        // (x and u back to the slot copies) and u is returned; otherwise the steps advance
        S.rejected = stop ? 1 : 0;
        if (!stop) {
          const double phi = 1.0 / sqrt(1.0 + 2.0 * S.cp_gamma * S.cp_tau);
          S.cp_tau *= phi;
          S.cp_sigma /= phi;
        }
      }
      if (obj_stop) S.stop_obj = 1;
      if (stop) {
        S.done = 1;
      } else if (o.r_safe < S.r_scr && (!a.screen_static || t == 1)) {
        S.r_scr = o.r_safe;
        S.r_slack = o.r_safe - o.r;
      }
      S.pending = 0;
      if (blockIdx.x == 0 && a.tele != nullptr && t - 1 < a.tele_cap) {
        TeleRec* rec = static_cast<TeleRec*>(a.tele) + (t - 1);
        rec->n_atoms = at;
        rec->n_units = kt;
        rec->n_support = ns;
        rec->nnz = nz;
        rec->r = o.r;
        rec->gap = o.gap;
      }
    }
    __syncthreads();
    if (S.rejected) {
      // undo the rejected step: x and u of the units it updated return to x_{t-1} and p
      constexpr int SEGCAP = GROUP ? SEGCAP_G : SEGCAP_L;
      const int nslots = a.grid_corr * SEGCAP;
      for (int s = blockIdx.x * BLK + tid; s < nslots; s += gridDim.x * BLK) {
        const int b = s / SEGCAP, kk = s % SEGCAP;
        const int j = GROUP ? kk / GMAX : kk;
        bool ok = j < a.seg_cnt[b];
        if (GROUP && ok) ok = kk % GMAX < a.urec_m[b * CBG + j];
        if (ok) {
          const int atom = a.seg_atom[s];
          a.x[atom] = a.seg_xo[s];
          a.u[atom] = a.seg_po[s];
        }
      }
    }
    if (S.done) {
      if (blockIdx.x == 0 && tid == 0) *sout = S;
      return;
    }
  }
  const bool rej = S.rejected != 0;
  if (blockIdx.x == 0 && tid == 0) {
    SolverState o = S;
    o.n_omp = nsg;  // the Omega partials this pass publishes
    *sout = o;
    a.counters[CNT_VID] = 0u;  // the correlation pass that used it has ended
  }
  const double r_keep = S.r_scr + S.marg_slack;
  const bool have_support = S.iter > 0 || S.warm;  // p_0 = 0 unless a warm start seeded it
  if (!have_support) {  // theta = -y, Omega(p_0) = 0
    if (static_cast<int>(blockIdx.x) < nrt)
      resid_finish_tile<T, V, VECTOR, RULE == RULE_CP>(a, blockIdx.x, 0, sd, S.cp_sigma, true);
    if (blockIdx.x == 0)
      for (int k = tid; k < nsg; k += BLK) a.omp[a.par * MAXITEM + k] = 0.0;
    return;
  }
  for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
    const int rt = item % nrt, sg = item / nrt;
    if (item != static_cast<int>(blockIdx.x)) load_slots(item, raw);
    const int r0 = rt * RT + lane * VR;
    double acc[VR];
#pragma unroll
    for (int e = 0; e < VR; ++e) acc[e] = 0.0;
    double om = 0.0;
    if constexpr (!GROUP) {
      // ---- the kept, non-zero support entries of segment group sg (in order) ----
      int cntv = 0;
      int e_atom[SPT];
      double e_val[SPT];
#pragma unroll
      for (int q = 0; q < SPT; ++q) {
        const int s = tid + q * BLK;  // slot within the item
        const int b = sg * SG + s / SEGCAP_L, j = s % SEGCAP_L;
        e_atom[q] = -1;
        e_val[q] = 0.0;
        if (b < a.grid_corr && j < raw[q].nk && !(raw[q].marg > r_keep)) {
          const double val = rej ? raw[q].valo : raw[q].val;  // a rejected step keeps p
          if (val != 0.0) {
            e_atom[q] = raw[q].atom;
            e_val[q] = val;
            ++cntv;
          }
          om += rej ? raw[q].omo : raw[q].om;
        }
      }
      if (rt == 0) {
        om = block_sum<double, NW>(om, sd);
        if (tid == 0) a.omp[a.par * MAXITEM + sg] = om;
      }
      int total;
      int off = block_exclusive_scan<NW>(cntv, scan, &total);
#pragma unroll
      for (int q = 0; q < SPT; ++q) {
        if (e_atom[q] >= 0) {
          l_idx[off] = e_atom[q];
          l_val[off] = e_val[q];
          ++off;
        }
      }
      __syncthreads();
      stream_list<T, V, VECTOR>(a, l_idx, l_val, r0, total, wave, acc);
    } else {
      // ---- groups: the atoms of the kept groups with a non-zero u_g, in order ----
      // Thread tid holds group record tid of the item; its m atoms occupy list positions
      // [off, off + m) after a block scan, and a chunk of positions is filled by locating
      // each position's record (binary search over the offsets) and reading its slot.
      const int b = sg * SG + tid / CBG, j = tid % CBG;
      int na = 0;
      if (b < a.grid_corr && j < raw[0].nk && !(raw[0].marg > r_keep)) {
        const double omg = rej ? raw[0].omo : raw[0].om;  // a rejected step keeps p
        om += omg;
        if (omg > 0.0) na = raw[0].m;
      }
      if (rt == 0) {
        om = block_sum<double, NW>(om, sd);
        if (tid == 0) a.omp[a.par * MAXITEM + sg] = om;
      }
      int total;
      const int off = block_exclusive_scan<NW>(na, scan, &total);
      s_goff[tid] = off;
      s_gbase[tid] = raw[0].atom;
      __syncthreads();
      for (int c0 = 0; c0 < total; c0 += LCAP) {
        const int nl = min(LCAP, total - c0);
        fill_group_list<V>(s_goff, s_gbase, c0, nl, a.seg_atom, rej ? a.seg_po : a.seg_val, l_idx, l_val);
        __syncthreads();
        stream_list<T, V, VECTOR>(a, l_idx, l_val, r0, nl, wave, acc);
        __syncthreads();
      }
    }
#pragma unroll
    for (int e = 0; e < VR; ++e) red[wave][lane * VR + e] = acc[e];
    __syncthreads();
    if (nsg == 1) {
      // one segment group (a short active list): the item holds its row tile's whole sum
      // and finishes the tile itself, without the publication and arrival round trips
      resid_finish_tile<T, V, VECTOR, RULE == RULE_CP>(a, rt, 1, sd, S.cp_sigma, S.iter == 0,
                                                       &red[0][0]);
      __syncthreads();
      continue;
    }
    for (int rr = tid; rr < RT; rr += BLK) {
      const int r = rt * RT + rr;
      if (r < a.N) {
        double s = red[0][rr];
#pragma unroll
        for (int w = 1; w < NW; ++w) s += red[w][rr];
        publish(&a.partial[static_cast<int64_t>(sg) * a.npad + r], s);
      }
    }
    if (arrive_last(&a.rt_cnt[rt], static_cast<unsigned>(nsg), &s_last))
      resid_finish_tile<T, V, VECTOR, RULE == RULE_CP>(a, rt, nsg, sd, S.cp_sigma, S.iter == 0);
    __syncthreads();
  }
}

// Backtracking check: ||D d||^2 for the step d = x' - p of the correlation pass that just
// ran (non-zero entries of its support slots), by the residual's work items: row tile x
// segment group, FP64 row partials published per item, and the item arriving last for a
// row tile adds the items' partials row by row and publishes the row tile's sum of squares.
template <typename T, typename V, bool VECTOR, bool GROUP>
__global__ __launch_bounds__(BLK) void k_dcheck(SingleArgs<T, V, double> a) {
  constexpr int VR = VECTOR ? Store<T>::VEC : 1;
  constexpr int RT = WAVE * VR;
  constexpr int SG = GROUP ? SGG : SGL;
  constexpr int SPI = GROUP ? SGG * CBG : SGL * SEGCAP_L;
  constexpr int SPT = SPI / BLK;
  __shared__ double red[NW][RT];
  __shared__ int l_idx[LCAP];
  __shared__ double l_val[LCAP];
  __shared__ double sd[NW];
  __shared__ int scan[NW];
  __shared__ int s_last;
  __shared__ int s_goff[GROUP ? BLK : 1], s_gbase[GROUP ? BLK : 1];
  const int tid = threadIdx.x, lane = tid % WAVE, wave = tid / WAVE;
  if ((a.st + a.par)->done) return;
  const int nrt = (a.N + RT - 1) / RT;
  const int nsg = (a.grid_corr + SG - 1) / SG;
  for (int item = blockIdx.x; item < nrt * nsg; item += gridDim.x) {
    const int rt = item % nrt, sg = item / nrt;
    const int r0 = rt * RT + lane * VR;
    double acc[VR];
#pragma unroll
    for (int e = 0; e < VR; ++e) acc[e] = 0.0;
    if constexpr (!GROUP) {
      int nk[SPT], atom[SPT];
      double dv[SPT];
#pragma unroll
      for (int q = 0; q < SPT; ++q) {  // unconditional loads at clamped indices
        const int s = tid + q * BLK;
        const int b = min(sg * SG + s / SEGCAP_L, a.grid_corr - 1);
        const int64_t slot = static_cast<int64_t>(b) * SEGCAP_L + s % SEGCAP_L;
        nk[q] = a.seg_cnt[b];
        atom[q] = a.seg_atom[slot];
        dv[q] = a.seg_d[slot];
      }
      int cnt = 0;
#pragma unroll
      for (int q = 0; q < SPT; ++q) {
        const int s = tid + q * BLK;
        const bool ok = sg * SG + s / SEGCAP_L < a.grid_corr && s % SEGCAP_L < nk[q] && dv[q] != 0.0;
        if (!ok) atom[q] = -1;
        cnt += ok ? 1 : 0;
      }
      int total;
      int off = block_exclusive_scan<NW>(cnt, scan, &total);
#pragma unroll
      for (int q = 0; q < SPT; ++q) {
        if (atom[q] >= 0) {
          l_idx[off] = atom[q];
          l_val[off] = dv[q];
          ++off;
        }
      }
      __syncthreads();
      stream_list<T, V, VECTOR>(a, l_idx, l_val, r0, total, wave, acc);
    } else {
      const int b = sg * SG + tid / CBG, j = tid % CBG;
      const int bc = min(b, a.grid_corr - 1);
      const int64_t rec = static_cast<int64_t>(bc) * CBG + j;
      const int nk = a.seg_cnt[bc], m = a.urec_m[rec];
      const double dn = a.urec_dn[rec];
      const int na = (b < a.grid_corr && j < nk && dn > 0.0) ? m : 0;
      int total;
      const int off = block_exclusive_scan<NW>(na, scan, &total);
      s_goff[tid] = off;
      s_gbase[tid] = bc * SEGCAP_G + j * GMAX;
      __syncthreads();
      for (int c0 = 0; c0 < total; c0 += LCAP) {
        const int nl = min(LCAP, total - c0);
        fill_group_list<double>(s_goff, s_gbase, c0, nl, a.seg_atom, a.seg_d, l_idx, l_val);
        __syncthreads();
        stream_list<T, V, VECTOR>(a, l_idx, l_val, r0, nl, wave, acc);
        __syncthreads();
      }
    }
#pragma unroll
    for (int e = 0; e < VR; ++e) red[wave][lane * VR + e] = acc[e];
    __syncthreads();
    for (int rr = tid; rr < RT; rr += BLK) {
      const int r = rt * RT + rr;
      if (r < a.N) {
        double s = red[0][rr];
#pragma unroll
        for (int w = 1; w < NW; ++w) s += red[w][rr];
        publish(&a.partial[static_cast<int64_t>(sg) * a.npad + r], s);
      }
    }
    if (arrive_last(&a.rt_cnt[rt], static_cast<unsigned>(nsg), &s_last)) {
      constexpr int FB = 32;
      double q2 = 0.0;
      const int r_end = min((rt + 1) * RT, a.N);
      for (int r = rt * RT + tid; r < r_end; r += BLK) {
        double s = 0.0;
        for (int c = 0; c < nsg; c += FB) {
          double pv[FB];
#pragma unroll
          for (int k2 = 0; k2 < FB; ++k2)
            pv[k2] = consume(&a.partial[static_cast<int64_t>(min(c + k2, nsg - 1)) * a.npad + r]);
#pragma unroll
          for (int k2 = 0; k2 < FB; ++k2) s += c + k2 < nsg ? pv[k2] : 0.0;
        }
        q2 = fma(s, s, q2);
      }
      q2 = block_sum<double, NW>(q2, sd);
      if (tid == 0) {
        a.dtn[rt] = q2;     // read by the next residual pass only
        a.rt_cnt[rt] = 0u;  // re-arm
      }
    }
    __syncthreads();
  }
}

// Wave-wide decoupled look-back (all 64 lanes call it): exclusive prefix of `agg` over
// virtual blocks 0..vb-1, 64 predecessors per probe.  Words are [epoch:16|flag:2|value:46],
// flag 1 = aggregate, 2 = inclusive prefix.  Virtual block ids are handed out in arrival
// order, so every predecessor has started and publishes without waiting on later blocks.
__device__ inline int lookback_wave(uint64_t* status, int vb, int agg, uint32_t epoch, int lane) {
  const uint64_t E = static_cast<uint64_t>(epoch) << 48;
  constexpr uint64_t FA = 1ull << 46, FI = 2ull << 46, VMASK = (1ull << 46) - 1ull;
  if (lane == 0)
    publish(&status[vb], E | (vb == 0 ? FI : FA) | static_cast<uint64_t>(agg));
  if (vb == 0) return 0;
  int64_t prefix = 0;
  int j0 = vb - 1;
  while (true) {
    const int j = j0 - lane;
    uint64_t w = FI;  // positions before block 0 never matter (block 0 is inclusive)
    if (j >= 0) w = consume(&status[j]);
    const uint64_t flag = (w >> 46) & 3ull;
    const bool valid = j < 0 || ((w >> 48) == epoch && flag != 0);
    const bool incl = valid && (j < 0 || flag == 2);
    const unsigned long long inc_mask = __ballot(incl);
    const unsigned long long bad_mask = __ballot(!valid);
    const int first_inc = inc_mask ? __ffsll(static_cast<long long>(inc_mask)) - 1 : WAVE;
    const int first_bad = bad_mask ? __ffsll(static_cast<long long>(bad_mask)) - 1 : WAVE;
    if (first_bad < first_inc || (first_inc == WAVE && first_bad < WAVE)) {
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    const int64_t v = (lane <= first_inc && j >= 0) ? static_cast<int64_t>(w & VMASK) : 0;
    prefix += wave_sum(v);
    if (first_inc < WAVE) break;
    j0 -= WAVE;
  }
  if (lane == 0) publish(&status[vb], E | FI | static_cast<uint64_t>(prefix + agg));
  return static_cast<int>(prefix);
}

// z = D_A^T theta over the active list with the fused epilogue.  Block b owns list
// entries [b*CBU, b*CBU + CBU); units screened at the previous iteration (margin above
// the screening radius) are skipped without touching their columns; the kept ones are
// streamed (the HBM-bound part, CPW columns per wave for the Lasso, one group per wave
// for the Group-Lasso) and the prox (eq. softTh / gr_softTh) and FISTA momentum
// (Table 1) update x and u in place.  The block publishes its partials and a support
// segment (the new u on its kept units, with their margins and Omega terms) for the next
// residual.  When flagged, it also rewrites the list without the screened entries
// (order preserved, offsets by decoupled look-back).
template <typename T, typename V, bool VECTOR, int RULE, bool GROUP>
__global__ __launch_bounds__(BLK) void k_corr(SingleArgs<T, V, double> a) {
  constexpr int CBU = GROUP ? CBG : CBL;
  constexpr int SEGCAP = GROUP ? SEGCAP_G : SEGCAP_L;
  static_assert(CBU <= WAVE, "one wave decides the block's list entries");
  __shared__ int s_vb, s_nk, s_kpre;
  __shared__ int klist[CBU];
  __shared__ double kmarg[CBU];
  __shared__ double sred[NW][6];
  __shared__ SolverState S;
  __shared__ int s_il[CBL];  // Lasso: the block's new x and u by list position
  __shared__ V s_xs[CBL], s_us[CBL], s_xo[CBL], s_po[CBL];
  // groups: the same by support slot (group j, atom k at j * GMAX + k), and per group its
  // first atom, size, Omega term and backtracking sums
  constexpr int GSL = GROUP ? SEGCAP_G : 1, GGR = GROUP ? CBG : 1;
  __shared__ V g_xs[GSL], g_us[GSL], g_xo[GSL], g_po[GSL];
  __shared__ int64_t g_a0[GGR];
  __shared__ int g_m[GGR];
  __shared__ double g_om[GGR], g_omo[GGR], g_dn[GGR];
  if (a.kclk != nullptr && threadIdx.x == 0) a.kclk[2 * blockIdx.x] = wall_clock64();
  const int tid = threadIdx.x, lane = tid % WAVE, wave = tid / WAVE;
  // One round trip for the state (one word per thread into LDS) and for the list entries
  // of virtual block blockIdx.x in both lists (the state says which list is current), at
  // clamped indices so that no load waits for another; a compacting pass reloads the
  // entries of the block it draws.
  constexpr int NWORDS = sizeof(SolverState) / 4;
  static_assert(NWORDS <= BLK, "state fits one word per thread");
  const int32_t sword = reinterpret_cast<const int32_t*>(a.st + a.par)[min(tid, NWORDS - 1)];
  const int n_units = GROUP ? a.G : a.K;
  int e_unit0 = 0, e_unit1 = 0;
  double e_marg0 = 0.0, e_marg1 = 0.0;
  if (wave == 0) {
    const int e = min(static_cast<int>(blockIdx.x) * CBU + lane, n_units - 1);
    e_unit0 = a.act[0][e];
    e_unit1 = a.act[1][e];
    e_marg0 = a.act_m[0][e];
    e_marg1 = a.act_m[1][e];
  }
  if (tid < NWORDS) reinterpret_cast<int32_t*>(&S)[tid] = sword;
  __syncthreads();
  const SolverState* st = &S;
  if (st->done) return;
  const bool compact = st->compact != 0;
  int vb = blockIdx.x;
  if (compact) {
    if (tid == 0) s_vb = static_cast<int>(atomicAdd(&a.counters[CNT_VID], 1u));
    __syncthreads();
    vb = s_vb;
  }
  const int n_old = st->n_active, cur = st->cur;
  const double r_keep = st->r_scr + st->marg_slack;
  const uint32_t epoch = static_cast<uint32_t>(st->iter + 1) & 0xffffu;
  const int base = vb * CBU;
  const int cnt = max(0, min(CBU, n_old - base));
  if (wave == 0) {
    int unit = cur ? e_unit1 : e_unit0;
    double m = cur ? e_marg1 : e_marg0;
    if (vb != static_cast<int>(blockIdx.x)) {
      const int e = min(base + lane, n_units - 1);
      unit = a.act[cur][e];
      m = a.act_m[cur][e];
    }
    const bool keep = lane < cnt && !(m > r_keep);
    const unsigned long long bal = __ballot(keep);
    const int pos = __popcll(bal & ((1ull << lane) - 1ull));
    if (keep) { klist[pos] = unit; kmarg[pos] = m; }
    const int nk0 = static_cast<int>(__popcll(bal));
    if (compact) {
      const int pre = lookback_wave(a.lbA, vb, nk0, epoch, lane);
      if (lane == 0) s_kpre = pre;
    }
    if (lane == 0) s_nk = nk0;
  }
  __syncthreads();
  const int nk = s_nk;

  const double lam = st->lam, L = st->L;
  // Chambolle-Pock: step tau instead of 1/L, prox from x_{t-1}, extrapolation weight phi
  const double invL = RULE == RULE_CP ? st->cp_tau : 1.0 / L;
  const double thr = RULE == RULE_CP ? lam * invL : lam / L;
  const double l_prev = st->l_prev;
  double beta = 0.0;
  if (RULE == RULE_FISTA) beta = (l_prev - 1.0) / (0.5 * (1.0 + sqrt(1.0 + 4.0 * l_prev * l_prev)));
  if (RULE == RULE_CP) beta = 1.0 / sqrt(1.0 + 2.0 * st->cp_gamma * st->cp_tau);
  double zsup = 0.0;  // max |z_i| (Lasso) or max ||z_g|| / w_g; rounding slack added later
  int nnz = 0, nsup = 0, natoms = 0;
  double dd = 0.0;    // backtracking: ||x' - p||^2 over this block's units
  double de = 0.0;    // SpaRSA: z^T d + lambda (Omega(x') - Omega(p)) over this block's units
  if constexpr (!GROUP) {
    for (int r0 = wave * CPW; r0 < nk; r0 += NW * CPW) {
      const int nc = min(CPW, nk - r0);
      const int jl = r0 + min(lane, nc - 1);
      const int i_l = klist[jl];
      // epilogue operands in flight together with the column stream
      const double p = static_cast<double>(a.u[i_l]);
      const double xo = static_cast<double>(a.x[i_l]);
      const T* cols[CPW];
#pragma unroll
      for (int c = 0; c < CPW; ++c)
        cols[c] = a.D + static_cast<int64_t>(klist[r0 + min(c, nc - 1)]) * a.ldd;
      double acc[CPW];
      wave_dots<T, V, CPW, VECTOR>(cols, a.theta, a.N, lane, acc);
#pragma unroll
      for (int c = 0; c < CPW; ++c) acc[c] = wave_sum(acc[c]);
      if (lane < nc) {
        const double z = pick(acc, lane);
        const double vv = (RULE == RULE_CP ? xo : p) - z * invL;
        const double mag = fabs(vv) - thr;
        const double xn = mag > 0.0 ? copysign(mag, vv) : 0.0;
        const double un = (RULE == RULE_FISTA || RULE == RULE_CP) ? xn + beta * (xn - xo) : xn;
        const V xs = static_cast<V>(xn), us = static_cast<V>(un);
        // staged in LDS and written once the block's rounds are done: a global store
        // here would hold up the next round's column loads until it completes
        s_il[jl] = i_l;
        s_xs[jl] = xs;
        s_us[jl] = us;
        if (a.bt) {  // keep p and x_{t-1} so that a rejected step can be undone
          const double dv = static_cast<double>(xs) - p;  // exact: two stored values
          s_xo[jl] = static_cast<V>(xo);
          s_po[jl] = static_cast<V>(p);
          dd = fma(dv, dv, dd);
          // SpaRSA: z_i d_i + lambda (|x'_i| - |p_i|), the first-order and penalty parts of
          // phi(x') - phi(p), unit by unit
          if constexpr (RULE == RULE_SPARSA)
            de += fma(z, dv, lam * (fabs(static_cast<double>(xs)) - fabs(p)));
        }
        zsup = fmax(zsup, fabs(z));
        nnz += xs != V(0) ? 1 : 0;
        nsup += us != V(0) ? 1 : 0;
      }
    }
    natoms = tid == 0 ? nk : 0;
  } else {
    constexpr int NS = GMAX / WAVE;  // atoms per lane: atom k of the group sits on lane k % 64
    // the offsets of the wave's (at most two) groups in one round trip: lane 2i + e reads
    // gptr[g_i + e] (lanes past 3 repeat lane 3's address)
    static_assert(CBG == 2 * NW, "two groups per wave");
    const int jq = wave + (min(lane, 3) >> 1) * NW;
    const int gq = nk > 0 ? klist[min(jq, nk - 1)] : 0;
    const long long goff = static_cast<long long>(a.gptr[gq + (min(lane, 3) & 1)]);
    int it = 0;
    for (int j = wave; j < nk; j += NW, ++it) {
      const int g = klist[j];
      const int64_t a0 = __shfl(goff, 2 * it);
      const int m = static_cast<int>(__shfl(goff, 2 * it + 1) - a0);
      double p[NS], xo[NS], vreg[NS], zk[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int li = min(lane + s * WAVE, m - 1);
        p[s] = static_cast<double>(a.u[a0 + li]);
        xo[s] = static_cast<double>(a.x[a0 + li]);
        vreg[s] = 0.0;
        zk[s] = 0.0;
      }
      double z2 = 0.0;
      for (int b0 = 0; b0 < m; b0 += CPW) {
        const int nc = min(CPW, m - b0);
        const T* cols[CPW];
#pragma unroll
        for (int c = 0; c < CPW; ++c) cols[c] = a.D + (a0 + b0 + min(c, nc - 1)) * a.ldd;
        double acc[CPW];
        wave_dots<T, V, CPW, VECTOR>(cols, a.theta, a.N, lane, acc);
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
          acc[c] = wave_sum(acc[c]);
          if (c < nc) {
            z2 = fma(acc[c], acc[c], z2);
#pragma unroll
            for (int s = 0; s < NS; ++s)
              if (b0 + c == lane + s * WAVE) zk[s] = acc[c];
          }
        }
      }
      // the gradient step after the stream, so that the u and x loads are not waited for
      // before the first columns are requested
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (lane + s * WAVE < m) vreg[s] = (RULE == RULE_CP ? xo[s] : p[s]) - zk[s] * invL;
      double vsq = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) vsq += vreg[s] * vreg[s];
      const double v2 = wave_sum(vsq);
      const double wg = a.w[g];
      const double nv = sqrt(v2);
      const double scale = nv > 0.0 ? fmax(0.0, (nv - thr * wg) / nv) : 0.0;
      int gnz = 0, gsup = 0;
      double un2 = 0.0, dn = 0.0, po2 = 0.0;
      double gzd = 0.0, gds = 0.0;  // SpaRSA: z_g^T d_g and d_g^T (x'_g + p_g)
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int ak = lane + s * WAVE;  // atom of the group
        if (ak < m) {
          const double xn = scale * vreg[s];
          const double un =
              (RULE == RULE_FISTA || RULE == RULE_CP) ? xn + beta * (xn - xo[s]) : xn;
          const V xs = static_cast<V>(xn), us = static_cast<V>(un);
          // staged in LDS and stored after the block's last group (a global store here
          // would hold up the wave's next loads until it completed)
          const int ls = j * GMAX + ak;
          g_xs[ls] = xs;
          g_us[ls] = us;
          if (a.bt) {
            const double dv = static_cast<double>(xs) - p[s];
            g_xo[ls] = static_cast<V>(xo[s]);
            g_po[ls] = static_cast<V>(p[s]);
            dn = fma(dv, dv, dn);
            po2 = fma(p[s], p[s], po2);
            if constexpr (RULE == RULE_SPARSA) {
              gzd = fma(zk[s], dv, gzd);
              gds = fma(dv, static_cast<double>(xs) + p[s], gds);
            }
          }
          gnz += xs != V(0) ? 1 : 0;
          gsup += us != V(0) ? 1 : 0;
          un2 = fma(static_cast<double>(us), static_cast<double>(us), un2);
        }
      }
      gnz = wave_sum(gnz);
      gsup = wave_sum(gsup);
      un2 = wave_sum(un2);
      if (a.bt) {
        dn = wave_sum(dn);
        po2 = wave_sum(po2);
        if constexpr (RULE == RULE_SPARSA) {
          gzd = wave_sum(gzd);
          gds = wave_sum(gds);
        }
      }
      if (lane == 0) {
        g_a0[j] = a0;
        g_m[j] = m;
        g_om[j] = wg * sqrt(un2);
        if (a.bt) {
          g_omo[j] = wg * sqrt(po2);
          g_dn[j] = dn;
          dd += dn;
          if constexpr (RULE == RULE_SPARSA) {
            // ||x'_g|| - ||p_g|| = d_g^T (x'_g + p_g) / (||x'_g|| + ||p_g||): no cancellation
            const double den = sqrt(un2) + sqrt(po2);
            de += gzd + (den > 0.0 ? lam * wg * (gds / den) : 0.0);
          }
        }
        zsup = fmax(zsup, sqrt(z2) / wg);
        nnz += gnz;
        nsup += gsup;
        natoms += m;
      }
    }
  }
  // block partials in one LDS pass (counts are exact in FP64)
  zsup = wave_max(zsup);
  const double cnz = wave_sum(static_cast<double>(nnz)), csup = wave_sum(static_cast<double>(nsup));
  const double cat = wave_sum(static_cast<double>(natoms));
  const double cdd = a.bt ? wave_sum(dd) : 0.0;
  const double cde = RULE == RULE_SPARSA ? wave_sum(de) : 0.0;
  if (lane == 0) {
    sred[wave][0] = zsup;
    sred[wave][1] = cnz;
    sred[wave][2] = csup;
    sred[wave][3] = cat;
    sred[wave][4] = cdd;
    if (RULE == RULE_SPARSA) sred[wave][5] = cde;
  }
  __syncthreads();
  // Global stores come after the column stream: a wave's loads wait for its earlier
  // stores to complete.
  if (compact && tid < nk) {
    a.act[1 - cur][s_kpre + tid] = klist[tid];
    a.act_m[1 - cur][s_kpre + tid] = kmarg[tid];
  }
  if (tid == 0) a.seg_cnt[vb] = nk;
  if constexpr (GROUP) {
    // the kept groups' x and u, support segment and group records
    for (int ls = tid; ls < nk * GMAX; ls += BLK) {
      const int j = ls / GMAX, ak = ls % GMAX;
      if (ak < g_m[j]) {
        const int64_t at = g_a0[j] + ak;
        const V xs = g_xs[ls], us = g_us[ls];
        a.x[at] = xs;
        a.u[at] = us;
        const int64_t slot = static_cast<int64_t>(vb) * SEGCAP + ls;
        a.seg_atom[slot] = static_cast<int32_t>(at);
        a.seg_val[slot] = us;
        if (a.bt) {
          const V po = g_po[ls];
          a.seg_xo[slot] = g_xo[ls];
          a.seg_po[slot] = po;
          a.seg_d[slot] = static_cast<double>(xs) - static_cast<double>(po);
        }
      }
    }
    if (tid < nk) {
      const int64_t rec = static_cast<int64_t>(vb) * CBU + tid;
      a.urec_marg[rec] = kmarg[tid];
      a.urec_om[rec] = g_om[tid];
      a.urec_m[rec] = g_m[tid];
      if (a.bt) {
        a.urec_omo[rec] = g_omo[tid];
        a.urec_dn[rec] = g_dn[tid];
      }
    }
  }
  if constexpr (!GROUP) {
    if (tid < nk) {  // the kept units' x and u, and the block's support segment
      const int i_l = s_il[tid];
      const V xs = s_xs[tid], us = s_us[tid];
      a.x[i_l] = xs;
      a.u[i_l] = us;
      const int64_t slot = static_cast<int64_t>(vb) * SEGCAP + tid;
      a.seg_atom[slot] = i_l;
      a.seg_val[slot] = us;
      a.urec_marg[slot] = kmarg[tid];
      a.urec_om[slot] = fabs(static_cast<double>(us));
      if (a.bt) {
        const double p = static_cast<double>(s_po[tid]);
        a.seg_xo[slot] = s_xo[tid];
        a.seg_po[slot] = s_po[tid];
        a.seg_d[slot] = static_cast<double>(xs) - p;
        a.urec_omo[slot] = fabs(p);
      }
    }
  }
  if (tid == 0) {  // read by the next residual pass only (after this kernel ends)
    double r0 = sred[0][0], r1 = sred[0][1], r2 = sred[0][2], r3 = sred[0][3], r4 = sred[0][4];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      r0 = fmax(r0, sred[w][0]);
      r1 += sred[w][1];
      r2 += sred[w][2];
      r3 += sred[w][3];
      r4 += sred[w][4];
    }
    double r5 = 0.0;
    if (RULE == RULE_SPARSA)
      for (int w = 0; w < NW; ++w) r5 += sred[w][5];
    if (a.bt) a.bpd[vb] = r4;
    if (RULE == RULE_SPARSA) a.bpe[vb] = r5;
    zsup = r0;
    nnz = static_cast<int>(r1);
    nsup = static_cast<int>(r2);
    natoms = static_cast<int>(r3);
    a.bp0[vb] = zsup;
    a.bpi[vb] = nnz;
    a.bpi[MAXB + vb] = nk;
    a.bpi[2 * MAXB + vb] = nsup;
    a.bpi[3 * MAXB + vb] = natoms;
    if (vb == 0) {
      SolverState* sw = a.st + a.par;
      sw->pending = 1;  // no block of this pass reads it after its prologue
    }
    if (a.kclk != nullptr) a.kclk[2 * blockIdx.x + 1] = wall_clock64();
  }
}

// Aligned copy of the observation (the caller's y may have any alignment).
template <typename V>
__global__ __launch_bounds__(BLK) void k_copy_y(const V* __restrict__ y, V* __restrict__ yc, int N,
                                                 int npad) {
  const int i = blockIdx.x * BLK + threadIdx.x;
  if (i < npad) yc[i] = i < N ? y[i] : V(0);
}

// Output: X = 0 outside the active units, x on them.
template <typename T, typename V, typename A>
__global__ __launch_bounds__(BLK) void k_zero_out(V* __restrict__ X, int K) {
  const int i = blockIdx.x * BLK + threadIdx.x;
  if (i < K) X[i] = V(0);
}
template <typename T, typename V, typename A>
__global__ __launch_bounds__(BLK) void k_scatter_out(SingleArgs<T, V, A> a, V* __restrict__ X) {
  const SolverState* st = a.st + a.par;
  const int j = blockIdx.x * BLK + threadIdx.x;
  if (st->status != 0 || j >= st->n_active) return;
  const int unit = a.act[st->cur][j];
  if (a.marg[unit] > st->r_scr + st->marg_slack) return;  // screened, not yet compacted away
  const V* src = a.rule == RULE_CP ? a.u : a.x;  // Chambolle-Pock returns u (certified)
  if (a.G > 0) {
    for (int64_t i = a.gptr[unit]; i < a.gptr[unit + 1]; ++i) X[i] = src[i];
  } else {
    X[unit] = src[unit];
  }
}

__global__ void k_fill_u8(uint8_t* __restrict__ p, int n, uint8_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
// Screened mask: 0 on the atoms of the active units (run after k_fill_u8(.., 1)).
template <typename T, typename V, typename A>
__global__ __launch_bounds__(BLK) void k_mark_active(SingleArgs<T, V, A> a, uint8_t* __restrict__ m) {
  const SolverState* st = a.st + a.par;
  const int j = blockIdx.x * BLK + threadIdx.x;
  if (st->status != 0 || j >= st->n_active) return;
  const int unit = a.act[st->cur][j];
  if (a.marg[unit] > st->r_scr + st->marg_slack) return;
  if (a.G > 0) {
    for (int64_t i = a.gptr[unit]; i < a.gptr[unit + 1]; ++i) m[i] = 0;
  } else {
    m[unit] = 0;
  }
}

// ============================================================== power iteration =====

// w = D v over all K columns, FP64: work items (row tile x chunk of PCH columns); each
// wave streams its share of the chunk's columns RPW at a time (16-byte loads when
// aligned), the block adds the waves' row partials in wave order and writes one partial
// per (chunk, row); k_pow_reduce adds the chunks in order.
constexpr int PCH = 512;
template <typename T, bool VECTOR>
__global__ __launch_bounds__(BLK) void k_pow_dv(const T* __restrict__ D, int64_t ldd, int N,
                                                 int K, const double* __restrict__ v,
                                                 double* __restrict__ part, int64_t npad) {
  constexpr int VR = VECTOR ? Store<T>::VEC : 1;
  constexpr int RT = WAVE * VR;
  __shared__ double red[NW][RT];
  const int tid = threadIdx.x, lane = tid % WAVE, wave = tid / WAVE;
  const int nrt = (N + RT - 1) / RT;
  const int nch = (K + PCH - 1) / PCH;
  for (int item = blockIdx.x; item < nrt * nch; item += gridDim.x) {
    const int rt = item % nrt, c = item / nrt;
    const int r0 = rt * RT + lane * VR;
    const int k1 = min((c + 1) * PCH, K);
    double acc[VR];
#pragma unroll
    for (int e = 0; e < VR; ++e) acc[e] = 0.0;
    for (int kb = c * PCH + wave * RPW; kb < k1; kb += NW * RPW) {
      int idx[RPW];
      double val[RPW];
#pragma unroll
      for (int p = 0; p < RPW; ++p) {
        const bool ok = kb + p < k1;
        idx[p] = ok ? kb + p : kb;
        val[p] = ok ? v[kb + p] : 0.0;
      }
      if (VECTOR && r0 + VR <= N) {
        if constexpr (VECTOR) {
          uint4 cv[RPW];
#pragma unroll
          for (int p = 0; p < RPW; ++p) cv[p] = ld16(D + static_cast<int64_t>(idx[p]) * ldd + r0);
#pragma unroll
          for (int p = 0; p < RPW; ++p) {
            double d[VR];
            widen<T>(cv[p], d);
#pragma unroll
            for (int e = 0; e < VR; ++e) acc[e] = fma(d[e], val[p], acc[e]);
          }
        }
      } else {
#pragma unroll
        for (int p = 0; p < RPW; ++p) {
          const T* col = D + static_cast<int64_t>(idx[p]) * ldd;
          for (int e = 0; e < VR; ++e)
            if (r0 + e < N) acc[e] = fma(to_double(col[r0 + e]), val[p], acc[e]);
        }
      }
    }
#pragma unroll
    for (int e = 0; e < VR; ++e) red[wave][lane * VR + e] = acc[e];
    __syncthreads();
    for (int rr = tid; rr < RT; rr += BLK) {
      const int r = rt * RT + rr;
      if (r < N) {
        double s = red[0][rr];
#pragma unroll
        for (int w = 1; w < NW; ++w) s += red[w][rr];
        part[static_cast<int64_t>(c) * npad + r] = s;
      }
    }
    __syncthreads();
  }
}
__global__ __launch_bounds__(BLK) void k_pow_reduce(const double* __restrict__ part, int nch,
                                                     int64_t npad, int N, double* __restrict__ w) {
  constexpr int FB = 16;  // chunk partials loaded at once (clamped indices, in order)
  const int r = blockIdx.x * BLK + threadIdx.x;
  if (r >= N) return;
  double s = 0.0;
  for (int c0 = 0; c0 < nch; c0 += FB) {
    double q[FB];
#pragma unroll
    for (int k = 0; k < FB; ++k) q[k] = part[static_cast<int64_t>(min(c0 + k, nch - 1)) * npad + r];
#pragma unroll
    for (int k = 0; k < FB; ++k) s += c0 + k < nch ? q[k] : 0.0;
  }
  w[r] = s;
}
__global__ __launch_bounds__(CBLK) void k_pow_dots(const double* __restrict__ a,
                                                    const double* __restrict__ b, int n,
                                                    double* __restrict__ out) {
  __shared__ double sd[CNW];
  double aa = 0.0, ab = 0.0, bb = 0.0;
  for (int i = threadIdx.x; i < n; i += CBLK) {
    aa = fma(a[i], a[i], aa);
    ab = fma(a[i], b[i], ab);
    bb = fma(b[i], b[i], bb);
  }
  aa = block_sum<double, CNW>(aa, sd);
  ab = block_sum<double, CNW>(ab, sd);
  bb = block_sum<double, CNW>(bb, sd);
  if (threadIdx.x == 0) { out[0] = aa; out[1] = ab; out[2] = bb; }
}
__global__ __launch_bounds__(BLK) void k_pow_scale(const double* __restrict__ src, int n,
                                                    const double* __restrict__ dots,
                                                    double* __restrict__ dst) {
  const int i = blockIdx.x * BLK + threadIdx.x;
  if (i >= n) return;
  const double nb = sqrt(dots[2]);
  dst[i] = nb > 0.0 ? src[i] / nb : 0.0;
}
// Zero n 32-bit words (counters and partials that must start at zero: a kernel rather than
// a memset, so that the clearing is an ordinary kernel node if a caller captures the work).
__global__ void k_zero_words(uint32_t* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = 0u;
}

// Default group weights w_g = sqrt(|g|) (the Group-Lasso section's choice).
__global__ void k_default_weights(const int64_t* __restrict__ gptr, int G, double* __restrict__ w) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < G) w[g] = sqrt(static_cast<double>(gptr[g + 1] - gptr[g]));
}

__global__ void k_fill(double* __restrict__ v, int n, double val) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = val;
}

}  // namespace ds
