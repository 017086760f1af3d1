// Single-signal kernels: Algorithm 3 with ISTA / FISTA (Table 1) and the sphere tests of
// Lemmas 1, 2, 4, 5 (through Lemma 6), one signal at a time.
//
// Per iteration four launches, all on one stream:
//   k_resid           theta partial sums  D_S p_S over the support S of the primal point p
//   k_resid_finalize  theta = sum(partials) - y, FP64 ||theta||^2 and theta^T y
//   k_corr_*          z = D_A^T theta over the active list A (the HBM stream), fused with the
//                     prox (eq. softTh / gr_softTh), the FISTA momentum, ||z||_inf or the
//                     group norms, Omega(p) and nnz; the last block to finish runs the
//                     FP64 screening scalars (dual scaling Lemma 7, radius, gap, stop rule)
//   k_compact         order-preserving compaction of A against the margins, plus the
//                     support list of the next primal point
// Every scalar is in device memory (SolverState); once `done` is set the kernels return
// immediately, so the host may enqueue iterations ahead of the stopping decision.
#pragma once
#include <cmath>

#include "ds_device.h"
#include "ds_state.h"

namespace ds {

constexpr int BLK = 256;         // threads per block of the streaming kernels
constexpr int NW = BLK / WAVE;   // waves per block
constexpr int CPW = 4;           // columns per wave in the correlation kernel
constexpr int RCH = 16;          // support columns per residual work item
constexpr int CBLK = 1024;       // threads of the single-block kernels
constexpr int CNW = CBLK / WAVE;
constexpr int MAXB = 2048;       // maximum grid of the kernels with block partials
constexpr int GMAX_REG = 4;      // group kernel: up to GMAX_REG * 64 atoms per group

enum CounterSlot { CNT_FIN = 0, CNT_CORR = 1, CNT_SETUP = 2, CNT_POW = 3 };

__device__ __forceinline__ double dinf() { return __builtin_huge_val(); }

// ---------------------------------------------------------------- vector loads ------
template <typename V, int VEC, typename A>
__device__ __forceinline__ void load_v(const V* __restrict__ p, A (&o)[VEC]) {
#pragma unroll
  for (int k = 0; k < VEC; ++k) o[k] = static_cast<A>(p[k]);
}

// Dot products of NC columns with a vector, by one wave.  Columns with c >= ncols are
// not read.  With VECTOR each lane issues 16-byte loads (columns must be 16-byte
// aligned); the tail N % VEC is read element-wise.
template <typename T, typename V, typename A, int NC, bool VECTOR>
__device__ __forceinline__ void wave_dots(const T* const (&cols)[NC], int ncols,
                                          const V* __restrict__ v, int N, int lane,
                                          A (&acc)[NC]) {
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = A(0);
  if constexpr (VECTOR) {
    constexpr int VEC = Store<T>::VEC;
    const int nfull = N / VEC;
#pragma unroll 2
    for (int q = lane; q < nfull; q += WAVE) {
      A vv[VEC];
      load_v<V, VEC, A>(v + q * VEC, vv);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if (c < ncols) {
          A d[VEC];
          load_vec<T, A>(cols[c] + static_cast<int64_t>(q) * VEC, d);
#pragma unroll
          for (int k = 0; k < VEC; ++k) acc[c] = fma(d[k], vv[k], acc[c]);
        }
      }
    }
    const int e = nfull * VEC + lane;
    if (e < N) {
      const A ve = static_cast<A>(v[e]);
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (c < ncols) acc[c] = fma(static_cast<A>(to_double(cols[c][e])), ve, acc[c]);
    }
  } else {
    for (int e = lane; e < N; e += WAVE) {
      const A ve = static_cast<A>(v[e]);
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (c < ncols) acc[c] = fma(static_cast<A>(to_double(cols[c][e])), ve, acc[c]);
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
    wave_dots<T, VV, double, CPW, VECTOR>(cols, nc, v, N, lane, acc);
    double sq[CPW];
    if constexpr (NORMS) {
#pragma unroll
      for (int c = 0; c < CPW; ++c) sq[c] = 0.0;
      for (int e = lane; e < N; e += WAVE) {
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
          if (c < nc) {
            const double d = to_double(cols[c][e]);
            sq[c] = fma(d, d, sq[c]);
          }
        }
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

// Group spectral norms ||D_g||_2 (Lemma 6) and Frobenius norms: one block per group
// forms the Gram matrix D_g^T D_g in FP64 and diagonalises it by cyclic Jacobi.
template <typename T>
__global__ __launch_bounds__(BLK) void k_group_norms(const T* __restrict__ D, int64_t ldd, int N,
                                                      int G, const int64_t* __restrict__ gptr,
                                                      double* __restrict__ gnorm,
                                                      double* __restrict__ fro) {
  constexpr int GM = 64;  // largest group handled by this kernel
  __shared__ double gram[GM * GM];
  __shared__ double red[NW];
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  for (int g = blockIdx.x; g < G; g += gridDim.x) {
    const int64_t a0 = gptr[g];
    const int m = static_cast<int>(gptr[g + 1] - a0);
    const int npairs = m * (m + 1) / 2;
    for (int pidx = wv; pidx < npairs; pidx += NW) {
      int a = 0, rem = pidx;
      while (rem >= m - a) { rem -= m - a; ++a; }
      const int b = a + rem;
      const T* ca = D + (a0 + a) * ldd;
      const T* cb = D + (a0 + b) * ldd;
      double s = 0.0;
      for (int e = lane; e < N; e += WAVE) s = fma(to_double(ca[e]), to_double(cb[e]), s);
      s = wave_sum(s);
      if (lane == 0) { gram[a * GM + b] = s; gram[b * GM + a] = s; }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double f2 = 0.0;
      for (int a = 0; a < m; ++a) f2 += gram[a * GM + a];
      // cyclic Jacobi sweeps until the off-diagonal mass is negligible
      for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < m; ++p)
          for (int q = p + 1; q < m; ++q) off += gram[p * GM + q] * gram[p * GM + q];
        if (off <= 1e-30 * f2 * f2) break;
        for (int p = 0; p < m; ++p) {
          for (int q = p + 1; q < m; ++q) {
            const double apq = gram[p * GM + q];
            if (apq == 0.0) continue;
            const double app = gram[p * GM + p], aqq = gram[q * GM + q];
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
            for (int k = 0; k < m; ++k) {
              const double akp = gram[k * GM + p], akq = gram[k * GM + q];
              gram[k * GM + p] = c * akp - s * akq;
              gram[k * GM + q] = s * akp + c * akq;
            }
            for (int k = 0; k < m; ++k) {
              const double apk = gram[p * GM + k], aqk = gram[q * GM + k];
              gram[p * GM + k] = c * apk - s * aqk;
              gram[q * GM + k] = s * apk + c * aqk;
            }
          }
        }
      }
      double lmax = 0.0;
      for (int a = 0; a < m; ++a) lmax = fmax(lmax, gram[a * GM + a]);
      gnorm[g] = sqrt(lmax);
      fro[g] = sqrt(f2);
    }
    __syncthreads();
  }
  (void)red;
}

// One block: ||y||^2, lambda_*, arg-max, lambda, centre data, state initialisation.
// Group problems: lambda_* = max_g ||z0_g|| / w_g (eq. (gstar)).
template <typename T, typename V, typename A>
__global__ __launch_bounds__(CBLK) void k_setup_scalars(SingleArgs<T, V, A> a, double lam_in,
                                                         int lam_relative, double L,
                                                         double gap_tol, int max_iter,
                                                         double gamma_z) {
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
  // centre of the DST3 / DGST3 sphere: n = d_* (Lasso) or D_g* D_g*^T y / lambda_* (groups)
  double nn = 0.0, ny = 0.0, wstar2 = 1.0;
  if (a.test == TEST_DST3 && !trivial && !bad) {
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
  if (tid == 0) {
    const double alpha = (a.test == TEST_DST3 && nn > 0.0) ? (ny / lam - wstar2) / nn : 0.0;
    st->lam = lam;
    st->lam_ratio = lam_relative ? lam_in : lam / lam_max;
    st->lam_max = lam_max;
    st->L = L;
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
// d_i^T c = z0_i / lambda - alpha * g_i with g = D^T n.
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
  } else {
    const double ci = a.z0[i] / lam - (dst3 ? alpha * a.g[i] : 0.0);
    const double nu = a.nu[i];
    m = nu > 0.0 ? (1.0 - fabs(ci)) / nu : dinf();
  }
  a.marg[i] = m;
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
  if (threadIdx.x == 0) {
    const double eps = (a.N + 16) * 0x1p-53;
    st->marg_slack = eps * kappa * (sqrt(st->yy) / st->lam + fabs(st->alpha) * sqrt(st->nn) + 1.0);
  }
}

// ============================================================== iteration kernels ===

// theta partial sums: item (row tile rt, chunk c) sums the support columns of chunk c.
template <typename T, typename V, typename A, bool VECTOR>
__global__ __launch_bounds__(BLK) void k_resid(SingleArgs<T, V, A> a) {
  const SolverState* st = a.st;
  if (st->done) return;
  constexpr int VR = VECTOR ? Store<T>::VEC : 1;
  const int nS = st->n_support;
  const int nch = (nS + RCH - 1) / RCH;
  const int RT = BLK * VR;
  const int nrt = (a.N + RT - 1) / RT;
  const int items = nrt * nch;
  for (int item = blockIdx.x; item < items; item += gridDim.x) {
    const int rt = item % nrt, c = item / nrt;
    const int r0 = rt * RT + threadIdx.x * VR;
    A acc[VR];
#pragma unroll
    for (int k = 0; k < VR; ++k) acc[k] = A(0);
    const int k0 = c * RCH, k1 = min(k0 + RCH, nS);
    if (r0 + VR <= a.N) {
      for (int k = k0; k < k1; ++k) {
        const A val = static_cast<A>(a.s_val[k]);
        const T* col = a.D + static_cast<int64_t>(a.s_idx[k]) * a.ldd + r0;
        if constexpr (VECTOR) {
          A d[VR];
          load_vec<T, A>(col, d);
#pragma unroll
          for (int e = 0; e < VR; ++e) acc[e] = fma(d[e], val, acc[e]);
        } else {
          acc[0] = fma(static_cast<A>(to_double(col[0])), val, acc[0]);
        }
      }
#pragma unroll
      for (int e = 0; e < VR; ++e) a.partial[static_cast<int64_t>(c) * a.npad + r0 + e] = acc[e];
    } else if (r0 < a.N) {
      for (int k = k0; k < k1; ++k) {
        const A val = static_cast<A>(a.s_val[k]);
        const T* col = a.D + static_cast<int64_t>(a.s_idx[k]) * a.ldd;
        for (int e = 0; e < VR; ++e)
          if (r0 + e < a.N) acc[e] = fma(static_cast<A>(to_double(col[r0 + e])), val, acc[e]);
      }
      for (int e = 0; e < VR; ++e)
        if (r0 + e < a.N) a.partial[static_cast<int64_t>(c) * a.npad + r0 + e] = acc[e];
    }
  }
}

// theta = sum of the chunk partials (fixed order) - y; FP64 ||theta||^2, theta^T y.
template <typename T, typename V, typename A>
__global__ __launch_bounds__(BLK) void k_resid_finalize(SingleArgs<T, V, A> a) {
  __shared__ double sd[NW];
  __shared__ int flag;
  SolverState* st = a.st;
  if (st->done) return;
  const int nch = (st->n_support + RCH - 1) / RCH;
  const int r = blockIdx.x * BLK + threadIdx.x;
  double tt = 0.0, ty = 0.0;
  if (r < a.N) {
    A s = A(0);
    for (int c = 0; c < nch; ++c) s += a.partial[static_cast<int64_t>(c) * a.npad + r];
    const V yv = a.y[r];
    const V th = static_cast<V>(s - static_cast<A>(yv));
    a.theta[r] = th;
    tt = static_cast<double>(th) * static_cast<double>(th);
    ty = static_cast<double>(th) * static_cast<double>(yv);
  }
  tt = block_sum<double, NW>(tt, sd);
  ty = block_sum<double, NW>(ty, sd);
  if (threadIdx.x == 0) { a.bp0[blockIdx.x] = tt; a.bp1[blockIdx.x] = ty; }
  if (last_block_arrive(&a.counters[CNT_FIN], &flag)) {
    double t2 = 0.0, y2 = 0.0;
    for (int b = threadIdx.x; b < static_cast<int>(gridDim.x); b += BLK) {
      t2 += a.bp0[b];
      y2 += a.bp1[b];
    }
    t2 = block_sum<double, NW>(t2, sd);
    y2 = block_sum<double, NW>(y2, sd);
    if (threadIdx.x == 0) {
      st->tt = t2;
      st->ty = y2;
      a.counters[CNT_FIN] = 0u;
    }
  }
}

// FP64 scalars of one iteration (thread 0 of the last correlation block).
// Dual scaling (Lemma 7), dual point v = mu theta, gap certificate, radius of the
// chosen sphere test, stopping rule; the screening radius carries a rounding slack.
__device__ inline void scalar_update(SolverState* st, int N, int test, double zsup,
                                     double omega, int nnz, double l_new) {
  const int t = st->iter + 1;
  const double tt = st->tt, ty = st->ty, lam = st->lam, yy = st->yy, rho2 = st->rho2;
  const double s = zsup > 0.0 ? 1.0 / zsup : dinf();
  double mu = 0.0;
  if (tt > 0.0) mu = fmin(fmax(ty / (lam * tt), -s), s);
  const double primal = 0.5 * tt + lam * omega;
  const double dual = lam * mu * ty - 0.5 * lam * lam * mu * mu * tt;
  const double gap = primal - dual;
  const double a1 = yy / (lam * lam), a2 = 2.0 * mu * ty / lam, a3 = mu * mu * tt;
  const double R2 = a1 - a2 + a3;
  double r = dinf(), r_safe = dinf();
  if (test != TEST_NONE) {
    const double q = R2 - (test == TEST_DST3 ? rho2 : 0.0);
    const double E = (N + 16) * 0x1p-53 * (a1 + fabs(a2) + a3 + rho2);
    r = sqrt(fmax(q, 0.0));
    r_safe = sqrt(fmax(q + E, 0.0));
  }
  st->iter = t;
  st->zsup = zsup;
  st->omega = omega;
  st->mu = mu;
  st->gap = gap;
  st->primal = primal;
  st->dual = dual;
  st->nnz = nnz;
  st->l_prev = l_new;
  st->r_last = r;
  st->r_min = fmin(st->r_min, r);
  const bool stop = (st->gap_tol_abs > 0.0 && gap <= st->gap_tol_abs) || t >= st->max_iter;
  if (stop) {
    st->done = 1;
  } else if (r_safe < st->r_scr) {
    st->r_scr = r_safe;
    st->r_slack = r_safe - r;
  }
}

// Correlation over the active atoms with the fused Lasso epilogue (one wave per CPW atoms).
template <typename T, typename V, typename A, bool VECTOR, int RULE>
__global__ __launch_bounds__(BLK) void k_corr_lasso(SingleArgs<T, V, A> a) {
  __shared__ double sd[NW];
  __shared__ int si[NW];
  __shared__ int flag;
  SolverState* st = a.st;
  if (st->done) return;
  const int n = st->n_active;
  const int32_t* __restrict__ act = a.act[st->cur];
  const double lam = st->lam, L = st->L;
  const A invL = static_cast<A>(1.0 / L);
  const A thr = static_cast<A>(lam / L);
  const double l_prev = st->l_prev;
  double l_new = l_prev;
  A beta = A(0);
  if (RULE == RULE_FISTA) {
    l_new = 0.5 * (1.0 + sqrt(1.0 + 4.0 * l_prev * l_prev));
    beta = static_cast<A>((l_prev - 1.0) / l_new);
  }
  const double gz = st->gamma_z * sqrt(st->tt);
  const int lane = threadIdx.x % WAVE;
  const int gw = blockIdx.x * NW + threadIdx.x / WAVE;
  const int nwaves = gridDim.x * NW;
  double zsup = 0.0, omega = 0.0;
  int nnz = 0;
  for (int base = gw * CPW; base < n; base += nwaves * CPW) {
    const int nc = min(CPW, n - base);
    int idx[CPW];
    const T* cols[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      idx[c] = act[base + min(c, nc - 1)];
      cols[c] = a.D + static_cast<int64_t>(idx[c]) * a.ldd;
    }
    A acc[CPW];
    wave_dots<T, V, A, CPW, VECTOR>(cols, nc, a.theta, a.N, lane, acc);
#pragma unroll
    for (int c = 0; c < CPW; ++c) acc[c] = wave_sum(acc[c]);
    if (lane < nc) {
      const A z = pick(acc, lane);
      const int i = pick(idx, lane);
      const V p = a.u[i];
      const A xo = static_cast<A>(a.x[i]);
      const A vv = static_cast<A>(p) - z * invL;
      const A mag = fabs(vv) - thr;
      const A xn = mag > A(0) ? copysign(mag, vv) : A(0);
      const A un = RULE == RULE_FISTA ? xn + beta * (xn - xo) : xn;
      a.x[i] = static_cast<V>(xn);
      a.u[i] = static_cast<V>(un);
      zsup = fmax(zsup, fabs(static_cast<double>(z)) + gz * a.nu[i]);
      omega += fabs(static_cast<double>(p));
      nnz += xn != A(0) ? 1 : 0;
    }
  }
  zsup = block_max<double, NW>(zsup, sd);
  omega = block_sum<double, NW>(omega, sd);
  nnz = block_sum<int, NW>(nnz, si);
  if (threadIdx.x == 0) {
    a.bp0[blockIdx.x] = zsup;
    a.bp1[blockIdx.x] = omega;
    a.bpi[blockIdx.x] = nnz;
  }
  if (last_block_arrive(&a.counters[CNT_CORR], &flag)) {
    double zs = 0.0, om = 0.0;
    int nz = 0;
    for (int b = threadIdx.x; b < static_cast<int>(gridDim.x); b += BLK) {
      zs = fmax(zs, a.bp0[b]);
      om += a.bp1[b];
      nz += a.bpi[b];
    }
    zs = block_max<double, NW>(zs, sd);
    om = block_sum<double, NW>(om, sd);
    nz = block_sum<int, NW>(nz, si);
    if (threadIdx.x == 0) {
      const int t = st->iter;  // index of this iteration's record
      scalar_update(st, a.N, a.test, zs, om, nz, l_new);
      if (a.tele != nullptr && t < a.tele_cap) {
        TeleRec* rec = static_cast<TeleRec*>(a.tele) + t;
        rec->n_atoms = st->n_active_atoms;
        rec->n_units = n;
        rec->n_support = st->n_support;
        rec->nnz = nz;
        rec->r = st->r_last;
        rec->gap = st->gap;
      }
      a.counters[CNT_CORR] = 0u;
    }
  }
}

// Correlation over the active groups with the fused Group-Lasso epilogue: one wave per
// group, the group's v = p - z / L kept in registers (lane k % 64 holds atom k).
template <typename T, typename V, typename A, bool VECTOR, int RULE>
__global__ __launch_bounds__(BLK) void k_corr_group(SingleArgs<T, V, A> a) {
  __shared__ double sd[NW];
  __shared__ int si[NW];
  __shared__ int flag;
  SolverState* st = a.st;
  if (st->done) return;
  const int n = st->n_active;
  const int32_t* __restrict__ act = a.act[st->cur];
  const double lam = st->lam, L = st->L;
  const A invL = static_cast<A>(1.0 / L);
  const double thr = lam / L;
  const double l_prev = st->l_prev;
  double l_new = l_prev;
  A beta = A(0);
  if (RULE == RULE_FISTA) {
    l_new = 0.5 * (1.0 + sqrt(1.0 + 4.0 * l_prev * l_prev));
    beta = static_cast<A>((l_prev - 1.0) / l_new);
  }
  const double thn = sqrt(st->tt);
  const double gz = st->gamma_z * thn;
  const int lane = threadIdx.x % WAVE;
  const int gw = blockIdx.x * NW + threadIdx.x / WAVE;
  const int nwaves = gridDim.x * NW;
  double zsup = 0.0, omega = 0.0;
  int nnz = 0;
  for (int j = gw; j < n; j += nwaves) {
    const int g = act[j];
    const int64_t a0 = a.gptr[g];
    const int m = static_cast<int>(a.gptr[g + 1] - a0);
    A vreg[GMAX_REG];
    A preg[GMAX_REG];
    double z2 = 0.0, p2 = 0.0, v2 = 0.0;
#pragma unroll
    for (int k = 0; k < GMAX_REG; ++k) { vreg[k] = A(0); preg[k] = A(0); }
    for (int base = 0; base < m; base += CPW) {
      const int nc = min(CPW, m - base);
      const T* cols[CPW];
#pragma unroll
      for (int c = 0; c < CPW; ++c) cols[c] = a.D + (a0 + base + min(c, nc - 1)) * a.ldd;
      A acc[CPW];
      wave_dots<T, V, A, CPW, VECTOR>(cols, nc, a.theta, a.N, lane, acc);
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        acc[c] = wave_sum(acc[c]);
        if (c < nc) z2 += static_cast<double>(acc[c]) * static_cast<double>(acc[c]);
      }
      // lane (base + c) % 64 keeps atom base + c
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const int k = base + c;
        if (c < nc && (k % WAVE) == lane) {
          const A p = static_cast<A>(a.u[a0 + k]);
          const A vv = p - acc[c] * invL;
#pragma unroll
          for (int r = 0; r < GMAX_REG; ++r)
            if (k / WAVE == r) { vreg[r] = vv; preg[r] = p; }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < GMAX_REG; ++r) {
      v2 += static_cast<double>(vreg[r]) * static_cast<double>(vreg[r]);
      p2 += static_cast<double>(preg[r]) * static_cast<double>(preg[r]);
    }
    v2 = wave_sum(v2);
    p2 = wave_sum(p2);
    const double wg = a.w[g];
    const double nv = sqrt(v2);
    const double scale = nv > 0.0 ? fmax(0.0, (nv - thr * wg) / nv) : 0.0;
    const A sc = static_cast<A>(scale);
    int gnz = 0;
#pragma unroll
    for (int r = 0; r < GMAX_REG; ++r) {
      const int k = r * WAVE + lane;
      if (k < m) {
        const int64_t i = a0 + k;
        const A xo = static_cast<A>(a.x[i]);
        const A xn = sc * vreg[r];
        const A un = RULE == RULE_FISTA ? xn + beta * (xn - xo) : xn;
        a.x[i] = static_cast<V>(xn);
        a.u[i] = static_cast<V>(un);
        gnz += xn != A(0) ? 1 : 0;
      }
    }
    gnz = wave_sum(gnz);
    if (lane == 0) {
      // rounding-safe bound of ||D_g^T theta|| / w_g
      zsup = fmax(zsup, (sqrt(z2) + gz * a.fro[g]) / wg);
      omega += wg * sqrt(p2);
      nnz += gnz;
    }
  }
  zsup = block_max<double, NW>(zsup, sd);
  omega = block_sum<double, NW>(omega, sd);
  nnz = block_sum<int, NW>(nnz, si);
  if (threadIdx.x == 0) {
    a.bp0[blockIdx.x] = zsup;
    a.bp1[blockIdx.x] = omega;
    a.bpi[blockIdx.x] = nnz;
  }
  if (last_block_arrive(&a.counters[CNT_CORR], &flag)) {
    double zs = 0.0, om = 0.0;
    int nz = 0;
    for (int b = threadIdx.x; b < static_cast<int>(gridDim.x); b += BLK) {
      zs = fmax(zs, a.bp0[b]);
      om += a.bp1[b];
      nz += a.bpi[b];
    }
    zs = block_max<double, NW>(zs, sd);
    om = block_sum<double, NW>(om, sd);
    nz = block_sum<int, NW>(nz, si);
    if (threadIdx.x == 0) {
      const int t = st->iter;  // index of this iteration's record
      scalar_update(st, a.N, a.test, zs, om, nz, l_new);
      if (a.tele != nullptr && t < a.tele_cap) {
        TeleRec* rec = static_cast<TeleRec*>(a.tele) + t;
        rec->n_atoms = st->n_active_atoms;
        rec->n_units = n;
        rec->n_support = st->n_support;
        rec->nnz = nz;
        rec->r = st->r_last;
        rec->gap = st->gap;
      }
      a.counters[CNT_CORR] = 0u;
    }
  }
}

// Order-preserving compaction of the active units against the margins (screened iff
// m > r_scr + slack, the strict test of the lemmas), and the support list of the new
// primal point.  One block; thread t handles a contiguous run of units.
template <typename T, typename V, typename A>
__global__ __launch_bounds__(CBLK) void k_compact(SingleArgs<T, V, A> a) {
  __shared__ int sc[CNW];
  SolverState* st = a.st;
  if (st->done) return;
  const int n = st->n_active;
  const int cur = st->cur;
  const int32_t* __restrict__ in = a.act[cur];
  int32_t* __restrict__ out = a.act[1 - cur];
  const double thr = st->r_scr + st->marg_slack;
  const int R = (n + CBLK - 1) / CBLK;
  const int lo = min(static_cast<int>(threadIdx.x) * R, n), hi = min(lo + R, n);
  int keep = 0, sup = 0, atoms = 0;
  for (int j = lo; j < hi; ++j) {
    const int unit = in[j];
    if (!(a.marg[unit] > thr)) {
      ++keep;
      const int64_t b = a.G > 0 ? a.gptr[unit] : unit;
      const int64_t e = a.G > 0 ? a.gptr[unit + 1] : unit + 1;
      atoms += static_cast<int>(e - b);
      for (int64_t i = b; i < e; ++i) sup += a.u[i] != V(0) ? 1 : 0;
    }
  }
  int tk, ts, ta;
  int pk = block_exclusive_scan<CNW>(keep, sc, &tk);
  int ps = block_exclusive_scan<CNW>(sup, sc, &ts);
  block_exclusive_scan<CNW>(atoms, sc, &ta);
  for (int j = lo; j < hi; ++j) {
    const int unit = in[j];
    if (!(a.marg[unit] > thr)) {
      out[pk++] = unit;
      const int64_t b = a.G > 0 ? a.gptr[unit] : unit;
      const int64_t e = a.G > 0 ? a.gptr[unit + 1] : unit + 1;
      for (int64_t i = b; i < e; ++i) {
        const V uv = a.u[i];
        if (uv != V(0)) {
          a.s_idx[ps] = static_cast<int32_t>(i);
          a.s_val[ps] = uv;
          ++ps;
        }
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    st->n_active = tk;
    st->n_support = ts;
    st->n_active_atoms = ta;
    st->cur = 1 - cur;
  }
}

// Output: X = 0 outside the active units, x on them.
template <typename T, typename V, typename A>
__global__ __launch_bounds__(BLK) void k_zero_out(V* __restrict__ X, int K) {
  const int i = blockIdx.x * BLK + threadIdx.x;
  if (i < K) X[i] = V(0);
}
template <typename T, typename V, typename A>
__global__ __launch_bounds__(BLK) void k_scatter_out(SingleArgs<T, V, A> a, V* __restrict__ X) {
  const SolverState* st = a.st;
  const int j = blockIdx.x * BLK + threadIdx.x;
  if (st->status != 0 || j >= st->n_active) return;
  const int unit = a.act[st->cur][j];
  if (a.G > 0) {
    for (int64_t i = a.gptr[unit]; i < a.gptr[unit + 1]; ++i) X[i] = a.x[i];
  } else {
    X[unit] = a.x[unit];
  }
}

__global__ void k_fill_u8(uint8_t* __restrict__ p, int n, uint8_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
// Screened mask: 0 on the atoms of the active units (run after k_fill_u8(.., 1)).
template <typename T, typename V, typename A>
__global__ __launch_bounds__(BLK) void k_mark_active(SingleArgs<T, V, A> a, uint8_t* __restrict__ m) {
  const SolverState* st = a.st;
  const int j = blockIdx.x * BLK + threadIdx.x;
  if (st->status != 0 || j >= st->n_active) return;
  const int unit = a.act[st->cur][j];
  if (a.G > 0) {
    for (int64_t i = a.gptr[unit]; i < a.gptr[unit + 1]; ++i) m[i] = 0;
  } else {
    m[unit] = 0;
  }
}

// ============================================================== power iteration =====

// w = D v over all K columns: partial sums over column chunks of PCH, FP64.
constexpr int PCH = 64;
template <typename T>
__global__ __launch_bounds__(BLK) void k_pow_dv(const T* __restrict__ D, int64_t ldd, int N,
                                                 int K, const double* __restrict__ v,
                                                 double* __restrict__ part, int64_t npad) {
  const int nrt = (N + BLK - 1) / BLK;
  const int nch = (K + PCH - 1) / PCH;
  for (int item = blockIdx.x; item < nrt * nch; item += gridDim.x) {
    const int rt = item % nrt, c = item / nrt;
    const int r = rt * BLK + threadIdx.x;
    if (r >= N) continue;
    double s = 0.0;
    const int k1 = min((c + 1) * PCH, K);
    for (int k = c * PCH; k < k1; ++k) s = fma(to_double(D[static_cast<int64_t>(k) * ldd + r]), v[k], s);
    part[static_cast<int64_t>(c) * npad + r] = s;
  }
}
__global__ __launch_bounds__(BLK) void k_pow_reduce(const double* __restrict__ part, int nch,
                                                     int64_t npad, int N, double* __restrict__ w) {
  const int r = blockIdx.x * BLK + threadIdx.x;
  if (r >= N) return;
  double s = 0.0;
  for (int c = 0; c < nch; ++c) s += part[static_cast<int64_t>(c) * npad + r];
  w[r] = s;
}
// out = [sum a_i^2, sum a_i b_i, sum b_i^2] over n (single block, FP64).
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
__global__ void k_fill(double* __restrict__ v, int n, double val) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = val;
}

}  // namespace ds
