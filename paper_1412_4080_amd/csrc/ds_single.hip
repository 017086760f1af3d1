// Single-signal solve: setup on the device, then chunks of iterations enqueued ahead of
// the device-side stopping decision (see ds_single_kernels.h for the kernels).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "ds_engine.h"
#include "ds_single_kernels.h"

static_assert(ds::GMAX == DS_GROUP_MAX, "group limit of the kernels and of the validation");

namespace ds {

namespace {

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

struct Layout {
  size_t off_state, off_act0, off_act1, off_actm0, off_actm1, off_x, off_u, off_theta, off_y,
      off_partial, off_z0, off_g, off_nu, off_fro, off_gnorm, off_marg, off_nvec, off_segcnt,
      off_segatom, off_segval, off_urm, off_uro, off_urn, off_bp0, off_bpi, off_rtn, off_omp,
      off_rtcnt, off_lba, off_cnt, off_gptr, off_w, off_tele, off_kclk, off_spans, off_pv, off_pw,
      off_pz, off_pd, off_segxo, off_segpo, off_segd, off_uromo, off_urdn, off_bpd, off_dtn, off_rtr, total;
  int64_t npad, grid_corr, nsg;
};

// Correlation grid and residual segment groups for a problem shape.
inline int64_t corr_blocks(int64_t K, int64_t G) {
  return G > 0 ? (G + CBG - 1) / CBG : (K + CBL - 1) / CBL;
}

Layout make_layout(int64_t N, int64_t K, int64_t G, size_t vsz, size_t asz, int64_t tele_cap,
                   bool power) {
  Layout l{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += static_cast<size_t>(round_up(static_cast<int64_t>(std::max<size_t>(bytes, 8)), 256));
    return at;
  };
  l.npad = round_up(N, 64);
  l.grid_corr = corr_blocks(K, G);
  const int64_t segcap = G > 0 ? SEGCAP_G : SEGCAP_L, ucap = G > 0 ? CBG : CBL;
  l.nsg = (l.grid_corr + (G > 0 ? SGG : SGL) - 1) / (G > 0 ? SGG : SGL);
  const int64_t units = G > 0 ? G : K;
  l.off_state = take(2 * sizeof(SolverState));
  l.off_act0 = take(units * 4);
  l.off_act1 = take(units * 4);
  l.off_actm0 = take(units * 8);
  l.off_actm1 = take(units * 8);
  l.off_x = take(K * vsz);
  l.off_u = take(K * vsz);
  l.off_theta = take(l.npad * vsz);
  l.off_y = take(l.npad * vsz);
  l.off_partial = take(l.nsg * l.npad * asz);
  l.off_z0 = take(K * 8);
  l.off_g = take(K * 8);
  l.off_nu = take(K * 8);
  l.off_fro = take(std::max<int64_t>(G, 1) * 8);
  l.off_gnorm = take(std::max<int64_t>(G, 1) * 8);
  l.off_marg = take(units * 8);
  l.off_nvec = take(l.npad * 8);
  l.off_segcnt = take(l.grid_corr * 4);
  l.off_segatom = take(l.grid_corr * segcap * 4);
  l.off_segval = take(l.grid_corr * segcap * vsz);
  l.off_urm = take(l.grid_corr * ucap * 8);
  l.off_uro = take(l.grid_corr * ucap * 8);
  l.off_urn = take(l.grid_corr * ucap * 4);
  l.off_bp0 = take(MAXB * 8);
  l.off_bpi = take(4 * MAXB * 4);
  l.off_segxo = take(l.grid_corr * segcap * vsz);
  l.off_segpo = take(l.grid_corr * segcap * vsz);
  l.off_segd = take(l.grid_corr * segcap * 8);
  l.off_uromo = take(l.grid_corr * ucap * 8);
  l.off_urdn = take(l.grid_corr * ucap * 8);
  l.off_bpd = take(2 * MAXB * 8);  // ||d||^2, then the SpaRSA partials
  l.off_rtr = take(2 * MAXRT * 8);  // Chambolle-Pock ||D u - y||^2 per row tile
  l.off_dtn = take(MAXRT * 8);
  l.off_rtn = take(2 * 2 * MAXRT * 8);
  l.off_omp = take(2 * MAXITEM * 8);
  l.off_rtcnt = take(MAXRT * 4);
  l.off_lba = take(MAXB * 8);
  l.off_cnt = take(32 * 4);
  l.off_gptr = take((std::max<int64_t>(G, 1) + 1) * 8);
  l.off_w = take(std::max<int64_t>(G, 1) * 8);
  l.off_tele = take(tele_cap * sizeof(Telemetry));
  l.off_kclk = take(2 * l.grid_corr * 8);
  l.off_spans = take((tele_cap + 1) * 8);
  if (power) {
    l.off_pv = take(K * 8);
    l.off_pz = take(K * 8);
    l.off_pw = take(l.npad * 8);
    l.off_pd = take(((K + PCH - 1) / PCH) * l.npad * 8 + 64);
  }
  l.total = o;
  return l;
}

template <typename T> struct Types { using V = typename Store<T>::V; using A = typename Store<T>::A; };

template <typename T>
bool vector_ok(const void* D, int64_t ldd) {
  return (reinterpret_cast<uintptr_t>(D) % 16 == 0) && ((ldd * sizeof(T)) % 16 == 0);
}

template <typename T>
SingleArgs<T, typename Types<T>::V, typename Types<T>::A> make_args(const ds_problem& P,
                                                                    const void* y, char* base,
                                                                    const Layout& l, int test,
                                                                    int rule) {
  using V = typename Types<T>::V;
  using A = typename Types<T>::A;
  SingleArgs<T, V, A> a{};
  a.D = static_cast<const T*>(P.D);
  a.ldd = P.ldd;
  a.N = static_cast<int32_t>(P.N);
  a.K = static_cast<int32_t>(P.K);
  a.G = static_cast<int32_t>(P.G);
  a.test = test;
  a.rule = rule;
  a.par = 0;
  a.grid_corr = static_cast<int32_t>(l.grid_corr);
  a.nsg_prev = static_cast<int32_t>(l.nsg);
  a.gptr = P.G > 0 ? reinterpret_cast<const int64_t*>(base + l.off_gptr) : nullptr;
  a.w = P.G > 0 ? reinterpret_cast<const double*>(base + l.off_w) : nullptr;
  a.y = reinterpret_cast<const V*>(base + l.off_y);
  (void)y;
  a.st = reinterpret_cast<SolverState*>(base + l.off_state);
  a.act[0] = reinterpret_cast<int32_t*>(base + l.off_act0);
  a.act[1] = reinterpret_cast<int32_t*>(base + l.off_act1);
  a.act_m[0] = reinterpret_cast<double*>(base + l.off_actm0);
  a.act_m[1] = reinterpret_cast<double*>(base + l.off_actm1);
  a.x = reinterpret_cast<V*>(base + l.off_x);
  a.u = reinterpret_cast<V*>(base + l.off_u);
  a.theta = reinterpret_cast<V*>(base + l.off_theta);
  a.partial = reinterpret_cast<A*>(base + l.off_partial);
  a.npad = l.npad;
  a.z0 = reinterpret_cast<double*>(base + l.off_z0);
  a.g = reinterpret_cast<double*>(base + l.off_g);
  a.nu = reinterpret_cast<double*>(base + l.off_nu);
  a.fro = reinterpret_cast<double*>(base + l.off_fro);
  a.gnorm = reinterpret_cast<double*>(base + l.off_gnorm);
  a.marg = reinterpret_cast<double*>(base + l.off_marg);
  a.nvec = reinterpret_cast<double*>(base + l.off_nvec);
  a.seg_cnt = reinterpret_cast<int32_t*>(base + l.off_segcnt);
  a.seg_atom = reinterpret_cast<int32_t*>(base + l.off_segatom);
  a.seg_val = reinterpret_cast<V*>(base + l.off_segval);
  a.urec_marg = reinterpret_cast<double*>(base + l.off_urm);
  a.urec_om = reinterpret_cast<double*>(base + l.off_uro);
  a.urec_m = reinterpret_cast<int32_t*>(base + l.off_urn);
  a.bp0 = reinterpret_cast<double*>(base + l.off_bp0);
  a.bpi = reinterpret_cast<int32_t*>(base + l.off_bpi);
  a.seg_xo = reinterpret_cast<V*>(base + l.off_segxo);
  a.seg_po = reinterpret_cast<V*>(base + l.off_segpo);
  a.seg_d = reinterpret_cast<double*>(base + l.off_segd);
  a.urec_omo = reinterpret_cast<double*>(base + l.off_uromo);
  a.urec_dn = reinterpret_cast<double*>(base + l.off_urdn);
  a.bpd = reinterpret_cast<double*>(base + l.off_bpd);
  a.bpe = a.bpd + MAXB;
  a.rtr = reinterpret_cast<double*>(base + l.off_rtr);
  a.dtn = reinterpret_cast<double*>(base + l.off_dtn);
  a.rtn = reinterpret_cast<double*>(base + l.off_rtn);
  a.omp = reinterpret_cast<double*>(base + l.off_omp);
  a.rt_cnt = reinterpret_cast<unsigned*>(base + l.off_rtcnt);
  a.lbA = reinterpret_cast<uint64_t*>(base + l.off_lba);
  a.counters = reinterpret_cast<unsigned*>(base + l.off_cnt);
  return a;
}

inline int grid_for(int64_t work, int per_block, int cap) {
  const int64_t g = (work + per_block - 1) / per_block;
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(g, cap)));
}

// Upload group offsets and weights into the workspace (default w_g = sqrt(|g|), formed on
// the device).  The copies read the caller's host arrays, which outlive the call.
ds_status upload_groups(const ds_problem& P, char* base, const Layout& l, hipStream_t s) {
  if (P.G <= 0) return DS_OK;
  DS_HIP(hipMemcpyAsync(base + l.off_gptr, P.group_ptr, (P.G + 1) * 8, hipMemcpyHostToDevice, s));
  if (P.w != nullptr) {
    DS_HIP(hipMemcpyAsync(base + l.off_w, P.w, P.G * 8, hipMemcpyHostToDevice, s));
  } else {
    hipLaunchKernelGGL(k_default_weights, dim3(grid_for(P.G, BLK, 1 << 20)), dim3(BLK), 0, s,
                       reinterpret_cast<const int64_t*>(base + l.off_gptr), static_cast<int>(P.G),
                       reinterpret_cast<double*>(base + l.off_w));
    DS_HIP(hipGetLastError());
  }
  return DS_OK;
}

// Several word ranges cleared by one launch (a fill kernel, not a memset: no memset node
// if the caller captures the stream).
struct ZeroRanges {
  static constexpr int MAX = 8;
  uint32_t* p[MAX];
  int64_t n[MAX];
  int count;
};
__global__ __launch_bounds__(BLK) void k_zero_ranges(ZeroRanges r) {
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * BLK + threadIdx.x;
  const int64_t step = static_cast<int64_t>(gridDim.x) * BLK;
  for (int k = 0; k < r.count; ++k)
    for (int64_t i = i0; i < r.n[k]; i += step) r.p[k][i] = 0u;
}


// Setup passes shared by lambda_max and the solve: z0 = D^T y, atom norms, group norms.
template <typename T, bool VEC>
ds_status launch_setup_corr(const ds_problem& P, const void* y, char* base, const Layout& l,
                            hipStream_t s) {
  using V = typename Types<T>::V;
  V* yc = reinterpret_cast<V*>(base + l.off_y);
  hipLaunchKernelGGL((k_copy_y<V>), dim3(grid_for(l.npad, BLK, 1 << 20)), dim3(BLK), 0, s,
                     static_cast<const V*>(y), yc, static_cast<int>(P.N),
                     static_cast<int>(l.npad));
  const int gridK = grid_for(P.K, NW * CPW, 4096);
  hipLaunchKernelGGL((k_setup_gemv<T, V, VEC, true>), dim3(gridK), dim3(BLK), 0, s,
                     static_cast<const T*>(P.D), P.ldd, static_cast<int>(P.N),
                     static_cast<int>(P.K), static_cast<const V*>(yc),
                     reinterpret_cast<double*>(base + l.off_z0),
                     reinterpret_cast<double*>(base + l.off_nu));
  DS_HIP(hipGetLastError());
  if (P.G > 0) {
    int64_t mmax = 1;  // largest group (validated: at most GMAX atoms)
    for (int64_t g = 0; g < P.G; ++g) mmax = std::max(mmax, P.group_ptr[g + 1] - P.group_ptr[g]);
    auto launch = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(grid_for(P.G, 1, 4096)), dim3(BLK), 0, s,
                         static_cast<const T*>(P.D), P.ldd, static_cast<int>(P.N),
                         static_cast<int>(P.G),
                         reinterpret_cast<const int64_t*>(base + l.off_gptr),
                         reinterpret_cast<double*>(base + l.off_gnorm),
                         reinterpret_cast<double*>(base + l.off_fro));
    };
    switch (gram_edge(static_cast<int>(mmax))) {
      case 16: launch(k_group_norms<T, 16>); break;
      case 32: launch(k_group_norms<T, 32>); break;
      case 64: launch(k_group_norms<T, 64>); break;
      default: launch(k_group_norms<T, 128>); break;
    }
    DS_HIP(hipGetLastError());
  }
  return DS_OK;
}

}  // namespace

// Spectral and Frobenius norms of contiguous groups of a bfloat16 dictionary (the batched
// path's padded copy), with the single-signal path's kernel.
ds_status group_norms_bf16(const uint16_t* D, int64_t ldd, int N, int G, const int64_t* gptr_dev,
                           int max_group, double* gnorm, double* fro, hipStream_t s) {
  auto launch = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(grid_for(G, 1, 4096)), dim3(BLK), 0, s, D, ldd, N, G, gptr_dev,
                       gnorm, fro);
  };
  switch (gram_edge(max_group)) {
    case 16: launch(k_group_norms<bf16_t, 16>); break;
    case 32: launch(k_group_norms<bf16_t, 32>); break;
    case 64: launch(k_group_norms<bf16_t, 64>); break;
    default: launch(k_group_norms<bf16_t, 128>); break;
  }
  DS_HIP(hipGetLastError());
  return DS_OK;
}

namespace {

template <typename T, bool VEC, int RULE>
ds_status run_single(const ds_problem& P, const void* y, double lam, const ds_params& prm,
                     void* x, ds_info* info, hipStream_t s, Workspace& ws,
                     std::vector<Telemetry>* tele_out, uint8_t* screened) {
  using V = typename Types<T>::V;
  using A = typename Types<T>::A;
  ds_status st_ = single_shape_check(P.dtype, P.N, P.K, P.G, VEC);
  if (st_ != DS_OK) return st_;
  const int64_t tele_cap = std::max<int32_t>(prm.max_iter, 1);
  const Layout l = make_layout(P.N, P.K, P.G, sizeof(V), sizeof(A), tele_cap, false);
  if ((st_ = ws.reserve(l.total)) != DS_OK) return st_;
  char* base = static_cast<char*>(ws.base);
  const int test = static_cast<int>(prm.test), rule = RULE;
  SingleArgs<T, V, A> a = make_args<T>(P, y, base, l, test, rule);
  Telemetry* tele = reinterpret_cast<Telemetry*>(base + l.off_tele);
  a.tele = tele;
  a.tele_cap = static_cast<int32_t>(tele_cap);
  a.screen_static = prm.screening;
  if ((st_ = upload_groups(P, base, l, s)) != DS_OK) return st_;
  {
    // counters, arrival counts, look-back words; the backtracking and Chambolle-Pock
    // partials (read by the residual pass before a correlation pass writes them)
    ZeroRanges zr{};
    auto add = [&](void* ptr, size_t bytes) {
      zr.p[zr.count] = static_cast<uint32_t*>(ptr);
      zr.n[zr.count] = static_cast<int64_t>(bytes / 4);
      ++zr.count;
    };
    add(a.counters, 32 * 4);
    add(a.rt_cnt, MAXRT * 4);
    add(a.lbA, MAXB * 8);
    add(a.bpd, 2 * MAXB * 8);
    add(a.rtr, 2 * MAXRT * 8);
    add(a.dtn, MAXRT * 8);
    hipLaunchKernelGGL(k_zero_ranges, dim3(64), dim3(BLK), 0, s, zr);
    DS_HIP(hipGetLastError());
  }

  // ---- setup (no host synchronisation) ----
  if ((st_ = launch_setup_corr<T, VEC>(P, y, base, l, s)) != DS_OK) return st_;
  // L: given, or estimated here (slow path); backtracking and SpaRSA start from step_L
  // when given, else from a bound the setup kernel computes on the device.  Both use the
  // step check and undo machinery (a.bt).
  // Chambolle-Pock uses the slot copies too (to return the certified point at the stop),
  // but no step check
  const bool line_search = prm.step_rule == DS_STEP_BACKTRACK || RULE == RULE_SPARSA;
  const bool bt = line_search || RULE == RULE_CP;
  const double eta = line_search ? (prm.bt_eta > 0.0 ? prm.bt_eta : 2.0) : 0.0;
  a.bt = bt ? 1 : 0;
  double L = prm.step_L;
  if (!(L > 0.0) && !line_search) {
    if (ws.fixed) {  // the estimate would need a workspace of its own
      set_error("the step constant must be given (step_L > 0) on this entry point");
      return DS_EINVAL;
    }
    // the power iteration uses its own (larger) workspace; keep ours intact by running it
    // on a private one
    Workspace tmp;
    tmp.device = ws.device;
    ds_status e = spectral_norm_impl(P, 0, &L, s, tmp);
    (void)hipStreamSynchronize(s);
    tmp.release();
    if (e != DS_OK) return e;
  }
  // Chambolle-Pock steps: tau_0 sigma_0 L = 1 by default
  const double cp_tau = prm.cp_tau > 0.0 ? prm.cp_tau : (L > 0.0 ? 1.0 / std::sqrt(L) : 1.0);
  const double cp_sigma = prm.cp_sigma > 0.0 ? prm.cp_sigma : (L > 0.0 ? 1.0 / (cp_tau * L) : 1.0);
  const double u_round = sizeof(A) == 4 ? 0x1p-24 : 0x1p-53;
  const double kchain = std::ceil(static_cast<double>(P.N) / WAVE) + Store<T>::VEC + 8;
  const double gamma_z = kchain * u_round / (1.0 - kchain * u_round);
  const bool relative = prm.lambda_mode == DS_LAMBDA_RELATIVE;
  hipLaunchKernelGGL((k_setup_scalars<T, V, A>), dim3(1), dim3(CBLK), 0, s, a, lam,
                     relative ? 1 : 0, L, prm.gap_tol, prm.max_iter, gamma_z, eta,
                     RULE == RULE_SPARSA ? prm.bb_memory : 0,
                     prm.bb_sigma > 0.0 ? prm.bb_sigma : 1e-5, cp_tau, cp_sigma, prm.cp_gamma,
                     prm.x0 != nullptr ? 1 : 0, prm.obj_tol);
  DS_HIP(hipGetLastError());
  if (prm.test == DS_TEST_DST3 || prm.test == DS_TEST_DOME) {
    hipLaunchKernelGGL((k_setup_normal<T, V, A>), dim3(grid_for(P.N, BLK, 1 << 20)), dim3(BLK),
                       0, s, a);
    DS_HIP(hipGetLastError());
    hipLaunchKernelGGL((k_setup_gemv<T, double, VEC, false>),
                       dim3(grid_for(P.K, NW * CPW, 4096)), dim3(BLK), 0, s, a.D, a.ldd, a.N,
                       a.K, static_cast<const double*>(a.nvec), a.g, nullptr);
    DS_HIP(hipGetLastError());
  }
  const int64_t units = P.G > 0 ? P.G : P.K;
  hipLaunchKernelGGL((k_setup_margins<T, V, A>), dim3(grid_for(std::max(units, P.K), BLK, 1 << 20)),
                     dim3(BLK), 0, s, a);
  DS_HIP(hipGetLastError());
  hipLaunchKernelGGL((k_setup_slack<T, V, A>), dim3(1), dim3(CBLK), 0, s, a);
  DS_HIP(hipGetLastError());
  if (prm.x0 != nullptr) {  // warm start: x_0 = u_0 = x0 and its support records
    hipLaunchKernelGGL((k_warm_seed<T, V, A>), dim3(grid_for(units, BLK, 1 << 20)), dim3(BLK), 0, s,
                       a, static_cast<const V*>(prm.x0));
    DS_HIP(hipGetLastError());
  }

  // ---- iterations ----
  constexpr int VR = VEC ? Store<T>::VEC : 1;
  const int nrt = static_cast<int>((P.N + WAVE * VR - 1) / (WAVE * VR));
  // The correlation grid covers the active list; the list never grows, so at each chunk
  // boundary the host shrinks the grid to the list length it reads from the state.  Each
  // residual pass reads the outputs of the correlation launch before it (its grid) and the
  // Omega partials of the residual pass before it (the segment groups of that pass).
  const int cbu = P.G > 0 ? CBG : CBL, sgu = P.G > 0 ? SGG : SGL;
  auto nsg_of = [&](int g) { return (g + sgu - 1) / sgu; };
  auto res_grid = [&](int g) {
    return std::max(nrt, grid_for(static_cast<int64_t>(nrt) * nsg_of(g), 1, 2048));
  };
  int grid_corr = static_cast<int>(l.grid_corr);  // correlation launches of this chunk
  int grid_res_read = grid_corr;                  // grid the last residual pass read
  StatAccum& S = stats();
  bool stat_on;
  {
    std::lock_guard<std::mutex> g(S.mu);
    stat_on = S.on && !ws.fixed;  // a fixed workspace creates no events
  }
  SolverState* hst = static_cast<SolverState*>(ws.host_pinned);
  // instrumented runs: each correlation block stamps the device wall clock at its start
  // and end; a one-block pass after the launch reduces the stamps to its span
  uint64_t* spans = reinterpret_cast<uint64_t*>(base + l.off_spans);
  int64_t nspan = 0;
  if (stat_on) a.kclk = reinterpret_cast<uint64_t*>(base + l.off_kclk);
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  size_t ev_used = 0;
  auto get_events = [&]() -> std::pair<hipEvent_t, hipEvent_t> {
    while (ws.events.size() < 2 * (ev_used + 1)) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return {nullptr, nullptr};
      ws.events.push_back(e);
    }
    auto p = std::make_pair(ws.events[2 * ev_used], ws.events[2 * ev_used + 1]);
    ++ev_used;
    return p;
  };
  // g: the grid of the correlation launch whose outputs the pass reads
  std::vector<std::pair<hipEvent_t, hipEvent_t>> evr;  // instrumented residual passes
  auto launch_resid = [&](int par, int g) {
    a.par = par;
    a.grid_corr = g;
    a.nsg_prev = nsg_of(grid_res_read);
    grid_res_read = g;
    std::pair<hipEvent_t, hipEvent_t> e{nullptr, nullptr};
    if (stat_on) e = get_events();
    if (P.G > 0)
      hipExtLaunchKernelGGL((k_resid<T, V, VEC, RULE, true>), dim3(res_grid(g)), dim3(BLK), 0, s,
                            e.first, e.second, 0, a);
    else
      hipExtLaunchKernelGGL((k_resid<T, V, VEC, RULE, false>), dim3(res_grid(g)), dim3(BLK), 0, s,
                            e.first, e.second, 0, a);
    if (stat_on && e.first) evr.push_back(e);
  };
  auto launch_dcheck = [&](int par, int g) {
    a.par = par;
    a.grid_corr = g;
    if (P.G > 0)
      hipLaunchKernelGGL((k_dcheck<T, V, VEC, true>), dim3(res_grid(g)), dim3(BLK), 0, s, a);
    else
      hipLaunchKernelGGL((k_dcheck<T, V, VEC, false>), dim3(res_grid(g)), dim3(BLK), 0, s, a);
  };
  auto launch_corr = [&](int par) {
    a.par = par;
    // instrumented launches carry start/stop events in the dispatch itself, so the
    // measured interval is the kernel's own execution
    std::pair<hipEvent_t, hipEvent_t> e{nullptr, nullptr};
    if (stat_on) e = get_events();
    if (P.G > 0)
      hipExtLaunchKernelGGL((k_corr<T, V, VEC, RULE, true>), dim3(grid_corr), dim3(BLK), 0, s,
                            e.first, e.second, 0, a);
    else
      hipExtLaunchKernelGGL((k_corr<T, V, VEC, RULE, false>), dim3(grid_corr), dim3(BLK), 0, s,
                            e.first, e.second, 0, a);
    if (stat_on && e.first) ev.push_back(e);
    if (stat_on && nspan < tele_cap) {
      hipLaunchKernelGGL(k_clock_span<0>, dim3(1), dim3(256), 0, s, a.kclk, grid_corr, spans + nspan);
      ++nspan;
    }
  };

  // iteration t: corr(t) with parity t%2, then resid(t+1) (scalars of t, theta_{t+1});
  // resid(1) forms theta_1 = -y.
  launch_resid(1, grid_corr);  // a warm start seeds the segments of the full grid
  // Chunk sizes.  Iterations enqueued past the stop return at once but still cost a
  // launch each, and every chunk costs a host round trip.  A fixed iteration count is
  // enqueued whole (up to 64 at a time); a gap target takes the iterations the gap's
  // geometric trend over the last chunk predicts (plus a quarter), between 4 and 64;
  // instrumented runs take one iteration per chunk, so that no launch runs past the stop.
  int t = 0, chunk = stat_on ? 1 : 4, last_par = 1;
  int t_prev = 0;
  double gap_prev = 0.0;
  bool finished = false;
  while (!finished && t < prm.max_iter) {
    const int nrun = std::min(chunk, prm.max_iter - t);
    for (int k = 0; k < nrun; ++k) {
      ++t;
      launch_corr(t % 2);
      if (line_search) launch_dcheck(t % 2, grid_corr);
      launch_resid((t + 1) % 2, grid_corr);
      last_par = (t + 1) % 2;
    }
    DS_HIP(hipGetLastError());
    DS_HIP(hipMemcpyAsync(hst, a.st + last_par, sizeof(SolverState), hipMemcpyDeviceToHost, s));
    DS_HIP(hipStreamSynchronize(s));
    finished = hst->done != 0;
    grid_corr = std::min(grid_corr, std::max(1, (hst->n_active + cbu - 1) / cbu));
    if (stat_on) {
      chunk = 1;
    } else if (prm.gap_tol <= 0.0 && prm.obj_tol <= 0.0) {
      chunk = 64;
    } else {
      int next = std::min(chunk * 2, 64);
      const double gap = hst->gap, tol = hst->gap_tol_abs;
      if (prm.obj_tol <= 0.0 && t_prev > 0 && gap > tol && gap < gap_prev && tol > 0.0) {
        const double rate = std::log(gap / gap_prev) / static_cast<double>(t - t_prev);
        const double need = std::log(tol / gap) / rate;  // iterations to the target
        if (need > 0.0 && need < 1e6) next = static_cast<int>(std::ceil(1.25 * need)) + 2;
      }
      chunk = std::max(4, std::min(next, 64));
      t_prev = t;
      gap_prev = gap;
    }
  }
  a.par = last_par;

  // ---- output ----
  V* X = static_cast<V*>(x);
  hipLaunchKernelGGL((k_zero_out<T, V, A>), dim3(grid_for(P.K, BLK, 1 << 20)), dim3(BLK), 0, s, X,
                     static_cast<int>(P.K));
  hipLaunchKernelGGL((k_scatter_out<T, V, A>), dim3(grid_for(units, BLK, 1 << 20)), dim3(BLK), 0,
                     s, a, X);
  DS_HIP(hipGetLastError());
  if (screened != nullptr) {
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(P.K, BLK, 1 << 20)), dim3(BLK), 0, s, screened,
                       static_cast<int>(P.K), static_cast<uint8_t>(1));
    hipLaunchKernelGGL((k_mark_active<T, V, A>), dim3(grid_for(units, BLK, 1 << 20)), dim3(BLK), 0,
                       s, a, screened);
    DS_HIP(hipGetLastError());
  }
  DS_HIP(hipMemcpyAsync(hst, a.st + last_par, sizeof(SolverState), hipMemcpyDeviceToHost, s));
  DS_HIP(hipStreamSynchronize(s));

  const int iters_run = hst->iter;
  std::vector<Telemetry> tl;
  if ((stat_on || tele_out) && iters_run > 0) {
    tl.resize(std::min<int64_t>(iters_run, tele_cap));
    DS_HIP(hipMemcpy(tl.data(), tele, tl.size() * sizeof(Telemetry), hipMemcpyDeviceToHost));
  }
  if (stat_on && !ev.empty()) {
    // algorithmic bytes of one correlation launch: the active columns of D, theta, the
    // read-modify-write of x and u on the active atoms and the active list
    double ms = 0.0, ms_ev = 0.0, bytes = 0.0, flops = 0.0;
    const size_t used = std::min({ev.size(), tl.size(), static_cast<size_t>(nspan)});
    std::vector<uint64_t> ticks(used);
    std::vector<ds_launch_stat> recs(used);
    int rate_khz = 0;
    DS_HIP(hipMemcpy(ticks.data(), spans, used * sizeof(uint64_t), hipMemcpyDeviceToHost));
    DS_HIP(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, ws.device));
    // residual pass k + 1 follows correlation pass k (pass 0 forms theta_1 = -y); it
    // streams the support of the new primal point, recorded with iteration k + 1
    double r_ms = 0.0, r_bytes = 0.0;
    int64_t r_n = 0;
    for (size_t k = 0; k < used; ++k) {
      float f = 0.f;
      if (hipEventElapsedTime(&f, ev[k].first, ev[k].second) == hipSuccess) ms_ev += f;
      const double mk = rate_khz > 0 ? static_cast<double>(ticks[k]) / rate_khz : 0.0;
      ms += mk;
      const double na = tl[k].n_atoms, nu = tl[k].n_units;
      const double bk = na * P.N * sizeof(T) + P.N * sizeof(V) + 4.0 * na * sizeof(V) + 4.0 * nu;
      bytes += bk;
      flops += 2.0 * na * P.N;
      recs[k] = ds_launch_stat{DS_STAT_CORR, tl[k].n_atoms, bk, mk};
      float fr = 0.f;
      if (k + 1 < evr.size() &&
          hipEventElapsedTime(&fr, evr[k + 1].first, evr[k + 1].second) == hipSuccess) {
        const double ns = k + 1 < tl.size() ? tl[k + 1].n_support : 0.0;
        const double rb = ns * P.N * sizeof(T) + 2.0 * P.N * sizeof(V);
        recs.push_back(ds_launch_stat{DS_STAT_RESID, tl[k].n_atoms, rb, fr});
        recs.push_back(ds_launch_stat{DS_STAT_ITER, tl[k].n_atoms, 0.0, f + fr});
        r_ms += fr;
        r_bytes += rb;
        ++r_n;
      }
    }
    std::lock_guard<std::mutex> g(S.mu);
    for (const ds_launch_stat& r : recs)
      if (S.launches.size() < StatAccum::MAX_LAUNCHES) S.launches.push_back(r);
    S.s[DS_STAT_RESID].launches += r_n;
    S.s[DS_STAT_RESID].ms_event += r_ms;
    S.s[DS_STAT_RESID].bytes += r_bytes;
    S.s[DS_STAT_CORR].launches += static_cast<int64_t>(used);
    S.s[DS_STAT_CORR].ms += ms;
    S.s[DS_STAT_CORR].ms_event += ms_ev;
    S.s[DS_STAT_CORR].bytes += bytes;
    S.s[DS_STAT_CORR].flops += flops;
  }
  if (tele_out) *tele_out = std::move(tl);

  if (hst->status < 0) {
    set_error(prm.x0 != nullptr ? "observation or initial point contains NaN or Inf"
                                : "observation contains NaN or Inf");
    return DS_EINVAL;
  }
  info->iters = hst->iter;
  info->n_active = hst->status == 1 ? 0 : hst->n_active_atoms;
  info->nnz = hst->status == 1 ? 0 : hst->nnz;
  info->lambda = hst->lam;
  info->lambda_max = hst->lam_max;
  info->primal = hst->primal;
  info->dual = hst->dual;
  info->gap = hst->gap;
  info->radius = hst->r_min;
  info->mu = hst->mu;
  info->L = hst->L;
  info->radius_slack = hst->r_slack + hst->marg_slack;
  const bool converged = hst->status == 1 || hst->stop_obj != 0 || prm.gap_tol <= 0.0 ||
                         hst->gap <= hst->gap_tol_abs;
  info->status = converged ? DS_OK : DS_NOT_CONVERGED;
  return converged ? DS_OK : DS_NOT_CONVERGED;
}

template <typename T>
ds_status dispatch_rule(const ds_problem& P, const void* y, double lam, const ds_params& prm,
                        void* x, ds_info* info, hipStream_t s, Workspace& ws,
                        std::vector<Telemetry>* tele, uint8_t* scr) {
  const bool vec = vector_ok<T>(P.D, P.ldd);
  if (prm.rule == DS_FISTA)
    return vec ? run_single<T, true, RULE_FISTA>(P, y, lam, prm, x, info, s, ws, tele, scr)
               : run_single<T, false, RULE_FISTA>(P, y, lam, prm, x, info, s, ws, tele, scr);
  if (prm.rule == DS_SPARSA)
    return vec ? run_single<T, true, RULE_SPARSA>(P, y, lam, prm, x, info, s, ws, tele, scr)
               : run_single<T, false, RULE_SPARSA>(P, y, lam, prm, x, info, s, ws, tele, scr);
  if (prm.rule == DS_CP)
    return vec ? run_single<T, true, RULE_CP>(P, y, lam, prm, x, info, s, ws, tele, scr)
               : run_single<T, false, RULE_CP>(P, y, lam, prm, x, info, s, ws, tele, scr);
  return vec ? run_single<T, true, RULE_ISTA>(P, y, lam, prm, x, info, s, ws, tele, scr)
             : run_single<T, false, RULE_ISTA>(P, y, lam, prm, x, info, s, ws, tele, scr);
}

}  // namespace

size_t single_workspace_bytes(const ds_problem& P, const ds_params& prm) {
  const size_t vsz = P.dtype == DS_F64 ? 8 : 4;
  const int64_t tele_cap = std::max<int32_t>(prm.max_iter, 1);
  return make_layout(P.N, P.K, P.G, vsz, sizeof(double), tele_cap, false).total;
}

ds_status single_shape_check(int32_t dtype, int64_t N, int64_t K, int64_t G, bool vec) {
  const int64_t esz = dtype == DS_F64 ? 8 : dtype == DS_F32 ? 4 : 2;
  const int64_t rows = static_cast<int64_t>(WAVE) * (vec ? 16 / esz : 1);  // rows of a row tile
  const int64_t nrt = (N + rows - 1) / rows;
  const int64_t gc = corr_blocks(K, G);
  const int64_t nsg = (gc + (G > 0 ? SGG : SGL) - 1) / (G > 0 ? SGG : SGL);
  if (nrt > MAXRT || gc > MAXB || nsg > MAXITEM) {
    set_error("problem too large for one device solve: N <= %lld rows (%s), at most %lld %s",
              static_cast<long long>(MAXRT) * rows,
              vec ? "16-byte aligned D and ldd" : "unaligned D or ldd",
              static_cast<long long>(MAXB) * (G > 0 ? CBG : CBL), G > 0 ? "groups" : "atoms");
    return DS_EINVAL;
  }
  return DS_OK;
}

ds_status single_shape_check(const ds_problem& P) {
  const size_t esz = P.dtype == DS_F64 ? 8 : P.dtype == DS_F32 ? 4 : 2;
  const bool vec = reinterpret_cast<uintptr_t>(P.D) % 16 == 0 && (P.ldd * esz) % 16 == 0;
  return single_shape_check(P.dtype, P.N, P.K, P.G, vec);
}

ds_status solve_single(const ds_problem& P, const void* y, double lam, const ds_params& prm,
                       void* x, ds_info* info, hipStream_t stream, Workspace& ws,
                       std::vector<Telemetry>* tele_out, uint8_t* scr) {
  switch (P.dtype) {
    case DS_F64: return dispatch_rule<double>(P, y, lam, prm, x, info, stream, ws, tele_out, scr);
    case DS_F32: return dispatch_rule<float>(P, y, lam, prm, x, info, stream, ws, tele_out, scr);
    case DS_BF16: return dispatch_rule<bf16_t>(P, y, lam, prm, x, info, stream, ws, tele_out, scr);
  }
  set_error("unknown dtype");
  return DS_EINVAL;
}

// ------------------------------------------------------------------ lambda_max -------
namespace {
template <typename T>
ds_status lambda_max_t(const ds_problem& P, const void* y, double* lmax, int64_t* arg,
                       hipStream_t s, Workspace& ws) {
  using V = typename Types<T>::V;
  using A = typename Types<T>::A;
  const Layout l = make_layout(P.N, P.K, P.G, sizeof(V), sizeof(A), 1, false);
  ds_status e = ws.reserve(l.total);
  if (e != DS_OK) return e;
  char* base = static_cast<char*>(ws.base);
  if ((e = upload_groups(P, base, l, s)) != DS_OK) return e;
  SingleArgs<T, V, A> a = make_args<T>(P, y, base, l, TEST_NONE, RULE_ISTA);
  e = vector_ok<T>(P.D, P.ldd) ? launch_setup_corr<T, true>(P, y, base, l, s)
                               : launch_setup_corr<T, false>(P, y, base, l, s);
  if (e != DS_OK) return e;
  hipLaunchKernelGGL((k_setup_scalars<T, V, A>), dim3(1), dim3(CBLK), 0, s, a, 1.0, 1, 1.0, 0.0,
                     1, 0.0, 0.0, 0, 1e-5, 1.0, 1.0, 0.0, 0, 0.0);
  DS_HIP(hipGetLastError());
  SolverState* hst = static_cast<SolverState*>(ws.host_pinned);
  DS_HIP(hipMemcpyAsync(hst, a.st, sizeof(SolverState), hipMemcpyDeviceToHost, s));
  DS_HIP(hipStreamSynchronize(s));
  if (hst->status < 0) {
    set_error("observation contains NaN or Inf");
    return DS_EINVAL;
  }
  *lmax = hst->lam_max;
  if (arg) *arg = hst->i_star;
  return DS_OK;
}

template <typename T>
ds_status spectral_t(const ds_problem& P, int iters, double* Lout, hipStream_t s, Workspace& ws) {
  using V = typename Types<T>::V;
  using A = typename Types<T>::A;
  const Layout l = make_layout(P.N, P.K, P.G, sizeof(V), sizeof(A), 1, true);
  ds_status e = ws.reserve(l.total);
  if (e != DS_OK) return e;
  char* base = static_cast<char*>(ws.base);
  double* v = reinterpret_cast<double*>(base + l.off_pv);
  double* zk = reinterpret_cast<double*>(base + l.off_pz);
  double* w = reinterpret_cast<double*>(base + l.off_pw);
  double* part = reinterpret_cast<double*>(base + l.off_pd);
  double* dots = reinterpret_cast<double*>(base + l.off_bp0);
  const int N = static_cast<int>(P.N), K = static_cast<int>(P.K);
  const T* D = static_cast<const T*>(P.D);
  const int nch = (K + PCH - 1) / PCH;
  const bool vec = vector_ok<T>(P.D, P.ldd);
  const int rt_rows = vec ? WAVE * Store<T>::VEC : WAVE;
  const int nrt = (N + rt_rows - 1) / rt_rows;
  const int gdv = grid_for(static_cast<int64_t>(nrt) * nch, 1, 4096);
  hipLaunchKernelGGL(k_fill, dim3(grid_for(K, BLK, 1 << 20)), dim3(BLK), 0, s, v, K,
                     1.0 / std::sqrt(static_cast<double>(K)));
  auto dv = [&](const double* src) {
    if (vec)
      hipLaunchKernelGGL((k_pow_dv<T, true>), dim3(gdv), dim3(BLK), 0, s, D, P.ldd, N, K, src, part, l.npad);
    else
      hipLaunchKernelGGL((k_pow_dv<T, false>), dim3(gdv), dim3(BLK), 0, s, D, P.ldd, N, K, src, part, l.npad);
    hipLaunchKernelGGL(k_pow_reduce, dim3(grid_for(N, BLK, 1 << 20)), dim3(BLK), 0, s, part, nch,
                       l.npad, N, w);
  };
  auto dtw = [&](double* dst) {
    if (vec)
      hipLaunchKernelGGL((k_setup_gemv<T, double, true, false>), dim3(grid_for(K, NW * CPW, 4096)),
                         dim3(BLK), 0, s, D, P.ldd, N, K, static_cast<const double*>(w), dst, nullptr);
    else
      hipLaunchKernelGGL((k_setup_gemv<T, double, false, false>), dim3(grid_for(K, NW * CPW, 4096)),
                         dim3(BLK), 0, s, D, P.ldd, N, K, static_cast<const double*>(w), dst, nullptr);
  };
  if (iters <= 0) iters = 200;
  for (int k = 0; k < iters; ++k) {
    dv(v);        // w = D v
    dtw(zk);      // zk = D^T D v
    hipLaunchKernelGGL(k_pow_dots, dim3(1), dim3(CBLK), 0, s, v, zk, K, dots);
    hipLaunchKernelGGL(k_pow_scale, dim3(grid_for(K, BLK, 1 << 20)), dim3(BLK), 0, s, zk, K, dots, v);
  }
  DS_HIP(hipGetLastError());
  // Rayleigh quotient rho = v^T D^T D v (v unit) and residual ||D^T D v - rho v||
  dv(v);
  dtw(zk);
  hipLaunchKernelGGL(k_pow_dots, dim3(1), dim3(CBLK), 0, s, v, zk, K, dots);
  double h[3];
  DS_HIP(hipMemcpyAsync(h, dots, sizeof(h), hipMemcpyDeviceToHost, s));
  DS_HIP(hipStreamSynchronize(s));
  const double vv = h[0], rho = h[1] / vv, zz = h[2] / vv;
  const double res2 = std::max(zz - rho * rho, 0.0);
  *Lout = (rho + std::sqrt(res2)) * (1.0 + 1e-12);
  return DS_OK;
}
}  // namespace

ds_status lambda_max_impl(const ds_problem& P, const void* y, double* lmax, int64_t* arg,
                          hipStream_t stream, Workspace& ws) {
  switch (P.dtype) {
    case DS_F64: return lambda_max_t<double>(P, y, lmax, arg, stream, ws);
    case DS_F32: return lambda_max_t<float>(P, y, lmax, arg, stream, ws);
    case DS_BF16: return lambda_max_t<bf16_t>(P, y, lmax, arg, stream, ws);
  }
  return DS_EINVAL;
}

ds_status spectral_norm_impl(const ds_problem& P, int iters, double* L, hipStream_t stream,
                             Workspace& ws) {
  switch (P.dtype) {
    case DS_F64: return spectral_t<double>(P, iters, L, stream, ws);
    case DS_F32: return spectral_t<float>(P, iters, L, stream, ws);
    case DS_BF16: return spectral_t<bf16_t>(P, iters, L, stream, ws);
  }
  return DS_EINVAL;
}

}  // namespace ds
