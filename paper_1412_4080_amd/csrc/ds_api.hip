// C-ABI entry points (include/dynscreen.h): argument validation, workspace management,
// dispatch to the single-signal and batched engines.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <atomic>
#include <map>
#include <memory>
#include <string>
#include <thread>

#include "ds_engine.h"

namespace ds {

namespace {
thread_local std::string g_err;
}

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}

StatAccum& stats() {
  static StatAccum s;
  return s;
}

Workspace::~Workspace() {
  // Cached per-device workspaces live until process exit, when the HIP runtime may
  // already be torn down; temporary ones call release() explicitly.
}

void Workspace::release() {
  if (fixed) return;  // memory owned elsewhere
  for (hipEvent_t e : events) (void)hipEventDestroy(e);
  events.clear();
  if (base != nullptr) (void)hipFree(base);
  if (host_pinned != nullptr) (void)hipHostFree(host_pinned);
  base = nullptr;
  host_pinned = nullptr;
  bytes = 0;
}

ds_status Workspace::reserve(size_t need) {
  if (fixed) {
    if (need <= bytes && base != nullptr && host_pinned != nullptr) return DS_OK;
    set_error("the problem needs %zu bytes of scratch memory; this entry point has %zu", need, bytes);
    return DS_EINVAL;
  }
  if (host_pinned == nullptr) {
    if (hipHostMalloc(&host_pinned, 4096, hipHostMallocDefault) != hipSuccess) {
      host_pinned = nullptr;
      set_error("hipHostMalloc of the staging area failed");
      return DS_ENOMEM;
    }
  }
  if (need <= bytes && base != nullptr) return DS_OK;
  if (base != nullptr) {
    DS_HIP(hipDeviceSynchronize());
    DS_HIP(hipFree(base));
    base = nullptr;
    bytes = 0;
  }
  const size_t want = need + need / 4;
  if (hipMalloc(&base, want) != hipSuccess) {
    (void)hipGetLastError();
    base = nullptr;
    set_error("hipMalloc of %zu workspace bytes failed", want);
    return DS_ENOMEM;
  }
  bytes = want;
  return DS_OK;
}

DeviceCtx& device_ctx(int device) {
  static std::mutex mu;
  static std::map<int, std::unique_ptr<DeviceCtx>> ctx;
  std::lock_guard<std::mutex> g(mu);
  auto& p = ctx[device];
  if (!p) {
    p = std::make_unique<DeviceCtx>();
    p->ws.device = device;
  }
  return *p;
}

size_t dtype_size(ds_dtype t) {
  switch (t) {
    case DS_F64: return 8;
    case DS_F32: return 4;
    case DS_BF16: return 2;
  }
  return 0;
}

// The integer a caller stored in an enumeration field: a C caller may store any int32 there,
// and reading a value outside the enumerators as the enumeration type is undefined in C++.
template <typename E>
int32_t enum_raw(const E& e) {
  static_assert(sizeof(E) == sizeof(int32_t), "enumerations of the boundary are 32-bit");
  int32_t v;
  std::memcpy(&v, &e, sizeof v);
  return v;
}

ds_status validate_problem(const ds_problem* p, bool group) {
  if (p == nullptr) { set_error("problem is NULL"); return DS_EINVAL; }
  const int32_t dt = enum_raw(p->dtype);
  if (dt != DS_F64 && dt != DS_F32 && dt != DS_BF16) {
    set_error("unknown dtype %d", static_cast<int>(dt));
    return DS_EINVAL;
  }
  if (p->N < 1 || p->K < 1 || p->N > (1ll << 24) || p->K > (1ll << 30)) {
    set_error("bad sizes N=%lld K=%lld", static_cast<long long>(p->N), static_cast<long long>(p->K));
    return DS_EINVAL;
  }
  if (p->ldd < p->N) { set_error("ldd < N"); return DS_EINVAL; }
  if (p->D == nullptr) { set_error("D is NULL"); return DS_EINVAL; }
  if (group) {
    if (p->G < 1 || p->group_ptr == nullptr) { set_error("group problem needs G > 0 and group_ptr"); return DS_EINVAL; }
    if (p->group_ptr[0] != 0 || p->group_ptr[p->G] != p->K) {
      set_error("group_ptr must start at 0 and end at K");
      return DS_EINVAL;
    }
    for (int64_t g = 0; g < p->G; ++g) {
      const int64_t sz = p->group_ptr[g + 1] - p->group_ptr[g];
      if (sz < 1) { set_error("group %lld is empty", static_cast<long long>(g)); return DS_EINVAL; }
      if (sz > DS_GROUP_MAX) {
        set_error("group %lld has %lld atoms; groups of at most %d atoms are supported",
                  static_cast<long long>(g), static_cast<long long>(sz), DS_GROUP_MAX);
        return DS_EINVAL;
      }
      if (p->w != nullptr && !(p->w[g] > 0.0 && std::isfinite(p->w[g]))) {
        set_error("group weight %lld must be positive and finite", static_cast<long long>(g));
        return DS_EINVAL;
      }
    }
  } else if (p->G != 0) {
    set_error("lasso_solve needs G == 0 (use glasso_solve for groups)");
    return DS_EINVAL;
  }
  return DS_OK;
}

ds_status validate_params(const ds_params* p) {
  if (p == nullptr) { set_error("params is NULL"); return DS_EINVAL; }
  const int32_t rule = enum_raw(p->rule), test = enum_raw(p->test);
  const int32_t lmode = enum_raw(p->lambda_mode), smode = enum_raw(p->screening);
  if (rule != DS_ISTA && rule != DS_FISTA && rule != DS_SPARSA && rule != DS_CP) {
    set_error("unknown rule");
    return DS_EINVAL;
  }
  if (test != DS_TEST_NONE && test != DS_TEST_SAFE && test != DS_TEST_DST3 && test != DS_TEST_DOME) {
    set_error("unknown test");
    return DS_EINVAL;
  }
  if (lmode != DS_LAMBDA_ABSOLUTE && lmode != DS_LAMBDA_RELATIVE) {
    set_error("unknown lambda mode");
    return DS_EINVAL;
  }
  if (!(p->gap_tol >= 0.0) || !std::isfinite(p->gap_tol)) { set_error("gap_tol must be >= 0"); return DS_EINVAL; }
  if (!(p->obj_tol >= 0.0) || !std::isfinite(p->obj_tol)) { set_error("obj_tol must be >= 0"); return DS_EINVAL; }
  if (p->batch_slots < 0) { set_error("batch_slots must be >= 0"); return DS_EINVAL; }
  if (p->max_iter < 1) { set_error("max_iter must be >= 1"); return DS_EINVAL; }
  if (!std::isfinite(p->step_L)) { set_error("step_L must be finite"); return DS_EINVAL; }
  if (smode != 0 && smode != 1) { set_error("screening must be 0 (dynamic) or 1 (static)"); return DS_EINVAL; }
  if (p->step_rule != DS_STEP_CONSTANT && p->step_rule != DS_STEP_BACKTRACK) {
    set_error("step_rule must be DS_STEP_CONSTANT or DS_STEP_BACKTRACK");
    return DS_EINVAL;
  }
  if (p->rule == DS_SPARSA && p->step_rule != DS_STEP_CONSTANT) {
    set_error("DS_SPARSA sets its own step: step_rule must be DS_STEP_CONSTANT");
    return DS_EINVAL;
  }
  if (p->rule == DS_CP) {
    if (p->step_rule != DS_STEP_CONSTANT) {
      set_error("DS_CP sets its own steps: step_rule must be DS_STEP_CONSTANT");
      return DS_EINVAL;
    }
    const double prm[3] = {p->cp_tau, p->cp_sigma, p->cp_gamma};
    for (double v : prm)
      if (!(v >= 0.0) || !std::isfinite(v)) {
        set_error("cp_tau, cp_sigma and cp_gamma must be finite and >= 0");
        return DS_EINVAL;
      }
    if (p->cp_tau > 0.0 && p->cp_sigma > 0.0 && p->step_L > 0.0 &&
        p->cp_tau * p->cp_sigma * p->step_L > 1.0 + 1e-12) {
      set_error("cp_tau * cp_sigma * step_L must be <= 1");
      return DS_EINVAL;
    }
  }
  const bool line_search = p->step_rule == DS_STEP_BACKTRACK || p->rule == DS_SPARSA;
  if (line_search && p->bt_eta != 0.0 && !(p->bt_eta > 1.0 && std::isfinite(p->bt_eta))) {
    set_error("bt_eta must be > 1 (or 0 for the default 2)");
    return DS_EINVAL;
  }
  if (p->rule == DS_SPARSA) {
    if (p->bb_memory < 0 || p->bb_memory > 15) {
      set_error("bb_memory must be in 0..15");
      return DS_EINVAL;
    }
    if (!(p->bb_sigma >= 0.0) || !std::isfinite(p->bb_sigma)) {
      set_error("bb_sigma must be >= 0 (0 selects 1e-5)");
      return DS_EINVAL;
    }
  }
  return DS_OK;
}

ds_status validate_test_for(const ds_params* p, bool group) {
  if (group && p->test == DS_TEST_DOME) {
    set_error("the Dome test is stated for the Lasso (use DS_TEST_DST3 for groups)");
    return DS_EINVAL;
  }
  return DS_OK;
}

namespace {

ds_status solve_common(const ds_problem* problem, const void* Y, int64_t B, int64_t ldy,
                       const double* lambdas, const ds_params* params, void* X, int64_t ldx,
                       ds_info* info, uint8_t* screened, void* stream, bool group) {
  ds_status e = validate_problem(problem, group);
  if (e != DS_OK) return e;
  if ((e = validate_params(params)) != DS_OK) return e;
  if ((e = validate_test_for(params, group)) != DS_OK) return e;
  if (Y == nullptr || X == nullptr || info == nullptr || lambdas == nullptr) {
    set_error("Y, X, lambdas and info must be non-NULL");
    return DS_EINVAL;
  }
  if (B < 1 || ldy < problem->N || ldx < problem->K) {
    set_error("bad B / ldy / ldx");
    return DS_EINVAL;
  }
  for (int64_t b = 0; b < B; ++b) {
    if (!(lambdas[b] > 0.0) || !std::isfinite(lambdas[b])) {
      set_error("lambda[%lld] must be positive and finite", static_cast<long long>(b));
      return DS_EINVAL;
    }
  }
  // every path but the batched bfloat16 one runs single-signal solves
  if (!(B > 1 && problem->dtype == DS_BF16) && (e = single_shape_check(*problem)) != DS_OK)
    return e;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0;
  DS_HIP(hipGetDevice(&dev));
  if (B > 1 && problem->dtype == DS_BF16) {
    if (params->step_rule == DS_STEP_BACKTRACK || params->rule == DS_SPARSA ||
        params->rule == DS_CP) {
      set_error("backtracking, SpaRSA and Chambolle-Pock are available on the single-signal path (B = 1 or FP32/FP64 D)");
      return DS_EINVAL;
    }
    if (params->x0 != nullptr || params->obj_tol > 0.0) {
      set_error("a warm start (x0) and the objective-change stop (obj_tol) are available on the single-signal path (B = 1 or FP32/FP64 D)");
      return DS_EINVAL;
    }
    return solve_batched_bf16(*problem, Y, B, ldy, lambdas, *params, X, ldx, info, screened, s);
  }
  DeviceCtx& ctx = device_ctx(dev);
  std::lock_guard<std::mutex> g(ctx.mu);
  const size_t vsz = problem->dtype == DS_F64 ? 8 : 4;
  auto one = [&](int64_t b, hipStream_t st, Workspace& ws) {
    const char* yb = static_cast<const char*>(Y) + b * ldy * vsz;
    char* xb = static_cast<char*>(X) + b * ldx * vsz;
    std::memset(&info[b], 0, sizeof(ds_info));
    ds_params pb = *params;  // column b of the warm start, laid out as X
    if (pb.x0 != nullptr) pb.x0 = static_cast<const char*>(params->x0) + b * ldx * vsz;
    return solve_single(*problem, yb, lambdas[b], pb, xb, &info[b], st, ws, nullptr,
                        screened != nullptr ? screened + b * problem->K : nullptr);
  };
  const int nl = static_cast<int>(std::min<int64_t>(B, SOLVE_LANES));
  if (nl == 1) return one(0, s, ctx.ws);
  // B > 1: the signals are independent solves.  Each lane (its own stream and workspace, on
  // a host thread of its own) takes the next waiting signal, smallest lambda first (those
  // usually need the most iterations, so the long solves start early).  Each solve is the
  // single-signal solve unchanged, so the results do not depend on the lanes.
  std::vector<int64_t> order(B);
  for (int64_t b = 0; b < B; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t c) { return lambdas[a] < lambdas[c]; });
  std::atomic<int64_t> next{0};
  hipEvent_t ready;
  DS_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  DS_HIP(hipEventRecord(ready, s));  // inputs written on the caller's stream
  for (int k = 0; k < nl; ++k) {
    SolveLane& ln = ctx.lanes[k];
    ln.ws.device = dev;
    if (ln.stream == nullptr) DS_HIP(hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking));
    DS_HIP(hipStreamWaitEvent(ln.stream, ready, 0));
  }
  std::vector<ds_status> st(nl, DS_OK);
  std::vector<std::string> msg(nl);
  auto lane = [&](int k) {
    if (hipSetDevice(dev) != hipSuccess) {
      st[k] = DS_EDEVICE;
      msg[k] = "hipSetDevice failed in a solve lane";
      return;
    }
    SolveLane& ln = ctx.lanes[k];
    for (int64_t q = next++; q < B; q = next++) {
      const ds_status r = one(order[q], ln.stream, ln.ws);
      if (r < 0) {
        st[k] = r;
        msg[k] = ds_last_error();
        next = B;  // the other lanes start no further signal
        return;
      }
      if (r == DS_NOT_CONVERGED) st[k] = DS_NOT_CONVERGED;
    }
  };
  // lanes 1 .. nl - 1 on threads of their own, lane 0 on the caller's thread; a lane whose
  // thread cannot be started runs on the caller's thread after lane 0 (no exception
  // crosses the boundary)
  std::vector<std::thread> th;
  std::vector<int> inline_lanes{0};
  for (int k = 1; k < nl; ++k) {
    try {
      th.emplace_back(lane, k);
    } catch (...) {
      inline_lanes.push_back(k);
    }
  }
  for (int k : inline_lanes) lane(k);
  for (auto& t : th) t.join();
  (void)hipEventDestroy(ready);
  ds_status worst = DS_OK;
  for (int k = 0; k < nl; ++k) {
    if (st[k] < 0) {
      set_error("%s", msg[k].c_str());
      return st[k];
    }
    if (st[k] == DS_NOT_CONVERGED) worst = DS_NOT_CONVERGED;
  }
  return worst;
}

}  // namespace
}  // namespace ds

using namespace ds;

extern "C" {

ds_status lasso_solve(const ds_problem* problem, const void* Y, int64_t B, int64_t ldy,
                      const double* lambdas, const ds_params* params, void* X, int64_t ldx,
                      ds_info* info, void* stream) {
  return solve_common(problem, Y, B, ldy, lambdas, params, X, ldx, info, nullptr, stream, false);
}

ds_status ds_solve_batch(const ds_problem* problem, const void* Y, int64_t B, int64_t ldy,
                         const double* lambdas, const ds_params* params, void* X, int64_t ldx,
                         ds_info* info, uint8_t* screened, void* stream) {
  const bool group = problem != nullptr && problem->G > 0;
  return solve_common(problem, Y, B, ldy, lambdas, params, X, ldx, info, screened, stream, group);
}

ds_status glasso_solve(const ds_problem* problem, const void* Y, int64_t B, int64_t ldy,
                       const double* lambdas, const ds_params* params, void* X, int64_t ldx,
                       ds_info* info, void* stream) {
  return solve_common(problem, Y, B, ldy, lambdas, params, X, ldx, info, nullptr, stream, true);
}

ds_status ds_solve_one(const ds_problem* problem, const void* y, double lambda,
                       const ds_params* params, void* x, uint8_t* screened, ds_trace* trace,
                       int32_t trace_cap, ds_info* info, void* stream) {
  const bool group = problem != nullptr && problem->G > 0;
  ds_status e = validate_problem(problem, group);
  if (e != DS_OK) return e;
  if ((e = validate_params(params)) != DS_OK) return e;
  if ((e = validate_test_for(params, group)) != DS_OK) return e;
  if (y == nullptr || x == nullptr || info == nullptr) {
    set_error("y, x and info must be non-NULL");
    return DS_EINVAL;
  }
  if (!(lambda > 0.0) || !std::isfinite(lambda)) { set_error("lambda must be positive"); return DS_EINVAL; }
  if (trace != nullptr && trace_cap < 0) { set_error("trace_cap < 0"); return DS_EINVAL; }
  if ((e = single_shape_check(*problem)) != DS_OK) return e;
  int dev = 0;
  DS_HIP(hipGetDevice(&dev));
  DeviceCtx& ctx = device_ctx(dev);
  std::lock_guard<std::mutex> g(ctx.mu);
  std::memset(info, 0, sizeof(ds_info));
  std::vector<Telemetry> tl;
  e = solve_single(*problem, y, lambda, *params, x, info, static_cast<hipStream_t>(stream), ctx.ws,
                   trace != nullptr ? &tl : nullptr, screened);
  if (e < 0) return e;
  if (trace != nullptr) {
    const size_t n = std::min<size_t>(tl.size(), static_cast<size_t>(trace_cap));
    for (size_t k = 0; k < n; ++k) {
      trace[k].n_active = tl[k].n_atoms;
      trace[k].n_units = tl[k].n_units;
      trace[k].n_support = tl[k].n_support;
      trace[k].nnz = tl[k].nnz;
      trace[k].radius = tl[k].r;
      trace[k].gap = tl[k].gap;
    }
  }
  return e;
}

ds_status ds_lambda_max(const ds_problem* problem, const void* y, double* lambda_max,
                        int64_t* argmax, void* stream) {
  ds_status e = validate_problem(problem, problem != nullptr && problem->G > 0);
  if (e != DS_OK) return e;
  if (y == nullptr || lambda_max == nullptr) { set_error("y and lambda_max must be non-NULL"); return DS_EINVAL; }
  int dev = 0;
  DS_HIP(hipGetDevice(&dev));
  DeviceCtx& ctx = device_ctx(dev);
  std::lock_guard<std::mutex> g(ctx.mu);
  return lambda_max_impl(*problem, y, lambda_max, argmax, static_cast<hipStream_t>(stream), ctx.ws);
}

ds_status ds_spectral_norm_sq(const ds_problem* problem, int32_t iters, double* L, void* stream) {
  ds_status e = validate_problem(problem, problem != nullptr && problem->G > 0);
  if (e != DS_OK) return e;
  if (L == nullptr) { set_error("L is NULL"); return DS_EINVAL; }
  int dev = 0;
  DS_HIP(hipGetDevice(&dev));
  DeviceCtx& ctx = device_ctx(dev);
  std::lock_guard<std::mutex> g(ctx.mu);
  return spectral_norm_impl(*problem, iters, L, static_cast<hipStream_t>(stream), ctx.ws);
}

void ds_stats_enable(int on) {
  StatAccum& S = stats();
  std::lock_guard<std::mutex> g(S.mu);
  S.on = on != 0;
}

void ds_stats_reset(void) {
  StatAccum& S = stats();
  std::lock_guard<std::mutex> g(S.mu);
  for (auto& k : S.s) k = ds_kernel_stat{};
  S.launches.clear();
}

int ds_stats_launches(ds_launch_stat* out, int n) {
  if (out == nullptr || n <= 0) return 0;
  StatAccum& S = stats();
  std::lock_guard<std::mutex> g(S.mu);
  const size_t m = std::min(S.launches.size(), static_cast<size_t>(n));
  for (size_t k = 0; k < m; ++k) out[k] = S.launches[k];
  return static_cast<int>(m);
}

int ds_stats_read(ds_kernel_stat* out, int n) {
  if (out == nullptr || n <= 0) return 0;
  StatAccum& S = stats();
  std::lock_guard<std::mutex> g(S.mu);
  const int m = n < DS_STAT_COUNT ? n : DS_STAT_COUNT;
  for (int k = 0; k < m; ++k) out[k] = S.s[k];
  return m;
}

const char* ds_last_error(void) { return g_err.c_str(); }

const char* ds_version(void) { return "dynscreen 0.1 (gfx950)"; }

}  // extern "C"
