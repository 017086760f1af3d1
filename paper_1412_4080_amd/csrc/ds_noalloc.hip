// Allocation-free single-signal solve (ds_solve_one_noalloc): the ds_solve_one path with
// its workspace carved from a file-scope device array instead of a device allocation, and
// its state read back through a static host buffer.  Each device holds its own copy of the
// array; its address is resolved once per device with hipGetSymbolAddress, and only that
// address (never the array's name) is used on the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "ds_engine.h"

namespace ds {
namespace {

constexpr size_t SCRATCH_BYTES = size_t(DS_NOALLOC_SCRATCH_MB) << 20;
constexpr int MAX_DEVICES = 64;

// The workspace of every call on a device.  Calls on one device are serialised by the
// per-device lock below; the array keeps the last call's contents, and every solve clears
// what must start at zero itself.
__device__ __align__(256) char scratch[SCRATCH_BYTES];

struct NoAllocCtx {
  std::mutex mu;
  void* ptr = nullptr;  // device address of this device's copy of `scratch`
  alignas(64) char stage[4096];  // host staging of the solver state (pageable)
};

NoAllocCtx g_ctx[MAX_DEVICES];

}  // namespace
}  // namespace ds

using namespace ds;

extern "C" ds_status ds_solve_one_noalloc(const ds_problem* problem, const void* y, double lambda,
                                          const ds_params* params, void* x, uint8_t* screened,
                                          ds_info* info, void* stream) {
  const bool group = problem != nullptr && problem->G > 0;
  ds_status e = validate_problem(problem, group);
  if (e != DS_OK) return e;
  if ((e = validate_params(params)) != DS_OK) return e;
  if ((e = validate_test_for(params, group)) != DS_OK) return e;
  if (y == nullptr || x == nullptr || info == nullptr) {
    set_error("y, x and info must be non-NULL");
    return DS_EINVAL;
  }
  if (!(lambda > 0.0) || !std::isfinite(lambda)) {
    set_error("lambda must be positive");
    return DS_EINVAL;
  }
  const bool line_search = params->step_rule == DS_STEP_BACKTRACK || params->rule == DS_SPARSA;
  if (!line_search && !(params->step_L > 0.0)) {
    set_error("ds_solve_one_noalloc needs step_L > 0 (estimating ||D||_2^2 would allocate; "
              "ds_spectral_norm_sq gives it once per dictionary)");
    return DS_EINVAL;
  }
  if ((e = single_shape_check(*problem)) != DS_OK) return e;
  const size_t need = single_workspace_bytes(*problem, *params);
  if (need > SCRATCH_BYTES) {
    set_error("the problem needs %zu bytes of scratch memory; ds_solve_one_noalloc has %zu "
              "(DS_NOALLOC_SCRATCH_MB)", need, SCRATCH_BYTES);
    return DS_EINVAL;
  }
  int dev = 0;
  DS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) {
    set_error("device ordinal %d out of range", dev);
    return DS_EINVAL;
  }
  NoAllocCtx& C = g_ctx[dev];
  std::lock_guard<std::mutex> g(C.mu);
  if (C.ptr == nullptr) {  // once per device, with that device current
    void* p = nullptr;
    DS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (p == nullptr) {
      set_error("hipGetSymbolAddress returned no address for the scratch array");
      return DS_EDEVICE;
    }
    C.ptr = p;
  }
  Workspace ws;
  ws.device = dev;
  ws.base = C.ptr;
  ws.bytes = SCRATCH_BYTES;
  ws.host_pinned = C.stage;
  ws.fixed = true;
  std::memset(info, 0, sizeof(ds_info));
  e = solve_single(*problem, y, lambda, *params, x, info, static_cast<hipStream_t>(stream), ws,
                   nullptr, screened);
  return e;
}
