// Batched path for many signals sharing one bfloat16 dictionary (placeholder: sequential
// single-signal solves until the MFMA engine lands).
#include <hip/hip_runtime.h>

#include <cstring>

#include "ds_engine.h"

namespace ds {

ds_status solve_batched_bf16(const ds_problem& P, const void* Y, int64_t B, int64_t ldy,
                             const double* lambdas, const ds_params& prm, void* X, int64_t ldx,
                             ds_info* info, hipStream_t stream) {
  int dev = 0;
  DS_HIP(hipGetDevice(&dev));
  DeviceCtx& ctx = device_ctx(dev);
  std::lock_guard<std::mutex> g(ctx.mu);
  ds_status worst = DS_OK;
  for (int64_t b = 0; b < B; ++b) {
    std::memset(&info[b], 0, sizeof(ds_info));
    const char* yb = static_cast<const char*>(Y) + b * ldy * 4;
    char* xb = static_cast<char*>(X) + b * ldx * 4;
    ds_status e = solve_single(P, yb, lambdas[b], prm, xb, &info[b], stream, ctx.ws, nullptr);
    if (e < 0) return e;
    if (e == DS_NOT_CONVERGED) worst = e;
  }
  return worst;
}

}  // namespace ds
