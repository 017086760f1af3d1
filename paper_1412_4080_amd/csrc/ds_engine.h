// Host-side engine shared by the C-ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dynscreen.h"

// Largest group the Group-Lasso kernels handle (two atoms per lane of a 64-wide wave).
constexpr int DS_GROUP_MAX = 128;

namespace ds {

void set_error(const char* fmt, ...);

#define DS_HIP(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) {                                                             \
      ::ds::set_error("HIP error %s at %s:%d: %s", hipGetErrorString(e_), __FILE__,     \
                      __LINE__, #expr);                                                 \
      return DS_EDEVICE;                                                                \
    }                                                                                   \
  } while (0)

// Per-iteration telemetry written on the device by the last correlation block: the
// quantities the paper's flops model needs (|I^c_t|, ||x_t||_0) plus radius and gap.
struct Telemetry {
  int32_t n_atoms;     // active atoms used by this iteration's update
  int32_t n_units;     // active units (atoms or groups)
  int32_t n_support;   // support size of the primal point theta was evaluated at
  int32_t nnz;         // non-zeros of x_t
  double r;            // radius r_t (no slack)
  double gap;          // gap certificate
};
static_assert(sizeof(Telemetry) == 32, "telemetry record layout");

// Kernel statistics (diagnostics API).
struct StatAccum {
  std::mutex mu;
  bool on = false;
  ds_kernel_stat s[DS_STAT_COUNT] = {};
  std::vector<ds_launch_stat> launches;  // per-launch records of the correlation pass
  static constexpr size_t MAX_LAUNCHES = size_t(1) << 20;
};
StatAccum& stats();

// One device allocation carved into the buffers of a single-signal solve.  A fixed
// workspace is memory the library does not own (base, bytes and a host staging area set
// by its owner): reserve() never allocates and refuses a larger need.
struct Workspace {
  int device = -1;
  void* base = nullptr;
  size_t bytes = 0;
  void* host_pinned = nullptr;  // small (pinned, unless fixed) staging area for the state
  bool fixed = false;
  std::vector<hipEvent_t> events;
  ~Workspace();
  ds_status reserve(size_t need);
  void release();  // frees everything (temporary workspaces; cached ones live until exit)
};

// A stream and workspace that run independent single-signal solves concurrently with the
// other lanes of the device (the B > 1 single-signal path).
struct SolveLane {
  hipStream_t stream = nullptr;
  Workspace ws;
};
constexpr int SOLVE_LANES = 4;  // one per hardware queue a process gets by default

// Per-device cache of workspaces (one in use at a time per lock holder).
struct DeviceCtx {
  std::mutex mu;
  Workspace ws;
  SolveLane lanes[SOLVE_LANES];
};
DeviceCtx& device_ctx(int device);

ds_status validate_problem(const ds_problem* p, bool group);
ds_status validate_params(const ds_params* p);
// The Dome test is stated for the Lasso: DS_EINVAL with a grouped problem.
ds_status validate_test_for(const ds_params* p, bool group);

// Whether the single-signal kernels cover a problem shape: the residual pass's row tiles
// and the correlation pass's blocks have fixed maxima.  DS_EINVAL, with the limits in the
// error string, otherwise.  Host arithmetic only; vec: the dictionary takes 16-byte loads
// (16-byte aligned base and column stride).
ds_status single_shape_check(int32_t dtype, int64_t N, int64_t K, int64_t G, bool vec);
ds_status single_shape_check(const ds_problem& P);
ds_status solve_single(const ds_problem& P, const void* y, double lam, const ds_params& prm,
                       void* x, ds_info* info, hipStream_t stream, Workspace& ws,
                       std::vector<Telemetry>* tele_out, uint8_t* screened = nullptr);
ds_status lambda_max_impl(const ds_problem& P, const void* y, double* lmax, int64_t* arg,
                          hipStream_t stream, Workspace& ws);
ds_status spectral_norm_impl(const ds_problem& P, int iters, double* L, hipStream_t stream,
                             Workspace& ws);
// Batched MFMA path (bfloat16 storage, B > 1).
ds_status solve_batched_bf16(const ds_problem& P, const void* Y, int64_t B, int64_t ldy,
                             const double* lambdas, const ds_params& prm, void* X, int64_t ldx,
                             ds_info* info, uint8_t* screened, hipStream_t stream);

// The batched engine's source and sink of signals.  Between graph replays the engine asks
// pull for up to `room` new signals (fills the Y / X column and the penalty of each, returns
// how many; 0 when none is waiting; a copy into Y enqueued on the engine's stream `s` is
// ordered before the signals' set-up) and hands finished ones to finish (their X columns
// and masks are written: the harvest that wrote them has completed).  The engine's stream
// may already run the next replay when finish is called.  A run ends when no slot holds a
// signal after a pull.
struct BatchFeed {
  std::function<int(int room, int* cols, double* lams, hipStream_t s)> pull;
  std::function<void(const int* cols, const ds_info* infos, int n, hipStream_t s)> finish;
};
struct BatchEngine;  // workspace, stream, graph and tuned shapes of one engine
BatchEngine* batch_engine_create(int device);
void batch_engine_destroy(BatchEngine* engine);
// Runs the signals the feed supplies with `nslot` resident slots on the bfloat16 dictionary
// P (Lasso; ISTA or FISTA with a constant step; SAFE, DST3 or no test).  Y: N x columns FP32
// (leading dimension ldy), X: K x columns FP32 (ldx), screened: K x columns or NULL.
ds_status run_batched(BatchEngine& engine, const ds_problem& P, const float* Y, int64_t ldy,
                      int nslot, const ds_params& prm, float* X, int64_t ldx,
                      uint8_t* screened, BatchFeed& feed, hipStream_t stream);
// Device bytes of a batched engine's workspace for this shape (G > 0: grouped).
size_t batched_workspace_bytes(int64_t N, int64_t K, int slots, int max_iter, int64_t G = 0);
// ||D_g||_2 and ||D_g||_F of the contiguous groups gptr_dev (device, G + 1 offsets) of a
// bfloat16 dictionary with leading dimension ldd; max_group: the largest group (<= 128).
ds_status group_norms_bf16(const uint16_t* D, int64_t ldd, int N, int G, const int64_t* gptr_dev,
                           int max_group, double* gnorm, double* fro, hipStream_t s);
// Gives an idle engine's device memory back (workspace and graph; tuned shapes are kept).
void batch_engine_trim(BatchEngine* engine);

size_t dtype_size(ds_dtype t);

// Device bytes a single-signal solve of this shape holds (its workspace).
size_t single_workspace_bytes(const ds_problem& P, const ds_params& prm);

}  // namespace ds
