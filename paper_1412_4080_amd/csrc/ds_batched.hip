// Batched path for many signals sharing one bfloat16 dictionary (Lasso, B > 1): host
// side.  Buffers live in one per-device workspace; a run of ITERS_PER_GRAPH iterations
// (an even number, so that it starts on the same parity of the u double buffer each time)
// is captured once as a HIP graph and replayed until every signal has finished.  The block
// shape of the Z = D^T Theta kernel is chosen per (N, K, B) by timing every eligible shape
// once (all shapes give the same results bit for bit), cached in memory and optionally in
// the file named by DS_AUTOTUNE_CACHE; DS_BATCH_TILE=<index> forces a shape.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <numeric>
#include <tuple>
#include <type_traits>
#include <vector>

#include "ds_batched_kernels.h"
#include "ds_engine.h"

namespace ds {
namespace {

using namespace batch;

constexpr int ITERS_PER_GRAPH = 8;  // iterations per graph replay (even)
constexpr int MAX_SLOTS = 512;      // resident signals when the caller does not set batch_slots

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
int round_up(int v, int m) { return (v + m - 1) / m * m; }

struct BLayout {
  int N, K, B, Np, Kp, Bp, nrb, G;
  size_t gptr, agrp, gw, gspec, gfro, Vd;  // groups only (zero bytes for the Lasso)
  size_t dcm, nu, dsc, Y, X, U0, U1, umask, Ths, th64, ptt, pty, marg, tminm, pz, pom, pact, Z, ccount, cidx, cval,
      inst, ctr, vlist, perm, slist, asig, alam, dflag, lam, z0, gn, Vn, kclk, spans, tX, tU, tZ, tpz, tpom,
      tpact, tmask, total;
  int nspan;
};

BLayout make_layout(int N, int K, int B, int max_iter, int G) {
  BLayout l{};
  l.N = N; l.K = K; l.B = B; l.G = G;
  l.Np = round_up(N, 64);
  l.Kp = round_up(K, KP_ALIGN);
  l.Bp = round_up(B, 64);
  l.nrb = (l.Np + TR - 1) / TR;
  const size_t np = l.Np, kp = l.Kp, bp = l.Bp, nt = l.Kp / MT;
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o = align256(o + bytes); return at; };
  l.dcm = take(kp * np * 2);
  l.nu = take(kp * 8);
  l.dsc = take(2 * 8);
  l.Y = take(bp * np * 4);
  l.X = take(bp * kp * 4);
  l.U0 = take(bp * kp * 4);
  l.U1 = take(bp * kp * 4);
  l.umask = take(nt * bp * 4);
  l.Ths = take(THP * bp * np * 2);
  l.th64 = take(bp * np * 8);
  l.ptt = take(static_cast<size_t>(l.nrb) * bp * 8);
  l.pty = take(static_cast<size_t>(l.nrb) * bp * 8);
  l.marg = take(bp * kp * 4);
  l.tminm = take(nt * bp * 4);
  l.pz = take(nt * bp * 8);
  l.pom = take(nt * bp * 8);
  l.pact = take(nt * bp * 4);
  l.Z = take(bp * kp * 4);
  l.ccount = take(bp * ((K + VC - 1) / VC) * 4);
  l.cidx = take(bp * kp * 4);
  l.cval = take(bp * kp * 8);
  l.inst = take(bp * sizeof(Inst));
  l.ctr = take(4 * sizeof(int));
  l.vlist = take(bp * 4);
  l.dflag = take(2 * bp * 4);  // harvest flags, two replays
  l.perm = take(bp * 4);
  l.lam = take(bp * 8);
  l.slist = take(bp * 4);  // slist, asig and alam are adjacent: one upload from the host
  l.asig = take(bp * 4);
  l.alam = take(bp * 8);
  l.z0 = take(bp * kp * 8);
  l.gn = take(bp * kp * 8);
  l.Vn = take(bp * np * 4);
  l.kclk = take(2 * static_cast<size_t>(l.Kp / 64) * (l.Bp / 64) * NWB * 8);
  l.nspan = max_iter + ITERS_PER_GRAPH;
  l.spans = take(static_cast<size_t>(l.nspan) * 8);
  // the autotuner's outputs (its trial launches write here instead of the solve's state)
  l.tX = take(bp * kp * 4);
  l.tU = take(bp * kp * 4);
  l.tZ = take(bp * kp * 4);
  l.tpz = take(nt * bp * 8);
  l.tpom = take(nt * bp * 8);
  l.tpact = take(nt * bp * 4);
  l.tmask = take(nt * bp * 4);
  const size_t ng = G > 0 ? static_cast<size_t>(G) : 0;
  l.gptr = take(G > 0 ? (ng + 1) * 8 : 0);
  l.agrp = take(G > 0 ? kp * 4 : 0);
  l.gw = take(ng * 8);
  l.gspec = take(ng * 8);
  l.gfro = take(ng * 8);
  l.Vd = take(G > 0 ? bp * np * 8 : 0);
  l.total = o;
  return l;
}

bool shape_fits(int k, const BLayout& l) {
  const ZShapeDesc& z = ZSHAPES[k];
  return l.Kp % (MT * z.ra * z.wa) == 0 && l.Bp % (MT * z.rb * z.wb) == 0;
}

template <int RA, int RB, int WA, int WB>
void launch_zgemm_t(const BLayout& l, hipStream_t s, hipEvent_t e0, hipEvent_t e1, const BArgs& a,
                    const float* Uin, float* Uout) {
  const dim3 g(l.Kp / (MT * RA * WA), l.Bp / (MT * RB * WB)), blk(BW * RA * RB);
  if (e0 != nullptr)
    hipExtLaunchKernelGGL((k_b_zgemm<RA, RB, WA, WB>), g, blk, 0, s, e0, e1, 0, a, Uin, Uout);
  else
    hipLaunchKernelGGL((k_b_zgemm<RA, RB, WA, WB>), g, blk, 0, s, a, Uin, Uout);
}

// Launch the Z-GEMM with block shape k (an index into ZSHAPES); returns its wave count.
int launch_zgemm(int k, const BLayout& l, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                 const BArgs& a, const float* Uin, float* Uout) {
  switch (k) {
    case 1: launch_zgemm_t<4, 2, 1, 1>(l, s, e0, e1, a, Uin, Uout); break;
    case 2: launch_zgemm_t<4, 1, 1, 1>(l, s, e0, e1, a, Uin, Uout); break;
    case 3: launch_zgemm_t<2, 4, 1, 1>(l, s, e0, e1, a, Uin, Uout); break;
    case 4: launch_zgemm_t<1, 4, 1, 1>(l, s, e0, e1, a, Uin, Uout); break;
    case 5: launch_zgemm_t<2, 2, 2, 1>(l, s, e0, e1, a, Uin, Uout); break;
    case 6: launch_zgemm_t<4, 1, 2, 1>(l, s, e0, e1, a, Uin, Uout); break;
    default: launch_zgemm_t<2, 2, 1, 1>(l, s, e0, e1, a, Uin, Uout); break;
  }
  const ZShapeDesc& z = ZSHAPES[k];
  return (l.Kp / (MT * z.ra * z.wa)) * (l.Bp / (MT * z.rb * z.wb)) * z.ra * z.rb;
}

}  // namespace

// State of one batched engine: workspace, a private stream (graph capture needs one that is
// not the legacy default stream), the last instantiated graph and the tuned block shapes.
// Each device has one for direct calls; a server has one per batched dictionary.
struct BatchEngine {
  std::mutex mu;
  Workspace ws;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  hipEvent_t evh[2] = {nullptr, nullptr};  // a replay's harvest results are on the host
  hipEvent_t evu = nullptr;                 // the last slot assignment has been uploaded
  hipGraphExec_t exec = nullptr;
  BArgs key{};
  int key_shape = -1;
  hipEvent_t tune0 = nullptr, tune1 = nullptr;  // timing events of the autotuner
  int last_shape = -1;                           // shape of the last solve (diagnostics)
  std::map<std::tuple<int, int, int>, int> tuned;  // (N, K, B) -> Z-GEMM block shape
  std::vector<std::pair<hipEvent_t, hipEvent_t>> evpool;
  size_t ev_used = 0;
  // pinned host staging of what a run exchanges with the device between replays (the
  // harvest flags and slot states, the slot assignment, penalties and set-up list), so
  // that those copies are plain asynchronous DMA
  void* pin = nullptr;
  size_t pin_bytes = 0;
};

BatchEngine* batch_engine_create(int device) {
  auto* E = new BatchEngine;
  E->ws.device = device;
  return E;
}

void batch_engine_destroy(BatchEngine* E) {
  if (E == nullptr) return;
  if (E->ws.device >= 0) (void)hipSetDevice(E->ws.device);
  if (E->stream != nullptr) (void)hipStreamSynchronize(E->stream);
  if (E->exec != nullptr) (void)hipGraphExecDestroy(E->exec);
  for (auto& p : E->evpool) {
    (void)hipEventDestroy(p.first);
    (void)hipEventDestroy(p.second);
  }
  if (E->tune0 != nullptr) (void)hipEventDestroy(E->tune0);
  if (E->tune1 != nullptr) (void)hipEventDestroy(E->tune1);
  if (E->ev != nullptr) (void)hipEventDestroy(E->ev);
  for (hipEvent_t h : E->evh)
    if (h != nullptr) (void)hipEventDestroy(h);
  if (E->evu != nullptr) (void)hipEventDestroy(E->evu);
  if (E->stream != nullptr) (void)hipStreamDestroy(E->stream);
  if (E->pin != nullptr) (void)hipHostFree(E->pin);
  E->ws.release();
  delete E;
}

void batch_engine_trim(BatchEngine* E) {
  if (E == nullptr) return;
  std::lock_guard<std::mutex> g(E->mu);
  if (E->ws.device >= 0) (void)hipSetDevice(E->ws.device);
  if (E->stream != nullptr) (void)hipStreamSynchronize(E->stream);
  if (E->exec != nullptr) (void)hipGraphExecDestroy(E->exec);
  E->exec = nullptr;
  E->key_shape = -1;
  E->ws.release();
}

namespace {

BatchEngine& batch_ctx(int device) {
  static std::mutex mu;
  static std::map<int, std::unique_ptr<BatchEngine>> ctx;
  std::lock_guard<std::mutex> g(mu);
  auto& p = ctx[device];
  if (!p) {
    p = std::make_unique<BatchEngine>();
    p->ws.device = device;
  }
  return *p;
}

// Autotuner: the Z-GEMM block shape for this (N, K, B).  DS_BATCH_TILE forces one; else the
// in-memory cache, then the file named by DS_AUTOTUNE_CACHE (lines "N K B bf16 shape"),
// then a timing of every shape that fits: one warm-up and three launches each, on the
// solve's first theta with every active tile of every signal in play, writing to scratch
// outputs so that the solve's state is untouched.  Returns the shape index.
int choose_shape(BatchEngine& C, const BLayout& l, char* base, const BArgs& a, hipStream_t s,
                 hipEvent_t e0, hipEvent_t e1) {
  if (const char* f = std::getenv("DS_BATCH_TILE")) {
    const int k = std::atoi(f);
    if (k >= 0 && k < NZSHAPE && shape_fits(k, l)) return k;
  }
  const auto key = std::make_tuple(l.N, l.K, l.B);
  auto it = C.tuned.find(key);
  if (it != C.tuned.end()) return it->second;
  const char* path = std::getenv("DS_AUTOTUNE_CACHE");
  if (path != nullptr) {
    if (FILE* fp = std::fopen(path, "r")) {
      int n, k, b, sh;
      char dt[16];
      int found = -1;
      while (std::fscanf(fp, "%d %d %d %15s %d", &n, &k, &b, dt, &sh) == 5)
        if (n == l.N && k == l.K && b == l.B && std::strcmp(dt, "bf16") == 0 && sh >= 0 &&
            sh < NZSHAPE && shape_fits(sh, l))
          found = sh;
      std::fclose(fp);
      if (found >= 0) return C.tuned[key] = found;
    }
  }
  BArgs t = a;
  t.X = reinterpret_cast<float*>(base + l.tX);
  t.Z = reinterpret_cast<float*>(base + l.tZ);
  t.pz = reinterpret_cast<double*>(base + l.tpz);
  t.pom = reinterpret_cast<double*>(base + l.tpom);
  t.pact = reinterpret_cast<int*>(base + l.tpact);
  t.umask = reinterpret_cast<uint32_t*>(base + l.tmask);
  t.kclk = nullptr;
  float* tU = reinterpret_cast<float*>(base + l.tU);
  if (hipMemsetAsync(t.X, 0, static_cast<size_t>(l.Bp) * l.Kp * 4, s) != hipSuccess) return 0;
  int best = 0;
  float best_ms = 1e30f;
  for (int k = 0; k < NZSHAPE; ++k) {
    if (!shape_fits(k, l)) continue;
    launch_zgemm(k, l, s, nullptr, nullptr, t, a.U0, tU);
    if (hipEventRecord(e0, s) != hipSuccess) return 0;
    for (int r = 0; r < 3; ++r) launch_zgemm(k, l, s, nullptr, nullptr, t, a.U0, tU);
    float ms = 1e30f;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess || hipGetLastError() != hipSuccess)
      return 0;
    if (ms < best_ms) {
      best_ms = ms;
      best = k;
    }
  }
  C.tuned[key] = best;
  if (path != nullptr) {
    if (FILE* fp = std::fopen(path, "a")) {
      std::fprintf(fp, "%d %d %d bf16 %d\n", l.N, l.K, l.B, best);
      std::fclose(fp);
    }
  }
  return best;
}

BArgs make_args(const BLayout& l, char* base, const ds_params& prm, double L) {
  BArgs a;
  std::memset(&a, 0, sizeof a);
  a.N = l.N; a.K = l.K; a.B = l.B; a.Np = l.Np; a.Kp = l.Kp; a.Bp = l.Bp; a.nrb = l.nrb;
  a.test = static_cast<int>(prm.test);
  a.rule = prm.rule == DS_FISTA ? 1 : 0;
  a.max_iter = prm.max_iter;
  a.screen_static = prm.screening;
  a.L = L;
  // |z_hat - d^T theta| <= gamma_acc ||d|| ||theta||: FP32 accumulation of the THP x 64
  // exact products of a row chunk (and the MFMA's internal sums) bounded with unit
  // roundoff 2^-23, the factor 1.02 covering the sum of the parts' magnitudes (at most
  // (1 + 2^-7) |v|); the FP64 sum of the chunk results; the FP32 rounding of theta; with
  // two parts, the part left out (at most 2^-16 of the FP32 theta, elementwise)
  const double n = THP * 64.0 + 32.0, u = 0x1p-23;
  a.gamma_acc = 1.02 * n * u / (1.0 - n * u) + (l.Np / 64 + 2) * 0x1p-52 + 0x1p-23 +
                (THP == 2 ? 0x1p-16 * (1.0 + 0x1p-20) : 0.0);
  a.gamma64 = 1.01 * (l.Np + 16) * 0x1p-53;
  a.dcm = reinterpret_cast<const uint16_t*>(base + l.dcm);
  a.dsc = reinterpret_cast<const double*>(base + l.dsc);
  a.nu = reinterpret_cast<const double*>(base + l.nu);
  a.Y = reinterpret_cast<const float*>(base + l.Y);
  a.X = reinterpret_cast<float*>(base + l.X);
  a.U0 = reinterpret_cast<float*>(base + l.U0);
  a.U1 = reinterpret_cast<float*>(base + l.U1);
  a.umask = reinterpret_cast<uint32_t*>(base + l.umask);
  a.Ths = reinterpret_cast<uint16_t*>(base + l.Ths);
  a.th64 = reinterpret_cast<double*>(base + l.th64);
  a.ptt = reinterpret_cast<double*>(base + l.ptt);
  a.pty = reinterpret_cast<double*>(base + l.pty);
  a.marg = reinterpret_cast<const float*>(base + l.marg);
  a.tminm = reinterpret_cast<const float*>(base + l.tminm);
  a.pz = reinterpret_cast<double*>(base + l.pz);
  a.pom = reinterpret_cast<double*>(base + l.pom);
  a.pact = reinterpret_cast<int*>(base + l.pact);
  a.Z = reinterpret_cast<float*>(base + l.Z);
  a.ccount = reinterpret_cast<int*>(base + l.ccount);
  a.cidx = reinterpret_cast<int*>(base + l.cidx);
  a.cval = reinterpret_cast<double*>(base + l.cval);
  a.inst = reinterpret_cast<Inst*>(base + l.inst);
  a.ndone = reinterpret_cast<int*>(base + l.ctr);
  a.vcount = reinterpret_cast<int*>(base + l.ctr) + 1;
  a.vlist = reinterpret_cast<int*>(base + l.vlist);
  a.G = l.G;
  if (l.G > 0) {
    a.gptr = reinterpret_cast<const int64_t*>(base + l.gptr);
    a.agrp = reinterpret_cast<const int*>(base + l.agrp);
    a.gw = reinterpret_cast<const double*>(base + l.gw);
    a.gspec = reinterpret_cast<const double*>(base + l.gspec);
    a.gfro = reinterpret_cast<const double*>(base + l.gfro);
  }
  return a;
}

}  // namespace

size_t batched_workspace_bytes(int64_t N, int64_t K, int slots, int max_iter, int64_t G) {
  return make_layout(static_cast<int>(N), static_cast<int>(K), slots, max_iter, static_cast<int>(G)).total;
}

namespace {

// The caller's record of a finished signal.
ds_info info_of(const Inst& h, double L) {
  ds_info r;
  std::memset(&r, 0, sizeof r);
  if (h.status < 0) {  // observation with NaN or Inf
    r.status = DS_EINVAL;
    return r;
  }
  r.iters = h.iter;
  r.n_active = h.n_active;
  r.nnz = h.nnz;
  r.lambda = h.lam;
  r.lambda_max = h.lam_max;
  r.primal = h.primal;
  r.dual = h.dual;
  r.gap = h.gap;
  r.radius = h.r_min;
  r.mu = h.mu;
  r.L = L;
  r.radius_slack = h.r_slack + h.marg_slack;
  r.status = (h.status == 1 || h.converged) ? DS_OK : DS_NOT_CONVERGED;
  return r;
}

}  // namespace

ds_status run_batched(BatchEngine& C, const ds_problem& P, const float* Y, int64_t ldy,
                      int nslot, const ds_params& prm, float* X, int64_t ldx,
                      uint8_t* screened, BatchFeed& feed, hipStream_t stream) {
  if (P.N > (1 << 24) || P.K > (1 << 24) || nslot < 1 || nslot > 32768) {
    set_error("batched path: N, K must be <= 2^24 and 1 <= batch_slots <= 32768");
    return DS_EINVAL;
  }
  int dev = 0;
  DS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> guard(C.mu);
  const BLayout l = make_layout(static_cast<int>(P.N), static_cast<int>(P.K), nslot, prm.max_iter,
                                static_cast<int>(P.G));
  ds_status e = C.ws.reserve(l.total);
  if (e != DS_OK) return e;
  if (C.stream == nullptr) {
    DS_HIP(hipStreamCreateWithFlags(&C.stream, hipStreamNonBlocking));
    DS_HIP(hipEventCreateWithFlags(&C.ev, hipEventDisableTiming));
    DS_HIP(hipEventCreateWithFlags(&C.evh[0], hipEventDisableTiming));
    DS_HIP(hipEventCreateWithFlags(&C.evh[1], hipEventDisableTiming));
    DS_HIP(hipEventCreateWithFlags(&C.evu, hipEventDisableTiming));
    DS_HIP(hipEventCreate(&C.tune0));
    DS_HIP(hipEventCreate(&C.tune1));
  }
  hipStream_t s = C.stream;
  // inputs written on the caller's stream are visible to ours
  DS_HIP(hipEventRecord(C.ev, stream));
  DS_HIP(hipStreamWaitEvent(s, C.ev, 0));

  // step constant
  double L = prm.step_L;
  if (!(L > 0.0)) {
    Workspace tmp;
    tmp.device = dev;
    e = spectral_norm_impl(P, 0, &L, s, tmp);
    tmp.release();
    if (e != DS_OK) return e;
  }

  char* base = static_cast<char*>(C.ws.base);
  BArgs a = make_args(l, base, prm, L);

  // Pinned staging (the engine's stream is idle between runs, so an old block can go):
  // harvest flags and slot states of two replays, and a slot assignment (slots, signals,
  // penalties) that mirrors the adjacent device arrays slist | asig | alam, so that one copy
  // uploads it.  The host writes the assignment only after a synchronization that followed
  // its last upload.
  const size_t bp = static_cast<size_t>(l.Bp);
  auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
  const size_t pin_need = 2 * al(bp * 4) + 2 * al(bp * sizeof(Inst)) + 2 * al(bp * 4) + al(bp * 8);
  const size_t up_bytes = 2 * al(bp * 4) + bp * 8;
  if (l.asig != l.slist + al(bp * 4) || l.alam != l.asig + al(bp * 4)) {
    set_error("batched path: internal layout error");
    return DS_EDEVICE;
  }
  if (C.pin_bytes < pin_need) {
    if (C.pin != nullptr) (void)hipHostFree(C.pin);
    C.pin = nullptr;
    C.pin_bytes = 0;
    DS_HIP(hipHostMalloc(&C.pin, pin_need, hipHostMallocDefault));
    C.pin_bytes = pin_need;
  }
  char* pp = static_cast<char*>(C.pin);
  int* h_flag[2] = {reinterpret_cast<int*>(pp), reinterpret_cast<int*>(pp + al(bp * 4))};
  pp += 2 * al(bp * 4);
  Inst* h_inst[2] = {reinterpret_cast<Inst*>(pp), reinterpret_cast<Inst*>(pp + al(bp * sizeof(Inst)))};
  pp += 2 * al(bp * sizeof(Inst));
  int* h_list = reinterpret_cast<int*>(pp);
  int* h_asig = reinterpret_cast<int*>(pp + al(bp * 4));
  double* h_alam = reinterpret_cast<double*>(pp + 2 * al(bp * 4));

  // The feed hands out signals (a column of Y and X, and a penalty) as slots free up;
  // slot k holds column slot_sig[k], or -1 when idle (the device's perm, which the harvest
  // clears and k_b_assign sets, mirrors it).
  std::vector<int> slot_sig(bp, -1);
  std::vector<int> cols(nslot);
  std::vector<double> lams(nslot);
  const int n0 = feed.pull(nslot, cols.data(), lams.data(), s);
  if (n0 <= 0) return DS_OK;
  for (int k = 0; k < l.Bp; ++k) {
    slot_sig[k] = k < n0 ? cols[k] : -1;
    h_list[k] = k;
    h_asig[k] = slot_sig[k];
    h_alam[k] = k < n0 ? lams[k] : 1.0;
  }
  int* d_perm = reinterpret_cast<int*>(base + l.perm);
  double* d_lam = reinterpret_cast<double*>(base + l.lam);
  int* d_list = reinterpret_cast<int*>(base + l.slist);
  // upload an assignment of n slots and apply it to perm and lam
  auto assign = [&](int n) -> ds_status {
    DS_HIP(hipMemcpyAsync(d_list, h_list, up_bytes, hipMemcpyHostToDevice, s));
    DS_HIP(hipEventRecord(C.evu, s));
    hipLaunchKernelGGL(k_b_assign, dim3((n + TB - 1) / TB), dim3(TB), 0, s, d_perm, d_lam,
                       static_cast<const int*>(d_list), reinterpret_cast<const int*>(base + l.asig),
                       reinterpret_cast<const double*>(base + l.alam), n);
    DS_HIP(hipGetLastError());
    return DS_OK;
  };
  if ((e = assign(l.Bp)) != DS_OK) return e;

  // ---------------------------------------------------------------- setup
  StatAccum& S = stats();
  bool stat_on;
  {
    std::lock_guard<std::mutex> g(S.mu);
    stat_on = S.on;
  }
  hipEvent_t su0 = nullptr, su1 = nullptr;
  if (stat_on) {
    DS_HIP(hipEventCreate(&su0));
    DS_HIP(hipEventCreate(&su1));
    DS_HIP(hipEventRecord(su0, s));
  }
  DS_HIP(hipMemsetAsync(base + l.ctr, 0, 4 * sizeof(int), s));
  uint16_t* dcm = reinterpret_cast<uint16_t*>(base + l.dcm);
  hipLaunchKernelGGL(k_b_prep, dim3(l.Kp, (l.Np + TB - 1) / TB), dim3(TB), 0, s,
                     static_cast<const uint16_t*>(P.D), P.ldd, l.N, l.K, l.Np, dcm);
  hipLaunchKernelGGL(k_b_norms, dim3(l.Kp / NWB), dim3(TB), 0, s, dcm, l.Np, l.Kp,
                     reinterpret_cast<double*>(base + l.nu));
  // groups: offsets, the group of each atom and the weights (default sqrt(|g|)) from the
  // host, the group norms of the stored values on the device
  std::vector<int64_t> h_gptr;
  std::vector<int> h_agrp;
  std::vector<double> h_gw;
  if (l.G > 0) {
    h_gptr.assign(P.group_ptr, P.group_ptr + l.G + 1);
    h_agrp.assign(l.Kp, -1);
    h_gw.resize(l.G);
    int mmax = 1;
    for (int g = 0; g < l.G; ++g) {
      for (int64_t k = h_gptr[g]; k < h_gptr[g + 1]; ++k) h_agrp[k] = g;
      mmax = std::max(mmax, static_cast<int>(h_gptr[g + 1] - h_gptr[g]));
      h_gw[g] = P.w != nullptr ? P.w[g] : std::sqrt(static_cast<double>(h_gptr[g + 1] - h_gptr[g]));
    }
    DS_HIP(hipMemcpyAsync(base + l.gptr, h_gptr.data(), h_gptr.size() * 8, hipMemcpyHostToDevice, s));
    DS_HIP(hipMemcpyAsync(base + l.agrp, h_agrp.data(), h_agrp.size() * 4, hipMemcpyHostToDevice, s));
    DS_HIP(hipMemcpyAsync(base + l.gw, h_gw.data(), h_gw.size() * 8, hipMemcpyHostToDevice, s));
    if ((e = group_norms_bf16(dcm, l.Np, l.N, l.G, reinterpret_cast<const int64_t*>(base + l.gptr),
                              mmax, reinterpret_cast<double*>(base + l.gspec),
                              reinterpret_cast<double*>(base + l.gfro), s)) != DS_OK)
      return e;
    hipLaunchKernelGGL(k_b_gdict_scalars, dim3(1), dim3(TB), 0, s, a,
                       reinterpret_cast<double*>(base + l.dsc));
  } else {
    hipLaunchKernelGGL(k_b_dict_scalars, dim3(1), dim3(TB), 0, s,
                       reinterpret_cast<const double*>(base + l.nu), l.K,
                       reinterpret_cast<double*>(base + l.dsc));
  }
  double* z0 = reinterpret_cast<double*>(base + l.z0);
  double* gn = reinterpret_cast<double*>(base + l.gn);
  float* Vn = reinterpret_cast<float*>(base + l.Vn);
  float* Yp = reinterpret_cast<float*>(base + l.Y);
  // per-slot set-up of the first n entries of d_list, of which the first nact hold signals
  // (the rest are idle slots, which need no products): y, cleared x / u / masks, D^T y,
  // lambda_* and the centre, D^T n (DST3), margins and their tile minima
  auto setup_slots = [&](int n, int nact) -> ds_status {
    hipLaunchKernelGGL(k_b_load_slots, dim3(std::max(1, (l.Kp + TB - 1) / TB), n), dim3(TB), 0, s, a,
                       Y, ldy, static_cast<const int*>(d_perm), static_cast<const int*>(d_list), Yp);
    // FP64 D^T v for the listed slots (tiles of 16 atoms x 16 slots on the matrix cores)
    auto dtv = [&](const auto* V, double* out) {
      using VT = std::remove_const_t<std::remove_pointer_t<decltype(V)>>;
      if (nact > 0)
        hipLaunchKernelGGL((k_b_dtv<VT>), dim3(l.Kp / 16, (nact + 15) / 16), dim3(TB), 0, s, dcm,
                           V, l.Np, l.Kp, out, static_cast<const int*>(d_list), nact);
    };
    dtv(a.Y, z0);
    const int lrel = prm.lambda_mode == DS_LAMBDA_RELATIVE ? 1 : 0;
    if (l.G > 0) {
      double* Vd = reinterpret_cast<double*>(base + l.Vd);
      hipLaunchKernelGGL(k_b_ginst_init, dim3(n), dim3(TB), 0, s, a, z0, d_lam, lrel, prm.gap_tol,
                         Vd, static_cast<const int*>(d_perm), static_cast<const int*>(d_list));
      if (prm.test == DS_TEST_DST3) dtv(static_cast<const double*>(Vd), gn);
      hipLaunchKernelGGL(k_b_gmargins, dim3((std::max(l.G, l.Kp) + TB - 1) / TB, n), dim3(TB), 0, s,
                         a, z0, gn, reinterpret_cast<float*>(base + l.marg),
                         static_cast<const int*>(d_perm), static_cast<const int*>(d_list));
    } else {
      hipLaunchKernelGGL(k_b_inst_init, dim3(n), dim3(TB), 0, s, a, z0, d_lam, lrel, prm.gap_tol,
                         Vn, static_cast<const int*>(d_perm), static_cast<const int*>(d_list));
      if (prm.test == DS_TEST_DST3 || prm.test == DS_TEST_DOME) dtv(static_cast<const float*>(Vn), gn);
      hipLaunchKernelGGL(k_b_margins, dim3((l.Kp + TB - 1) / TB, n), dim3(TB), 0, s, a, z0, gn,
                         reinterpret_cast<float*>(base + l.marg), static_cast<const int*>(d_perm),
                         static_cast<const int*>(d_list));
    }
    hipLaunchKernelGGL(k_b_tile_min, dim3((l.Kp / MT + TB - 1) / TB, n), dim3(TB), 0, s, a,
                       reinterpret_cast<float*>(base + l.tminm), static_cast<const int*>(d_list));
    DS_HIP(hipGetLastError());
    return DS_OK;
  };
  if ((e = setup_slots(l.Bp, n0)) != DS_OK) return e;
  if (stat_on) DS_HIP(hipEventRecord(su1, s));

  // ---------------------------------------------------------------- iteration
  const dim3 g_theta(l.nrb, l.Bp);
  // block shape of the Z-GEMM; tuning needs the first theta (theta_1 = -y; the first
  // iteration recomputes it identically)
  int shape = -1;
  {
    const auto key = std::make_tuple(l.N, l.K, l.B);
    if (std::getenv("DS_BATCH_TILE") == nullptr && C.tuned.find(key) == C.tuned.end()) {
      hipLaunchKernelGGL(k_b_theta, g_theta, dim3(TB), 0, s, a, static_cast<const float*>(a.U0));
      DS_HIP(hipGetLastError());
    }
    shape = choose_shape(C, l, base, a, s, C.tune0, C.tune1);
    DS_HIP(hipGetLastError());
    C.last_shape = shape;
  }
  const dim3 g_slot4(l.Bp / NWB);
  const dim3 g_vca((l.K + VC - 1) / VC, VG), g_vdot(512);
  const dim3 g_scr((l.Kp / 4 + TB - 1) / TB, l.Bp);
  std::vector<std::pair<hipEvent_t, hipEvent_t>> evz, evt;
  // instrumented runs: every Z-GEMM wave stamps the device wall clock at its start and
  // end; a one-block pass after the launch reduces the stamps to the launch's span
  uint64_t* spans = reinterpret_cast<uint64_t*>(base + l.spans);
  int nspan = 0;
  const ZShapeDesc& zs = ZSHAPES[shape];
  const int zwaves = (l.Kp / (MT * zs.ra * zs.wa)) * (l.Bp / (MT * zs.rb * zs.wb)) * zs.ra * zs.rb;
  if (stat_on) a.kclk = reinterpret_cast<uint64_t*>(base + l.kclk);
  auto events = [&]() -> std::pair<hipEvent_t, hipEvent_t> {
    if (C.ev_used == C.evpool.size()) {
      hipEvent_t e0, e1;
      if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return {nullptr, nullptr};
      C.evpool.push_back({e0, e1});
    }
    return C.evpool[C.ev_used++];
  };
  auto iteration = [&](int t, bool timed) {
    float* Uin = (t % 2 == 1) ? a.U0 : a.U1;
    float* Uout = (t % 2 == 1) ? a.U1 : a.U0;
    std::pair<hipEvent_t, hipEvent_t> et{nullptr, nullptr}, ez{nullptr, nullptr};
    if (timed) { et = events(); ez = events(); }
    // instrumented launches carry start/stop events in the dispatch itself
    if (timed)
      hipExtLaunchKernelGGL(k_b_theta, g_theta, dim3(TB), 0, s, et.first, et.second, 0, a,
                            static_cast<const float*>(Uin));
    else
      hipLaunchKernelGGL(k_b_theta, g_theta, dim3(TB), 0, s, a, static_cast<const float*>(Uin));
    launch_zgemm(shape, l, s, timed ? ez.first : nullptr, timed ? ez.second : nullptr, a, Uin,
                 Uout);
    if (timed && nspan < l.nspan) {
      hipLaunchKernelGGL(k_clock_span<0>, dim3(1), dim3(256), 0, s, a.kclk, zwaves, spans + nspan);
      ++nspan;
    }
    if (l.G > 0)
      hipLaunchKernelGGL(k_b_gprox, dim3((l.G + TB - 1) / TB, l.Bp), dim3(TB), 0, s, a,
                         static_cast<const float*>(Uin), Uout);
    hipLaunchKernelGGL(k_b_scalars, dim3(l.Bp / 16), dim3(TB), 0, s, a);
    if (l.G > 0) {
      hipLaunchKernelGGL(k_b_gvcand, g_vca, dim3(TB), 0, s, a);
      hipLaunchKernelGGL(k_b_gvdot, g_vdot, dim3(TB), 0, s, a);
    } else {
      hipLaunchKernelGGL(k_b_vcand, g_vca, dim3(TB), 0, s, a);
      hipLaunchKernelGGL(k_b_vdot, g_vdot, dim3(TB), 0, s, a);
    }
    hipLaunchKernelGGL(k_b_vfin, g_slot4, dim3(TB), 0, s, a);
    hipLaunchKernelGGL(k_b_screen, g_scr, dim3(TB), 0, s, a);
    if (timed && et.first) { evt.push_back(et); evz.push_back(ez); }
  };

  if (!stat_on &&
      (C.exec == nullptr || std::memcmp(&C.key, &a, sizeof a) != 0 || C.key_shape != shape)) {
    if (C.exec != nullptr) {
      DS_HIP(hipGraphExecDestroy(C.exec));
      C.exec = nullptr;
    }
    hipGraph_t graph;
    DS_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (int k = 1; k <= ITERS_PER_GRAPH; ++k) iteration(k, false);
    const hipError_t ce = hipGetLastError();
    DS_HIP(hipStreamEndCapture(s, &graph));
    DS_HIP(ce);
    const hipError_t ie = hipGraphInstantiate(&C.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
      C.exec = nullptr;
      DS_HIP(ie);
    }
    C.key = a;
    C.key_shape = shape;
  }
  if (stat_on) C.ev_used = 0;

  // Runs of ITERS_PER_GRAPH iterations (graph replays, or direct launches when instrumented)
  // while any slot holds a signal.  After each run the device harvests the signals that
  // finished (counts, x into column perm[k] of X, the screened mask) and the harvest flags
  // and slot states go to the host; the finished signals report (the feed's finish) and
  // free slots take the signals the feed has waiting.  When the feed had nothing waiting
  // at the last pull, the next run is enqueued before the host waits for the current one
  // (finished signals are frozen and harvested once, so the extra run only delays the
  // refill of their slots); instrumented runs do not overlap.
  int* d_flag = reinterpret_cast<int*>(base + l.dflag);
  std::vector<int> fcols;
  std::vector<ds_info> finfo;
  double act = 0.0, sup = 0.0;  // work of the finished signals (statistics)
  int nactive = n0;             // slots holding a signal
  int t = 0;
  auto enqueue_run = [&](int buf) -> ds_status {
    if (stat_on) {
      for (int k = 0; k < ITERS_PER_GRAPH; ++k) iteration(++t, true);
      DS_HIP(hipGetLastError());
    } else {
      DS_HIP(hipGraphLaunch(C.exec, s));
      t += ITERS_PER_GRAPH;
    }
    int* fl = d_flag + buf * l.Bp;
    hipLaunchKernelGGL(k_b_harvest, dim3(l.Bp), dim3(TB), 0, s, a, d_perm, X, ldx, screened, fl);
    DS_HIP(hipGetLastError());
    DS_HIP(hipMemcpyAsync(h_flag[buf], fl, bp * sizeof(int), hipMemcpyDeviceToHost, s));
    DS_HIP(hipMemcpyAsync(h_inst[buf], a.inst, bp * sizeof(Inst), hipMemcpyDeviceToHost, s));
    DS_HIP(hipEventRecord(C.evh[buf], s));
    return DS_OK;
  };
  // the host's part of a run whose results are in buffer buf
  auto collect = [&](int buf) -> ds_status {
    DS_HIP(hipEventSynchronize(C.evh[buf]));
    fcols.clear();
    finfo.clear();
    for (int k = 0; k < l.Bp; ++k) {
      if (h_flag[buf][k] == 0) continue;
      fcols.push_back(slot_sig[k]);
      finfo.push_back(info_of(h_inst[buf][k], L));
      act += h_inst[buf][k].act_sum;
      sup += h_inst[buf][k].sup_sum;
      slot_sig[k] = -1;
      --nactive;
    }
    if (!fcols.empty()) feed.finish(fcols.data(), finfo.data(), static_cast<int>(fcols.size()), s);
    return DS_OK;
  };
  bool waiting = true;  // the feed may have signals waiting
  int cur = 0;
  if ((e = enqueue_run(cur)) != DS_OK) return e;
  for (;;) {
    const bool ahead = !stat_on && !waiting;
    if (ahead && (e = enqueue_run(cur ^ 1)) != DS_OK) return e;
    if ((e = collect(cur)) != DS_OK) return e;
    const int room = nslot - nactive;
    const int got = room > 0 ? feed.pull(room, cols.data(), lams.data(), s) : 0;
    if (room > 0) waiting = got == room;  // (no room: as after the last pull)
    if (got > 0) {
      DS_HIP(hipEventSynchronize(C.evu));  // the staging of the previous assignment is free
      int nref = 0;
      for (int k = 0, q = 0; k < nslot && q < got; ++k) {
        if (slot_sig[k] >= 0) continue;
        slot_sig[k] = cols[q];
        h_list[nref] = k;
        h_asig[nref] = cols[q];
        h_alam[nref] = lams[q];
        ++nref;
        ++q;
      }
      nactive += got;
      if ((e = assign(nref)) != DS_OK) return e;
      if ((e = setup_slots(got, got)) != DS_OK) return e;
    }
    cur ^= 1;
    if (ahead) {
      if (nactive == 0) {  // the run enqueued ahead found nothing to do
        if ((e = collect(cur)) != DS_OK) return e;
        break;
      }
    } else {
      if (nactive == 0) break;
      if ((e = enqueue_run(cur)) != DS_OK) return e;
    }
  }
  DS_HIP(hipStreamSynchronize(s));

  if (stat_on) {
    double ms_z = 0.0, ms_zev = 0.0, ms_t = 0.0, ms_s = 0.0;
    std::vector<uint64_t> ticks(nspan);
    int rate_khz = 0;
    DS_HIP(hipMemcpy(ticks.data(), spans, nspan * sizeof(uint64_t), hipMemcpyDeviceToHost));
    DS_HIP(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev));
    for (uint64_t tk : ticks) if (rate_khz > 0) ms_z += static_cast<double>(tk) / rate_khz;
    for (auto& p : evz) { float m = 0.f; if (hipEventElapsedTime(&m, p.first, p.second) == hipSuccess) ms_zev += m; }
    for (auto& p : evt) { float m = 0.f; if (hipEventElapsedTime(&m, p.first, p.second) == hipSuccess) ms_t += m; }
    { float m = 0.f; if (hipEventElapsedTime(&m, su0, su1) == hipSuccess) ms_s = m; }
    std::lock_guard<std::mutex> g(S.mu);
    // algorithmic work: 2 N flops per active (atom, signal) pair for Z, per support entry
    // of the primal point for Theta; bytes: D once plus the per-signal vectors
    ds_kernel_stat& z = S.s[DS_STAT_BATCH];
    z.launches += static_cast<int64_t>(nspan);
    z.ms += ms_z;
    z.ms_event += ms_zev;
    z.flops += 2.0 * l.N * act;
    z.bytes += static_cast<double>(nspan) * (2.0 * l.N * l.K) + 22.0 * act;
    ds_kernel_stat& th = S.s[DS_STAT_BATCH_THETA];
    th.launches += static_cast<int64_t>(evt.size());
    th.ms += ms_t;
    th.ms_event += ms_t;
    th.flops += 2.0 * l.N * sup;
    th.bytes += 2.0 * l.N * sup + static_cast<double>(evt.size()) * 26.0 * l.N * l.B;
    S.s[DS_STAT_SETUP].launches += 1;
    S.s[DS_STAT_SETUP].ms += ms_s;
  }
  if (su0) (void)hipEventDestroy(su0);
  if (su1) (void)hipEventDestroy(su1);

  return DS_OK;
}

ds_status solve_batched_bf16(const ds_problem& P, const void* Y, int64_t B, int64_t ldy,
                             const double* lambdas, const ds_params& prm, void* X, int64_t ldx,
                             ds_info* info, uint8_t* screened, hipStream_t stream) {
  // resident slots: all signals up to MAX_SLOTS, or the caller's batch_slots; the rest wait
  // and take the slots of finished signals (continuous batching)
  const int64_t want = prm.batch_slots > 0 ? prm.batch_slots : std::min<int64_t>(B, MAX_SLOTS);
  const int64_t nslot = std::min<int64_t>(want, B);
  if (nslot > 32768 || B > (int64_t(1) << 30)) {
    set_error("batched path: batch_slots must be <= 32768 and B <= 2^30");
    return DS_EINVAL;
  }
  // signals in order of increasing penalty: neighbouring slots hold signals that finish
  // together (whole tiles fall idle), and when signals wait for slots the slow ones (small
  // lambda needs the most iterations) start first, which keeps the end of the run short
  std::vector<int> order(B);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int i, int j) { return lambdas[i] < lambdas[j]; });
  for (int64_t b = 0; b < B; ++b) std::memset(&info[b], 0, sizeof(ds_info));
  int64_t next = 0;
  bool bad = false;
  ds_status worst = DS_OK;
  BatchFeed feed;
  feed.pull = [&](int room, int* cols, double* lams, hipStream_t) {
    int n = 0;
    for (; n < room && next < B; ++n, ++next) {
      cols[n] = order[next];
      lams[n] = lambdas[order[next]];
    }
    return n;
  };
  feed.finish = [&](const int* cols, const ds_info* inf, int n, hipStream_t) {
    for (int j = 0; j < n; ++j) {
      info[cols[j]] = inf[j];
      if (inf[j].status == DS_EINVAL) bad = true;
      if (inf[j].status == DS_NOT_CONVERGED) worst = DS_NOT_CONVERGED;
    }
  };
  int dev = 0;
  DS_HIP(hipGetDevice(&dev));
  const ds_status e = run_batched(batch_ctx(dev), P, static_cast<const float*>(Y), ldy,
                                  static_cast<int>(nslot), prm, static_cast<float*>(X), ldx,
                                  screened, feed, stream);
  if (e < 0) return e;
  if (bad) {
    set_error("observation contains NaN or Inf");
    return DS_EINVAL;
  }
  return worst;
}

}  // namespace ds

extern "C" int ds_batch_shape(int* atoms, int* signals) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  ds::BatchEngine& C = ds::batch_ctx(dev);
  std::lock_guard<std::mutex> g(C.mu);
  const int k = C.last_shape;
  if (k >= 0) {
    const ds::batch::ZShapeDesc& z = ds::batch::ZSHAPES[k];
    if (atoms != nullptr) *atoms = ds::batch::MT * z.ra * z.wa;
    if (signals != nullptr) *signals = ds::batch::MT * z.rb * z.wb;
  }
  return k;
}
