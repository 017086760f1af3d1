// Serving: a continuous request loop over resident dictionaries.
//
// Dictionaries are copied into server-owned device memory at registration (column-major,
// leading dimension padded to 16 bytes, optionally rounded from FP32 to bfloat16) with
// ||D||_2^2 computed once.  Requests carry y on the host and wait in a queue.  Each of
// max_slots worker threads owns a HIP stream, a solver workspace and device buffers for
// y and x; a worker takes the oldest queued request whose device footprint fits the part
// of the HBM budget not held by the other workers, so requests are admitted as slots and
// memory free up, and the resident requests' kernels run concurrently on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ds_engine.h"

namespace ds {
namespace {

using Clock = std::chrono::steady_clock;

constexpr int SKIP_SCAN = 64;    // queued requests a worker looks at for one that fits
constexpr int SKIP_LIMIT = 16;   // a request passed over this often blocks later ones

// RNE rounding of FP32 columns to bfloat16 with a new leading dimension.
__global__ void k_f32_to_bf16(const float* __restrict__ src, int64_t lds, uint16_t* __restrict__ dst,
                              int64_t ldd, int64_t N, int64_t K) {
  const int64_t i = blockIdx.y;
  for (int64_t n = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; n < N;
       n += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const uint32_t u = __float_as_uint(src[i * lds + n]);
    const uint32_t lsb = (u >> 16) & 1u;
    dst[i * ldd + n] = static_cast<uint16_t>((u + 0x7fffu + lsb) >> 16);
  }
}

struct Dict {
  ds_dtype store;
  int64_t N, K, G, ldd;
  void* D = nullptr;
  std::vector<int64_t> gptr;
  std::vector<double> w;
  bool has_w = false;
  double L = 0.0;
  ds_problem view() const {
    ds_problem p{};
    p.dtype = store;
    p.N = N;
    p.K = K;
    p.ldd = ldd;
    p.D = D;
    p.G = G;
    p.group_ptr = G > 0 ? gptr.data() : nullptr;
    p.w = has_w ? w.data() : nullptr;
    return p;
  }
};

enum ReqState { QUEUED, RUNNING, DONE };

struct Request {
  uint64_t id;
  int dict;
  std::vector<char> y, x, x0;  // x0: the warm start when one was given (else empty)
  double lam;
  ds_params prm;
  size_t need;  // device bytes while it runs
  int skipped = 0;
  ReqState state = QUEUED;
  ds_status status = DS_OK;
  ds_info info{};
  std::string error;
  Clock::time_point t_submit, t_start, t_end;
};

struct Worker {
  std::thread th;
  hipStream_t stream = nullptr;
  Workspace ws;
  void* io = nullptr;
  size_t io_bytes = 0;
  size_t held = 0;  // device bytes charged to the budget for this worker
};

size_t vec_size(ds_dtype t) { return t == DS_F64 ? 8 : 4; }
size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Device bytes a worker holds to run request r: the solver workspace (reserved with the
// 25% headroom Workspace::reserve adds) plus y, x and the warm start.
size_t request_need(const Dict& d, const ds_params& prm) {
  const size_t ws = single_workspace_bytes(d.view(), prm);
  const size_t xb = align256(d.K * vec_size(d.store));
  const size_t io = align256(d.N * vec_size(d.store)) + xb + (prm.x0 != nullptr ? xb : 0);
  return ws + ws / 4 + io;
}

}  // namespace

struct Server {
  ds_server_config cfg{};
  std::mutex mu;
  std::condition_variable cv_work;
  std::map<int, std::unique_ptr<Dict>> dicts;
  int next_dict = 0;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  uint64_t next_id = 1;
  size_t held = 0;  // sum of the workers' charged bytes
  bool stop = false;
  // Failure injection for tests of the failure path: the request with this id (0: none,
  // read from DS_SERVE_FAIL_REQUEST at creation) has its slot marked failed after its solve
  // ran; it completes with DS_EDEVICE and no x, the other requests are unaffected.  Host
  // side only: no device fault is involved.
  uint64_t fail_request = 0;
  std::vector<std::unique_ptr<Worker>> workers;
  hipStream_t admin = nullptr;  // registration work

  void worker_loop(Worker* w);
  void run(Worker* w, Request* r, const Dict& d);
};

void Server::run(Worker* w, Request* r, const Dict& d) {
  const ds_problem P = d.view();
  const size_t vsz = vec_size(d.store);
  const size_t yb = align256(d.N * vsz), xb = align256(d.K * vsz);
  const size_t x0b = r->x0.empty() ? 0 : xb;
  auto fail = [&](ds_status st) {
    r->status = st;
    r->error = ds_last_error();
  };
  if (w->io_bytes < yb + xb + x0b) {
    if (w->io != nullptr) {
      (void)hipStreamSynchronize(w->stream);
      (void)hipFree(w->io);
      w->io = nullptr;
      w->io_bytes = 0;
    }
    if (hipMalloc(&w->io, yb + xb + x0b) != hipSuccess) {
      (void)hipGetLastError();
      set_error("hipMalloc of %zu request bytes failed", yb + xb + x0b);
      return fail(DS_ENOMEM);
    }
    w->io_bytes = yb + xb + x0b;
  }
  char* y = static_cast<char*>(w->io);
  char* x = y + yb;
  char* x0 = x + xb;
  if (hipMemcpyAsync(y, r->y.data(), d.N * vsz, hipMemcpyHostToDevice, w->stream) != hipSuccess ||
      (x0b > 0 && hipMemcpyAsync(x0, r->x0.data(), d.K * vsz, hipMemcpyHostToDevice, w->stream) !=
                      hipSuccess)) {
    set_error("upload of y or x0 failed");
    return fail(DS_EDEVICE);
  }
  ds_params prm = r->prm;
  prm.x0 = x0b > 0 ? x0 : nullptr;
  if (!(prm.step_L > 0.0) && prm.step_rule == DS_STEP_CONSTANT && prm.rule != DS_SPARSA)
    prm.step_L = d.L;
  ds_info info{};
  const ds_status st = solve_single(P, y, r->lam, prm, x, &info, w->stream, w->ws, nullptr);
  if (st < 0) return fail(st);
  if (r->id == fail_request) {
    (void)hipStreamSynchronize(w->stream);
    set_error("the slot of request %llu was marked failed (DS_SERVE_FAIL_REQUEST)",
              static_cast<unsigned long long>(r->id));
    return fail(DS_EDEVICE);
  }
  r->x.resize(d.K * vsz);
  if (hipMemcpyAsync(r->x.data(), x, d.K * vsz, hipMemcpyDeviceToHost, w->stream) != hipSuccess ||
      hipStreamSynchronize(w->stream) != hipSuccess) {
    set_error("download of x failed");
    return fail(DS_EDEVICE);
  }
  r->info = info;
  r->status = st;
}

void Server::worker_loop(Worker* w) {
  (void)hipSetDevice(cfg.device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    Request* pick = nullptr;
    size_t grow_to = 0;
    while (!stop) {
      // oldest queued request whose footprint fits next to what the other workers hold
      int scanned = 0;
      for (auto it = queue.begin(); it != queue.end() && scanned < SKIP_SCAN; ++it, ++scanned) {
        Request* r = reqs[*it].get();
        const size_t want = std::max(w->held, r->need);
        if (held - w->held + want <= cfg.hbm_budget_bytes) {
          pick = r;
          grow_to = want;
          queue.erase(it);
          break;
        }
        if (++r->skipped > SKIP_LIMIT) break;  // no overtaking a long-waiting request
      }
      if (pick != nullptr) break;
      if (!queue.empty() && w->held > 0) {
        // nothing queued fits next to what the workers hold: give this worker's memory
        // back so that a waiting request can be admitted by whoever has room
        const size_t h = w->held;
        lk.unlock();
        (void)hipStreamSynchronize(w->stream);
        w->ws.release();
        if (w->io != nullptr) (void)hipFree(w->io);
        w->io = nullptr;
        w->io_bytes = 0;
        lk.lock();
        held -= h;
        w->held = 0;
        cv_work.notify_all();
        continue;
      }
      cv_work.wait(lk);
    }
    if (stop) return;
    held += grow_to - w->held;
    w->held = grow_to;
    pick->state = RUNNING;
    pick->t_start = Clock::now();
    const Dict& d = *dicts.at(pick->dict);
    lk.unlock();
    run(w, pick, d);
    lk.lock();
    pick->t_end = Clock::now();
    pick->state = DONE;
    cv_work.notify_all();
  }
}

namespace {

Server* as_server(void* s) { return static_cast<Server*>(s); }

ds_status submit_impl(void* server, int32_t dict_id, const void* y_host, double lambda,
                      const ds_params* params, uint64_t* request_id) {
  Server* S = as_server(server);
  if (S == nullptr || y_host == nullptr || request_id == nullptr) {
    set_error("server, y_host and request_id must be non-NULL");
    return DS_EINVAL;
  }
  ds_status e = validate_params(params);
  if (e != DS_OK) return e;
  if (!(lambda > 0.0) || !std::isfinite(lambda)) {
    set_error("lambda must be positive and finite");
    return DS_EINVAL;
  }
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->dicts.find(dict_id);
  if (it == S->dicts.end()) {
    set_error("unknown dictionary id %d", dict_id);
    return DS_ENOTFOUND;
  }
  const Dict& d = *it->second;
  if ((e = validate_test_for(params, d.G > 0)) != DS_OK) return e;
  if (static_cast<int64_t>(S->queue.size()) >= S->cfg.max_queue) {
    set_error("request queue full (%d waiting)", S->cfg.max_queue);
    return DS_EBUSY;
  }
  const size_t need = request_need(d, *params);
  if (need > S->cfg.hbm_budget_bytes) {
    set_error("request needs %zu device bytes, budget is %zu", need, S->cfg.hbm_budget_bytes);
    return DS_ENOMEM;
  }
  auto r = std::make_unique<Request>();
  r->id = S->next_id++;
  r->dict = dict_id;
  const size_t vsz = vec_size(d.store);
  r->y.assign(static_cast<const char*>(y_host), static_cast<const char*>(y_host) + d.N * vsz);
  if (params->x0 != nullptr)
    r->x0.assign(static_cast<const char*>(params->x0), static_cast<const char*>(params->x0) + d.K * vsz);
  r->lam = lambda;
  r->prm = *params;
  r->prm.x0 = nullptr;  // the copy above is uploaded by the worker
  r->need = need;
  r->t_submit = Clock::now();
  *request_id = r->id;
  S->queue.push_back(r->id);
  S->reqs.emplace(r->id, std::move(r));
  // every worker looks: an idle worker that still holds memory must see a request that
  // does not fit next to it (and give the memory back), which a worker holding nothing
  // woken alone would leave waiting
  S->cv_work.notify_all();
  return DS_OK;
}

}  // namespace
}  // namespace ds

using namespace ds;

extern "C" {

ds_status ds_server_create(const ds_server_config* config, void** server) {
  if (config == nullptr || server == nullptr) {
    set_error("config and server must be non-NULL");
    return DS_EINVAL;
  }
  if (config->max_slots < 1 || config->max_queue < 1 || config->hbm_budget_bytes == 0 ||
      config->reserved != 0 || config->device < 0) {
    set_error("bad server config (max_slots >= 1, max_queue >= 1, budget > 0, reserved = 0)");
    return DS_EINVAL;
  }
  int ndev = 0;
  DS_HIP(hipGetDeviceCount(&ndev));
  if (config->device >= ndev) {
    set_error("device %d not present", config->device);
    return DS_EINVAL;
  }
  DS_HIP(hipSetDevice(config->device));
  auto S = std::make_unique<Server>();
  S->cfg = *config;
  if (const char* f = std::getenv("DS_SERVE_FAIL_REQUEST")) S->fail_request = std::strtoull(f, nullptr, 10);
  DS_HIP(hipStreamCreateWithFlags(&S->admin, hipStreamNonBlocking));
  for (int k = 0; k < config->max_slots; ++k) {
    auto w = std::make_unique<Worker>();
    w->ws.device = config->device;
    DS_HIP(hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking));
    S->workers.push_back(std::move(w));
  }
  for (auto& w : S->workers) {
    Worker* wp = w.get();
    Server* sp = S.get();
    w->th = std::thread([sp, wp] { sp->worker_loop(wp); });
  }
  *server = S.release();
  return DS_OK;
}

ds_status ds_server_add_dict(void* server, const ds_problem* problem, ds_dtype store,
                             int32_t* dict_id) {
  Server* S = as_server(server);
  if (S == nullptr || dict_id == nullptr) {
    set_error("server and dict_id must be non-NULL");
    return DS_EINVAL;
  }
  const bool group = problem != nullptr && problem->G > 0;
  ds_status e = validate_problem(problem, group);
  if (e != DS_OK) return e;
  const bool convert = problem->dtype == DS_F32 && store == DS_BF16;
  if (store != problem->dtype && !convert) {
    set_error("store precision must equal the input's, or be DS_BF16 for DS_F32 input");
    return DS_EINVAL;
  }
  DS_HIP(hipSetDevice(S->cfg.device));
  auto d = std::make_unique<Dict>();
  d->store = store;
  d->N = problem->N;
  d->K = problem->K;
  d->G = problem->G;
  const size_t tsz = dtype_size(store), isz = dtype_size(problem->dtype);
  const int64_t per16 = static_cast<int64_t>(16 / tsz);
  d->ldd = (problem->N + per16 - 1) / per16 * per16;
  if (group) {
    d->gptr.assign(problem->group_ptr, problem->group_ptr + problem->G + 1);
    if (problem->w != nullptr) {
      d->w.assign(problem->w, problem->w + problem->G);
      d->has_w = true;
    }
  }
  hipPointerAttribute_t attr{};
  const bool on_device = hipPointerGetAttributes(&attr, problem->D) == hipSuccess &&
                         attr.type == hipMemoryTypeDevice;
  (void)hipGetLastError();
  if (hipMalloc(&d->D, static_cast<size_t>(d->ldd) * d->K * tsz) != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipMalloc of the dictionary failed");
    return DS_ENOMEM;
  }
  hipStream_t s = S->admin;
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  ds_status st = DS_OK;
  void* stage = nullptr;
  if (!convert) {
    if (hipMemcpy2DAsync(d->D, d->ldd * tsz, problem->D, problem->ldd * isz, problem->N * isz,
                         problem->K, kind, s) != hipSuccess)
      st = DS_EDEVICE;
  } else {
    const float* src = static_cast<const float*>(problem->D);
    int64_t lds = problem->ldd;
    if (!on_device) {
      if (hipMalloc(&stage, static_cast<size_t>(problem->N) * problem->K * 4) != hipSuccess ||
          hipMemcpy2DAsync(stage, problem->N * 4, problem->D, problem->ldd * 4, problem->N * 4,
                           problem->K, hipMemcpyHostToDevice, s) != hipSuccess) {
        st = DS_EDEVICE;
      }
      src = static_cast<const float*>(stage);
      lds = problem->N;
    }
    if (st == DS_OK) {
      const int gx = static_cast<int>(std::min<int64_t>((problem->N + 255) / 256, 64));
      hipLaunchKernelGGL(k_f32_to_bf16, dim3(gx, static_cast<unsigned>(problem->K)), dim3(256), 0, s,
                         src, lds, static_cast<uint16_t*>(d->D), d->ldd, problem->N, problem->K);
      if (hipGetLastError() != hipSuccess) st = DS_EDEVICE;
    }
  }
  if (st == DS_OK) {
    Workspace tmp;
    tmp.device = S->cfg.device;
    st = spectral_norm_impl(d->view(), 0, &d->L, s, tmp);
    tmp.release();
  } else {
    set_error("copy of the dictionary failed");
  }
  if (hipStreamSynchronize(s) != hipSuccess && st == DS_OK) st = DS_EDEVICE;
  if (stage != nullptr) (void)hipFree(stage);
  if (st != DS_OK) {
    (void)hipFree(d->D);
    return st;
  }
  std::lock_guard<std::mutex> g(S->mu);
  *dict_id = S->next_dict++;
  S->dicts.emplace(*dict_id, std::move(d));
  return DS_OK;
}

ds_status ds_submit(void* server, int32_t dict_id, const void* y_host, double lambda,
                    const ds_params* params, uint64_t* request_id) {
  return submit_impl(server, dict_id, y_host, lambda, params, request_id);
}

ds_status lasso_submit(void* server, int32_t dict_id, const void* y_host, double lambda,
                       const ds_params* params, uint64_t* request_id) {
  return submit_impl(server, dict_id, y_host, lambda, params, request_id);
}

ds_status lasso_poll(void* server, uint64_t request_id, void* x_host, ds_info* info) {
  Server* S = as_server(server);
  if (S == nullptr) {
    set_error("server must be non-NULL");
    return DS_EINVAL;
  }
  std::unique_ptr<Request> r;
  {
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->reqs.find(request_id);
    if (it == S->reqs.end()) {
      set_error("unknown request id %llu", static_cast<unsigned long long>(request_id));
      return DS_ENOTFOUND;
    }
    if (it->second->state != DONE) return DS_PENDING;
    r = std::move(it->second);
    S->reqs.erase(it);
  }
  if (r->status < 0) {
    set_error("%s", r->error.c_str());
    return r->status;
  }
  if (x_host != nullptr) std::memcpy(x_host, r->x.data(), r->x.size());
  if (info != nullptr) {
    *info = r->info;
    info->queue_ms = std::chrono::duration<double, std::milli>(r->t_start - r->t_submit).count();
    info->run_ms = std::chrono::duration<double, std::milli>(r->t_end - r->t_start).count();
  }
  return r->status;
}

ds_status ds_server_destroy(void* server) {
  Server* S = as_server(server);
  if (S == nullptr) {
    set_error("server must be non-NULL");
    return DS_EINVAL;
  }
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  for (auto& w : S->workers)
    if (w->th.joinable()) w->th.join();
  (void)hipSetDevice(S->cfg.device);
  for (auto& w : S->workers) {
    if (w->stream != nullptr) (void)hipStreamSynchronize(w->stream);
    w->ws.release();
    if (w->io != nullptr) (void)hipFree(w->io);
    if (w->stream != nullptr) (void)hipStreamDestroy(w->stream);
  }
  for (auto& kv : S->dicts) (void)hipFree(kv.second->D);
  if (S->admin != nullptr) (void)hipStreamDestroy(S->admin);
  delete S;
  return DS_OK;
}

}  // extern "C"
