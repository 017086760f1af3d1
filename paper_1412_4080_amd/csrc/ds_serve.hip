// Serving: a continuous request loop over resident dictionaries.
//
// Dictionaries are copied into server-owned device memory at registration (column-major,
// leading dimension padded to 16 bytes, optionally rounded from FP32 to bfloat16) with
// ||D||_2^2 computed once.  Requests carry y on the host and wait in a queue.  Each of
// max_slots worker threads owns a HIP stream, a solver workspace and device buffers for
// y and x; a worker takes the oldest queued request whose device footprint fits the part
// of the HBM budget not held by the other workers, so requests are admitted as slots and
// memory free up, and the resident requests' kernels run concurrently on the device.
// With batch_slots > 0 each bfloat16 dictionary also has a batched engine run by a
// thread of its own: its requests wait in the dictionary's queue, join the engine's
// resident signals whenever a slot is free at a graph-replay boundary (the ones with the
// parameters of the running batch), and leave when they finish.
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
#include <string>
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
  bool batched = false;  // routed to the dictionary's batched engine
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

// The batched engine of one bfloat16 dictionary (Lasso or groups) and its requests.
struct BatchLane {
  int dict = -1;
  std::thread th;
  BatchEngine* eng = nullptr;
  std::deque<uint64_t> queue;  // requests waiting for this engine
  // staging in coherent pinned host memory, read and written by the engine's kernels
  // directly: column c of Y (leading dimension ldy) and of X (K)
  float* Ys = nullptr;
  float* Xs = nullptr;
  float* Ys_dev = nullptr;  // the same memory as the device addresses it
  float* Xs_dev = nullptr;
  int64_t ldy = 0;
  size_t held = 0;             // device bytes charged to the budget for this engine
  bool waiting = false;        // needs memory that others hold
};

size_t vec_size(ds_dtype t) { return t == DS_F64 ? 8 : 4; }
size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Requests the batched engine can run (the parameters lasso_solve's batched path takes).
bool batch_eligible(const ds_params& p) {
  return (p.rule == DS_ISTA || p.rule == DS_FISTA) && p.step_rule == DS_STEP_CONSTANT &&
         (p.test == DS_TEST_NONE || p.test == DS_TEST_SAFE || p.test == DS_TEST_DST3 ||
          p.test == DS_TEST_DOME) &&
         p.x0 == nullptr && p.obj_tol == 0.0;
}

// Requests share a batched run when the engine's parameters agree.
bool same_run(const ds_params& a, const ds_params& b) {
  return a.rule == b.rule && a.test == b.test && a.screening == b.screening &&
         a.lambda_mode == b.lambda_mode && a.gap_tol == b.gap_tol && a.max_iter == b.max_iter &&
         a.step_L == b.step_L;
}

// Bytes a batched engine is charged: its device workspace (with the 25% headroom of
// Workspace::reserve) and its staging columns (pinned host memory, counted as well).
size_t lane_need(int64_t N, int64_t K, int64_t G, int slots, int max_iter) {
  const size_t ws = batched_workspace_bytes(N, K, slots, max_iter, G);
  const int64_t ldy = (N + 3) / 4 * 4;
  return ws + ws / 4 + align256(static_cast<size_t>(ldy) * slots * 4) +
         align256(static_cast<size_t>(K) * slots * 4);
}

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
  std::map<int, std::unique_ptr<BatchLane>> lanes;  // by dictionary id
  int lanes_waiting = 0;         // batched engines waiting for memory
  hipStream_t admin = nullptr;  // registration work

  void worker_loop(Worker* w);
  void run(Worker* w, Request* r, const Dict& d);
  void lane_loop(BatchLane* b);
  void run_lane(BatchLane* b, const Dict& d, const ds_params& key);
  void release_lane(BatchLane* b, std::unique_lock<std::mutex>& lk);
  size_t pending() const {
    size_t n = queue.size();
    for (const auto& kv : lanes) n += kv.second->queue.size();
    return n;
  }
  void finish(Request* r, ds_status st, const std::string& err) {  // with mu held
    r->status = st;
    r->error = err;
    r->t_end = Clock::now();
    r->state = DONE;
  }
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
      if ((!queue.empty() || lanes_waiting > 0) && w->held > 0) {
        // nothing queued fits next to what the workers hold (or a batched engine waits for
        // memory): give this worker's memory back so that whoever has room can admit
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

void Server::release_lane(BatchLane* b, std::unique_lock<std::mutex>& lk) {
  const size_t h = b->held;
  lk.unlock();
  batch_engine_trim(b->eng);
  if (b->Ys != nullptr) (void)hipHostFree(b->Ys);
  if (b->Xs != nullptr) (void)hipHostFree(b->Xs);
  b->Ys = b->Xs = b->Ys_dev = b->Xs_dev = nullptr;
  lk.lock();
  held -= h;
  b->held = 0;
  cv_work.notify_all();
}

void Server::lane_loop(BatchLane* b) {
  (void)hipSetDevice(cfg.device);
  std::unique_lock<std::mutex> lk(mu);
  const Dict& d = *dicts.at(b->dict);
  for (;;) {
    if (stop) break;
    if (b->queue.empty()) {
      // idle: give the memory back when others wait for some
      if (b->held > 0 && (!queue.empty() || lanes_waiting > 0)) {
        release_lane(b, lk);
        continue;
      }
      cv_work.wait(lk);
      continue;
    }
    const ds_params key = reqs.at(b->queue.front())->prm;
    const size_t need = lane_need(d.N, d.K, d.G, cfg.batch_slots, key.max_iter);
    const size_t want = std::max(b->held, need);
    if (held - b->held + want > cfg.hbm_budget_bytes) {
      if (b->held > 0) {  // hold nothing while waiting
        release_lane(b, lk);
        continue;
      }
      if (!b->waiting) {
        b->waiting = true;
        ++lanes_waiting;
        cv_work.notify_all();
      }
      cv_work.wait(lk);
      continue;
    }
    if (b->waiting) {
      b->waiting = false;
      --lanes_waiting;
    }
    held += want - b->held;
    b->held = want;
    lk.unlock();
    run_lane(b, d, key);
    lk.lock();
    cv_work.notify_all();
  }
  if (b->waiting) {
    b->waiting = false;
    --lanes_waiting;
  }
}

// One run of the batched engine: requests with the parameters `key` join while slots are
// free, until none holds a signal.
void Server::run_lane(BatchLane* b, const Dict& d, const ds_params& key) {
  const int slots = cfg.batch_slots;
  const int64_t ldy = (d.N + 3) / 4 * 4;  // 16-byte columns
  std::vector<Request*> in_col(slots, nullptr);
  std::vector<int> free_cols;
  for (int c = slots - 1; c >= 0; --c) free_cols.push_back(c);
  auto fail_waiting = [&](ds_status st) {  // the requests of this run still queued
    const std::string err = ds_last_error();
    std::lock_guard<std::mutex> g(mu);
    for (auto it = b->queue.begin(); it != b->queue.end();) {
      Request* r = reqs.at(*it).get();
      if (!same_run(r->prm, key)) {
        ++it;
        continue;
      }
      it = b->queue.erase(it);
      r->t_start = Clock::now();
      finish(r, st, err);
    }
    cv_work.notify_all();
  };
  if (b->eng == nullptr) b->eng = batch_engine_create(cfg.device);
  if (b->Ys == nullptr) {
    // coherent: a column is rewritten by the host for each new request, so the device must
    // not read it through a cache that could hold the previous request's values
    void *py = nullptr, *px = nullptr, *dy = nullptr, *dx = nullptr;
    if (hipHostMalloc(&py, static_cast<size_t>(ldy) * slots * 4, hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc(&px, static_cast<size_t>(d.K) * slots * 4, hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer(&dy, py, 0) != hipSuccess ||
        hipHostGetDevicePointer(&dx, px, 0) != hipSuccess) {
      (void)hipGetLastError();
      if (py != nullptr) (void)hipHostFree(py);
      if (px != nullptr) (void)hipHostFree(px);
      set_error("pinned host staging columns of the batched engine could not be allocated");
      return fail_waiting(DS_ENOMEM);
    }
    b->Ys = static_cast<float*>(py);
    b->Xs = static_cast<float*>(px);
    b->Ys_dev = static_cast<float*>(dy);
    b->Xs_dev = static_cast<float*>(dx);
    b->ldy = ldy;
  }
  ds_params prm = key;
  if (!(prm.step_L > 0.0)) prm.step_L = d.L;
  const size_t vsz = 4;  // FP32 observations and solutions
  BatchFeed feed;
  feed.pull = [&](int room, int* cols, double* lams, hipStream_t s) -> int {
    std::vector<Request*> got;
    {
      std::lock_guard<std::mutex> g(mu);
      if (stop) return 0;
      // Requests of other parameters wait for this run to end.  The ones queued behind them
      // may overtake them, but a waiting request is overtaken by at most SKIP_LIMIT pulls;
      // then this run admits nothing more, drains, and the next run starts with it.
      std::vector<Request*> passed;
      size_t overtaken = 0;  // the first `overtaken` of `passed` were overtaken here
      for (auto it = b->queue.begin();
           it != b->queue.end() && static_cast<int>(got.size()) < room &&
           got.size() < free_cols.size();) {
        Request* r = reqs.at(*it).get();
        if (!same_run(r->prm, key)) {
          if (r->skipped >= SKIP_LIMIT) break;
          passed.push_back(r);
          ++it;
          continue;
        }
        it = b->queue.erase(it);
        r->state = RUNNING;
        r->t_start = Clock::now();
        got.push_back(r);
        overtaken = passed.size();
      }
      for (size_t k = 0; k < overtaken; ++k) ++passed[k]->skipped;
    }
    int n = 0;
    for (Request* r : got) {
      const int c = free_cols.back();
      free_cols.pop_back();
      in_col[c] = r;
      // the column is free: no kernel reads it until the set-up this pull precedes
      std::memcpy(b->Ys + static_cast<int64_t>(c) * ldy, r->y.data(), d.N * vsz);
      cols[n] = c;
      lams[n] = r->lam;
      ++n;
    }
    return n;
  };
  feed.finish = [&](const int* cols, const ds_info* infos, int n, hipStream_t) {
    // the engine's stream has been synchronized after the harvest wrote these columns
    for (int j = 0; j < n; ++j) {
      Request* r = in_col[cols[j]];
      r->x.resize(d.K * vsz);
      std::memcpy(r->x.data(), b->Xs + static_cast<int64_t>(cols[j]) * d.K, d.K * vsz);
    }
    std::lock_guard<std::mutex> g(mu);
    for (int j = 0; j < n; ++j) {
      Request* r = in_col[cols[j]];
      in_col[cols[j]] = nullptr;
      free_cols.push_back(cols[j]);
      r->info = infos[j];
      if (infos[j].status == DS_EINVAL) {
        finish(r, DS_EINVAL, "observation contains NaN or Inf");
      } else if (r->id == fail_request) {
        finish(r, DS_EDEVICE,
               "the slot of request " + std::to_string(r->id) + " was marked failed (DS_SERVE_FAIL_REQUEST)");
      } else {
        finish(r, static_cast<ds_status>(infos[j].status), std::string());
      }
    }
    cv_work.notify_all();
  };
  const ds_problem P = d.view();
  const ds_status e = run_batched(*b->eng, P, b->Ys_dev, ldy, slots, prm, b->Xs_dev, d.K, nullptr,
                                  feed, nullptr);
  if (e < 0) {  // the signals in the engine fail with the run
    const std::string err = ds_last_error();
    std::lock_guard<std::mutex> g(mu);
    for (Request* r : in_col)
      if (r != nullptr) finish(r, e, err);
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
  if (static_cast<int64_t>(S->pending()) >= S->cfg.max_queue) {
    set_error("request queue full (%d waiting)", S->cfg.max_queue);
    return DS_EBUSY;
  }
  auto lane = S->lanes.find(dict_id);
  const bool batched = lane != S->lanes.end() && batch_eligible(*params) &&
                       lane_need(d.N, d.K, d.G, S->cfg.batch_slots, params->max_iter) <=
                           S->cfg.hbm_budget_bytes;
  const size_t need = batched ? 0 : request_need(d, *params);
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
  r->batched = batched;
  r->t_submit = Clock::now();
  *request_id = r->id;
  if (batched)
    lane->second->queue.push_back(r->id);
  else
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
      config->batch_slots < 0 || config->batch_slots > 32768 || config->device < 0) {
    set_error("bad server config (max_slots >= 1, max_queue >= 1, budget > 0, "
              "0 <= batch_slots <= 32768)");
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
    try {
      w->th = std::thread([sp, wp] { sp->worker_loop(wp); });
    } catch (...) {  // stop the workers already running; no exception crosses the boundary
      {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
      }
      S->cv_work.notify_all();
      for (auto& v : S->workers) {
        if (v->th.joinable()) v->th.join();
        if (v->stream != nullptr) (void)hipStreamDestroy(v->stream);
      }
      (void)hipStreamDestroy(S->admin);
      set_error("could not start the server's worker threads");
      return DS_EDEVICE;
    }
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
  int32_t store_raw;  // a C caller may pass any int32 here
  std::memcpy(&store_raw, &store, sizeof store_raw);
  if (store_raw != DS_F64 && store_raw != DS_F32 && store_raw != DS_BF16) {
    set_error("unknown store precision %d", static_cast<int>(store_raw));
    return DS_EINVAL;
  }
  const bool convert = problem->dtype == DS_F32 && store == DS_BF16;
  if (store != problem->dtype && !convert) {
    set_error("store precision must equal the input's, or be DS_BF16 for DS_F32 input");
    return DS_EINVAL;
  }
  // the workers serve every dictionary with single-signal solves on the server's copy,
  // whose base and column stride are 16-byte aligned
  if ((e = single_shape_check(store_raw, problem->N, problem->K, problem->G, true)) != DS_OK)
    return e;
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
  const bool lane = S->cfg.batch_slots > 0 && store == DS_BF16;
  std::lock_guard<std::mutex> g(S->mu);
  *dict_id = S->next_dict++;
  S->dicts.emplace(*dict_id, std::move(d));
  if (lane) {
    auto b = std::make_unique<BatchLane>();
    b->dict = *dict_id;
    BatchLane* bp = b.get();
    Server* sp = S;
    try {
      b->th = std::thread([sp, bp] { sp->lane_loop(bp); });
    } catch (...) {  // no engine: the dictionary's requests run on the workers
      return DS_OK;
    }
    S->lanes.emplace(*dict_id, std::move(b));
  }
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
  for (auto& kv : S->lanes)
    if (kv.second->th.joinable()) kv.second->th.join();
  (void)hipSetDevice(S->cfg.device);
  for (auto& kv : S->lanes) {
    batch_engine_destroy(kv.second->eng);
    if (kv.second->Ys != nullptr) (void)hipHostFree(kv.second->Ys);
    if (kv.second->Xs != nullptr) (void)hipHostFree(kv.second->Xs);
  }
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
