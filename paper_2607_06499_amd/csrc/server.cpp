// server.cpp -- served form: continuous batching of replan requests over
// device-resident planner sessions.
//
// Sessions are planners opened before start, admitted while their device
// memory fits the budget.  Requests carry host inputs (state, obstacles) and
// are queued.  A scheduler thread retires finished launches (event polls) and
// forms new launches from the pending requests of idle sessions, in arrival
// order, at most one request per session per launch and max_batch requests per
// launch.  Up to max_inflight launches run at once on their own streams, so
// requests that arrive while others are on the GPU start as soon as a launch
// context frees up, and their work overlaps on the device.  A launch stages
// the inputs with one host-to-device copy, runs the batched replan of its
// members and copies the outputs back with one device-to-host copy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cemppi.h"
#include "device.hpp"
#include "planner.hpp"

using namespace cemppi;

namespace {

using Clock = std::chrono::steady_clock;

double seconds_since(Clock::time_point t0) {
  return std::chrono::duration<double>(Clock::now() - t0).count();
}

constexpr int kInStride = 12 + kMaxObs * 4;  // floats: state, then obstacle rows
constexpr int kOutFloats = kMaxCtrl;         // u_out
constexpr int kMaxInflight = 3;
// Launches of at most this many requests run each request's own
// single-planner replan (eight kernels, back to back on the launch stream)
// instead of the batched chain, whose per-phase persistent kernels cost more
// than they share at these sizes; both give the same bits.
constexpr int kSingleMax = 2;

struct Request {
  uint64_t ticket = 0;
  int session = 0;
  int n_obs = 0;
  double t_arrival = 0.0, t_done = 0.0;
  float in[kInStride];
  float u[kOutFloats];
  ce_mppi_info info;
  bool done = false;
};

struct Launch {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  float* d_in = nullptr;   // [max_batch][kInStride]
  float* d_out = nullptr;  // [max_batch][kOutFloats]
  char* d_info = nullptr;  // [max_batch] ce_mppi_info
  float* h_in = nullptr;   // pinned mirrors
  float* h_out = nullptr;
  char* h_info = nullptr;
  std::vector<Request*> reqs;
  bool busy = false;
};

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

}  // namespace

struct ce_mppi_server {
  ce_mppi_server_config cfg{};
  uint64_t budget = 0, used = 0;
  std::vector<ce_mppi_planner*> sessions;
  ce_mppi_batch* batch = nullptr;
  Launch launch[kMaxInflight];
  Clock::time_point t0 = Clock::now();
  // request bookkeeping (guarded by mu)
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> pending;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  std::vector<char> session_busy;
  uint64_t next_ticket = 1;
  bool started = false, stop = false;
  std::string thread_error;
  std::thread worker;
  // statistics (guarded by mu)
  uint64_t n_launches = 0, n_served = 0, max_members = 0;
  uint64_t sum_members = 0;
  int max_inflight_seen = 0;
};

namespace {

void retire(ce_mppi_server* S, Launch& L) {
  const double now = seconds_since(S->t0);
  std::lock_guard<std::mutex> g(S->mu);
  for (size_t q = 0; q < L.reqs.size(); ++q) {
    Request* r = L.reqs[q];
    std::memcpy(r->u, L.h_out + q * kOutFloats, sizeof(r->u));
    std::memcpy(&r->info, L.h_info + q * sizeof(ce_mppi_info), sizeof(ce_mppi_info));
    r->t_done = now;
    r->done = true;
    S->session_busy[r->session] = 0;
    ++S->n_served;
  }
  L.reqs.clear();
  L.busy = false;
  S->cv_done.notify_all();
}

// One launch over the given requests (launch context L is free).
hipError_t start_launch(ce_mppi_server* S, Launch& L, std::vector<Request*>& take) {
  const int count = (int)take.size();
  std::vector<int32_t> members(count);
  std::vector<ce_mppi_batch_io> io(count);
  for (int q = 0; q < count; ++q) {
    Request* r = take[q];
    std::memcpy(L.h_in + (size_t)q * kInStride, r->in, sizeof(r->in));
    members[q] = r->session;
    ce_mppi_batch_io& e = io[q];
    e.x_t = L.d_in + (size_t)q * kInStride;
    e.obstacles = r->n_obs > 0 ? L.d_in + (size_t)q * kInStride + 12 : nullptr;
    e.n_obs = r->n_obs;
    e.reserved = 0;
    e.u_out = L.d_out + (size_t)q * kOutFloats;
    e.U_out = nullptr;
    e.info = L.d_info + (size_t)q * sizeof(ce_mppi_info);
  }
  hipError_t e = hipMemcpyAsync(L.d_in, L.h_in, sizeof(float) * kInStride * count,
                                hipMemcpyHostToDevice, L.stream);
  if (e != hipSuccess) return e;
  if (S->cfg.mode == CE_SERVE_PLAIN || count <= kSingleMax) {
    // each request through its session's own single-planner replan
    for (int q = 0; q < count; ++q) {
      const ce_mppi_batch_io& a = io[q];
      // the scheduler orders each session's requests (one in flight at most)
      if (replan_unchecked(S->sessions[members[q]], a.x_t, a.obstacles, a.n_obs, a.u_out, nullptr,
                           static_cast<ce_mppi_info*>(a.info), L.stream) != CE_OK)
        return hipErrorUnknown;
    }
  } else if (ce_mppi_batch_replan_subset(S->batch, members.data(), count, io.data(), L.stream) != CE_OK) {
    return hipErrorUnknown;
  }
  e = hipMemcpyAsync(L.h_out, L.d_out, sizeof(float) * kOutFloats * count, hipMemcpyDeviceToHost,
                     L.stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(L.h_info, L.d_info, sizeof(ce_mppi_info) * count, hipMemcpyDeviceToHost,
                       L.stream);
  if (e == hipSuccess) e = hipEventRecord(L.done, L.stream);
  if (e != hipSuccess) return e;
  L.reqs = take;
  L.busy = true;
  return hipSuccess;
}

void worker_loop(ce_mppi_server* S) {
  (void)hipSetDevice(S->cfg.device);
  const int max_batch = S->cfg.max_batch;
  const int max_inflight = S->cfg.max_inflight;
  std::vector<Request*> take;
  take.reserve(max_batch);
  while (true) {
    bool progressed = false;
    int inflight = 0;
    for (int i = 0; i < max_inflight; ++i) {
      Launch& L = S->launch[i];
      if (!L.busy) continue;
      const hipError_t q = hipEventQuery(L.done);
      if (q == hipSuccess) {
        retire(S, L);
        progressed = true;
      } else if (q != hipErrorNotReady) {
        std::lock_guard<std::mutex> g(S->mu);
        S->thread_error = std::string("launch failed: ") + hipGetErrorString(q);
        S->stop = true;
        S->cv_done.notify_all();
        return;
      } else {
        ++inflight;
      }
    }
    Launch* freeL = nullptr;
    for (int i = 0; i < max_inflight && !freeL; ++i)
      if (!S->launch[i].busy) freeL = &S->launch[i];
    take.clear();
    {
      std::lock_guard<std::mutex> g(S->mu);
      if (S->stop && S->pending.empty() && inflight == 0) return;
      if (freeL) {
        // arrival order; one request per session per launch; idle sessions only
        std::vector<char> in_this(S->sessions.size(), 0);
        for (auto it = S->pending.begin(); it != S->pending.end() && (int)take.size() < max_batch;) {
          Request* r = *it;
          if (!S->session_busy[r->session] && !in_this[r->session]) {
            in_this[r->session] = 1;
            S->session_busy[r->session] = 1;
            take.push_back(r);
            it = S->pending.erase(it);
          } else {
            ++it;
          }
        }
      }
    }
    if (!take.empty()) {
      const hipError_t e = start_launch(S, *freeL, take);
      std::lock_guard<std::mutex> g(S->mu);
      if (e != hipSuccess) {
        S->thread_error = std::string("launch start failed: ") + hipGetErrorString(e);
        S->stop = true;
        S->cv_done.notify_all();
        return;
      }
      ++S->n_launches;
      S->sum_members += take.size();
      S->max_members = std::max<uint64_t>(S->max_members, take.size());
      S->max_inflight_seen = std::max(S->max_inflight_seen, inflight + 1);
      progressed = true;
    }
    if (!progressed) {
      std::unique_lock<std::mutex> g(S->mu);
      const bool idle = S->pending.empty();
      if (idle && inflight == 0 && !S->stop)
        S->cv_work.wait_for(g, std::chrono::milliseconds(2));
      // otherwise poll again: launches finish within microseconds
    }
  }
}

void free_launches(ce_mppi_server* S) {
  for (Launch& L : S->launch) {
    if (L.stream) (void)hipStreamSynchronize(L.stream);
    if (L.done) (void)hipEventDestroy(L.done);
    if (L.stream) (void)hipStreamDestroy(L.stream);
    if (L.d_in) (void)hipFree(L.d_in);
    if (L.d_out) (void)hipFree(L.d_out);
    if (L.d_info) (void)hipFree(L.d_info);
    if (L.h_in) (void)hipHostFree(L.h_in);
    if (L.h_out) (void)hipHostFree(L.h_out);
    if (L.h_info) (void)hipHostFree(L.h_info);
    L = Launch{};
  }
}

}  // namespace

extern "C" {

ce_status ce_mppi_server_create(const ce_mppi_server_config* cfg, ce_mppi_server** out) {
  if (!cfg || !out) return set_error(CE_EINVAL, "NULL argument");
  *out = nullptr;
  if (cfg->max_batch < 1 || cfg->max_batch > CE_MPPI_MAX_BATCH)
    return set_error(CE_EINVAL, "max_batch out of range 1..1024");
  if (cfg->max_inflight < 1 || cfg->max_inflight > kMaxInflight)
    return set_error(CE_EINVAL, "max_inflight out of range 1..3");
  if (cfg->mode != CE_SERVE_BATCHED && cfg->mode != CE_SERVE_PLAIN)
    return set_error(CE_EINVAL, "unknown mode");
  if (cfg->mode == CE_SERVE_PLAIN && (cfg->max_batch != 1 || cfg->max_inflight != 1))
    return set_error(CE_EINVAL, "the plain form serves one request at a time (max_batch = max_inflight = 1)");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0)
    return set_error(CE_EDEVICE, "no HIP device available");
  if (cfg->device < 0 || cfg->device >= ndev) return set_error(CE_EINVAL, "device ordinal out of range");
  DeviceGuard guard(cfg->device);
  ce_mppi_server* S = new (std::nothrow) ce_mppi_server();
  if (!S) return set_error(CE_ENOMEM, "host allocation failed");
  S->cfg = *cfg;
  S->budget = cfg->memory_budget;
  if (S->budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      delete S;
      return set_error(CE_EDEVICE, "hipMemGetInfo failed");
    }
    S->budget = (uint64_t)(0.9 * (double)fr);
  }
  *out = S;
  return CE_OK;
}

ce_status ce_mppi_server_open_session(ce_mppi_server* S, const ce_mppi_config* cfg, const float* U0,
                                      int32_t* session) {
  if (!S || !cfg || !session) return set_error(CE_EINVAL, "NULL argument");
  if (S->started) return set_error(CE_EINVAL, "sessions are opened before ce_mppi_server_start");
  if ((int)S->sessions.size() >= CE_MPPI_MAX_BATCH)
    return set_error(CE_EBUSY, "session limit reached");
  if (cfg->device != S->cfg.device) return set_error(CE_EINVAL, "session on another device");
  ce_mppi_planner* P = nullptr;
  ce_status st = ce_mppi_create(cfg, &P);
  if (st != CE_OK) return st;
  if (S->used + P->arena_bytes > S->budget) {
    ce_mppi_destroy(P);
    return set_error(CE_EBUSY, "device memory budget exhausted");
  }
  DeviceGuard guard(S->cfg.device);
  if (U0) {
    // the nominal sequence through a device bounce buffer
    float* d = nullptr;
    const size_t bytes = sizeof(float) * P->c.NM;
    hipError_t e = hipMalloc(&d, bytes);
    if (e == hipSuccess) e = hipMemcpy(d, U0, bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) st = ce_mppi_set_nominal(P, d, nullptr);
    if (e == hipSuccess && st == CE_OK) e = hipDeviceSynchronize();
    if (d) (void)hipFree(d);
    if (e != hipSuccess || st != CE_OK) {
      ce_mppi_destroy(P);
      return e != hipSuccess ? set_hip_error(e, "open_session") : st;
    }
  }
  S->used += P->arena_bytes;
  *session = (int32_t)S->sessions.size();
  S->sessions.push_back(P);
  return CE_OK;
}

ce_status ce_mppi_server_start(ce_mppi_server* S) {
  if (!S) return set_error(CE_EINVAL, "server is NULL");
  if (S->started) return set_error(CE_EINVAL, "already started");
  if (S->sessions.empty()) return set_error(CE_EINVAL, "no session opened");
  DeviceGuard guard(S->cfg.device);
  ce_status st = ce_mppi_batch_create(S->sessions.data(), (int32_t)S->sessions.size(), &S->batch);
  if (st != CE_OK) return st;
  const int mb = S->cfg.max_batch;
  hipError_t e = hipSuccess;
  for (int i = 0; i < S->cfg.max_inflight && e == hipSuccess; ++i) {
    Launch& L = S->launch[i];
    e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(&L.d_in, sizeof(float) * kInStride * mb);
    if (e == hipSuccess) e = hipMalloc(&L.d_out, sizeof(float) * kOutFloats * mb);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&L.d_info), sizeof(ce_mppi_info) * mb);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&L.h_in), sizeof(float) * kInStride * mb, 0);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&L.h_out), sizeof(float) * kOutFloats * mb, 0);
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void**>(&L.h_info), sizeof(ce_mppi_info) * mb, 0);
  }
  if (e != hipSuccess) {
    free_launches(S);
    ce_mppi_batch_destroy(S->batch);
    S->batch = nullptr;
    return set_hip_error(e, "server_start");
  }
  {
    // every session builds its replan graph and picks its faster launch mode
    // before the first request (tune_launch restores each session's state)
    Launch& L = S->launch[0];
    e = hipMemsetAsync(L.d_in, 0, sizeof(float) * kInStride, L.stream);
    for (size_t q = 0; q < S->sessions.size() && st == CE_OK && e == hipSuccess; ++q)
      st = ce_mppi_tune_launch(S->sessions[q], L.d_in, nullptr, 0, L.d_out, 8, L.stream, nullptr,
                               nullptr);
    if (st == CE_OK && e == hipSuccess) e = hipStreamSynchronize(L.stream);
    if (st != CE_OK || e != hipSuccess) {
      free_launches(S);
      ce_mppi_batch_destroy(S->batch);
      S->batch = nullptr;
      return st != CE_OK ? st : set_hip_error(e, "server warm-up");
    }
  }
  if (S->cfg.mode == CE_SERVE_BATCHED) {
    // warm-up: one launch through every subset area, so that graph builds and
    // first kernel loads happen before the first request (session 0 replans a
    // zero state without obstacles; its state is saved before and restored)
    size_t bytes = 0;
    st = ce_mppi_state_size(S->sessions[0], &bytes);
    std::vector<char> saved(bytes);
    if (st == CE_OK) st = ce_mppi_get_state(S->sessions[0], saved.data(), bytes, S->launch[0].stream);
    Launch& L = S->launch[0];
    if (st == CE_OK) e = hipMemsetAsync(L.d_in, 0, sizeof(float) * kInStride, L.stream);
    for (int k = 0; k < 3 && st == CE_OK && e == hipSuccess; ++k) {
      const int32_t m = 0;
      ce_mppi_batch_io io{};
      io.x_t = L.d_in;
      io.u_out = L.d_out;
      io.info = L.d_info;
      st = ce_mppi_batch_replan_subset(S->batch, &m, 1, &io, L.stream);
    }
    if (st == CE_OK && e == hipSuccess) e = hipStreamSynchronize(L.stream);
    if (st == CE_OK && e == hipSuccess)
      st = ce_mppi_set_state(S->sessions[0], saved.data(), bytes, L.stream);
    if (st != CE_OK || e != hipSuccess) {
      free_launches(S);
      ce_mppi_batch_destroy(S->batch);
      S->batch = nullptr;
      return st != CE_OK ? st : set_hip_error(e, "server warm-up");
    }
  }
  S->session_busy.assign(S->sessions.size(), 0);
  S->started = true;
  S->t0 = Clock::now();
  S->worker = std::thread(worker_loop, S);
  return CE_OK;
}

ce_status ce_mppi_server_submit(ce_mppi_server* S, int32_t session, const float* x_t,
                                const float* obstacles, int32_t n_obs, uint64_t* ticket) {
  if (!S || !x_t || !ticket) return set_error(CE_EINVAL, "NULL argument");
  if (!S->started) return set_error(CE_EINVAL, "server not started");
  if (session < 0 || session >= (int)S->sessions.size()) return set_error(CE_EINVAL, "unknown session");
  const ce_mppi_planner* P = S->sessions[session];
  if (n_obs < 0 || n_obs > P->c.max_obs) return set_error(CE_EINVAL, "n_obs out of range");
  if (n_obs > 0 && !obstacles) return set_error(CE_EINVAL, "obstacles is NULL");
  auto r = std::make_unique<Request>();
  r->session = session;
  r->n_obs = n_obs;
  std::memset(r->in, 0, sizeof(r->in));
  std::memcpy(r->in, x_t, sizeof(float) * P->c.n);
  if (n_obs > 0) std::memcpy(r->in + 12, obstacles, sizeof(float) * n_obs * (P->c.p + 1));
  std::lock_guard<std::mutex> g(S->mu);
  if (S->stop) return set_error(CE_EDEVICE, "server stopped: " + S->thread_error);
  r->ticket = S->next_ticket++;
  r->t_arrival = seconds_since(S->t0);
  *ticket = r->ticket;
  S->pending.push_back(r.get());
  S->reqs.emplace(r->ticket, std::move(r));
  S->cv_work.notify_one();
  return CE_OK;
}

ce_status ce_mppi_server_wait(ce_mppi_server* S, uint64_t ticket, float* u_out, ce_mppi_info* info,
                              double* latency_s) {
  if (!S) return set_error(CE_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> g(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return set_error(CE_EINVAL, "unknown ticket");
  Request* r = it->second.get();
  S->cv_done.wait(g, [&] { return r->done || S->stop; });
  if (!r->done) return set_error(CE_EDEVICE, "server stopped: " + S->thread_error);
  const ce_mppi_planner* P = S->sessions[r->session];
  if (u_out) std::memcpy(u_out, r->u, sizeof(float) * P->c.m);
  if (info) *info = r->info;
  if (latency_s) *latency_s = r->t_done - r->t_arrival;
  S->reqs.erase(it);
  return CE_OK;
}

ce_status ce_mppi_server_run_trace(ce_mppi_server* S, int32_t n, const double* t_arrival,
                                   const int32_t* session, const float* x_t, const float* obstacles,
                                   const int32_t* n_obs, double* latency_s, float* u_out) {
  if (!S || !t_arrival || !session || !x_t || !n_obs || n < 0)
    return set_error(CE_EINVAL, "NULL argument");
  if (!S->started) return set_error(CE_EINVAL, "server not started");
  std::vector<uint64_t> tickets(n);
  const Clock::time_point start = Clock::now();
  for (int i = 0; i < n; ++i) {
    // release each request at its arrival time
    while (std::chrono::duration<double>(Clock::now() - start).count() < t_arrival[i]) {
    }
    const float* obs = obstacles ? obstacles + (size_t)i * kMaxObs * 4 : nullptr;
    ce_status st = ce_mppi_server_submit(S, session[i], x_t + (size_t)i * 12, obs, n_obs[i], &tickets[i]);
    if (st != CE_OK) return st;
  }
  for (int i = 0; i < n; ++i) {
    double lat = 0.0;
    ce_status st = ce_mppi_server_wait(S, tickets[i], u_out ? u_out + (size_t)i * kMaxCtrl : nullptr,
                                       nullptr, &lat);
    if (st != CE_OK) return st;
    if (latency_s) latency_s[i] = lat;
  }
  return CE_OK;
}

ce_status ce_mppi_server_get_stats(ce_mppi_server* S, ce_mppi_server_stats* out) {
  if (!S || !out) return set_error(CE_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> g(S->mu);
  out->launches = S->n_launches;
  out->served = S->n_served;
  out->mean_batch = S->n_launches ? (double)S->sum_members / (double)S->n_launches : 0.0;
  out->max_batch = (int32_t)S->max_members;
  out->max_inflight = S->max_inflight_seen;
  out->sessions = (int32_t)S->sessions.size();
  out->reserved = 0;
  out->session_bytes = S->used;
  out->budget_bytes = S->budget;
  return CE_OK;
}

void ce_mppi_server_destroy(ce_mppi_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
    S->cv_work.notify_all();
  }
  if (S->worker.joinable()) S->worker.join();
  DeviceGuard guard(S->cfg.device);
  free_launches(S);
  if (S->batch) ce_mppi_batch_destroy(S->batch);
  for (ce_mppi_planner* P : S->sessions) ce_mppi_destroy(P);
  delete S;
}

ce_mppi_planner* ce_mppi_server_session_planner(ce_mppi_server* S, int32_t session) {
  if (!S || session < 0 || session >= (int)S->sessions.size()) return nullptr;
  return S->sessions[session];
}

}  // extern "C"
