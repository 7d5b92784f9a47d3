// Serving loop (C ABI, include/mss.h): continuous batching of simulation
// requests of mixed spin and length on one GPU.
//
//  * Memory: one device pool of the HBM budget, carved first-fit into one
//    block per admitted request (final state, operators, states, scan
//    scratch).  A request is admitted (FIFO) only when its block fits and
//    an active slot is free; otherwise it waits in the queue
//    (back-pressure).  Blocks return to the pool on release.  Parameters
//    and initial states travel with each round's descriptors (one pinned
//    upload per round).
//  * Scheduling: a host thread runs rounds.  Each round gives every active
//    request with intervals left a share of the round's work budget (whole
//    64-interval items), integrates all those interval ranges in one
//    persistent-integrator launch, and scans the requests whose last range
//    is in the round.  A request's intervals are split over 2^s lanes each,
//    s fixed per request (by default the least s for which its intervals
//    times 2^s fill the device's resident lanes, at most its fine steps), so
//    a short request alone is not held up by one lane's serial steps and
//    its results never depend on the other requests.  Requests that arrive meanwhile join the next round,
//    so work of different requests overlaps on the device.  Two rounds are
//    kept in flight (descriptor buffers are double-buffered behind events).
//  * Results stay in the request's device block until release.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mss_work.h"

using namespace mss;

namespace {

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

// First-fit allocator over [0, size) with coalescing of free ranges.
class Pool {
 public:
  void reset(size_t size) {
    free_.clear();
    free_[0] = size;
    used_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = a256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t roff = it->first + bytes;
        free_.erase(it);
        if (rest) free_[roff] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = a256(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0;
};

struct Request {
  uint64_t ticket = 0;
  mss_problem prob{};
  std::vector<mss_term> terms;
  std::vector<double> params, psi0;
  int N = 0;
  int slices_log2 = 0;
  size_t bytes = 0, off = 0;
  double *d_fin = nullptr, *d_U = nullptr, *d_psi = nullptr, *d_scan = nullptr;
  int64_t next_k = 0;
  int32_t state = MSS_REQ_QUEUED;
  double t_submit = 0, t_admit = 0, t_done = 0;
};

size_t request_bytes(const mss_problem& p) {
  const int N = p.spin_twice + 1;
  size_t b = a256((size_t)N * 16);
  b += a256((size_t)p.n_samples * N * N * 16) + a256((size_t)p.n_samples * N * 16);
  b += scan_scratch_bytes(N, p.n_samples);
  return b;
}

struct Inflight {
  int slot;
  std::vector<uint64_t> finishing;
};

}  // namespace

struct mss_server {
  int device = 0;
  mss_server_options opt{};
  char* pool_base = nullptr;
  Pool pool;
  size_t peak = 0;
  hipStream_t stream = nullptr;
  // per round slot: device image, pinned staging of the same capacity,
  // completion event
  static constexpr int kSlots = 2;
  void* desc[kSlots] = {};
  char* staging[kSlots] = {};
  size_t cap[kSlots] = {};
  hipEvent_t done[kSlots] = {};
  int grid_cap = 0;
  int64_t lanes = 0;  // resident lanes of the device: CUs x 4 SIMDs x 2 waves x 64
  std::chrono::steady_clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> queue;
  std::vector<uint64_t> active;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::string fatal;
  int64_t submitted = 0, completed = 0, rounds = 0;
  double fine_steps = 0;
  std::thread worker;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void run();
  hipError_t ensure_slot(int slot, size_t bytes);
  int request_slices_log2(const mss_problem& p) const;
};

// Grow a slot's buffers to at least bytes (the slot must be idle).
hipError_t mss_server::ensure_slot(int slot, size_t bytes) {
  if (bytes <= cap[slot]) return hipSuccess;
  const size_t want = std::max(a256(bytes), 2 * cap[slot]);
  if (desc[slot]) (void)hipFree(desc[slot]);
  if (staging[slot]) (void)hipHostFree(staging[slot]);
  desc[slot] = nullptr;
  staging[slot] = nullptr;
  cap[slot] = 0;
  hipError_t e = hipMalloc(&desc[slot], want);
  if (e == hipSuccess) e = hipHostMalloc((void**)&staging[slot], want);
  if (e != hipSuccess) return e;
  cap[slot] = want;
  return hipSuccess;
}

int mss_server::request_slices_log2(const mss_problem& p) const {
  const int top = api_ilog2(std::min(64, p.n_fine));
  if (opt.slices > 0) return std::min(api_ilog2(opt.slices), top);
  int s = 0;
  while (s < top && (p.n_samples << s) < lanes) ++s;
  return s;
}

namespace {

void fail_all(mss_server* S, const std::string& msg) {
  std::lock_guard<std::mutex> lock(S->mu);
  S->fatal = msg;
  for (auto& kv : S->reqs)
    if (kv.second->state != MSS_REQ_DONE) kv.second->state = MSS_REQ_FAILED;
  S->cv_done.notify_all();
}

}  // namespace

void mss_server::run() {
  (void)hipSetDevice(device);
  std::deque<Inflight> inflight;
  int round = 0;
  for (;;) {
    std::vector<Request*> work;
    {
      std::unique_lock<std::mutex> lock(mu);
      for (;;) {
        if (stop) break;
        // admission: FIFO while a slot and pool memory are available
        while (!queue.empty() && (int)active.size() < opt.max_active) {
          Request* r = reqs[queue.front()].get();
          size_t off = 0;
          if (!pool.alloc(r->bytes, &off)) break;
          peak = std::max(peak, pool.used());
          r->off = off;
          char* b = pool_base + off;
          const int N = r->N;
          const int64_t K = r->prob.n_samples;
          r->d_fin = (double*)b;
          b += a256((size_t)N * 16);
          r->d_U = (double*)b;
          b += a256((size_t)K * N * N * 16);
          r->d_psi = (double*)b;
          b += a256((size_t)K * N * 16);
          r->d_scan = (double*)b;
          r->state = MSS_REQ_RUNNING;
          r->t_admit = now();
          queue.pop_front();
          active.push_back(r->ticket);
        }
        for (uint64_t t : active) {
          Request* r = reqs[t].get();
          if (r->next_k < r->prob.n_samples) work.push_back(r);
        }
        if (!work.empty() || !inflight.empty()) break;
        cv_work.wait_for(lock, std::chrono::milliseconds(50));
      }
      if (stop && work.empty() && inflight.empty()) break;
    }
    hipError_t e = hipSuccess;
    if (!work.empty()) {
      const int slot = round % kSlots;
      if (inflight.size() >= (size_t)kSlots) {
        // the slot's previous round must be complete before its buffers are reused
        e = hipEventSynchronize(done[slot]);
      }
      // shares: the round budget split evenly (spin-1/2 steps weigh 1/16)
      double cost_left = opt.iteration_steps;
      std::sort(work.begin(), work.end(), [](const Request* a, const Request* b) {
        return a->ticket < b->ticket;
      });
      const double share = cost_left / (double)work.size();
      WorkSet ws;
      Inflight inf;
      inf.slot = slot;
      double round_steps = 0;
      for (Request* r : work) {
        const double w = (r->N == 3 ? 1.0 : 1.0 / 16.0) * r->prob.n_fine;
        const int per = 64 >> r->slices_log2;
        int64_t k = (int64_t)(share / w);
        k = std::max<int64_t>(per, k / per * per);
        k = std::min<int64_t>(k, r->prob.n_samples - r->next_k);
        const bool last = r->next_k + k == r->prob.n_samples;
        mss_problem q = r->prob;
        q.terms = r->terms.data();
        ws.add(q, r->slices_log2, r->next_k, k, last);
        SimDesc& d = ws.sims.back();
        d.psi = r->d_psi;
        d.psi_final = r->d_fin;
        d.U = r->d_U;
        d.scan_ws = r->d_scan;
        r->next_k += k;
        round_steps += (double)k * r->prob.n_fine;
        if (last) inf.finishing.push_back(r->ticket);
      }
      ws.finalize();
      // the image: the work queue counter (uploaded as zero), descriptors,
      // then every range's parameters and initial state
      const size_t base = 256 + a256(ws.packed_bytes());
      size_t total = base;
      std::vector<size_t> o_par(work.size()), o_psi0(work.size());
      for (size_t i = 0; i < work.size(); ++i) {
        o_par[i] = total;
        total += a256((size_t)std::max(1, work[i]->prob.n_params) * 8);
        o_psi0[i] = total;
        total += a256((size_t)work[i]->N * 16);
      }
      e = ensure_slot(slot, total);
      size_t o_sims, o_terms;
      std::vector<size_t> o_red, o_app;
      if (e == hipSuccess) {
        char* dev = (char*)desc[slot];
        for (size_t i = 0; i < work.size(); ++i) {
          const Request* r = work[i];
          SimDesc& d = ws.sims[i];
          d.params = r->prob.n_params > 0 ? (const double*)(dev + o_par[i]) : nullptr;
          d.psi0 = (const double*)(dev + o_psi0[i]);
          if (r->prob.n_params > 0)
            memcpy(staging[slot] + o_par[i], r->params.data(), r->params.size() * 8);
          memcpy(staging[slot] + o_psi0[i], r->psi0.data(), r->psi0.size() * 8);
        }
        memset(staging[slot], 0, 256);
        ws.pack(staging[slot] + 256, &o_sims, &o_terms, &o_red, &o_app);
        e = hipMemcpyAsync(desc[slot], staging[slot], total, hipMemcpyHostToDevice, stream);
      }
      if (e == hipSuccess) {
        DevWork dw = device_view(ws, (const char*)desc[slot] + 256, o_sims, o_terms, o_red, o_app);
        const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(grid_cap, (ws.n_items + 3) / 4));
        e = launch_work_integrate(dw, (unsigned long long*)desc[slot], blocks, stream, nullptr,
                                  true);
        if (e == hipSuccess) e = launch_work_scan(dw, stream);
        if (e == hipSuccess) e = hipEventRecord(done[slot], stream);
      }
      if (e == hipSuccess) {
        inflight.push_back(inf);
        ++round;
        std::lock_guard<std::mutex> lock(mu);
        ++rounds;
        fine_steps += round_steps;
      }
    }
    if (e != hipSuccess) {
      fail_all(this, std::string("serving round: ") + hipGetErrorString(e));
      return;
    }
    // retire the oldest round when two are in flight, or when there is no new work
    while (!inflight.empty() && (inflight.size() >= (size_t)kSlots || work.empty())) {
      Inflight f = inflight.front();
      inflight.pop_front();
      e = hipEventSynchronize(done[f.slot]);
      if (e != hipSuccess) {
        fail_all(this, std::string("serving round: ") + hipGetErrorString(e));
        return;
      }
      std::lock_guard<std::mutex> lock(mu);
      const double t = now();
      for (uint64_t tk : f.finishing) {
        auto it = reqs.find(tk);
        if (it == reqs.end()) continue;
        it->second->state = MSS_REQ_DONE;
        it->second->t_done = t;
        ++completed;
        active.erase(std::find(active.begin(), active.end(), tk));
      }
      cv_done.notify_all();
      if (!work.empty()) break;
    }
  }
  (void)hipStreamSynchronize(stream);
}

namespace {

void destroy(mss_server* S) {
  if (!S) return;
  if (S->worker.joinable()) {
    {
      std::lock_guard<std::mutex> lock(S->mu);
      S->stop = true;
    }
    S->cv_work.notify_all();
    S->worker.join();
  }
  if (S->stream) (void)hipStreamSynchronize(S->stream);
  for (int i = 0; i < mss_server::kSlots; ++i) {
    if (S->done[i]) (void)hipEventDestroy(S->done[i]);
    if (S->desc[i]) (void)hipFree(S->desc[i]);
    if (S->staging[i]) (void)hipHostFree(S->staging[i]);
  }
  if (S->stream) (void)hipStreamDestroy(S->stream);
  if (S->pool_base) (void)hipFree(S->pool_base);
  delete S;
}

void fill_info(const Request& r, mss_request_info* out) {
  out->state = r.state;
  out->spin_twice = r.prob.spin_twice;
  out->n_samples = r.prob.n_samples;
  const bool done = r.state == MSS_REQ_DONE;
  out->psi = done ? r.d_psi : nullptr;
  out->psi_final = done ? r.d_fin : nullptr;
  out->U = done ? r.d_U : nullptr;
  out->t_submit = r.t_submit;
  out->t_admit = r.t_admit;
  out->t_done = r.t_done;
}

}  // namespace

extern "C" {

mss_status mss_server_create(const mss_server_options* options, mss_server** out) {
  if (!out) return api_fail(MSS_E_INVALID, "out is NULL");
  *out = nullptr;
  mss_server_options opt{};
  if (options) opt = *options;
  if (opt.max_active < 0 || opt.slices < 0 || opt.slices > 64 ||
      (opt.slices & (opt.slices - 1)) != 0 || !(opt.iteration_steps >= 0.0))
    return api_fail(MSS_E_INVALID, "bad server options");
  if (!opt.max_active) opt.max_active = 512;
  if (opt.iteration_steps == 0.0) opt.iteration_steps = 3e7;
  mss_server* S = new (std::nothrow) mss_server();
  if (!S) return api_fail(MSS_E_NOMEM, "host allocation failed");
  S->t0 = std::chrono::steady_clock::now();
  hipError_t e = hipGetDevice(&S->device);
  if (e != hipSuccess) {
    delete S;
    return api_hip_fail(e, "no device");
  }
  if (!opt.hbm_budget) {
    size_t fr = 0, tot = 0;
    e = hipMemGetInfo(&fr, &tot);
    if (e != hipSuccess) {
      delete S;
      return api_hip_fail(e, "hipMemGetInfo");
    }
    opt.hbm_budget = (size_t)(0.8 * (double)fr);
  }
  opt.hbm_budget = opt.hbm_budget & ~(size_t)255;
  S->opt = opt;
  e = hipMalloc((void**)&S->pool_base, opt.hbm_budget);
  if (e != hipSuccess) {
    delete S;
    if (e == hipErrorOutOfMemory) return api_fail(MSS_E_NOMEM, "cannot reserve the HBM budget");
    return api_hip_fail(e, "hipMalloc");
  }
  S->pool.reset(opt.hbm_budget);
  // initial slot capacity: descriptors of max_active requests of up to
  // MSS_MAX_TERMS terms and 8 scan levels, and a spin-1 initial state and
  // 32 parameters each (a slot grows when a round needs more)
  const size_t slot_bytes = a256((size_t)opt.max_active * sizeof(SimDesc)) +
                            a256((size_t)opt.max_active * MSS_MAX_TERMS * sizeof(mss_term)) +
                            17 * a256(((size_t)opt.max_active + 1) * 8) +
                            (size_t)opt.max_active * (a256(48) + a256(32 * 8)) + 4096;
  e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
  for (int i = 0; i < mss_server::kSlots && e == hipSuccess; ++i) {
    e = S->ensure_slot(i, slot_bytes);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&S->done[i], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    destroy(S);
    return api_hip_fail(e, "server setup");
  }
  S->grid_cap = api_device_cu_count() * 2;
  S->lanes = (int64_t)api_device_cu_count() * 4 * 2 * 64;
  S->worker = std::thread([S] { S->run(); });
  *out = S;
  return api_ok();
}

mss_status mss_server_submit(mss_server* S, const mss_problem* p, const double* params,
                             const double* psi0, uint64_t* ticket) {
  if (!S || !ticket) return api_fail(MSS_E_INVALID, "server and ticket are required");
  mss_status s = api_validate_problem(p);
  if (s != MSS_OK) return s;
  if (p->n_params > 0 && !params) return api_fail(MSS_E_INVALID, "params is NULL");
  if (!psi0) return api_fail(MSS_E_INVALID, "psi0 is NULL");
  std::unique_ptr<Request> r(new (std::nothrow) Request());
  if (!r) return api_fail(MSS_E_NOMEM, "host allocation failed");
  r->prob = *p;
  r->terms.assign(p->terms, p->terms + p->n_terms);
  r->prob.terms = r->terms.data();
  r->params.assign(params, params + std::max(0, p->n_params));
  r->N = p->spin_twice + 1;
  r->psi0.assign(psi0, psi0 + 2 * r->N);
  r->bytes = request_bytes(*p);
  r->slices_log2 = S->request_slices_log2(*p);
  if (r->bytes > S->opt.hbm_budget)
    return api_fail(MSS_E_NOMEM, "request needs %zu bytes, the budget is %zu", r->bytes,
                    S->opt.hbm_budget);
  std::lock_guard<std::mutex> lock(S->mu);
  if (!S->fatal.empty()) return api_fail(MSS_E_DEVICE, "%s", S->fatal.c_str());
  r->ticket = S->next_ticket++;
  r->t_submit = S->now();
  *ticket = r->ticket;
  S->queue.push_back(r->ticket);
  S->reqs.emplace(r->ticket, std::move(r));
  ++S->submitted;
  S->cv_work.notify_all();
  return api_ok();
}

mss_status mss_server_poll(mss_server* S, uint64_t ticket, mss_request_info* out) {
  if (!S || !out) return api_fail(MSS_E_INVALID, "server and out are required");
  std::lock_guard<std::mutex> lock(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return api_fail(MSS_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  fill_info(*it->second, out);
  return api_ok();
}

mss_status mss_server_wait(mss_server* S, uint64_t ticket, double timeout_s,
                           mss_request_info* out) {
  if (!S || !out) return api_fail(MSS_E_INVALID, "server and out are required");
  std::unique_lock<std::mutex> lock(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return api_fail(MSS_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  Request* r = it->second.get();
  const auto deadline = std::chrono::steady_clock::now() +
                        std::chrono::microseconds((int64_t)(std::max(0.0, timeout_s) * 1e6));
  while (r->state != MSS_REQ_DONE && r->state != MSS_REQ_FAILED) {
    if (S->cv_done.wait_until(lock, deadline) == std::cv_status::timeout &&
        r->state != MSS_REQ_DONE && r->state != MSS_REQ_FAILED) {
      fill_info(*r, out);
      return api_fail(MSS_E_NOTREADY, "request %llu not done", (unsigned long long)ticket);
    }
  }
  fill_info(*r, out);
  if (r->state == MSS_REQ_FAILED) return api_fail(MSS_E_DEVICE, "%s", S->fatal.c_str());
  return api_ok();
}

mss_status mss_server_copy_out(mss_server* S, uint64_t ticket, double* psi, double* psi_final,
                               double* U, void* stream) {
  if (!S) return api_fail(MSS_E_INVALID, "server is NULL");
  const double *sp, *sf, *su;
  size_t np, nf, nu;
  {
    std::lock_guard<std::mutex> lock(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return api_fail(MSS_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
    const Request& r = *it->second;
    if (r.state != MSS_REQ_DONE) return api_fail(MSS_E_NOTREADY, "request not done");
    sp = r.d_psi;
    sf = r.d_fin;
    su = r.d_U;
    np = (size_t)r.prob.n_samples * r.N * 16;
    nf = (size_t)r.N * 16;
    nu = (size_t)r.prob.n_samples * r.N * r.N * 16;
  }
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  if (psi) e = hipMemcpyAsync(psi, sp, np, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess && psi_final) e = hipMemcpyAsync(psi_final, sf, nf, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess && U) e = hipMemcpyAsync(U, su, nu, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return api_hip_fail(e, "copy out");
  return api_ok();
}

mss_status mss_server_release(mss_server* S, uint64_t ticket) {
  if (!S) return api_fail(MSS_E_INVALID, "server is NULL");
  std::lock_guard<std::mutex> lock(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return api_fail(MSS_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  Request& r = *it->second;
  if (r.state == MSS_REQ_RUNNING) return api_fail(MSS_E_BUSY, "request is still running");
  if (r.state == MSS_REQ_QUEUED) {
    S->queue.erase(std::find(S->queue.begin(), S->queue.end(), ticket));
  } else if (r.state == MSS_REQ_DONE || (r.state == MSS_REQ_FAILED && r.d_psi)) {
    S->pool.release(r.off, r.bytes);
  }
  S->reqs.erase(it);
  S->cv_work.notify_all();
  return api_ok();
}

mss_status mss_server_stats_get(mss_server* S, mss_server_stats* out) {
  if (!S || !out) return api_fail(MSS_E_INVALID, "server and out are required");
  std::lock_guard<std::mutex> lock(S->mu);
  out->submitted = S->submitted;
  out->completed = S->completed;
  out->rounds = S->rounds;
  out->queued = (int32_t)S->queue.size();
  out->active = (int32_t)S->active.size();
  out->fine_steps = S->fine_steps;
  out->bytes_in_use = S->pool.used();
  out->bytes_peak = S->peak;
  out->budget = S->opt.hbm_budget;
  return api_ok();
}

mss_status mss_server_request_slices(const mss_server* S, const mss_problem* p,
                                     int32_t* slices) {
  if (!S || !slices) return api_fail(MSS_E_INVALID, "server and slices are required");
  mss_status s = api_validate_problem(p);
  if (s != MSS_OK) return s;
  *slices = 1 << S->request_slices_log2(*p);
  return api_ok();
}

double mss_server_clock(const mss_server* S) { return S ? S->now() : 0.0; }

void mss_server_destroy(mss_server* S) { destroy(S); }

}  // extern "C"
