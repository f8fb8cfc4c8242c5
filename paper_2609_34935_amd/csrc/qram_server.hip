// Request server: continuous batching of simulation requests on one GPU.
//
// A host thread owns every request context.  Requests wait in arrival order
// until their device footprint (tables, work buffers for one chunk, the
// per-trajectory result array) fits the HBM budget and an execution slot is
// free; each admitted request then runs chunk by chunk on its slot's stream,
// so chunks of different requests overlap on the device and a long request
// never holds the GPU for its whole length.  Results stay on the device
// until the request completes.  A request's trajectories are indexed by
// (seed, traj0 + i) exactly as in a direct call, so its results do not depend
// on what else is in flight.
#include "qram_internal.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Req {
  uint64_t ticket = 0;
  qram_request q{};
  std::vector<uint32_t> mem;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int state = 0;  // 0 waiting, 1 running, 2 done, 3 failed
  qram_status status = QRAM_OK;
  std::string err;
  uint64_t footprint = 0;
  qram_ctx *ctx = nullptr;
  double *d_fid = nullptr;
  std::vector<double> fid;
  double mean = 0, sem = 0;
  uint32_t next = 0, inflight = 0;
  int slot = -1;
};

}  // namespace

struct qram_server {
  uint64_t budget = 0;
  int max_active = 0;
  uint32_t chunk = 0;
  int device = 0;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  std::vector<int> free_slots;
  std::mutex mu;
  std::condition_variable wake, done;
  std::deque<Req *> waiting;
  std::vector<Req *> running;
  std::unordered_map<uint64_t, Req *> all;
  std::vector<std::pair<qram_ctx *, double *>> parked;  // released at idle points
  uint64_t used = 0, parked_bytes = 0, next_ticket = 1;
  bool stop = false;
  std::thread th;
  std::string err;
};

namespace {

void fail_req(Req *r, qram_status st, const std::string &msg) {
  r->state = 3;
  r->status = st;
  r->err = msg;
  r->t_done = now_ms();
}

// Destroy finished contexts.  hipFree waits for the device, so this runs
// only when no chunk is in flight or when admission needs the memory.
void release_parked(qram_server *s) {
  for (auto &p : s->parked) {
    if (p.second) (void)hipFree(p.second);
    qram_destroy(p.first);
  }
  s->parked.clear();
  s->used -= s->parked_bytes;
  s->parked_bytes = 0;
}

// Create the context of the request at the head of the queue and size it
// for chunks of `chunk` trajectories.
bool prepare(qram_server *s, Req *r) {
  if (r->ctx) return true;
  qram_status st = qram_create(r->q.n_addr, r->q.k_data, r->q.enc, r->q.gamma, r->mem.data(), &r->ctx);
  if (st) {
    std::lock_guard<std::mutex> lk(s->mu);
    fail_req(r, st, qram_last_error(nullptr));
    return false;
  }
  uint64_t fp = 0;
  st = qram_footprint(r->ctx, r->q.mode, std::min<uint32_t>(r->q.shots, s->chunk), &fp);
  if (st) {
    std::lock_guard<std::mutex> lk(s->mu);
    fail_req(r, st, qram_last_error(r->ctx));
    qram_destroy(r->ctx);
    r->ctx = nullptr;
    return false;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  r->footprint = fp + (uint64_t)r->q.shots * sizeof(double);
  return true;
}

void finish(qram_server *s, Req *r) {
  hipStream_t st = s->streams[r->slot];
  r->fid.resize(r->q.shots);
  hipError_t e = hipMemcpyAsync(r->fid.data(), r->d_fid, (size_t)r->q.shots * sizeof(double),
                                hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  const qram_status ke = e == hipSuccess ? qram_errors(r->ctx) : QRAM_E_DEVICE;
  std::lock_guard<std::mutex> lk(s->mu);
  if (e != hipSuccess) {
    fail_req(r, QRAM_E_DEVICE, hipGetErrorString(e));
  } else if (ke != QRAM_OK) {
    fail_req(r, ke, qram_last_error(r->ctx));
  } else {
    qram_fidelity(r->fid.data(), r->q.shots, &r->mean, &r->sem);
    r->state = 2;
    r->t_done = now_ms();
  }
  s->parked.emplace_back(r->ctx, r->d_fid);
  s->parked_bytes += r->footprint;
  r->ctx = nullptr;
  r->d_fid = nullptr;
  s->free_slots.push_back(r->slot);
  s->done.notify_all();
}

void serve(qram_server *s) {
  (void)hipSetDevice(s->device);
  std::vector<Req *> run;
  for (;;) {
    bool progress = false;
    // admission in arrival order
    for (;;) {
      Req *r;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->waiting.empty() || s->free_slots.empty()) break;
        r = s->waiting.front();
      }
      if (!prepare(s, r)) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->waiting.pop_front();
        s->done.notify_all();
        progress = true;
        continue;
      }
      if (r->footprint > s->budget) {
        std::lock_guard<std::mutex> lk(s->mu);
        fail_req(r, QRAM_E_CAPACITY, "request footprint exceeds the server's memory budget");
        s->parked.emplace_back(r->ctx, nullptr);
        r->ctx = nullptr;
        s->waiting.pop_front();
        s->done.notify_all();
        progress = true;
        continue;
      }
      if (s->used + r->footprint > s->budget) {
        if (s->parked.empty()) break;  // wait for running requests to finish
        release_parked(s);
        if (s->used + r->footprint > s->budget) break;
      }
      qram_status st = qram_reserve(r->ctx, r->q.mode, std::min<uint32_t>(r->q.shots, s->chunk));
      hipError_t e = st ? hipSuccess : hipMalloc(reinterpret_cast<void **>(&r->d_fid), (size_t)r->q.shots * sizeof(double) + 8);
      std::lock_guard<std::mutex> lk(s->mu);
      s->waiting.pop_front();
      if (st || e != hipSuccess) {
        fail_req(r, st ? st : QRAM_E_NOMEM, st ? qram_last_error(r->ctx) : "device allocation failed");
        s->parked.emplace_back(r->ctx, nullptr);
        r->ctx = nullptr;
        s->done.notify_all();
        progress = true;
        continue;
      }
      r->slot = s->free_slots.back();
      s->free_slots.pop_back();
      s->used += r->footprint;
      r->state = 1;
      r->t_admit = now_ms();
      run.push_back(r);
      progress = true;
    }
    // one chunk in flight per running request
    for (Req *r : run) {
      if (r->inflight || r->next >= r->q.shots || r->state != 1) continue;
      const uint32_t cnt = std::min<uint32_t>(s->chunk, r->q.shots - r->next);
      hipStream_t st = s->streams[r->slot];
      const qram_status q = r->q.mode == QRAM_MODE_PRUNED
                                ? qram_run_pruned_async(r->ctx, r->q.seed, r->q.traj0 + r->next, cnt, r->d_fid + r->next, nullptr, st)
                                : qram_run_full_async(r->ctx, r->q.seed, r->q.traj0 + r->next, cnt, r->d_fid + r->next, nullptr, st);
      if (q != QRAM_OK || hipEventRecord(s->events[r->slot], st) != hipSuccess) {
        std::lock_guard<std::mutex> lk(s->mu);
        fail_req(r, q ? q : QRAM_E_DEVICE, qram_last_error(r->ctx));
        continue;
      }
      r->inflight = cnt;
      progress = true;
    }
    // completions
    bool any_inflight = false;
    for (size_t i = 0; i < run.size();) {
      Req *r = run[i];
      if (r->inflight) {
        const hipError_t e = hipEventQuery(s->events[r->slot]);
        if (e == hipSuccess) {
          r->next += r->inflight;
          r->inflight = 0;
          progress = true;
        } else if (e != hipErrorNotReady) {
          std::lock_guard<std::mutex> lk(s->mu);
          fail_req(r, QRAM_E_DEVICE, hipGetErrorString(e));
          r->inflight = 0;
        } else {
          any_inflight = true;
        }
      }
      if (!r->inflight && (r->next >= r->q.shots || r->state == 3)) {
        if (r->state == 3) {  // failed while running
          (void)hipStreamSynchronize(s->streams[r->slot]);
          std::lock_guard<std::mutex> lk(s->mu);
          s->parked.emplace_back(r->ctx, r->d_fid);
          s->parked_bytes += r->footprint;
          r->ctx = nullptr;
          r->d_fid = nullptr;
          s->free_slots.push_back(r->slot);
          s->done.notify_all();
        } else {
          finish(s, r);
        }
        run.erase(run.begin() + i);
        progress = true;
        continue;
      }
      ++i;
    }
    if (!any_inflight && !s->parked.empty()) release_parked(s);
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->stop && run.empty() && s->waiting.empty()) break;
    if (!progress) {
      if (run.empty() && s->waiting.empty())
        s->wake.wait(lk, [s] { return s->stop || !s->waiting.empty(); });
      else
        s->wake.wait_for(lk, std::chrono::microseconds(50));
    }
  }
  release_parked(s);
}

void fill_result(const Req *r, qram_result *out) {
  std::memset(out, 0, sizeof(*out));
  out->ticket = r->ticket;
  out->state = r->state;
  out->status = r->status;
  out->mean = r->mean;
  out->sem = r->sem;
  out->shots = r->q.shots;
  out->footprint_bytes = r->footprint;
  out->queue_ms = r->t_admit > 0 ? r->t_admit - r->t_submit : 0.0;
  out->latency_ms = r->t_done > 0 ? r->t_done - r->t_submit : 0.0;
}

}  // namespace

extern "C" {

qram_status qram_server_create(uint64_t hbm_budget_bytes, int max_active,
                               uint32_t chunk, qram_server **out) {
  if (!out || hbm_budget_bytes == 0 || max_active < 1 || max_active > 64 || chunk == 0)
    return QRAM_E_INVAL;
  *out = nullptr;
  qram_server *s = new (std::nothrow) qram_server();
  if (!s) return QRAM_E_NOMEM;
  s->budget = hbm_budget_bytes;
  s->max_active = max_active;
  s->chunk = chunk;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return QRAM_E_DEVICE;
  }
  for (int i = 0; i < max_active; ++i) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      if (st) (void)hipStreamDestroy(st);
      for (auto x : s->streams) (void)hipStreamDestroy(x);
      for (auto x : s->events) (void)hipEventDestroy(x);
      delete s;
      return QRAM_E_DEVICE;
    }
    s->streams.push_back(st);
    s->events.push_back(ev);
    s->free_slots.push_back(max_active - 1 - i);
  }
  s->th = std::thread(serve, s);
  *out = s;
  return QRAM_OK;
}

qram_status qram_server_submit(qram_server *s, const qram_request *req,
                               uint64_t *ticket) {
  if (!s || !req || !ticket || !req->memory_bits) return QRAM_E_INVAL;
  if (req->n_addr < 1 || req->n_addr > 15) return QRAM_E_RANGE;
  if (req->mode != QRAM_MODE_FULL && req->mode != QRAM_MODE_PRUNED) return QRAM_E_INVAL;
  if (req->shots == 0) return QRAM_E_INVAL;
  if (req->traj0 + (uint64_t)req->shots > (1ull << 32)) return QRAM_E_RANGE;
  Req *r = new (std::nothrow) Req();
  if (!r) return QRAM_E_NOMEM;
  r->q = *req;
  r->mem.assign(req->memory_bits, req->memory_bits + ((size_t)1 << req->n_addr));
  r->q.memory_bits = nullptr;
  r->t_submit = now_ms();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      delete r;
      return QRAM_E_INVAL;
    }
    r->ticket = s->next_ticket++;
    s->all[r->ticket] = r;
    s->waiting.push_back(r);
  }
  s->wake.notify_all();
  *ticket = r->ticket;
  return QRAM_OK;
}

qram_status qram_server_poll(qram_server *s, uint64_t ticket, qram_result *out) {
  if (!s || !out) return QRAM_E_INVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return QRAM_E_INVAL;
  fill_result(it->second, out);
  return QRAM_OK;
}

qram_status qram_server_wait(qram_server *s, uint64_t ticket, double timeout_ms,
                             qram_result *out) {
  if (!s || !out) return QRAM_E_INVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return QRAM_E_INVAL;
  Req *r = it->second;
  auto ready = [r] { return r->state >= 2; };
  if (timeout_ms < 0)
    s->done.wait(lk, ready);
  else
    s->done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), ready);
  fill_result(r, out);
  return QRAM_OK;
}

qram_status qram_server_fidelities(qram_server *s, uint64_t ticket,
                                   double *fid, uint32_t n) {
  if (!s || !fid) return QRAM_E_INVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return QRAM_E_INVAL;
  const Req *r = it->second;
  if (r->state != 2) return QRAM_E_INVAL;
  if (n < r->q.shots) return QRAM_E_RANGE;
  std::memcpy(fid, r->fid.data(), (size_t)r->q.shots * sizeof(double));
  return QRAM_OK;
}

qram_status qram_server_release(qram_server *s, uint64_t ticket) {
  if (!s) return QRAM_E_INVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return QRAM_E_INVAL;
  if (it->second->state < 2) return QRAM_E_INVAL;
  delete it->second;
  s->all.erase(it);
  return QRAM_OK;
}

void qram_server_destroy(qram_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->wake.notify_all();
  if (s->th.joinable()) s->th.join();
  for (auto x : s->streams) (void)hipStreamDestroy(x);
  for (auto x : s->events) (void)hipEventDestroy(x);
  for (auto &kv : s->all) delete kv.second;
  delete s;
}

}  // extern "C"
