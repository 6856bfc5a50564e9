// Request server over resident tracks: callers submit (track, H_t, W)
// requests from any thread; a dispatcher thread gathers the pending requests
// into batched launches (at most one request per track per launch, in
// submission order per track) and a completion thread stamps each request
// once its launch has finished on the GPU.  Mode UPDATE runs Alg. 2 on the
// track (rzf_update_batch); mode FULL computes the full-inversion RZF of the
// request's snapshot with the track's alpha and P (the track state is not
// touched), the baseline on the same request stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <mutex>
#include <new>
#include <set>
#include <thread>
#include <vector>

#include "runtime.h"

using namespace rzfrt;

namespace {

struct Request {
  rzf_track* tr;
  const rzf_c32* H;
  int ldh;
  rzf_c32* W;
  int ldw;
  uint64_t tag;
  double t_submit;
};

struct Batch {
  std::vector<Request> reqs;
  hipEvent_t ev = nullptr;
  DevInfo* slots = nullptr;
  double t_launch = 0.0;
  rzf_status st = RZF_OK;
};

using Clock = std::chrono::steady_clock;

}  // namespace

struct rzf_server {
  rzf_ctx* ctx = nullptr;
  rzf_server_params prm{};
  Clock::time_point t0;
  std::mutex m;
  std::condition_variable cv_pending, cv_inflight, cv_done;
  std::list<Request> pending;
  std::deque<Batch> inflight;
  std::deque<rzf_completion> done;
  std::vector<hipEvent_t> ev_free;
  std::vector<DevInfo*> slot_free;
  DevInfo* slot_base = nullptr;
  bool stop = false, dispatcher_done = false;
  uint64_t submitted = 0, completed = 0;
  std::thread dispatcher, completer;

  double now() const { return std::chrono::duration<double, std::micro>(Clock::now() - t0).count(); }
};

namespace {

void dispatch_loop(rzf_server* S) {
  (void)hipSetDevice(S->ctx->device);
  const int maxb = S->prm.max_batch;
  std::unique_lock<std::mutex> lk(S->m);
  for (;;) {
    S->cv_pending.wait(lk, [&] { return S->stop || !S->pending.empty(); });
    if (S->pending.empty()) break;   // stop requested and nothing left
    // a fuller batch, until the oldest request has waited max_wait_us
    const double deadline = S->pending.front().t_submit + S->prm.max_wait_us;
    while (!S->stop && (int)S->pending.size() < maxb && S->now() < deadline) {
      const auto tp = S->t0 + std::chrono::duration_cast<Clock::duration>(
                                  std::chrono::duration<double, std::micro>(deadline));
      S->cv_pending.wait_until(lk, tp);
    }
    S->cv_inflight.wait(lk, [&] { return (int)S->inflight.size() < S->prm.max_inflight; });
    Batch b;
    std::set<rzf_track*> used;
    for (auto it = S->pending.begin(); it != S->pending.end() && (int)b.reqs.size() < maxb;) {
      if (used.insert(it->tr).second) {
        b.reqs.push_back(*it);
        it = S->pending.erase(it);
      } else {
        ++it;   // a later request of a track already in this batch waits for the next one
      }
    }
    b.ev = S->ev_free.back();
    S->ev_free.pop_back();
    b.slots = S->slot_free.back();
    S->slot_free.pop_back();
    lk.unlock();
    const int n = (int)b.reqs.size();
    rzf_ctx* c = S->ctx;
    {
      std::lock_guard<std::mutex> cl(c->mu);
      if (S->prm.mode == RZF_SERVE_FULL) {
        std::vector<rzf_full_item> items(n);
        for (int i = 0; i < n; ++i) {
          const Request& r = b.reqs[i];
          items[i] = rzf_full_item{r.tr->K, r.tr->N, r.H, r.ldh, r.tr->alpha, r.tr->prm.P, r.W, r.ldw,
                                   r.tr->prm.precision};
        }
        b.st = full_batch_locked(c, n, items.data());
      } else {
        std::vector<rzf_update_item> items(n);
        std::vector<DevInfo*> slots(n);
        for (int i = 0; i < n; ++i) {
          const Request& r = b.reqs[i];
          items[i] = rzf_update_item{r.tr, r.H, r.ldh, r.W, r.ldw, nullptr};
          slots[i] = b.slots + i;
        }
        b.st = update_batch_locked(c, n, items.data(), S->prm.tol, slots.data());
      }
      if (b.st == RZF_OK && hipEventRecord(b.ev, c->stream) != hipSuccess) b.st = RZF_E_DEVICE;
    }
    b.t_launch = S->now();
    lk.lock();
    S->inflight.push_back(std::move(b));
    S->cv_inflight.notify_all();
  }
  S->dispatcher_done = true;
  S->cv_inflight.notify_all();
}

void complete_loop(rzf_server* S) {
  (void)hipSetDevice(S->ctx->device);
  std::unique_lock<std::mutex> lk(S->m);
  for (;;) {
    S->cv_inflight.wait(lk, [&] { return !S->inflight.empty() || S->dispatcher_done; });
    if (S->inflight.empty()) break;   // the dispatcher has stopped and nothing is in flight
    Batch b = std::move(S->inflight.front());
    S->inflight.pop_front();
    lk.unlock();
    rzf_status st = b.st;
    if (st == RZF_OK && hipEventSynchronize(b.ev) != hipSuccess) st = RZF_E_DEVICE;
    const double t_done = S->now();
    lk.lock();
    for (size_t i = 0; i < b.reqs.size(); ++i) {
      rzf_completion cpl;
      std::memset(&cpl, 0, sizeof(cpl));
      cpl.tag = b.reqs[i].tag;
      cpl.status = st;
      if (st == RZF_OK && S->prm.mode != RZF_SERVE_FULL)
        std::memcpy(&cpl.info, b.slots + i, sizeof(rzf_update_info));
      cpl.t_submit_us = b.reqs[i].t_submit;
      cpl.t_launch_us = b.t_launch;
      cpl.t_done_us = t_done;
      S->done.push_back(cpl);
    }
    S->completed += b.reqs.size();
    S->ev_free.push_back(b.ev);
    S->slot_free.push_back(b.slots);
    S->cv_inflight.notify_all();
    S->cv_done.notify_all();
  }
}

rzf_status enqueue(rzf_server* S, rzf_track* tr, const rzf_c32* H, int ldh, rzf_c32* W, int ldw,
                   uint64_t tag) {
  if (!tr || !H || !W || tr->ctx != S->ctx) return RZF_E_INVALID;
  if (ldh < tr->N || ldw < tr->K) return RZF_E_SHAPE;
  std::lock_guard<std::mutex> lk(S->m);
  if (S->stop) return RZF_E_INVALID;
  S->pending.push_back(Request{tr, H, ldh, W, ldw, tag, S->now()});
  ++S->submitted;
  S->cv_pending.notify_one();
  return RZF_OK;
}

}  // namespace

extern "C" {

rzf_status rzf_server_params_default(rzf_server_params* p) {
  if (!p) return RZF_E_INVALID;
  std::memset(p, 0, sizeof(*p));
  p->max_batch = 512;
  p->max_wait_us = 1000.0;
  p->tol = 0.999;
  p->mode = RZF_SERVE_UPDATE;
  p->max_inflight = 2;
  return RZF_OK;
}

rzf_status rzf_server_create(rzf_ctx* c, const rzf_server_params* p, rzf_server** out) {
  if (!c || !p || !out) return RZF_E_INVALID;
  *out = nullptr;
  if (p->max_batch < 1 || p->max_batch > RZF_BATCH_MAX || !(p->max_wait_us >= 0.0) ||
      !(p->tol > 0.0 && p->tol <= 1.0) || (p->mode != RZF_SERVE_UPDATE && p->mode != RZF_SERVE_FULL) ||
      p->max_inflight < 1 || p->max_inflight > 8)
    return RZF_E_INVALID;
  rzf_server* S = new (std::nothrow) rzf_server();
  if (!S) return RZF_E_NOMEM;
  S->ctx = c;
  S->prm = *p;
  S->t0 = Clock::now();
  if (hipSetDevice(c->device) != hipSuccess) { delete S; return RZF_E_DEVICE; }
  const int pools = p->max_inflight + 1;
  if (hipHostMalloc((void**)&S->slot_base, sizeof(DevInfo) * p->max_batch * pools, hipHostMallocDefault) !=
      hipSuccess) {
    delete S;
    return RZF_E_DEVICE;
  }
  for (int k = 0; k < pools; ++k) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      for (hipEvent_t x : S->ev_free) (void)hipEventDestroy(x);
      (void)hipHostFree(S->slot_base);
      delete S;
      return RZF_E_DEVICE;
    }
    S->ev_free.push_back(e);
    S->slot_free.push_back(S->slot_base + (size_t)k * p->max_batch);
  }
  S->dispatcher = std::thread(dispatch_loop, S);
  S->completer = std::thread(complete_loop, S);
  *out = S;
  return RZF_OK;
}

rzf_status rzf_server_submit(rzf_server* S, rzf_track* tr, const rzf_c32* H_t, int ldh, rzf_c32* W,
                             int ldw, uint64_t tag) {
  if (!S) return RZF_E_INVALID;
  return enqueue(S, tr, H_t, ldh, W, ldw, tag);
}

rzf_status rzf_server_replay(rzf_server* S, int n, const rzf_serve_request* reqs) {
  if (!S || n < 0 || (n > 0 && !reqs)) return RZF_E_INVALID;
  for (int i = 0; i < n; ++i)
    if (!reqs[i].track || !reqs[i].H || !reqs[i].W || reqs[i].track->ctx != S->ctx ||
        !(reqs[i].t_arrival_us >= 0.0) || (i > 0 && reqs[i].t_arrival_us < reqs[i - 1].t_arrival_us))
      return RZF_E_INVALID;
  const double base = S->now();
  for (int i = 0; i < n; ++i) {
    const double due = base + reqs[i].t_arrival_us;
    while (S->now() < due) {
      if (due - S->now() > 200.0) std::this_thread::sleep_for(std::chrono::microseconds(50));
      else std::this_thread::yield();
    }
    const rzf_serve_request& r = reqs[i];
    const rzf_status st = enqueue(S, r.track, r.H, r.ldh, r.W, r.ldw, r.tag);
    if (st != RZF_OK) return st;
  }
  return RZF_OK;
}

rzf_status rzf_server_poll(rzf_server* S, rzf_completion* out, int max, int* n_out) {
  if (!S || !n_out || max < 0 || (max > 0 && !out)) return RZF_E_INVALID;
  std::lock_guard<std::mutex> lk(S->m);
  int k = 0;
  while (k < max && !S->done.empty()) {
    out[k++] = S->done.front();
    S->done.pop_front();
  }
  *n_out = k;
  return RZF_OK;
}

rzf_status rzf_server_drain(rzf_server* S) {
  if (!S) return RZF_E_INVALID;
  std::unique_lock<std::mutex> lk(S->m);
  S->cv_pending.notify_all();
  S->cv_done.wait(lk, [&] { return S->completed == S->submitted; });
  return RZF_OK;
}

double rzf_server_now_us(rzf_server* S) { return S ? S->now() : 0.0; }

rzf_status rzf_server_destroy(rzf_server* S) {
  if (!S) return RZF_E_INVALID;
  {
    std::lock_guard<std::mutex> lk(S->m);
    S->stop = true;   // pending requests are still dispatched
  }
  S->cv_pending.notify_all();
  S->dispatcher.join();
  S->completer.join();
  (void)hipSetDevice(S->ctx->device);
  for (hipEvent_t e : S->ev_free) (void)hipEventDestroy(e);
  (void)hipHostFree(S->slot_base);
  delete S;
  return RZF_OK;
}

}  // extern "C"
