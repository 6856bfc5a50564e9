// Request server over resident tracks, with continuous batching.
//
// Callers submit (track, H_t, W) requests from any thread.  Requests go to a
// lane by the kernel family of their track (K <= 64: the kernels whose working
// set sits in LDS; K > 64: the blocked large-track kernels), and each lane
// launches on a stream of its own, so the two families' batches run on the
// device at the same time instead of the small tracks waiting behind the
// large ones.  A dispatcher thread forms a lane's next batch whenever that
// lane has a free in-flight slot and either max_batch of its requests are
// pending or the oldest has waited max_wait_us: requests that arrive while
// earlier batches run are admitted as soon as a slot frees.  A batch takes
// at most one request per track, in submission order per track; a track's
// later requests go to later batches of the same lane, which run in order on
// its stream.  One completion thread per lane waits on the lane's batches in
// launch order and stamps each request, with the batch's own device error
// status (every in-flight slot has its own error word).
//
// Mode UPDATE runs Alg. 2 on the track (the batched rzf_update); mode FULL
// computes the full-inversion RZF of the request's snapshot with the track's
// alpha and P, using the track's own Gram and partial-sum buffers as scratch
// (the track's state is not changed): the baseline on the same requests.
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

constexpr int NLANES = 2;   // K <= KS, K > KS

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
  int slot = 0;
  double t_launch = 0.0;
  rzf_status st = RZF_OK;
};

struct Lane {
  hipStream_t stream = nullptr;
  std::list<Request> pending;
  std::deque<Batch> inflight;      // in launch order
  std::vector<int> free_slots;
  // per in-flight slot
  std::vector<hipEvent_t> ev;
  std::vector<DevInfo*> info;      // pinned, max_batch records
  std::vector<int*> d_err;         // device error word
  std::vector<int*> h_err;         // pinned copy of it, valid once ev has completed
  std::thread completer;
};

using Clock = std::chrono::steady_clock;

int lane_of(const rzf_track* t) { return t->K > KS ? 1 : 0; }

rzf_status status_of(int code) {
  if (code == DEV_ERR_NOT_HPD) return RZF_E_NOT_HPD;
  if (code == DEV_ERR_NONFINITE) return RZF_E_NONFINITE;
  return code ? RZF_E_DEVICE : RZF_OK;
}

}  // namespace

struct rzf_server {
  rzf_ctx* ctx = nullptr;
  rzf_server_params prm{};
  Clock::time_point t0;
  std::mutex m;
  std::condition_variable cv_work, cv_done;
  Lane lanes[NLANES];
  std::deque<rzf_completion> done;
  DevInfo* info_base = nullptr;
  int* d_err_base = nullptr;
  int* h_err_base = nullptr;
  bool stop = false, dispatcher_done = false;
  uint64_t submitted = 0, completed = 0;
  std::thread dispatcher;

  double now() const { return std::chrono::duration<double, std::micro>(Clock::now() - t0).count(); }
};

namespace {

// A lane may launch now: a free slot and a full batch, a request past its
// wait, or the server stopping.
bool lane_ready(const rzf_server* S, const Lane& L, double now) {
  if (L.pending.empty() || L.free_slots.empty()) return false;
  return S->stop || (int)L.pending.size() >= S->prm.max_batch ||
         now >= L.pending.front().t_submit + S->prm.max_wait_us;
}

// Launch one batch of lane l from slot b.slot (S->m not held).
void launch_batch(rzf_server* S, int l, Batch& b) {
  rzf_ctx* c = S->ctx;
  Lane& L = S->lanes[l];
  const int n = (int)b.reqs.size();
  const int k = b.slot;
  std::lock_guard<std::mutex> cl(c->mu);
  hipStream_t s = L.stream;
  if (hipMemsetAsync(L.d_err[k], 0, sizeof(int), s) != hipSuccess) {
    b.st = RZF_E_DEVICE;
    return;
  }
  if (S->prm.mode == RZF_SERVE_FULL) {
    std::vector<rzf_full_item> items(n);
    std::vector<FullScratch> scr(n);
    for (int i = 0; i < n; ++i) {
      const Request& r = b.reqs[i];
      items[i] = rzf_full_item{r.tr->K, r.tr->N, r.H, r.ldh, r.tr->alpha, r.tr->prm.P, r.W, r.ldw,
                               r.tr->prm.precision};
      scr[i] = FullScratch{r.tr->h_desc.Anew, r.tr->h_desc.wpart};
    }
    b.st = full_batch_locked(c, n, items.data(), scr.data(), s, L.d_err[k]);
  } else {
    std::vector<rzf_update_item> items(n);
    std::vector<DevInfo*> slots(n);
    for (int i = 0; i < n; ++i) {
      const Request& r = b.reqs[i];
      items[i] = rzf_update_item{r.tr, r.H, r.ldh, r.W, r.ldw, nullptr};
      slots[i] = L.info[k] + i;
    }
    b.st = update_batch_locked(c, n, items.data(), S->prm.tol, slots.data(), s, L.d_err[k]);
  }
  if (b.st == RZF_OK &&
      (hipMemcpyAsync(L.h_err[k], L.d_err[k], sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
       hipEventRecord(L.ev[k], s) != hipSuccess))
    b.st = RZF_E_DEVICE;
}

void dispatch_loop(rzf_server* S) {
  (void)hipSetDevice(S->ctx->device);
  const int maxb = S->prm.max_batch;
  std::unique_lock<std::mutex> lk(S->m);
  for (;;) {
    const double now = S->now();
    int l = -1;
    for (int q = 0; q < NLANES && l < 0; ++q)
      if (lane_ready(S, S->lanes[q], now)) l = q;
    if (l < 0) {
      bool any_pending = false;
      double wake = 1e300;   // the earliest deadline of a lane that has a free slot
      for (const Lane& L : S->lanes) {
        if (L.pending.empty()) continue;
        any_pending = true;
        if (!L.free_slots.empty()) wake = std::min(wake, L.pending.front().t_submit + S->prm.max_wait_us);
      }
      if (S->stop && !any_pending) break;
      if (wake < 1e300) {
        const auto tp = S->t0 + std::chrono::duration_cast<Clock::duration>(
                                    std::chrono::duration<double, std::micro>(wake));
        S->cv_work.wait_until(lk, tp);
      } else {
        S->cv_work.wait(lk);   // a new request, a freed slot or stop
      }
      continue;
    }
    Lane& L = S->lanes[l];
    Batch b;
    std::set<rzf_track*> used;
    for (auto it = L.pending.begin(); it != L.pending.end() && (int)b.reqs.size() < maxb;) {
      if (used.insert(it->tr).second) {
        b.reqs.push_back(*it);
        it = L.pending.erase(it);
      } else {
        ++it;   // a later request of a track already in this batch waits for the next one
      }
    }
    b.slot = L.free_slots.back();
    L.free_slots.pop_back();
    lk.unlock();
    launch_batch(S, l, b);
    b.t_launch = S->now();
    lk.lock();
    L.inflight.push_back(std::move(b));
    S->cv_done.notify_all();   // wakes this lane's completion thread
  }
  S->dispatcher_done = true;
  S->cv_done.notify_all();
}

void complete_loop(rzf_server* S, int l) {
  (void)hipSetDevice(S->ctx->device);
  Lane& L = S->lanes[l];
  std::unique_lock<std::mutex> lk(S->m);
  for (;;) {
    S->cv_done.wait(lk, [&] { return !L.inflight.empty() || S->dispatcher_done; });
    if (L.inflight.empty()) break;   // the dispatcher has stopped and nothing is in flight
    Batch& b = L.inflight.front();
    const int k = b.slot;
    rzf_status st = b.st;
    lk.unlock();
    if (st == RZF_OK) st = hipEventSynchronize(L.ev[k]) == hipSuccess ? status_of(*L.h_err[k]) : RZF_E_DEVICE;
    const double t_done = S->now();
    lk.lock();
    for (size_t i = 0; i < b.reqs.size(); ++i) {
      rzf_completion cpl;
      std::memset(&cpl, 0, sizeof(cpl));
      cpl.tag = b.reqs[i].tag;
      cpl.status = st;
      if (b.st == RZF_OK && S->prm.mode != RZF_SERVE_FULL)
        std::memcpy(&cpl.info, L.info[k] + i, sizeof(rzf_update_info));
      cpl.t_submit_us = b.reqs[i].t_submit;
      cpl.t_launch_us = b.t_launch;
      cpl.t_done_us = t_done;
      S->done.push_back(cpl);
    }
    S->completed += b.reqs.size();
    L.inflight.pop_front();
    L.free_slots.push_back(k);
    S->cv_work.notify_all();
    S->cv_done.notify_all();
  }
}

rzf_status enqueue(rzf_server* S, rzf_track* tr, const rzf_c32* H, int ldh, rzf_c32* W, int ldw,
                   uint64_t tag) {
  if (!tr || !H || !W || tr->ctx != S->ctx) return RZF_E_INVALID;
  if (ldh < tr->N || ldw < tr->K) return RZF_E_SHAPE;
  std::lock_guard<std::mutex> lk(S->m);
  if (S->stop) return RZF_E_INVALID;
  S->lanes[lane_of(tr)].pending.push_back(Request{tr, H, ldh, W, ldw, tag, S->now()});
  ++S->submitted;
  S->cv_work.notify_all();
  return RZF_OK;
}

void release(rzf_server* S) {
  for (Lane& L : S->lanes) {
    for (hipEvent_t e : L.ev)
      if (e) (void)hipEventDestroy(e);
    if (L.stream) (void)hipStreamDestroy(L.stream);
  }
  if (S->info_base) (void)hipHostFree(S->info_base);
  if (S->h_err_base) (void)hipHostFree(S->h_err_base);
  if (S->d_err_base) (void)hipFree(S->d_err_base);
  delete S;
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
  const int slots = p->max_inflight;
  const int total = NLANES * slots;
  bool ok = hipSetDevice(c->device) == hipSuccess &&
            hipHostMalloc((void**)&S->info_base, sizeof(DevInfo) * p->max_batch * total, hipHostMallocDefault) ==
                hipSuccess &&
            hipHostMalloc((void**)&S->h_err_base, sizeof(int) * 64 * total, hipHostMallocDefault) == hipSuccess &&
            hipMalloc((void**)&S->d_err_base, sizeof(int) * 64 * total) == hipSuccess;
  for (int l = 0; l < NLANES && ok; ++l) {
    Lane& L = S->lanes[l];
    // default priority (the streams of one process keep equal priorities)
    ok = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) == hipSuccess;
    for (int k = 0; k < slots && ok; ++k) {
      hipEvent_t e = nullptr;
      ok = hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
      L.ev.push_back(e);
      const int g = l * slots + k;
      L.info.push_back(S->info_base + (size_t)g * p->max_batch);
      L.d_err.push_back(S->d_err_base + 64 * g);   // one 256-byte line per word
      L.h_err.push_back(S->h_err_base + 64 * g);
      L.free_slots.push_back(slots - 1 - k);
    }
  }
  if (!ok) {
    release(S);
    return RZF_E_DEVICE;
  }
  S->dispatcher = std::thread(dispatch_loop, S);
  for (int l = 0; l < NLANES; ++l) S->lanes[l].completer = std::thread(complete_loop, S, l);
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
  S->cv_work.notify_all();
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
  S->cv_work.notify_all();
  S->dispatcher.join();
  for (Lane& L : S->lanes) L.completer.join();
  (void)hipSetDevice(S->ctx->device);
  release(S);
  return RZF_OK;
}

}  // extern "C"
