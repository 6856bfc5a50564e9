// Captured steps (rzf_graph_*): one update or full-inversion step, and
// optionally its sum rate, recorded from the context's stream into HIP graphs
// by the same launch code as the eager calls, then replayed by one
// hipGraphLaunch per step.  Job arrays and scratch live in an arena region
// of the graph, uploaded once before the capture, so a replay copies nothing
// and allocates nothing.  The step index and the two-phase tag number come
// from the track descriptors on the device (advanced by each step's last
// launch), so a replay of the same launches computes the next step.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <vector>

#include "runtime.h"

using namespace rzfrt;

struct rzf_graph {
  rzf_ctx* c = nullptr;
  bool update = false;
  std::vector<rzf_track*> tracks;
  hipGraphExec_t exec[2] = {nullptr, nullptr};   // [0] a Woodbury (or full-inversion) step,
                                                 // [1] an FP64 re-inversion step
  size_t off = 0, bytes = 0;                     // arena region: job arrays, then scratch
};

namespace {

#define HIP_OK(x) do { if ((x) != hipSuccess) return RZF_E_DEVICE; } while (0)

// Record what launch(s) enqueues as an executable graph (c->mu held).  The
// launches are recorded on a private stream (the context's may be the null
// stream, which cannot be captured); the graph is later launched on the
// context's stream.  No timing events are recorded meanwhile.
template <class F>
rzf_status capture(rzf_ctx* c, const F& launch, hipGraphExec_t* exec) {
  hipStream_t s = nullptr;
  HIP_OK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipStreamDestroy(s);
    return RZF_E_DEVICE;
  }
  c->capturing = true;
  launch(s);
  c->capturing = false;
  hipGraph_t g = nullptr;
  const hipError_t e1 = hipStreamEndCapture(s, &g);
  (void)hipStreamDestroy(s);
  if (e1 != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return RZF_E_DEVICE;
  }
  const hipError_t e2 = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e2 == hipSuccess ? RZF_OK : RZF_E_DEVICE;
}

// Frees what the graph holds (c->mu held).
void release(rzf_graph* g) {
  for (hipGraphExec_t& e : g->exec)
    if (e) { (void)hipGraphExecDestroy(e); e = nullptr; }
  if (g->bytes) arena_give(g->c, g->off, g->bytes);
  for (rzf_track* t : g->tracks) t->graphs -= 1;
  g->c->graphs.erase(g);
  delete g;
}

bool rate_ok(const rzf_graph_rate* r) {
  return !r || (r->sums && std::isfinite(r->P) && r->P > 0.0 && std::isfinite(r->sigma2) && r->sigma2 >= 0.0);
}

// Job arrays in the graph's region: built on the host, copied once on the
// context stream (ordered after any earlier use of the region's memory).
struct Upload {
  std::vector<char> host;
  Stager st;
  // `bytes` bounds what the plans put (their bytes() include the alignment)
  explicit Upload(char* dev, size_t bytes) : host(bytes + 256), st{host.data(), dev} {}
  rzf_status commit(hipStream_t s) {
    if (st.used > host.size() - 256) return RZF_E_INVALID;
    if (st.used == 0) return RZF_OK;
    HIP_OK(hipMemcpyAsync(st.d, st.h, st.used, hipMemcpyHostToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
    return RZF_OK;
  }
};

// A new graph object on context c with an arena region of `bytes` (c->mu held).
rzf_status graph_new(rzf_ctx* c, bool update, size_t bytes, rzf_graph** out) {
  rzf_graph* g = new (std::nothrow) rzf_graph();
  if (!g) return RZF_E_NOMEM;
  g->c = c;
  g->update = update;
  if (bytes) {
    if (!arena_take(c, bytes, &g->off)) { delete g; return RZF_E_NOMEM; }
    g->bytes = bytes;
  }
  c->graphs.insert(g);
  *out = g;
  return RZF_OK;
}

std::vector<rzf_rate_item> rate_items_of(int n, const int* K, const int* N, const rzf_c32* const* H,
                                         const int* ldh, rzf_c32* const* W, const int* ldw,
                                         const rzf_graph_rate* rate) {
  std::vector<rzf_rate_item> ri(n);
  for (int i = 0; i < n; ++i)
    ri[i] = rzf_rate_item{K[i], N[i], H[i], ldh[i], W[i], ldw[i], nullptr, rate->sums + i, -1.0};
  return ri;
}

}  // namespace

namespace rzfrt {

void graphs_release_all(rzf_ctx* c) {
  while (!c->graphs.empty()) {
    rzf_graph* g = *c->graphs.begin();
    g->bytes = 0;   // the arena goes with the context
    release(g);
  }
}

}  // namespace rzfrt

extern "C" {

rzf_status rzf_graph_update(rzf_ctx* c, int n, const rzf_update_item* items, double tol,
                            const rzf_graph_rate* rate, rzf_graph** out) {
  if (!out) return RZF_E_INVALID;
  *out = nullptr;
  const rzf_status st0 = check_update_items(c, n, items, tol);
  if (st0 != RZF_OK) return st0;
  if (!rate_ok(rate)) return RZF_E_INVALID;
  std::lock_guard<std::mutex> lk(c->mu);
  HIP_OK(hipSetDevice(c->device));
  const rzf_track* t0 = items[0].track;
  for (int i = 1; i < n; ++i) {
    const rzf_track* t = items[i].track;
    if (t->prm.reset_period != t0->prm.reset_period || t->since_reset != t0->since_reset)
      return RZF_E_INVALID;
  }
  const int nexec = t0->prm.reset_period > 0 ? 2 : 1;
  std::vector<int> K(n), N(n), ldh(n), ldw(n);
  std::vector<const rzf_c32*> H(n);
  std::vector<rzf_c32*> W(n);
  for (int i = 0; i < n; ++i) {
    K[i] = items[i].track->K; N[i] = items[i].track->N;
    H[i] = items[i].H; W[i] = items[i].W; ldh[i] = items[i].ldh; ldw[i] = items[i].ldw;
  }
  // n > 1: both steps' job arrays, the sum rate's job array and scratch
  UpdatePlan up[2];
  RatePlan rp;
  std::vector<rzf_rate_item> ri;
  size_t jobs = 0, part = 0;
  if (n > 1) {
    for (int e = 0; e < nexec; ++e) {
      plan_update(up[e], n, items, tol, e);
      jobs += up[e].bytes();
    }
    if (rate) {
      jobs += sizeof(RateJob) * n + 64;
      for (int i = 0; i < n; ++i) part += rate_scratch_bytes(K[i]);
    }
  }
  jobs = align_up(jobs);
  rzf_graph* g = nullptr;
  rzf_status st = graph_new(c, true, jobs + part, &g);
  if (st != RZF_OK) return st;
  for (int i = 0; i < n; ++i) {
    g->tracks.push_back(items[i].track);
    items[i].track->graphs += 1;
  }
  if (rate) ri = rate_items_of(n, K.data(), N.data(), H.data(), ldh.data(), W.data(), ldw.data(), rate);
  if (n > 1) {
    char* base = c->arena + g->off;
    if (rate) plan_rate(rp, n, ri.data(), rate->P, rate->sigma2, base + jobs, c->d_counts);
    Upload u(base, jobs);
    for (int e = 0; e < nexec; ++e) up[e].put(u.st);
    if (rate) rp.put(u.st);
    st = u.commit(c->stream);
  }
  for (int e = 0; e < nexec && st == RZF_OK; ++e) {
    st = capture(c, [&](hipStream_t s) {
      if (n > 1) {
        up[e].launch(c, s, c->d_err);
        if (rate) rp.launch(c, s, c->d_err);
      } else {
        rzf_track* t = items[0].track;
        const float2* Hf = reinterpret_cast<const float2*>(items[0].H);
        float2* Wf = reinterpret_cast<float2*>(items[0].W);
        update_single_launch(c, t, Hf, items[0].ldh, tol, Wf, items[0].ldw, e == 1, s);
        if (rate)
          rate_single_launch(c, t->K, t->N, Hf, items[0].ldh, Wf, items[0].ldw, rate->P, rate->sigma2, nullptr,
                             rate->sums, s);
      }
    }, &g->exec[e]);
  }
  if (st != RZF_OK) {
    release(g);
    return st;
  }
  *out = g;
  return RZF_OK;
}

rzf_status rzf_graph_full(rzf_ctx* c, int n, const rzf_full_item* items, const rzf_graph_rate* rate,
                          rzf_graph** out) {
  if (!c || !out) return RZF_E_INVALID;
  *out = nullptr;
  const rzf_status st0 = check_full_items(n, items);
  if (st0 != RZF_OK) return st0;
  if (!rate_ok(rate)) return RZF_E_INVALID;
  std::lock_guard<std::mutex> lk(c->mu);
  HIP_OK(hipSetDevice(c->device));
  // one FP32 item is rzf_full; anything else is rzf_full_batch
  const bool single = n == 1 && items[0].precision == RZF_PREC_FP32;
  std::vector<int> K(n), N(n), ldh(n), ldw(n);
  std::vector<const rzf_c32*> H(n);
  std::vector<rzf_c32*> W(n);
  for (int i = 0; i < n; ++i) {
    K[i] = items[i].K; N[i] = items[i].N;
    H[i] = items[i].H; W[i] = items[i].W; ldh[i] = items[i].ldh; ldw[i] = items[i].ldw;
  }
  size_t jobs = 0, scratch = 0, part = 0;
  if (!single) {
    jobs += (sizeof(GramJob) + sizeof(Inv32Job) + sizeof(PrecJob) + sizeof(ScaleJob)) * n + 64;
    for (int i = 0; i < n; ++i) scratch += full_scratch_bytes(items[i]);
    if (rate) {
      jobs += sizeof(RateJob) * n + 64;
      for (int i = 0; i < n; ++i) part += rate_scratch_bytes(K[i]);
    }
  }
  jobs = align_up(jobs);
  rzf_graph* g = nullptr;
  rzf_status st = graph_new(c, false, jobs + scratch + part, &g);
  if (st != RZF_OK) return st;
  std::vector<rzf_rate_item> ri;
  if (rate) ri = rate_items_of(n, K.data(), N.data(), H.data(), ldh.data(), W.data(), ldw.data(), rate);
  FullPlan fp;
  RatePlan rp;
  if (!single) {
    char* base = c->arena + g->off;
    std::vector<FullScratch> scr(n);
    char* p = base + jobs;
    for (int i = 0; i < n; ++i) {
      scr[i] = full_scratch_at(items[i], p);
      p += full_scratch_bytes(items[i]);
    }
    plan_full(fp, n, items, scr.data());
    if (rate) plan_rate(rp, n, ri.data(), rate->P, rate->sigma2, p, c->d_counts);
    Upload u(base, jobs);
    fp.put(u.st);
    if (rate) rp.put(u.st);
    st = u.commit(c->stream);
  }
  if (st == RZF_OK)
    st = capture(c, [&](hipStream_t s) {
      if (!single) {
        fp.launch(c, s, c->d_err);
        if (rate) rp.launch(c, s, c->d_err);
      } else {
        const rzf_full_item& it = items[0];
        const float2* Hf = reinterpret_cast<const float2*>(it.H);
        float2* Wf = reinterpret_cast<float2*>(it.W);
        full_single_launch(c, it.K, it.N, Hf, it.ldh, it.alpha, it.P, Wf, it.ldw, s);
        if (rate)
          rate_single_launch(c, it.K, it.N, Hf, it.ldh, Wf, it.ldw, rate->P, rate->sigma2, nullptr, rate->sums, s);
      }
    }, &g->exec[0]);
  if (st != RZF_OK) {
    release(g);
    return st;
  }
  *out = g;
  return RZF_OK;
}

rzf_status rzf_graph_launch(rzf_graph* g) {
  if (!g) return RZF_E_INVALID;
  rzf_ctx* c = g->c;
  std::lock_guard<std::mutex> lk(c->mu);
  HIP_OK(hipSetDevice(c->device));
  int e = 0;
  if (g->update) {
    const rzf_track* t0 = g->tracks[0];
    for (const rzf_track* t : g->tracks)
      if (t->since_reset != t0->since_reset) return RZF_E_INVALID;
    e = reset_due(t0) ? 1 : 0;
  }
  if (!g->exec[e]) return RZF_E_INVALID;
  HIP_OK(hipGraphLaunch(g->exec[e], c->stream));
  if (g->update) {
    const std::vector<int> flag(g->tracks.size(), e);
    advance_tracks((int)g->tracks.size(), g->tracks.data(), flag);
  }
  return RZF_OK;
}

rzf_status rzf_graph_destroy(rzf_graph* g) {
  if (!g) return RZF_E_INVALID;
  rzf_ctx* c = g->c;
  std::lock_guard<std::mutex> lk(c->mu);
  HIP_OK(hipSetDevice(c->device));
  HIP_OK(hipStreamSynchronize(c->stream));
  release(g);
  return RZF_OK;
}

}  // extern "C"
