// Host runtime behind rzf.h: context (device, stream, arena, error word),
// track state in the arena, launch sequences of rzf_init / rzf_update /
// rzf_full / rzf_sum_rate, and deferred info records.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <vector>

#include "runtime.h"

using namespace rzfrt;

namespace {

const char* const KERNEL_NAMES[] = {"gram", "gram64", "inv64", "inv32", "arsvd_wb",
                                    "precoder", "scale", "sum_rate", "beam_resp", "beam_select"};
static_assert(sizeof(KERNEL_NAMES) / sizeof(KERNEL_NAMES[0]) == KN_COUNT, "one name per kernel");

}  // namespace

namespace {

// Batches from these sizes on take the batch launch shapes: a Gram workgroup
// per track (which needs the batch to fill the CUs) and the batch entry of the
// precoder's rows; smaller ones the single-track shapes.
constexpr int GRAM_TRACK_MIN = 256;
constexpr int PREC_BATCH_MIN = 128;

size_t sr_single_doubles() { return std::max(sum_rate_scratch_doubles(KM), sum_rate_split_scratch_doubles()); }

size_t scratch_bytes() {
  return align_up(sizeof(int) * 64) + align_up(sizeof(unsigned) * RZF_BATCH_MAX) +
         2 * align_up(sizeof(float2) * KM * KM) +
         align_up(sizeof(double) * ((RZF_NMAX + 15) / 16)) + align_up(sizeof(double) * 8) +
         align_up(sizeof(double) * sr_single_doubles()) + align_up(SPEC_BYTES) +
         NSTAGE * STAGE_BYTES;
}

struct Layout {
  size_t desc, ainv, hprev, anew, da, a64, wpart, rfb, xw, xd, ym, qm, zm, pm, aug, total;
};

Layout track_layout(int K, int N) {
  Layout L{};
  size_t o = 0;
  L.desc = o; o += align_up(sizeof(TrackDesc));
  L.ainv = o; o += align_up(sizeof(float2) * K * K);
  L.hprev = o; o += align_up(sizeof(float2) * (size_t)K * N);
  L.anew = o; o += align_up(sizeof(float2) * K * K);
  L.da = o; o += align_up(sizeof(float2) * K * K);
  L.a64 = o; o += align_up(sizeof(double2) * K * K);
  L.wpart = o; o += align_up(sizeof(double) * precoder_scratch(N));
  L.rfb = o; o += align_up(sizeof(float2) * K * K);
  L.xw = o; o += align_up(sizeof(float2) * K * K);   // full-width SVD basis
  if (K <= KS) {
    L.xd = o; o += align_up(sizeof(float2) * K * K);   // basis of the last narrower SVD
  }
  if (K > KS) {
    // working set of the large-track kernels
    L.ym = o; o += align_up(sizeof(float2) * K * K);
    L.qm = o; o += align_up(sizeof(float2) * K * K);
    L.zm = o; o += align_up(sizeof(float2) * K * K);
    L.pm = o; o += align_up(sizeof(float2) * K * (K / 2));
    L.aug = o; o += align_up(sizeof(double2) * (K / 2) * (K / 2 + K));
  }
  L.total = o;
  return L;
}

bool arena_alloc(rzf_ctx* c, size_t bytes, size_t* off) {
  for (auto it = c->free_blocks.begin(); it != c->free_blocks.end(); ++it) {
    if (it->second >= bytes) {
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t noff = it->first + bytes;
      c->free_blocks.erase(it);
      if (rest) c->free_blocks[noff] = rest;
      return true;
    }
  }
  return false;
}

void arena_free(rzf_ctx* c, size_t off, size_t bytes) {
  auto it = c->free_blocks.emplace(off, bytes).first;
  auto nx = std::next(it);
  if (nx != c->free_blocks.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    c->free_blocks.erase(nx);
  }
  if (it != c->free_blocks.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      c->free_blocks.erase(it);
    }
  }
}

DevInfo* pin_slot(rzf_ctx* c) {
  const size_t chunk = c->pin_used / PIN_CHUNK, idx = c->pin_used % PIN_CHUNK;
  if (chunk >= c->pin_chunks.size()) {
    DevInfo* p = nullptr;
    if (hipHostMalloc((void**)&p, sizeof(DevInfo) * PIN_CHUNK, hipHostMallocDefault) != hipSuccess)
      return nullptr;
    c->pin_chunks.push_back(p);
  }
  ++c->pin_used;
  return c->pin_chunks[chunk] + idx;
}

hipEvent_t ev_get(rzf_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Run `launch` between an event pair when timing is on.
template <class F>
void timed(rzf_ctx* c, int kernel, hipStream_t s, F launch) {
  if (!c->prof_on || c->capturing) { launch(); return; }
  hipEvent_t a = ev_get(c), b = ev_get(c);
  if (!a || !b) { launch(); return; }
  (void)hipEventRecord(a, s);
  launch();
  (void)hipEventRecord(b, s);
  c->prof.push_back(ProfRec{kernel, a, b});
}

void prof_drain(rzf_ctx* c) {
  for (const ProfRec& r : c->prof) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      c->prof_count[r.kernel] += 1;
      c->prof_ms[r.kernel] += ms;
    }
    c->ev_pool.push_back(r.a);
    c->ev_pool.push_back(r.b);
  }
  c->prof.clear();
}

rzf_status dev_status(int code) {
  if (code == DEV_ERR_NOT_HPD) return RZF_E_NOT_HPD;
  if (code == DEV_ERR_NONFINITE) return RZF_E_NONFINITE;
  if (code == DEV_ERR_BEAM) return RZF_E_INVALID;
  return code ? RZF_E_DEVICE : RZF_OK;
}

#define HIP_OK(x) do { if ((x) != hipSuccess) return RZF_E_DEVICE; } while (0)

// Tracks created in this process: a track's two-phase tag numbers start at its
// number times 2^32 (unique across the process, so that no tag left in reused
// device memory by another track or an earlier context can match).
std::atomic<unsigned long long> g_track_uid{0};

// Kernel families by track size: K <= KS keeps the working set in LDS, larger
// tracks use the blocked kernels on a global workspace.
void inv64_any(const Inv64Job& j, int* err, hipStream_t s) {
  if (j.K > KS) launch_inv64_big(j, nullptr, 1, err, s); else launch_inv64(j, nullptr, 1, err, s);
}
void inv32_any(const Inv32Job& j, int* err, hipStream_t s) {
  if (j.K > KS) launch_inv32_big(j, nullptr, 1, err, s); else launch_inv32(j, nullptr, 1, err, s);
}
// A single track's step: K <= KS tracks run the two-phase form, whose
// speculated iterations of Alg. 1 use otherwise idle CUs (same results as
// the one-launch form); larger tracks run the blocked kernel.
void arsvd_single(rzf_ctx* c, ArsvdJob j, int K, hipStream_t s) {
  if (K > KS) {
    launch_arsvd_big(j, nullptr, 1, c->d_err, s);
  } else {
    j.spec = c->d_spec;
    j.stage = reinterpret_cast<char*>(c->d_spec) + SPEC_STAGE_OFF;
    launch_arsvd_wb_spec(j, c->d_err, s);
  }
}

bool params_valid(const rzf_params* p) {
  return p->k_init >= 1 && p->k_init <= RZF_KMAX && p->p >= 0 && p->p <= RZF_KMAX &&
         p->i_max >= 0 && p->i_max <= 64 &&
         std::isfinite(p->switch_ratio) && p->switch_ratio > 0.0 && p->switch_ratio <= 1.0 &&
         p->reset_period >= 0 && std::isfinite(p->P) && p->P > 0.0 &&
         (p->kinit_policy == RZF_KINIT_FIXED || p->kinit_policy == RZF_KINIT_WARM) &&
         (p->early_fallback == 0 || p->early_fallback == 1) &&
         p->precision >= RZF_PREC_FP32 && p->precision <= RZF_PREC_BF16X3 &&
         (p->error_feedback == 0 || p->error_feedback == 1);
}

// Largest rank the Woodbury branch of a K x K track can take: the LDS
// kernels hold WB_RMAX columns, the large-track workspace K / 2.
int wb_capacity(int K) { return std::min(K, std::max(WB_RMAX, K / 2)); }

// Alg. 2's switch as a rank: Woodbury when k_est <= floor(switch_ratio K).
int switch_rank(double ratio, int K) { return (int)std::floor(ratio * K); }

// The track's parameters fit a K-user track: Alg. 2's switch must stay within
// the Woodbury workspace (a larger ratio is refused rather than capped).
bool params_fit(const rzf_params* p, int K) { return switch_rank(p->switch_ratio, K) <= wb_capacity(K); }

int default_imax(int K, int k_init, int p) {
  int i = 1;
  long k0 = k_init;
  while (k0 + p < K) { k0 *= 2; ++i; }
  return i;
}

// Wait for the stream, fill the pending info records, and move the device
// error word into *code (clearing it on the device).
rzf_status take_device_error(rzf_ctx* c, int* code) {
  *code = 0;
  HIP_OK(hipStreamSynchronize(c->stream));
  for (const Pending& pd : c->pending) {
    if (pd.dst) std::memcpy(pd.dst, pd.slot, sizeof(rzf_update_info));
  }
  c->pending.clear();
  c->pin_used = 0;
  HIP_OK(hipMemcpy(c->h_err, c->d_err, sizeof(int), hipMemcpyDeviceToHost));
  *code = *c->h_err;
  if (*code) {
    *c->h_err = 0;
    HIP_OK(hipMemcpy(c->d_err, c->h_err, sizeof(int), hipMemcpyHostToDevice));
  }
  return RZF_OK;
}

// rzf_sync: the first error recorded since the last rzf_sync, then cleared
// (one kept aside by a synchronous call comes first).
rzf_status sync_and_collect(rzf_ctx* c) {
  int code = 0;
  const rzf_status st = take_device_error(c, &code);
  const int first = c->held_err ? c->held_err : code;
  c->held_err = 0;
  if (st != RZF_OK) return st;
  return dev_status(first);
}

// Before a synchronous call's own launches: an error that earlier
// asynchronous work left on the device is kept for the next rzf_sync.
rzf_status hold_earlier_error(rzf_ctx* c) {
  int code = 0;
  const rzf_status st = take_device_error(c, &code);
  if (code && !c->held_err) c->held_err = code;
  return st;
}

// After a synchronous call's own launches: their device error only.
rzf_status own_device_error(rzf_ctx* c) {
  int code = 0;
  const rzf_status st = take_device_error(c, &code);
  return st != RZF_OK ? st : dev_status(code);
}

}  // namespace

namespace {

// Arena space and host descriptor of a new track (no device work; the
// caller fills the state and uploads the descriptor).  nullptr if the arena
// or the host heap is full.
rzf_track* track_new(rzf_ctx* c, int K, int N, const rzf_params& prm, double alpha) {
  const Layout L = track_layout(K, N);
  size_t off = 0;
  if (!arena_alloc(c, L.total, &off)) return nullptr;
  rzf_track* t = new (std::nothrow) rzf_track();
  if (!t) { arena_free(c, off, L.total); return nullptr; }
  char* base = c->arena + off;
  t->ctx = c; t->K = K; t->N = N; t->prm = prm; t->alpha = alpha; t->off = off; t->bytes = L.total;
  t->i_max = prm.i_max > 0 ? prm.i_max : default_imax(K, prm.k_init, prm.p);
  TrackDesc& d = t->h_desc;
  std::memset(&d, 0, sizeof(d));
  d.K = K; d.N = N; d.alpha = alpha; d.P = prm.P; d.switch_ratio = prm.switch_ratio;
  d.k_init = prm.k_init; d.p = prm.p; d.i_max = t->i_max; d.kinit_policy = prm.kinit_policy;
  d.seed = prm.seed; d.track_id = prm.track_id;
  d.early_fallback = prm.early_fallback;
  d.prec = prm.precision;
  d.error_feedback = prm.error_feedback;
  // Alg. 2's switch (params_fit keeps it within the Woodbury workspace)
  d.wb_limit = switch_rank(prm.switch_ratio, K);
  d.Ainv = reinterpret_cast<float2*>(base + L.ainv);
  d.Hprev = reinterpret_cast<float2*>(base + L.hprev);
  d.Anew = reinterpret_cast<float2*>(base + L.anew);
  d.dA = reinterpret_cast<float2*>(base + L.da);
  d.A64 = reinterpret_cast<double2*>(base + L.a64);
  d.wpart = reinterpret_cast<double*>(base + L.wpart);
  d.Rfb = reinterpret_cast<float2*>(base + L.rfb);
  d.Xw = reinterpret_cast<float2*>(base + L.xw);
  if (K <= KS) d.Xd = reinterpret_cast<float2*>(base + L.xd);
  if (K > KS) {
    d.Ym = reinterpret_cast<float2*>(base + L.ym);
    d.Qm = reinterpret_cast<float2*>(base + L.qm);
    d.Zm = reinterpret_cast<float2*>(base + L.zm);
    d.Pm = reinterpret_cast<float2*>(base + L.pm);
    d.Aug = reinterpret_cast<double2*>(base + L.aug);
  }
  d.last_r = 0;
  d.t_dev = 0;
  d.seq_dev = (++g_track_uid) << 32;
  t->d_desc = reinterpret_cast<TrackDesc*>(base + L.desc);
  return t;
}

// Checkpoint blob of one track: this header, then A^-1 (K x K) and H_prev
// (K x N) row-major, the error-feedback residual R (K x K, row-major) and
// the full-width SVD basis and that of the last narrower SVD (K x K each,
// column-major; the second zero for K > KS), all complex64.
struct TrackBlob {
  char magic[8];
  uint32_t version, header_bytes;
  int32_t K, N;
  rzf_params prm;
  double alpha;
  int32_t step, since_reset, last_r, warm, dwarm;
  int32_t nsig, spec_hint, pad;   // d of the last SVD; Alg. 1 iterations of the last step
};
const char BLOB_MAGIC[8] = {'R', 'Z', 'F', 'T', 'R', 'A', 'C', 'K'};
constexpr uint32_t BLOB_VERSION = 6;   // 3: params gained early_fallback, precision, error
                                       // feedback; the residual R follows H_prev.
                                       // 4: the full-width SVD basis follows R.
                                       // 5: nsig and spec_hint; the basis for every K.
                                       // 6: the narrower basis (dwarm columns)

size_t blob_bytes(int K, int N) {
  return sizeof(TrackBlob) + sizeof(float2) * (4 * (size_t)K * K + (size_t)K * N);
}

}  // namespace

static_assert(sizeof(DevInfo) == sizeof(rzf_update_info), "info layout");

extern "C" {

const char* rzf_status_string(rzf_status s) {
  switch (s) {
    case RZF_OK: return "ok";
    case RZF_E_INVALID: return "invalid argument";
    case RZF_E_SHAPE: return "size out of range";
    case RZF_E_NOMEM: return "arena full";
    case RZF_E_NOT_HPD: return "Gram matrix not positive definite";
    case RZF_E_NONFINITE: return "non-finite value";
    case RZF_E_DEVICE: return "HIP runtime error";
  }
  return "unknown status";
}

rzf_status rzf_params_default(rzf_params* p) {
  if (!p) return RZF_E_INVALID;
  std::memset(p, 0, sizeof(*p));
  p->k_init = 2;
  p->p = 5;
  p->i_max = 0;
  p->switch_ratio = 0.5;
  p->reset_period = 0;
  p->P = 1.0;
  p->seed = 0;
  p->track_id = 0;
  p->kinit_policy = RZF_KINIT_FIXED;
  return RZF_OK;
}

rzf_status rzf_params_check(const rzf_params* p, int K) {
  if (K < 1 || K > RZF_KMAX) return RZF_E_SHAPE;
  if (!p || !params_valid(p) || !params_fit(p, K)) return RZF_E_INVALID;
  return RZF_OK;
}

size_t rzf_track_bytes(int K, int N) {
  if (K < 1 || K > RZF_KMAX || N < 1 || N > RZF_NMAX) return 0;
  return track_layout(K, N).total;
}

rzf_status rzf_ctx_create(int device, void* hip_stream, void* arena, size_t arena_bytes,
                          rzf_ctx** out) {
  if (!out) return RZF_E_INVALID;
  *out = nullptr;
  const size_t scr = scratch_bytes();
  if (arena_bytes < scr + ALIGN) return RZF_E_NOMEM;
  if (arena && (reinterpret_cast<uintptr_t>(arena) % ALIGN)) return RZF_E_INVALID;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return RZF_E_DEVICE;
  HIP_OK(hipSetDevice(device));
  rzf_ctx* c = new (std::nothrow) rzf_ctx();
  if (!c) return RZF_E_NOMEM;
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (arena) {
    c->arena = static_cast<char*>(arena);
  } else {
    if (hipMalloc((void**)&c->arena, arena_bytes) != hipSuccess) { delete c; return RZF_E_NOMEM; }
    c->own_arena = true;
  }
  c->arena_bytes = arena_bytes;
  char* p = c->arena;
  c->d_err = reinterpret_cast<int*>(p); p += align_up(sizeof(int) * 64);
  c->d_counts = reinterpret_cast<unsigned*>(p); p += align_up(sizeof(unsigned) * RZF_BATCH_MAX);
  c->d_fullA = reinterpret_cast<float2*>(p); p += align_up(sizeof(float2) * KM * KM);
  c->d_fullAinv = reinterpret_cast<float2*>(p); p += align_up(sizeof(float2) * KM * KM);
  c->d_fullwpart = reinterpret_cast<double*>(p); p += align_up(sizeof(double) * ((RZF_NMAX + 15) / 16));
  c->d_sum = reinterpret_cast<double*>(p); p += align_up(sizeof(double) * 8);
  c->d_srpart = reinterpret_cast<double*>(p); p += align_up(sizeof(double) * sr_single_doubles());
  c->d_spec = reinterpret_cast<float2*>(p); p += align_up(SPEC_BYTES);
  c->d_stage = p;
  c->free_blocks[scr] = arena_bytes - scr;
  if (hipHostMalloc((void**)&c->h_sum, sizeof(double) * 8, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->h_err, sizeof(int) * 8, hipHostMallocDefault) != hipSuccess) {
    if (c->own_arena) (void)hipFree(c->arena);
    delete c;
    return RZF_E_DEVICE;
  }
  *c->h_err = 0;
  bool stage_ok = hipHostMalloc((void**)&c->h_stage, NSTAGE * STAGE_BYTES, hipHostMallocDefault) == hipSuccess;
  for (int k = 0; k < NSTAGE && stage_ok; ++k)
    stage_ok = hipEventCreateWithFlags(&c->stage_ev[k], hipEventDisableTiming) == hipSuccess;
  // the completion counts of the context's sum-rate launches start at zero
  if (stage_ok) stage_ok = hipMemset(c->d_counts, 0, sizeof(unsigned) * RZF_BATCH_MAX) == hipSuccess;
  // the speculation area starts with no iteration posted (its tags zero)
  if (stage_ok)
    stage_ok = hipMemset(reinterpret_cast<char*>(c->d_spec) + sizeof(float2) * 2 * KS * KS * SPEC_MAX, 0,
                         SPEC_STAGE_OFF - sizeof(float2) * 2 * KS * KS * SPEC_MAX) == hipSuccess;
  if (!stage_ok || hipMemcpy(c->d_err, c->h_err, sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
    for (int k = 0; k < NSTAGE; ++k) if (c->stage_ev[k]) (void)hipEventDestroy(c->stage_ev[k]);
    if (c->h_stage) (void)hipHostFree(c->h_stage);
    (void)hipHostFree(c->h_sum);
    (void)hipHostFree(c->h_err);
    if (c->own_arena) (void)hipFree(c->arena);
    delete c;
    return RZF_E_DEVICE;
  }
  *out = c;
  return RZF_OK;
}

rzf_status rzf_ctx_destroy(rzf_ctx* c) {
  if (!c) return RZF_E_INVALID;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  graphs_release_all(c);
  for (rzf_track* t : c->tracks) delete t;
  c->tracks.clear();
  prof_drain(c);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  for (int k = 0; k < NSTAGE; ++k) if (c->stage_ev[k]) (void)hipEventDestroy(c->stage_ev[k]);
  if (c->h_stage) (void)hipHostFree(c->h_stage);
  for (DevInfo* p : c->pin_chunks) (void)hipHostFree(p);
  if (c->h_sum) (void)hipHostFree(c->h_sum);
  if (c->h_err) (void)hipHostFree(c->h_err);
  if (c->own_arena) (void)hipFree(c->arena);
  delete c;
  return RZF_OK;
}

rzf_status rzf_sync(rzf_ctx* c) {
  if (!c) return RZF_E_INVALID;
  std::lock_guard<std::mutex> lk(c->mu);
  HIP_OK(hipSetDevice(c->device));
  return sync_and_collect(c);
}

rzf_status rzf_init(rzf_ctx* c, int K, int N, const rzf_c32* H, int ldh, double alpha,
                    const rzf_params* params, rzf_track** out) {
  if (!c || !H || !out) return RZF_E_INVALID;
  *out = nullptr;
  if (K < 1 || K > RZF_KMAX || N < 1 || N > RZF_NMAX || ldh < N) return RZF_E_SHAPE;
  if (!std::isfinite(alpha) || alpha < 0.0) return RZF_E_INVALID;
  rzf_params prm;
  if (params) prm = *params; else rzf_params_default(&prm);
  if (!params_valid(&prm) || !params_fit(&prm, K)) return RZF_E_INVALID;
  std::lock_guard<std::mutex> lk(c->mu);
  HIP_OK(hipSetDevice(c->device));
  // an error of earlier asynchronous work stays pending for the next rzf_sync
  rzf_status st0 = hold_earlier_error(c);
  if (st0 != RZF_OK) return st0;

  rzf_track* t = track_new(c, K, N, prm, alpha);
  if (!t) return RZF_E_NOMEM;
  const TrackDesc& d = t->h_desc;
  hipStream_t s = c->stream;
  const float2* Hf = reinterpret_cast<const float2*>(H);
  bool ok = hipMemcpyAsync(t->d_desc, &d, sizeof(d), hipMemcpyHostToDevice, s) == hipSuccess;
  if (ok) {
    const Gram64Job gj{Hf, d.A64, K, N, ldh, alpha};
    launch_gram64(gj, nullptr, 1, K, s);
    const Inv64Job ij{d.A64, d.Ainv, nullptr, nullptr, K, d.Rfb};
    inv64_any(ij, c->d_err, s);
    ok = hipMemcpy2DAsync(d.Hprev, sizeof(float2) * N, Hf, sizeof(float2) * ldh,
                          sizeof(float2) * N, K, hipMemcpyDeviceToDevice, s) == hipSuccess;
    ok = ok && hipGetLastError() == hipSuccess;
  }
  rzf_status st = ok ? own_device_error(c) : RZF_E_DEVICE;
  if (st != RZF_OK) {
    arena_free(c, t->off, t->bytes);
    delete t;
    return st;
  }
  c->tracks.insert(t);
  *out = t;
  return RZF_OK;
}

rzf_status rzf_update(rzf_track* t, const rzf_c32* H_t, int ldh, double tol, rzf_c32* W, int ldw,
                      rzf_update_info* info) {
  if (!t || !H_t || !W) return RZF_E_INVALID;
  if (!(tol > 0.0 && tol <= 1.0)) return RZF_E_INVALID;
  if (ldh < t->N || ldw < t->K) return RZF_E_SHAPE;
  rzf_ctx* c = t->ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  HIP_OK(hipSetDevice(c->device));
  hipStream_t s = c->stream;
  const float2* Hf = reinterpret_cast<const float2*>(H_t);
  float2* Wf = reinterpret_cast<float2*>(W);
  DevInfo* slot = nullptr;
  if (info) {
    slot = pin_slot(c);
    if (!slot) return RZF_E_DEVICE;
  }
  const int step = t->t + 1;
  const bool reset = reset_due(t);
  update_single_launch(c, t, Hf, ldh, tol, Wf, ldw, reset, s);
  if (hipGetLastError() != hipSuccess) return RZF_E_DEVICE;
  if (slot) {
    HIP_OK(hipMemcpyAsync(slot, &t->d_desc->info, sizeof(DevInfo), hipMemcpyDeviceToHost, s));
    c->pending.push_back(Pending{slot, info});
  }
  t->t = step;
  t->since_reset = reset ? 0 : t->since_reset + 1;
  return RZF_OK;
}


}  // extern "C"

namespace {

// Reserve the next staging slot (waits until the launches that last used it
// have consumed their job arrays).  Returns the slot index or -1.
int stage_acquire(rzf_ctx* c) {
  const int k = c->stage_next;
  c->stage_next = (k + 1) % NSTAGE;
  if (c->stage_used[k] && hipEventSynchronize(c->stage_ev[k]) != hipSuccess) return -1;
  c->stage_used[k] = false;
  return k;
}

}  // namespace

namespace rzfrt {

rzf_status check_update_items(rzf_ctx* c, int n, const rzf_update_item* items, double tol) {
  if (!c || !items || n < 1 || n > RZF_BATCH_MAX) return RZF_E_INVALID;
  if (!(tol > 0.0 && tol <= 1.0)) return RZF_E_INVALID;
  std::set<rzf_track*> seen;
  for (int i = 0; i < n; ++i) {
    const rzf_update_item& it = items[i];
    if (!it.track || !it.H || !it.W || it.track->ctx != c) return RZF_E_INVALID;
    if (!seen.insert(it.track).second) return RZF_E_INVALID;
    if (it.ldh < it.track->N || it.ldw < it.track->K) return RZF_E_SHAPE;
  }
  return RZF_OK;
}

void plan_update(UpdatePlan& P, int n, const rzf_update_item* items, double tol, int force_reset) {
  P = UpdatePlan{};
  P.reset_flag.resize(n);
  for (int i = 0; i < n; ++i) {
    rzf_track* t = items[i].track;
    const TrackDesc& d = t->h_desc;
    const int K = t->K, N = t->N;
    const float2* Hf = reinterpret_cast<const float2*>(items[i].H);
    float2* Wf = reinterpret_cast<float2*>(items[i].W);
    const bool reset = force_reset < 0 ? reset_due(t) : force_reset != 0;
    P.reset_flag[i] = reset;
    if (reset) {
      P.g64.push_back(Gram64Job{Hf, d.A64, K, N, items[i].ldh, t->alpha});
      (K > KS ? P.i64b : P.i64).push_back(Inv64Job{d.A64, d.Ainv, &t->d_desc->info, nullptr, K, d.Rfb,
                                                   &t->d_desc->hold});
      P.maxKr = std::max(P.maxKr, K);
    } else {
      P.gj.push_back(GramJob{Hf, d.Hprev, d.Anew, d.dA, K, N, items[i].ldh, N, (float)t->alpha, d.prec});
      (K > KS ? P.ajb : P.aj).push_back(ArsvdJob{t->d_desc, nullptr, tol, t->i_max});
    }
    P.pj.push_back(PrecJob{Hf, d.Ainv, Wf, d.wpart, d.Hprev, K, N, items[i].ldh, items[i].ldw, d.prec,
                           &t->d_desc->hold});
    P.sj.push_back(ScaleJob{Wf, d.wpart, d.P, K, N, items[i].ldw, precoder_blocks(N), t->d_desc});
    P.maxNK = std::max(P.maxNK, N * K);
    P.maxK = std::max(P.maxK, K);
    P.maxN = std::max(P.maxN, N);
  }
}

size_t UpdatePlan::bytes() const {
  return sizeof(GramJob) * gj.size() + 2 * sizeof(ArsvdJob) * (aj.size() + ajb.size()) +
         sizeof(Gram64Job) * g64.size() + sizeof(Inv64Job) * (i64.size() + i64b.size()) +
         sizeof(PrecJob) * pj.size() + sizeof(ScaleJob) * sj.size() + 16 * 12;
}

void UpdatePlan::put(Stager& st) {
  if (!gj.empty()) st.put(gj.data(), (int)gj.size(), &d_gj);
  if (!aj.empty()) {
    st.put(aj.data(), (int)aj.size(), &d_aj);
    st.put(aj.data(), (int)aj.size(), &d_ajo);   // reordered on the device before use
  }
  if (!ajb.empty()) {
    st.put(ajb.data(), (int)ajb.size(), &d_ajb);
    st.put(ajb.data(), (int)ajb.size(), &d_ajbo);
  }
  if (!g64.empty()) st.put(g64.data(), (int)g64.size(), &d_g64);
  if (!i64.empty()) st.put(i64.data(), (int)i64.size(), &d_i64);
  if (!i64b.empty()) st.put(i64b.data(), (int)i64b.size(), &d_i64b);
  st.put(pj.data(), (int)pj.size(), &d_pj);
  st.put(sj.data(), (int)sj.size(), &d_sj);
}

void UpdatePlan::launch(rzf_ctx* c, hipStream_t s, int* err) const {
  const int n = (int)pj.size();
  if (!gj.empty()) {
    bool fp32 = (int)gj.size() >= GRAM_TRACK_MIN;
    for (const GramJob& g : gj) fp32 = fp32 && g.prec == RZF_PREC_FP32;
    timed(c, KN_GRAM, s, [&] { launch_gram(gj[0], d_gj, (int)gj.size(), maxK, fp32, s); });
    timed(c, KN_ARSVD, s, [&] {
      // longest-first order over the CUs for a batch that spans more than one
      // wave of workgroups
      if (!aj.empty()) {
        const bool ord = aj.size() > 64 && aj.size() <= RZF_BATCH_MAX;
        if (ord) launch_arsvd_order(d_aj, d_ajo, (int)aj.size(), s);
        launch_arsvd_wb(aj[0], ord ? d_ajo : d_aj, (int)aj.size(), err, s);
      }
      if (!ajb.empty()) {
        const bool ord = ajb.size() > 64 && ajb.size() <= RZF_BATCH_MAX;
        if (ord) launch_arsvd_order(d_ajb, d_ajbo, (int)ajb.size(), s);
        launch_arsvd_big(ajb[0], ord ? d_ajbo : d_ajb, (int)ajb.size(), err, s);
      }
    });
  }
  if (!g64.empty()) {
    timed(c, KN_GRAM64, s, [&] { launch_gram64(g64[0], d_g64, (int)g64.size(), maxKr, s); });
    timed(c, KN_INV64, s, [&] {
      if (!i64.empty()) launch_inv64(i64[0], d_i64, (int)i64.size(), err, s);
      if (!i64b.empty()) launch_inv64_big(i64b[0], d_i64b, (int)i64b.size(), err, s);
    });
  }
  const rzf_tune_entry te = tune_for(c, maxK, maxN);
  const int pb = (int)pj.size() >= PREC_BATCH_MIN ? te.batch_precoder_rows : te.precoder_rows;
  bool scaled = false;
  timed(c, KN_PRECODER, s, [&] { scaled = launch_precoder(pj[0], d_pj, sj[0], d_sj, n, maxN, maxK, pb, s); });
  if (!scaled) timed(c, KN_SCALE, s, [&] { launch_scale(sj[0], d_sj, n, maxNK, s); });
}

void advance_tracks(int n, rzf_track* const* tracks, const std::vector<int>& reset_flag) {
  for (int i = 0; i < n; ++i) {
    rzf_track* t = tracks[i];
    t->t += 1;
    t->since_reset = reset_flag[i] ? 0 : t->since_reset + 1;
  }
}

rzf_status update_batch_locked(rzf_ctx* c, int n, const rzf_update_item* items, double tol,
                               DevInfo* const* slots, hipStream_t s, int* err) {
  UpdatePlan P;
  plan_update(P, n, items, tol, -1);
  if (P.bytes() > STAGE_BYTES) return RZF_E_INVALID;
  const int slot = stage_acquire(c);
  if (slot < 0) return RZF_E_DEVICE;
  Stager st{c->h_stage + slot * STAGE_BYTES, c->d_stage + slot * STAGE_BYTES};
  P.put(st);
  HIP_OK(hipMemcpyAsync(st.d, st.h, st.used, hipMemcpyHostToDevice, s));
  P.launch(c, s, err);
  HIP_OK(hipEventRecord(c->stage_ev[slot], s));
  c->stage_used[slot] = true;
  if (hipGetLastError() != hipSuccess) return RZF_E_DEVICE;
  std::vector<rzf_track*> tr(n);
  for (int i = 0; i < n; ++i) {
    tr[i] = items[i].track;
    if (slots[i])
      HIP_OK(hipMemcpyAsync(slots[i], &tr[i]->d_desc->info, sizeof(DevInfo), hipMemcpyDeviceToHost, s));
  }
  advance_tracks(n, tr.data(), P.reset_flag);
  return RZF_OK;
}


rzf_status check_full_items(int n, const rzf_full_item* items) {
  if (!items || n < 1 || n > RZF_BATCH_MAX) return RZF_E_INVALID;
  for (int i = 0; i < n; ++i) {
    const rzf_full_item& it = items[i];
    if (!it.H || !it.W) return RZF_E_INVALID;
    if (it.K < 1 || it.K > RZF_KMAX || it.N < 1 || it.N > RZF_NMAX || it.ldh < it.N || it.ldw < it.K)
      return RZF_E_SHAPE;
    if (!std::isfinite(it.alpha) || it.alpha < 0.0 || !std::isfinite(it.P) || it.P <= 0.0)
      return RZF_E_INVALID;
    if (it.precision < RZF_PREC_FP32 || it.precision > RZF_PREC_BF16X3) return RZF_E_INVALID;
  }
  return RZF_OK;
}

size_t full_scratch_bytes(const rzf_full_item& it) {
  return align_up(sizeof(float2) * it.K * it.K) + align_up(sizeof(double) * precoder_scratch(it.N));
}

FullScratch full_scratch_at(const rzf_full_item& it, char* p) {
  return FullScratch{reinterpret_cast<float2*>(p),
                     reinterpret_cast<double*>(p + align_up(sizeof(float2) * it.K * it.K))};
}

void plan_full(FullPlan& P, int n, const rzf_full_item* items, const FullScratch* scr) {
  P = FullPlan{};
  P.gj.resize(n);
  P.pj.resize(n);
  P.sj.resize(n);
  for (int i = 0; i < n; ++i) {
    const rzf_full_item& it = items[i];
    float2* A = scr[i].A;
    double* wp = scr[i].wpart;
    const float2* Hf = reinterpret_cast<const float2*>(it.H);
    float2* Wf = reinterpret_cast<float2*>(it.W);
    P.gj[i] = GramJob{Hf, nullptr, A, nullptr, it.K, it.N, it.ldh, 0, (float)it.alpha, it.precision};
    (it.K > KS ? P.vjb : P.vj).push_back(Inv32Job{A, A, it.K});
    P.pj[i] = PrecJob{Hf, A, Wf, wp, nullptr, it.K, it.N, it.ldh, it.ldw, it.precision, nullptr};
    P.sj[i] = ScaleJob{Wf, wp, it.P, it.K, it.N, it.ldw, precoder_blocks(it.N), nullptr};
    P.maxK = std::max(P.maxK, it.K);
    P.maxN = std::max(P.maxN, it.N);
    P.maxNK = std::max(P.maxNK, it.N * it.K);
  }
}

size_t FullPlan::bytes() const {
  return (sizeof(GramJob) + sizeof(Inv32Job) + sizeof(PrecJob) + sizeof(ScaleJob)) * gj.size() + 64;
}

void FullPlan::put(Stager& st) {
  const int n = (int)gj.size();
  st.put(gj.data(), n, &d_gj);
  if (!vj.empty()) st.put(vj.data(), (int)vj.size(), &d_vj);
  if (!vjb.empty()) st.put(vjb.data(), (int)vjb.size(), &d_vjb);
  st.put(pj.data(), n, &d_pj);
  st.put(sj.data(), n, &d_sj);
}

void FullPlan::launch(rzf_ctx* c, hipStream_t s, int* err) const {
  const int n = (int)gj.size();
  bool fp32 = n >= GRAM_TRACK_MIN;
  for (const GramJob& g : gj) fp32 = fp32 && g.prec == RZF_PREC_FP32;
  timed(c, KN_GRAM, s, [&] { launch_gram(gj[0], d_gj, n, maxK, fp32, s); });
  timed(c, KN_INV32, s, [&] {
    if (!vj.empty()) launch_inv32(vj[0], d_vj, (int)vj.size(), err, s);
    if (!vjb.empty()) launch_inv32_big(vjb[0], d_vjb, (int)vjb.size(), err, s);
  });
  const rzf_tune_entry te = tune_for(c, maxK, maxN);
  const int pb = (int)pj.size() >= PREC_BATCH_MIN ? te.batch_precoder_rows : te.precoder_rows;
  bool scaled = false;
  timed(c, KN_PRECODER, s, [&] { scaled = launch_precoder(pj[0], d_pj, sj[0], d_sj, n, maxN, maxK, pb, s); });
  if (!scaled) timed(c, KN_SCALE, s, [&] { launch_scale(sj[0], d_sj, n, maxNK, s); });
}

rzf_status full_batch_locked(rzf_ctx* c, int n, const rzf_full_item* items, const FullScratch* scr,
                             hipStream_t s, int* err) {
  std::vector<FullScratch> own;
  if (!scr) {
    size_t need = 0;
    for (int i = 0; i < n; ++i) need += full_scratch_bytes(items[i]);
    if (need > c->batch_full_bytes) {
      // grow: the old region may still be read by queued work
      HIP_OK(hipStreamSynchronize(c->stream));
      if (c->d_batch_full) arena_free(c, c->batch_full_off, c->batch_full_bytes);
      c->d_batch_full = nullptr;
      c->batch_full_bytes = 0;
      size_t off = 0;
      if (!arena_alloc(c, need, &off)) return RZF_E_NOMEM;
      c->batch_full_off = off;
      c->batch_full_bytes = need;
      c->d_batch_full = c->arena + off;
    }
    own.resize(n);
    char* p = c->d_batch_full;
    for (int i = 0; i < n; ++i) {
      own[i] = full_scratch_at(items[i], p);
      p += full_scratch_bytes(items[i]);
    }
    scr = own.data();
  }
  FullPlan P;
  plan_full(P, n, items, scr);
  if (P.bytes() > STAGE_BYTES) return RZF_E_INVALID;
  const int slot = stage_acquire(c);
  if (slot < 0) return RZF_E_DEVICE;
  Stager st{c->h_stage + slot * STAGE_BYTES, c->d_stage + slot * STAGE_BYTES};
  P.put(st);
  HIP_OK(hipMemcpyAsync(st.d, st.h, st.used, hipMemcpyHostToDevice, s));
  P.launch(c, s, err);
  HIP_OK(hipEventRecord(c->stage_ev[slot], s));
  c->stage_used[slot] = true;
  return hipGetLastError() == hipSuccess ? RZF_OK : RZF_E_DEVICE;
}

size_t rate_scratch_bytes(int K) { return align_up(sizeof(double) * sum_rate_scratch_doubles(K)); }

void plan_rate(RatePlan& P, int n, const rzf_rate_item* items, double Pw, double sigma2, char* part,
               unsigned* counts) {
  P = RatePlan{};
  P.rj.resize(n);
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    const rzf_rate_item& it = items[i];
    P.rj[i] = RateJob{reinterpret_cast<const float2*>(it.H), reinterpret_cast<const float2*>(it.W),
                      reinterpret_cast<double*>(part + off), it.rates, it.sum_rate, it.K, it.N, it.ldh, it.ldw,
                      Pw, it.sigma2 >= 0.0 ? it.sigma2 : sigma2, counts + i};
    off += rate_scratch_bytes(it.K);
    P.maxK = std::max(P.maxK, it.K);
  }
}

size_t RatePlan::bytes() const { return sizeof(RateJob) * rj.size() + 64; }

void RatePlan::put(Stager& st) { st.put(rj.data(), (int)rj.size(), &d_rj); }

void RatePlan::launch(rzf_ctx* c, hipStream_t s, int* err) const {
  timed(c, KN_SUMRATE, s, [&] { launch_sum_rate(rj[0], d_rj, (int)rj.size(), maxK, 1, err, s); });
}

void update_single_launch(rzf_ctx* c, rzf_track* t, const float2* Hf, int ldh, double tol, float2* Wf, int ldw,
                          bool reset, hipStream_t s) {
  const TrackDesc& d = t->h_desc;
  const int K = t->K, N = t->N;
  if (reset) {
    const Gram64Job gj{Hf, d.A64, K, N, ldh, t->alpha};
    const Inv64Job ij{d.A64, d.Ainv, &t->d_desc->info, nullptr, K, d.Rfb, &t->d_desc->hold};
    timed(c, KN_GRAM64, s, [&] { launch_gram64(gj, nullptr, 1, K, s); });
    timed(c, KN_INV64, s, [&] { inv64_any(ij, c->d_err, s); });
  } else {
    const GramJob gj{Hf, d.Hprev, d.Anew, d.dA, K, N, ldh, N, (float)t->alpha, d.prec};
    const ArsvdJob aj{t->d_desc, nullptr, tol, t->i_max};
    timed(c, KN_GRAM, s, [&] { launch_gram(gj, nullptr, 1, K, false, s); });
    timed(c, KN_ARSVD, s, [&] { arsvd_single(c, aj, K, s); });
  }
  const PrecJob pj{Hf, d.Ainv, Wf, d.wpart, d.Hprev, K, N, ldh, ldw, d.prec, &t->d_desc->hold};
  const ScaleJob sj{Wf, d.wpart, d.P, K, N, ldw, precoder_blocks(N), t->d_desc};
  const int pb = tune_for(c, K, N).precoder_rows;
  bool scaled = false;
  timed(c, KN_PRECODER, s, [&] { scaled = launch_precoder(pj, nullptr, sj, nullptr, 1, N, K, pb, s); });
  if (!scaled) timed(c, KN_SCALE, s, [&] { launch_scale(sj, nullptr, 1, N * K, s); });
}

void full_single_launch(rzf_ctx* c, int K, int N, const float2* Hf, int ldh, double alpha, double P, float2* Wf,
                        int ldw, hipStream_t s) {
  const GramJob gj{Hf, nullptr, c->d_fullA, nullptr, K, N, ldh, 0, (float)alpha, RZF_PREC_FP32};
  const PrecJob pj{Hf, c->d_fullAinv, Wf, c->d_fullwpart, nullptr, K, N, ldh, ldw, RZF_PREC_FP32, nullptr};
  const ScaleJob sj{Wf, c->d_fullwpart, P, K, N, ldw, precoder_blocks(N), nullptr};
  timed(c, KN_GRAM, s, [&] { launch_gram(gj, nullptr, 1, K, false, s); });
  const Inv32Job vj{c->d_fullA, c->d_fullAinv, K};
  timed(c, KN_INV32, s, [&] { inv32_any(vj, c->d_err, s); });
  const int pb = tune_for(c, K, N).precoder_rows;
  bool scaled = false;
  timed(c, KN_PRECODER, s, [&] { scaled = launch_precoder(pj, nullptr, sj, nullptr, 1, N, K, pb, s); });
  if (!scaled) timed(c, KN_SCALE, s, [&] { launch_scale(sj, nullptr, 1, N * K, s); });
}

void rate_single_launch(rzf_ctx* c, int K, int N, const float2* H, int ldh, const float2* W, int ldw, double P,
                        double sigma2, float* rates, double* sum, hipStream_t s) {
  const RateJob rj{H, W, c->d_srpart, rates, sum, K, N, ldh, ldw, P, sigma2, c->d_counts};
  const int ns = tune_for(c, K, N).rate_splits;
  timed(c, KN_SUMRATE, s, [&] { launch_sum_rate(rj, nullptr, 1, K, ns, c->d_err, s); });
}

rzf_tune_entry tune_for(const rzf_ctx* c, int K, int N) {
  rzf_tune_entry best{K, N, 0, 0, 0};
  double bd = 1e300;
  for (const rzf_tune_entry& e : c->tune) {
    const double d = std::fabs(std::log2((double)K / e.K)) + std::fabs(std::log2((double)N / e.N));
    // nearest; ties to the lower K, then the lower N
    if (d < bd || (d == bd && (e.K < best.K || (e.K == best.K && e.N < best.N)))) {
      bd = d;
      best = e;
    }
  }
  if (best.precoder_rows == 0) best.precoder_rows = 64;
  if (best.batch_precoder_rows == 0) best.batch_precoder_rows = 64;
  if (best.rate_splits == 0) best.rate_splits = sum_rate_splits(K, N);
  return best;
}

bool arena_take(rzf_ctx* c, size_t bytes, size_t* off) { return arena_alloc(c, bytes, off); }
void arena_give(rzf_ctx* c, size_t off, size_t bytes) { arena_free(c, off, bytes); }
bool reset_due(const rzf_track* t) {
  return t->prm.reset_period > 0 && t->since_reset + 1 >= t->prm.reset_period;
}

}  // namespace rzfrt

extern "C" {

rzf_status rzf_update_batch(rzf_ctx* c, int n, const rzf_update_item* items, double tol) {
  const rzf_status st = check_update_items(c, n, items, tol);
  if (st != RZF_OK) return st;
  std::lock_guard<std::mutex> lk(c->mu);
  HIP_OK(hipSetDevice(c->device));
  std::vector<DevInfo*> slots(n, nullptr);
  for (int i = 0; i < n; ++i) {
    if (!items[i].info) continue;
    slots[i] = pin_slot(c);
    if (!slots[i]) return RZF_E_DEVICE;
  }
  const rzf_status s2 = update_batch_locked(c, n, items, tol, slots.data(), c->stream, c->d_err);
  if (s2 != RZF_OK) return s2;
  for (int i = 0; i < n; ++i)
    if (slots[i]) c->pending.push_back(Pending{slots[i], items[i].info});
  return RZF_OK;
}

rzf_status rzf_full_batch(rzf_ctx* c, int n, const rzf_full_item* items) {
  if (!c) return RZF_E_INVALID;
  const rzf_status st = check_full_items(n, items);
  if (st != RZF_OK) return st;
  std::lock_guard<std::mutex> lk(c->mu);
  HIP_OK(hipSetDevice(c->device));
  return full_batch_locked(c, n, items, nullptr, c->stream, c->d_err);
}

rzf_status rzf_sum_rate_batch(rzf_ctx* c, int n, const rzf_rate_item* items, double P, double sigma2) {
  if (!c || !items || n < 1 || n > RZF_BATCH_MAX) return RZF_E_INVALID;
  if (!std::isfinite(P) || P <= 0.0 || !std::isfinite(sigma2) || sigma2 < 0.0) return RZF_E_INVALID;
  size_t want = 0;   // per-item partial sums, packed
  for (int i = 0; i < n; ++i) {
    const rzf_rate_item& it = items[i];
    if (!it.H || !it.W) return RZF_E_INVALID;
    if (it.K < 1 || it.K > RZF_KMAX || it.N < 1 || it.N > RZF_NMAX || it.ldh < it.N || it.ldw < it.K)
      return RZF_E_SHAPE;
    if (std::isnan(it.sigma2)) return RZF_E_INVALID;
    want += rate_scratch_bytes(it.K);
  }
  std::lock_guard<std::mutex> lk(c->mu);
  HIP_OK(hipSetDevice(c->device));
  hipStream_t s = c->stream;
  if (want > c->batch_part_bytes) {
    // grow: the old region may still be read by queued work
    HIP_OK(hipStreamSynchronize(c->stream));
    if (c->d_batch_part) arena_free(c, c->batch_part_off, c->batch_part_bytes);
    c->d_batch_part = nullptr;
    c->batch_part_bytes = 0;
    size_t off = 0;
    if (!arena_alloc(c, want, &off)) return RZF_E_NOMEM;
    c->batch_part_off = off;
    c->batch_part_bytes = want;
    c->d_batch_part = reinterpret_cast<double*>(c->arena + off);
  }
  RatePlan R;
  plan_rate(R, n, items, P, sigma2, reinterpret_cast<char*>(c->d_batch_part), c->d_counts);
  const int slot = stage_acquire(c);
  if (slot < 0) return RZF_E_DEVICE;
  Stager st{c->h_stage + slot * STAGE_BYTES, c->d_stage + slot * STAGE_BYTES};
  R.put(st);
  HIP_OK(hipMemcpyAsync(st.d, st.h, st.used, hipMemcpyHostToDevice, s));
  R.launch(c, s, c->d_err);
  HIP_OK(hipEventRecord(c->stage_ev[slot], s));
  c->stage_used[slot] = true;
  return hipGetLastError() == hipSuccess ? RZF_OK : RZF_E_DEVICE;
}

}  // extern "C"

extern "C" {

rzf_status rzf_full(rzf_ctx* c, int K, int N, const rzf_c32* H, int ldh, double alpha, double P,
                    rzf_c32* W, int ldw) {
  if (!c || !H || !W) return RZF_E_INVALID;
  if (K < 1 || K > RZF_KMAX || N < 1 || N > RZF_NMAX || ldh < N || ldw < K) return RZF_E_SHAPE;
  if (!std::isfinite(alpha) || alpha < 0.0 || !std::isfinite(P) || P <= 0.0) return RZF_E_INVALID;
  std::lock_guard<std::mutex> lk(c->mu);
  HIP_OK(hipSetDevice(c->device));
  hipStream_t s = c->stream;
  full_single_launch(c, K, N, reinterpret_cast<const float2*>(H), ldh, alpha, P, reinterpret_cast<float2*>(W), ldw,
                     s);
  return hipGetLastError() == hipSuccess ? RZF_OK : RZF_E_DEVICE;
}

rzf_status rzf_sum_rate(rzf_ctx* c, int K, int N, const rzf_c32* H, int ldh, const rzf_c32* W,
                        int ldw, double P, double sigma2, float* rates, double* sum_rate) {
  if (!c || !H || !W) return RZF_E_INVALID;
  if (K < 1 || K > RZF_KMAX || N < 1 || N > RZF_NMAX || ldh < N || ldw < K) return RZF_E_SHAPE;
  if (!std::isfinite(P) || P <= 0.0 || !std::isfinite(sigma2) || sigma2 < 0.0) return RZF_E_INVALID;
  std::lock_guard<std::mutex> lk(c->mu);
  HIP_OK(hipSetDevice(c->device));
  hipStream_t s = c->stream;
  rate_single_launch(c, K, N, reinterpret_cast<const float2*>(H), ldh, reinterpret_cast<const float2*>(W), ldw, P,
                     sigma2, rates, c->d_sum, s);
  if (hipGetLastError() != hipSuccess) return RZF_E_DEVICE;
  if (sum_rate) {
    HIP_OK(hipMemcpyAsync(c->h_sum, c->d_sum, sizeof(double), hipMemcpyDeviceToHost, s));
    rzf_status st = sync_and_collect(c);
    if (st != RZF_OK) return st;
    *sum_rate = *c->h_sum;
  }
  return RZF_OK;
}

rzf_status rzf_tune_switch(rzf_ctx* c, int K, int N, int precision, double* switch_ratio,
                           double* direct_cycles, double* wb_cycles_a, double* wb_cycles_b) {
  if (!c || !switch_ratio || K < 2 || K > RZF_KMAX || N < K || N > RZF_NMAX ||
      precision < RZF_PREC_FP32 || precision > RZF_PREC_BF16X3)
    return RZF_E_INVALID;
  const size_t kn = (size_t)K * N;
  // synthetic inputs from a fixed 64-bit LCG: H0 with entries uniform in
  // [-1/2, 1/2)^2, and per rank m the change X Y^H / 1000 (X K x m, Y N x m),
  // with alpha = 100: a small change, so that ||V~^H A^-1 U|| stays well
  // below 1/4 and the Woodbury step solves its capacitance by the passes, as
  // on a slowly varying channel.  eta = 1 - 1e-4 keeps the 2m components of
  // Delta A (their energy is known to FP32 accuracy, about 1e-6 relative)
  // and none of those of the FP32 rounding of H1 (about 1e-8 of the energy)
  uint64_t rs = 0x2545F4914F6CDD1Dull;
  auto unif = [&rs]() {
    rs = rs * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(rs >> 11) * 0x1.0p-53 - 0.5;
  };
  std::vector<rzf_c32> h0(kn), h1(kn);
  for (rzf_c32& v : h0) {
    v.re = (float)unif();
    v.im = (float)unif();
  }
  size_t off = 0;
  const size_t bytes = align_up(sizeof(rzf_c32) * 3 * kn);
  {
    std::lock_guard<std::mutex> lk(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return RZF_E_DEVICE;
    // an error of earlier asynchronous work stays pending for the next rzf_sync
    if (hold_earlier_error(c) != RZF_OK) return RZF_E_DEVICE;
    if (!arena_alloc(c, bytes, &off)) return RZF_E_NOMEM;
  }
  rzf_c32* dH0 = reinterpret_cast<rzf_c32*>(c->arena + off);
  rzf_c32* dH1 = dH0 + kn;
  rzf_c32* dW = dH1 + kn;   // N x K
  rzf_status st = RZF_OK;
  // cycles after the SVD of one update H0 -> H1 (fresh track, d = K at the
  // first iteration), the least of three runs; the rank and path it took
  auto measure = [&](double ratio, double* cyc, int* r_out, int* path_out) -> rzf_status {
    rzf_params prm;
    rzf_params_default(&prm);
    prm.k_init = K;
    prm.p = 0;
    prm.switch_ratio = ratio;
    prm.precision = precision;
    double best = 0.0;
    for (int rep = 0; rep < 3; ++rep) {
      rzf_track* t = nullptr;
      rzf_status s1 = rzf_init(c, K, N, dH0, N, 100.0, &prm, &t);
      if (s1 != RZF_OK) return s1;
      rzf_update_info info;
      s1 = rzf_update(t, dH1, N, 1.0 - 1e-4, dW, K, &info);
      if (s1 == RZF_OK) {
        std::lock_guard<std::mutex> lk(c->mu);
        s1 = own_device_error(c);
      }
      int v[8] = {0};
      if (s1 == RZF_OK) s1 = rzf_debug_counters(t, v, 8);
      rzf_track_destroy(t);
      if (s1 != RZF_OK) return s1;
      const double cy = (double)(unsigned)v[6];
      if (rep == 0 || cy < best) best = cy;
      *r_out = info.r;
      *path_out = info.path;
    }
    *cyc = best;
    return RZF_OK;
  };
  auto set_change = [&](int m) -> rzf_status {
    std::vector<rzf_c32> X((size_t)K * m), Y((size_t)N * m);
    for (rzf_c32& v : X) { v.re = (float)unif(); v.im = (float)unif(); }
    for (rzf_c32& v : Y) { v.re = (float)unif(); v.im = (float)unif(); }
    for (int i = 0; i < K; ++i)
      for (int n = 0; n < N; ++n) {
        double re = h0[(size_t)i * N + n].re, im = h0[(size_t)i * N + n].im;
        for (int q = 0; q < m; ++q) {   // + X[i, q] conj(Y[n, q]) / 1000
          const rzf_c32 x = X[(size_t)i * m + q], y = Y[(size_t)n * m + q];
          re += 1e-3 * ((double)x.re * y.re + (double)x.im * y.im);
          im += 1e-3 * ((double)x.im * y.re - (double)x.re * y.im);
        }
        h1[(size_t)i * N + n].re = (float)re;
        h1[(size_t)i * N + n].im = (float)im;
      }
    if (hipSetDevice(c->device) != hipSuccess ||
        hipMemcpy(dH1, h1.data(), sizeof(rzf_c32) * kn, hipMemcpyHostToDevice) != hipSuccess)
      return RZF_E_DEVICE;
    return RZF_OK;
  };
  const int cap = wb_capacity(K);   // Woodbury workspace
  std::vector<double> rr, cc;
  double direct = 0.0;
  int r = 0, path = 0;
  if (hipSetDevice(c->device) != hipSuccess ||
      hipMemcpy(dH0, h0.data(), sizeof(rzf_c32) * kn, hipMemcpyHostToDevice) != hipSuccess)
    st = RZF_E_DEVICE;
  // the direct inversion (switch below 1/K: every rank inverts), at the largest change
  if (st == RZF_OK) st = set_change(std::max(1, cap / 2));
  if (st == RZF_OK) st = measure(0.5 / K, &direct, &r, &path);
  if (st == RZF_OK && path != RZF_PATH_FULL_RANK) st = RZF_E_DEVICE;
  // the Woodbury branch at change ranks m (Delta A of rank 2m)
  for (int m = 1; st == RZF_OK && 2 * m <= cap; m = (m < 4) ? 2 * m : m + 4) {
    st = set_change(m);
    double cy = 0.0;
    if (st == RZF_OK) st = measure(std::min(1.0, (cap + 0.5) / K), &cy, &r, &path);
    if (st == RZF_OK && path == RZF_PATH_WB && r > 0) {
      rr.push_back(r);
      cc.push_back(cy);
    }
  }
  {
    std::lock_guard<std::mutex> lk(c->mu);
    if (hipStreamSynchronize(c->stream) != hipSuccess) st = RZF_E_DEVICE;
    arena_free(c, off, bytes);
  }
  if (st != RZF_OK) return st;
  if (rr.size() < 2) return RZF_E_DEVICE;
  // least-squares line through (r, cycles)
  double sr = 0, sc = 0, srr = 0, src = 0;
  const double n = (double)rr.size();
  for (size_t i = 0; i < rr.size(); ++i) {
    sr += rr[i]; sc += cc[i]; srr += rr[i] * rr[i]; src += rr[i] * cc[i];
  }
  const double den = n * srr - sr * sr;
  const double b = den != 0.0 ? (n * src - sr * sc) / den : 0.0;
  const double a = (sc - b * sr) / n;
  int rstar = 0;   // largest whole rank with a + b r <= direct
  for (int k = 1; k <= cap; ++k)
    if (a + b * k <= direct) rstar = k;
  *switch_ratio = (double)rstar / K;
  if (direct_cycles) *direct_cycles = direct;
  if (wb_cycles_a) *wb_cycles_a = a;
  if (wb_cycles_b) *wb_cycles_b = b;
  return RZF_OK;
}

rzf_status rzf_beamspace(rzf_ctx* c, int K, int nx, int ny, const rzf_c32* H, int ldh, int n_rf,
                         int select, int* beams, rzf_c32* H_eff, int ld_eff) {
  if (!c || !H || !beams || !H_eff || (select != 0 && select != 1)) return RZF_E_INVALID;
  if (K < 1 || K > RZF_KMAX || nx < 1 || ny < 1 || nx > RZF_NMAX || ny > RZF_NMAX / nx) return RZF_E_SHAPE;
  const int N = nx * ny;
  if (ldh < N || n_rf < (select ? K : 1) || n_rf > N || ld_eff < n_rf) return RZF_E_SHAPE;
  std::lock_guard<std::mutex> lk(c->mu);
  HIP_OK(hipSetDevice(c->device));
  hipStream_t s = c->stream;
  const size_t want = sizeof(float2) * (size_t)K * N;
  if (want > c->beam_g_bytes) {
    // grow: the old region may still be read by queued work
    HIP_OK(hipStreamSynchronize(c->stream));
    if (c->d_beam_g) arena_free(c, c->beam_g_off, c->beam_g_bytes);
    c->d_beam_g = nullptr;
    c->beam_g_bytes = 0;
    size_t off = 0;
    if (!arena_alloc(c, want, &off)) return RZF_E_NOMEM;
    c->beam_g_off = off;
    c->beam_g_bytes = want;
    c->d_beam_g = reinterpret_cast<float2*>(c->arena + off);
  }
  const float2* Hf = reinterpret_cast<const float2*>(H);
  timed(c, KN_BEAM_RESP, s, [&] { launch_beam_resp(Hf, ldh, K, nx, ny, c->d_beam_g, s); });
  timed(c, KN_BEAM_SELECT, s, [&] {
    launch_beam_select(c->d_beam_g, K, N, n_rf, select, beams, reinterpret_cast<float2*>(H_eff), ld_eff,
                       c->d_err, s);
  });
  return hipGetLastError() == hipSuccess ? RZF_OK : RZF_E_DEVICE;
}

rzf_status rzf_get_inverse(rzf_track* t, rzf_c32* Ainv) {
  if (!t || !Ainv) return RZF_E_INVALID;
  rzf_ctx* c = t->ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  HIP_OK(hipSetDevice(c->device));
  HIP_OK(hipMemcpyAsync(Ainv, t->h_desc.Ainv, sizeof(float2) * t->K * t->K,
                        hipMemcpyDeviceToDevice, c->stream));
  return RZF_OK;
}

rzf_status rzf_track_query(rzf_track* t, int* K, int* N, int* step, int* since_reset, int* last_r) {
  if (!t) return RZF_E_INVALID;
  rzf_ctx* c = t->ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  HIP_OK(hipSetDevice(c->device));
  HIP_OK(hipStreamSynchronize(c->stream));
  if (K) *K = t->K;
  if (N) *N = t->N;
  if (step) *step = t->t;
  if (since_reset) *since_reset = t->since_reset;
  if (last_r) {
    int v = 0;
    HIP_OK(hipMemcpy(&v, &t->d_desc->last_r, sizeof(int), hipMemcpyDeviceToHost));
    *last_r = v;
  }
  return RZF_OK;
}

rzf_status rzf_debug_counters(rzf_track* t, int* out, int n) {
  if (!t || !out || n < 0) return RZF_E_INVALID;
  rzf_ctx* c = t->ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  HIP_OK(hipSetDevice(c->device));
  HIP_OK(hipStreamSynchronize(c->stream));
  int v[8];
  HIP_OK(hipMemcpy(v, t->d_desc->dbg, sizeof(v), hipMemcpyDeviceToHost));
  for (int i = 0; i < n && i < 8; ++i) out[i] = v[i];
  return RZF_OK;
}

rzf_status rzf_debug_sigma2(rzf_track* t, double* out, int n, int* d_out) {
  if (!t || !d_out || (n > 0 && !out)) return RZF_E_INVALID;
  rzf_ctx* c = t->ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  HIP_OK(hipSetDevice(c->device));
  HIP_OK(hipStreamSynchronize(c->stream));
  int d = 0;
  HIP_OK(hipMemcpy(&d, &t->d_desc->nsig, sizeof(int), hipMemcpyDeviceToHost));
  if (d < 0 || d > KM) d = 0;
  const int m = n < d ? n : d;
  if (m > 0) HIP_OK(hipMemcpy(out, t->d_desc->sig2, sizeof(double) * m, hipMemcpyDeviceToHost));
  *d_out = d;
  return RZF_OK;
}

rzf_status rzf_track_export(rzf_track* t, void* buf, size_t* bytes) {
  if (!t || !bytes) return RZF_E_INVALID;
  const size_t need = blob_bytes(t->K, t->N);
  if (!buf) { *bytes = need; return RZF_OK; }
  if (*bytes < need) { *bytes = need; return RZF_E_INVALID; }
  rzf_ctx* c = t->ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  HIP_OK(hipSetDevice(c->device));
  HIP_OK(hipStreamSynchronize(c->stream));
  TrackBlob h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, BLOB_MAGIC, sizeof(h.magic));
  h.version = BLOB_VERSION;
  h.header_bytes = sizeof(TrackBlob);
  h.K = t->K; h.N = t->N; h.prm = t->prm; h.alpha = t->alpha;
  h.step = t->t; h.since_reset = t->since_reset;
  HIP_OK(hipMemcpy(&h.last_r, &t->d_desc->last_r, sizeof(int), hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(&h.warm, &t->d_desc->warm, sizeof(int), hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(&h.dwarm, &t->d_desc->dwarm, sizeof(int), hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(&h.nsig, &t->d_desc->nsig, sizeof(int), hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(&h.spec_hint, &t->d_desc->spec_hint, sizeof(int), hipMemcpyDeviceToHost));
  char* p = static_cast<char*>(buf);
  std::memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  HIP_OK(hipMemcpy(p, t->h_desc.Ainv, sizeof(float2) * t->K * t->K, hipMemcpyDeviceToHost));
  p += sizeof(float2) * t->K * t->K;
  HIP_OK(hipMemcpy(p, t->h_desc.Hprev, sizeof(float2) * (size_t)t->K * t->N, hipMemcpyDeviceToHost));
  p += sizeof(float2) * (size_t)t->K * t->N;
  HIP_OK(hipMemcpy(p, t->h_desc.Rfb, sizeof(float2) * t->K * t->K, hipMemcpyDeviceToHost));
  p += sizeof(float2) * t->K * t->K;
  if (t->h_desc.Xw)
    HIP_OK(hipMemcpy(p, t->h_desc.Xw, sizeof(float2) * t->K * t->K, hipMemcpyDeviceToHost));
  else
    std::memset(p, 0, sizeof(float2) * t->K * t->K);
  p += sizeof(float2) * t->K * t->K;
  if (t->h_desc.Xd)
    HIP_OK(hipMemcpy(p, t->h_desc.Xd, sizeof(float2) * t->K * t->K, hipMemcpyDeviceToHost));
  else
    std::memset(p, 0, sizeof(float2) * t->K * t->K);
  *bytes = need;
  return RZF_OK;
}

rzf_status rzf_track_import(rzf_ctx* c, const void* buf, size_t bytes, rzf_track** out) {
  if (!c || !buf || !out) return RZF_E_INVALID;
  *out = nullptr;
  if (bytes < sizeof(TrackBlob)) return RZF_E_INVALID;
  TrackBlob h;
  std::memcpy(&h, buf, sizeof(h));
  if (std::memcmp(h.magic, BLOB_MAGIC, sizeof(h.magic)) != 0 || h.version != BLOB_VERSION ||
      h.header_bytes != sizeof(TrackBlob))
    return RZF_E_INVALID;
  if (h.K < 1 || h.K > RZF_KMAX || h.N < 1 || h.N > RZF_NMAX) return RZF_E_SHAPE;
  if (bytes < blob_bytes(h.K, h.N)) return RZF_E_INVALID;
  if (!params_valid(&h.prm) || !params_fit(&h.prm, h.K) || !std::isfinite(h.alpha) || h.alpha < 0.0 || h.step < 0 ||
      h.since_reset < 0 || h.last_r < 0 || h.last_r > h.K || (h.warm != 0 && h.warm != 1) ||
      h.dwarm < 0 || h.dwarm >= h.K || (h.dwarm > 0 && h.K > KS) || h.nsig < 0 || h.nsig > h.K ||
      h.spec_hint < 0 || h.spec_hint > 64)
    return RZF_E_INVALID;
  std::lock_guard<std::mutex> lk(c->mu);
  HIP_OK(hipSetDevice(c->device));
  rzf_status st0 = hold_earlier_error(c);
  if (st0 != RZF_OK) return st0;
  rzf_track* t = track_new(c, h.K, h.N, h.prm, h.alpha);
  if (!t) return RZF_E_NOMEM;
  t->t = h.step;
  t->since_reset = h.since_reset;
  t->h_desc.last_r = h.last_r;
  t->h_desc.t_dev = h.step;
  t->h_desc.seq_dev += (unsigned)h.step;
  t->h_desc.warm = h.warm;
  t->h_desc.dwarm = h.dwarm;
  t->h_desc.nsig = h.nsig;
  t->h_desc.spec_hint = h.spec_hint;
  const char* p = static_cast<const char*>(buf) + sizeof(h);
  bool ok = hipMemcpy(t->d_desc, &t->h_desc, sizeof(TrackDesc), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(t->h_desc.Ainv, p, sizeof(float2) * h.K * h.K, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(t->h_desc.Hprev, p + sizeof(float2) * h.K * h.K, sizeof(float2) * (size_t)h.K * h.N,
                      hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(t->h_desc.Rfb, p + sizeof(float2) * ((size_t)h.K * h.K + (size_t)h.K * h.N),
                      sizeof(float2) * h.K * h.K, hipMemcpyHostToDevice) == hipSuccess &&
            (!t->h_desc.Xw ||
             hipMemcpy(t->h_desc.Xw, p + sizeof(float2) * (2 * (size_t)h.K * h.K + (size_t)h.K * h.N),
                       sizeof(float2) * h.K * h.K, hipMemcpyHostToDevice) == hipSuccess) &&
            (!t->h_desc.Xd ||
             hipMemcpy(t->h_desc.Xd, p + sizeof(float2) * (3 * (size_t)h.K * h.K + (size_t)h.K * h.N),
                       sizeof(float2) * h.K * h.K, hipMemcpyHostToDevice) == hipSuccess);
  if (!ok) {
    arena_free(c, t->off, t->bytes);
    delete t;
    return RZF_E_DEVICE;
  }
  c->tracks.insert(t);
  *out = t;
  return RZF_OK;
}

rzf_status rzf_track_destroy(rzf_track* t) {
  if (!t) return RZF_E_INVALID;
  rzf_ctx* c = t->ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  if (t->graphs > 0) return RZF_E_INVALID;   // a captured step still updates it
  (void)hipSetDevice(c->device);
  HIP_OK(hipStreamSynchronize(c->stream));
  c->tracks.erase(t);
  arena_free(c, t->off, t->bytes);
  delete t;
  return RZF_OK;
}

rzf_status rzf_debug_sketch(rzf_ctx* c, uint64_t seed, uint64_t track_id, int t, int it, int K, int d,
                            rzf_c32* Omega, uint64_t* words) {
  if (!c || (!Omega && !words)) return RZF_E_INVALID;
  if (K < 1 || K > 1024 || d < 1 || d > K || t < 0 || it < 0) return RZF_E_SHAPE;
  std::lock_guard<std::mutex> lk(c->mu);
  HIP_OK(hipSetDevice(c->device));
  launch_debug_sketch(seed, track_id, t, it, K, d, reinterpret_cast<float2*>(Omega), words, c->stream);
  return hipGetLastError() == hipSuccess ? RZF_OK : RZF_E_DEVICE;
}

rzf_status rzf_tune_table(rzf_ctx* c, int n, const rzf_tune_entry* entries) {
  if (!c || n < 0 || n > 4096 || (n > 0 && !entries)) return RZF_E_INVALID;
  for (int i = 0; i < n; ++i) {
    const rzf_tune_entry& e = entries[i];
    if (e.K < 1 || e.K > RZF_KMAX || e.N < 1 || e.N > RZF_NMAX) return RZF_E_INVALID;
    for (int v : {e.precoder_rows, e.batch_precoder_rows})
      if (v != 0 && v != 32 && v != 64 && v != 256) return RZF_E_INVALID;
    if (e.rate_splits < 0 || e.rate_splits > 8) return RZF_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(c->mu);
  c->tune.assign(entries, entries + n);
  return RZF_OK;
}

rzf_status rzf_profile(rzf_ctx* c, int enable) {
  if (!c) return RZF_E_INVALID;
  std::lock_guard<std::mutex> lk(c->mu);
  HIP_OK(hipSetDevice(c->device));
  if (enable) {
    prof_drain(c);
    for (int k = 0; k < KN_COUNT; ++k) { c->prof_count[k] = 0; c->prof_ms[k] = 0.0; }
  }
  c->prof_on = enable != 0;
  return RZF_OK;
}

rzf_status rzf_profile_read(rzf_ctx* c, rzf_profile_entry* out, int max, int* n) {
  if (!c || !n || (max > 0 && !out)) return RZF_E_INVALID;
  std::lock_guard<std::mutex> lk(c->mu);
  HIP_OK(hipSetDevice(c->device));
  HIP_OK(hipStreamSynchronize(c->stream));
  prof_drain(c);
  int m = 0;
  for (int k = 0; k < KN_COUNT; ++k) {
    if (!c->prof_count[k]) continue;
    if (m < max) {
      std::memset(out[m].name, 0, sizeof(out[m].name));
      std::strncpy(out[m].name, KERNEL_NAMES[k], sizeof(out[m].name) - 1);
      out[m].count = c->prof_count[k];
      out[m].total_ms = c->prof_ms[k];
    }
    ++m;
  }
  *n = m;
  return RZF_OK;
}

}  // extern "C"
