// Host runtime state behind rzf.h, shared by the entry points (api.cpp) and
// the request server (server.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <vector>

#include "rzf.h"
#include "rzf_internal.h"

namespace rzfrt {

constexpr size_t ALIGN = 256;
constexpr int PIN_CHUNK = 4096;   // info records per pinned chunk
constexpr int NSTAGE = 4;
constexpr size_t STAGE_BYTES = 1 << 20;   // per slot

inline size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

struct Pending {
  DevInfo* slot;
  rzf_update_info* dst;
};

struct ProfRec {
  int kernel;
  hipEvent_t a, b;
};

enum { KN_GRAM, KN_GRAM64, KN_INV64, KN_INV32, KN_ARSVD, KN_PRECODER, KN_SCALE, KN_SUMRATE,
       KN_BEAM_RESP, KN_BEAM_SELECT, KN_COUNT };

}  // namespace rzfrt

struct rzf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  bool own_arena = false;
  std::map<size_t, size_t> free_blocks;   // offset -> size
  // fixed scratch at the front of the arena
  int* d_err = nullptr;
  unsigned* d_counts = nullptr;         // completion counts of the context's sum-rate launches (item i at i)
  int held_err = 0;                     // device error of earlier work, kept for rzf_sync
  float2* d_fullA = nullptr;
  float2* d_fullAinv = nullptr;
  double* d_fullwpart = nullptr;
  double* d_sum = nullptr;
  double* d_srpart = nullptr;
  float2* d_spec = nullptr;             // speculated iterations of a single-track arSVD step
  // pinned host staging
  double* h_sum = nullptr;
  int* h_err = nullptr;
  std::vector<DevInfo*> pin_chunks;
  size_t pin_used = 0;
  std::vector<rzfrt::Pending> pending;
  std::set<rzf_track*> tracks;
  std::set<rzf_graph*> graphs;          // captured steps on this context
  std::vector<rzf_tune_entry> tune;     // launch shapes by track size (rzf_tune_table)
  std::mutex mu;
  // batched calls: ring of pinned host / device staging slots for job arrays
  char* h_stage = nullptr;
  char* d_stage = nullptr;
  hipEvent_t stage_ev[rzfrt::NSTAGE] = {};
  bool stage_used[rzfrt::NSTAGE] = {};
  int stage_next = 0;
  double* d_batch_part = nullptr;       // sum-rate scratch of batched calls
  size_t batch_part_off = 0, batch_part_bytes = 0;
  char* d_batch_full = nullptr;         // Gram / partial-norm scratch of rzf_full_batch
  size_t batch_full_off = 0, batch_full_bytes = 0;
  float2* d_beam_g = nullptr;           // beam responses of rzf_beamspace
  size_t beam_g_off = 0, beam_g_bytes = 0;
  bool capturing = false;               // a step is being captured into a graph (no timing events)
  // event timing
  bool prof_on = false;
  std::vector<rzfrt::ProfRec> prof;
  std::vector<hipEvent_t> ev_pool;
  int prof_count[rzfrt::KN_COUNT] = {};
  double prof_ms[rzfrt::KN_COUNT] = {};
};

struct rzf_track {
  rzf_ctx* ctx = nullptr;
  int K = 0, N = 0;
  rzf_params prm{};
  double alpha = 0.0;
  size_t off = 0, bytes = 0;
  TrackDesc* d_desc = nullptr;
  TrackDesc h_desc{};
  int t = 0;
  int since_reset = 0;
  int i_max = 0;
  int graphs = 0;   // captured steps (rzf_graph) that update this track
};

namespace rzfrt {

// Argument checks of rzf_update_batch / rzf_full_batch (no device work).
rzf_status check_update_items(rzf_ctx* c, int n, const rzf_update_item* items, double tol);
rzf_status check_full_items(int n, const rzf_full_item* items);

// Launch one batched update (c->mu held, items checked) on stream s, device
// errors recorded in *err.  For every i with slots[i] != nullptr the step's
// info record is copied into that pinned host slot on s after the update;
// the caller decides when it is valid (an event, or rzf_sync).
rzf_status update_batch_locked(rzf_ctx* c, int n, const rzf_update_item* items, double tol,
                               DevInfo* const* slots, hipStream_t s, int* err);
// Per-item scratch of a batched full inversion: the K x K Gram matrix (then
// its inverse) and the precoder's partial sums.
struct FullScratch {
  float2* A;
  double* wpart;
};
// Launch one batched full-inversion RZF (c->mu held, items checked) on
// stream s, device errors in *err.  scr: per-item scratch, or nullptr for
// the context's own (grown on demand; then only on the context stream).
rzf_status full_batch_locked(rzf_ctx* c, int n, const rzf_full_item* items, const FullScratch* scr,
                             hipStream_t s, int* err);

// Job arrays of a batched launch: written into a host buffer h and given the
// matching addresses in device memory d (the caller copies h to d once).
struct Stager {
  char* h;
  char* d;
  size_t used = 0;
  template <class T>
  T* put(const T* src, int n, T** dev) {
    used = (used + 15) & ~size_t(15);
    T* hp = reinterpret_cast<T*>(h + used);
    *dev = reinterpret_cast<T*>(d + used);
    std::memcpy(hp, src, sizeof(T) * n);
    used += sizeof(T) * n;
    return hp;
  }
};

// The launches of one batched update step over their job arrays.  bytes()
// bounds what put() writes; launch() needs the arrays in device memory.
struct UpdatePlan {
  std::vector<GramJob> gj;
  std::vector<ArsvdJob> aj, ajb;   // LDS kernels (K <= KS) / large tracks
  std::vector<Gram64Job> g64;
  std::vector<Inv64Job> i64, i64b;
  std::vector<PrecJob> pj;
  std::vector<ScaleJob> sj;
  std::vector<int> reset_flag;
  int maxK = 1, maxN = 1, maxKr = 1, maxNK = 1;
  GramJob* d_gj = nullptr;
  ArsvdJob* d_aj = nullptr;
  ArsvdJob* d_ajb = nullptr;
  ArsvdJob* d_ajo = nullptr;    // d_aj, d_ajb in longest-first order (written on the device)
  ArsvdJob* d_ajbo = nullptr;
  Gram64Job* d_g64 = nullptr;
  Inv64Job* d_i64 = nullptr;
  Inv64Job* d_i64b = nullptr;
  PrecJob* d_pj = nullptr;
  ScaleJob* d_sj = nullptr;
  size_t bytes() const;
  void put(Stager& st);
  void launch(rzf_ctx* c, hipStream_t s, int* err) const;
};
// force_reset < 0: each track's own reset schedule; 0 or 1: every item takes
// a Woodbury step, or an FP64 re-inversion.
void plan_update(UpdatePlan& P, int n, const rzf_update_item* items, double tol, int force_reset);
// Host step counters after a step of these tracks.
void advance_tracks(int n, rzf_track* const* tracks, const std::vector<int>& reset_flag);
bool reset_due(const rzf_track* t);

struct FullPlan {
  std::vector<GramJob> gj;
  std::vector<Inv32Job> vj, vjb;
  std::vector<PrecJob> pj;
  std::vector<ScaleJob> sj;
  int maxK = 1, maxN = 1, maxNK = 1;
  GramJob* d_gj = nullptr;
  Inv32Job* d_vj = nullptr;
  Inv32Job* d_vjb = nullptr;
  PrecJob* d_pj = nullptr;
  ScaleJob* d_sj = nullptr;
  size_t bytes() const;
  void put(Stager& st);
  void launch(rzf_ctx* c, hipStream_t s, int* err) const;
};
void plan_full(FullPlan& P, int n, const rzf_full_item* items, const FullScratch* scr);
size_t full_scratch_bytes(const rzf_full_item& it);
FullScratch full_scratch_at(const rzf_full_item& it, char* p);

struct RatePlan {
  std::vector<RateJob> rj;
  int maxK = 1;
  RateJob* d_rj = nullptr;
  size_t bytes() const;
  void put(Stager& st);
  void launch(rzf_ctx* c, hipStream_t s, int* err) const;
};
// part: the items' scratch packed in item order (rate_scratch_bytes(K) each);
// counts: one completion count per item, zero between launches.
void plan_rate(RatePlan& P, int n, const rzf_rate_item* items, double Pw, double sigma2, char* part,
               unsigned* counts);
size_t rate_scratch_bytes(int K);

// One track's launches (c->mu held, arguments checked), as rzf_update,
// rzf_full and rzf_sum_rate make them.
void update_single_launch(rzf_ctx* c, rzf_track* t, const float2* H, int ldh, double tol, float2* W, int ldw,
                          bool reset, hipStream_t s);
void full_single_launch(rzf_ctx* c, int K, int N, const float2* H, int ldh, double alpha, double P, float2* W,
                        int ldw, hipStream_t s);
void rate_single_launch(rzf_ctx* c, int K, int N, const float2* H, int ldh, const float2* W, int ldw, double P,
                        double sigma2, float* rates, double* sum, hipStream_t s);

// The launch shapes for a (K, N) track: the table's entry (exact, else
// nearest), knobs left at 0 resolved to the defaults.
rzf_tune_entry tune_for(const rzf_ctx* c, int K, int N);

// Frees every graph of a context that is being destroyed.
void graphs_release_all(rzf_ctx* c);

// Device memory from the context's arena (c->mu held).
bool arena_take(rzf_ctx* c, size_t bytes, size_t* off);
void arena_give(rzf_ctx* c, size_t off, size_t bytes);

}  // namespace rzfrt
