// Host/device shared definitions of the HIP implementation behind rzf.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rzf.h"

#define KM RZF_KMAX     // largest K of any track
#define KS 64           // largest K whose working set fits one workgroup's LDS
#define WB_RMAX 32      // largest Woodbury rank of the LDS kernels (= KS / 2)

// Device-side error codes (first one wins; rzf_sync maps them to rzf_status).
#define DEV_ERR_NOT_HPD 1
#define DEV_ERR_NONFINITE 2
#define DEV_ERR_BEAM 3        // a given beam index outside the codebook

// Per-update outcome, same layout as rzf_update_info.
struct DevInfo {
  int r, iters, path, d;
  double dA_fro2, captured;
};

// One track, resident in device memory (in the context arena).
struct TrackDesc {
  int K, N;
  double alpha, P, switch_ratio;
  int k_init, p, i_max, kinit_policy;
  int early_fallback, wb_limit;   // policy flag; largest rank the Woodbury branch takes
  int prec, error_feedback;       // rzf_precision of the Gram and precoder operands; policy
  float2* Rfb;     // K x K, ld K: error-feedback residual (zero unless the policy is on)
  float2* Xw;      // K x K, column-major ld K: normalised columns z_j / sigma_j
                   // of the last full-width (d = K) SVD, the next one's starting point
  float2* Xd;      // K x K, column-major ld K (K <= KS): the last SVD below full width
                   // (and at least 32 wide), its dwarm normalised columns z_j / sigma_j
                   // by descending sigma_j
  uint64_t seed, track_id;
  float2* Ainv;    // K x K, ld K: stored inverse
  float2* Hprev;   // K x N, ld N: previous snapshot
  float2* Anew;    // K x K, ld K: A' of the current step (FP32)
  float2* dA;      // K x K, ld K: Delta A of the current step
  double2* A64;    // K x K, ld K: FP64 Gram for init / reset
  double* wpart;   // precoder scratch: partial ||W||^2 of its blocks, then its completion count
  // working set of the large-track kernels (K > KS), null otherwise; all
  // column-major with leading dimension K
  float2* Ym;      // K x K: sketch Y, the Householder vectors, Q^H Delta A Z_r, then P = A^-1 U
  float2* Qm;      // K x K: Q
  float2* Zm;      // K x K: Z = Delta A Q, rotated by the Jacobi sweeps
  float2* Pm;      // K x K/2: Delta A Z_r, then U_r
  double2* Aug;    // (K/2) x (K/2 + K), row-major: [C | V~^H A^-1] in FP64
  // written by the device
  int last_r;
  int spec_hint;   // Alg. 1 iterations of the last step that ran it (speculation depth)
  int warm;        // Xw holds a basis
  int dwarm;       // columns of Xd that hold a basis (0: none)
  int hold;        // the current step met a non-finite snapshot (or its reset failed):
                   // the precoder keeps H_prev, so the track's state stays as it was
  DevInfo info;
  int dbg[8];      // last update: [0] Jacobi sweeps, [1] Jacobi rounds, [2] QR columns
  int nsig;        // number of sigma^2 below (d of the last SVD, 0 if none)
  int t_dev;       // steps done (the host's count, advanced on the device by the step's
                   // last launch, so that a captured step replays with the right index)
  unsigned long long seq_dev;   // the two-phase form's tag number of the next step: unique to
                                // the track in the process (its number times 2^32), plus t_dev
  double sig2[KM]; // last SVD: sigma_j^2, descending
};

// A track descriptor addressed as global memory.  A descriptor pointer read
// from a job array in device memory is a generic pointer, and a generic load
// may reach per-lane scratch, so every field read through it would count as a
// per-lane value and occupy vector registers; through this type the fields
// stay in scalar registers.  Whole-struct copies go through the plain type.
using GTrackDesc = __attribute__((address_space(1))) TrackDesc;

// Work descriptors.  Every kernel takes one descriptor by value (a single
// call) or a device array of them indexed by blockIdx.y (a batch); blocks
// beyond a descriptor's own grid extent return at once.  The two forms are
// separate instantiations (template flag MANY), so profiles tell them apart.
struct GramJob {
  const float2* Ht; const float2* Hp; float2* Anew; float2* dA;
  int K, N, ldh, ldp;
  float alpha;
  int prec;        // rzf_precision of the operands
};
struct Gram64Job {
  const float2* H; double2* A;
  int K, N, ldh;
  double alpha;
};
struct Inv64Job {
  const double2* A; float2* Ainv; DevInfo* info; DevInfo* out;   // out: extra copy of info, or null
  int K;
  float2* zero;    // K x K cleared alongside (the error-feedback residual), or null
  int* hold;       // reset step: set to 1 (state kept, nothing written) if the
                   // inversion fails, else 0; null for rzf_init
};
struct Inv32Job {
  const float2* A; float2* Ainv;   // may alias: A is read into LDS first
  int K;
};
struct ArsvdJob {
  TrackDesc* td;   // the step index (sketch counter) and the two-phase tag number come from
                   // td->t_dev and td->seq_dev
  DevInfo* out;    // extra copy of the step's info (batched calls), or null
  double eta;
  int i_max;
  float2* spec;    // speculative-iteration workspace (SPEC_BYTES), two-phase single-track form only
  char* stage;     // staging area of the job's full-width step (two-phase form), or null
};
// Two-phase single-track form of the K <= KS arSVD kernel: up to SPEC_MAX
// iterations of Alg. 1 are computed at once, one workgroup each, into
// [SPEC_MAX][Q, Z][KS x KS] complex values followed by SPEC_MAX doubles
// (||Z||_F^2), one more (||Delta A||_F^2) and SPEC_MAX + 1 64-bit tags (the
// launch number once the iteration's ||Z||_F^2 is posted; the last one once
// the full-width iteration has written the whole step to the track).  The workgroup of the first full-width iteration (d = K) also
// carries the step through when its energy test passes, into a staging area
// (after those doubles) that the second phase copies to the track if that
// iteration decides: SpecStage, sigma^2 (KS doubles), then A'^-1 and R
// (K x K, ld K, row-major) and the rotated basis (K x K, ld K, column-major).
#define SPEC_MAX 8
struct SpecStage {
  DevInfo info;
  int warm, nsig, err, pad_;   // warm: the staged basis may start the next full-width step
  int dbg[8];
};
inline constexpr size_t stage_bytes(int K) {
  return (sizeof(SpecStage) + sizeof(double) * KS + sizeof(float2) * 3 * (size_t)K * K + 255) & ~size_t(255);
}
#define SPEC_STAGE_OFF (sizeof(float2) * 2 * KS * KS * SPEC_MAX + sizeof(double) * (2 * SPEC_MAX + 2))
#define SPEC_BYTES (SPEC_STAGE_OFF + stage_bytes(KS))
struct PrecJob {
  const float2* H; const float2* X; float2* W; double* wpart; float2* Hcopy;
  int K, N, ldh, ldw;
  int prec;        // rzf_precision of the operands
  const int* hold; // if set and nonzero when the kernel runs, H is not copied to Hcopy
};
struct ScaleJob {
  float2* W; const double* wpart;
  double P;
  int K, N, ldw, nparts;
  TrackDesc* adv;   // a track's step ends here: its t_dev and seq_dev advance (or null)
};
struct RateJob {
  const float2* H; const float2* W; double* part; float* rates; double* sum;
  int K, N, ldh, ldw;
  double P, sigma2;
  unsigned* count; // the launch's completion count: zero before, left at zero after
};

template <bool MANY, class J>
__device__ __forceinline__ const J& job_of(const J& one, const J* many) {
  if constexpr (MANY) return many[blockIdx.y]; else return one;
}

// Position (x, item) of this workgroup in a batched launch of gridDim.x
// workgroups per item, relabelled so that one item's workgroups run on one
// XCD: the hardware hands consecutive workgroups to the 8 XCDs in turn, each
// with its own L2, so linear id L runs on XCD L mod 8, and the logical id
// (L mod 8) * share + L / 8 makes consecutive logical ids (an item's
// workgroups, which read the same operands) share that XCD's L2.  A bijection
// of the grid whatever the dispatch order, so it moves only time.
struct GridPos { int x, item; };
__device__ __forceinline__ GridPos xcd_grid_pos() {
  constexpr int NX = 8;
  const int gx = gridDim.x, total = gridDim.x * gridDim.y;
  const int L = blockIdx.y * gx + blockIdx.x;
  const int per = total / NX, rem = total - per * NX;
  const int xcd = L % NX, slot = L / NX;
  const int logical = xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
  return {logical % gx, logical / gx};
}
template <bool MANY>
__device__ __forceinline__ GridPos grid_pos() {
  if constexpr (MANY) return xcd_grid_pos(); else return GridPos{(int)blockIdx.x, 0};
}
template <bool MANY, class J>
__device__ __forceinline__ const J& job_at(const J& one, const J* many, int item) {
  if constexpr (MANY) return many[item]; else return one;
}

// Launchers (defined next to their kernels).  `many` == nullptr launches the
// single job `one`; otherwise `n` jobs read from device memory, with the grid
// sized by the largest job (`maxK`, `maxN`).
// per_track: a batch of FP32 jobs with K <= 64 may run one workgroup per
// track (same results as the tile kernel); any other launch ignores it.
void launch_gram(const GramJob& one, const GramJob* many, int n, int maxK, bool per_track, hipStream_t s);
void launch_gram64(const Gram64Job& one, const Gram64Job* many, int n, int maxK, hipStream_t s);
void launch_inv64(const Inv64Job& one, const Inv64Job* many, int n, int* err, hipStream_t s);
void launch_inv32(const Inv32Job& one, const Inv32Job* many, int n, int* err, hipStream_t s);
// Precoder workgroups of an N-antenna track, and the doubles of its scratch
// wpart (the workgroups' partial sums).
int precoder_blocks(int N);
int precoder_scratch(int N);
// pb: rows of W per workgroup (32 or 64, or 256 with maxK <= 64; any other value takes 64).
// Returns true when the launch also normalised W (every track in one
// workgroup: the scale jobs' P and adv are used); otherwise launch_scale
// over the same scale jobs follows.
bool launch_precoder(const PrecJob& one, const PrecJob* many, const ScaleJob& sone, const ScaleJob* smany, int n,
                     int maxN, int maxK, int pb, hipStream_t s);
// W <- W sqrt(P / ||W||_F^2) from the precoder's partial sums (maxNK: the
// largest N K of the launch).
void launch_scale(const ScaleJob& one, const ScaleJob* many, int n, int maxNK, hipStream_t s);
void launch_arsvd_wb(const ArsvdJob& one, const ArsvdJob* many, int n, int* err, hipStream_t s);
// The same step for one track in two launches (one.spec set): the iterations
// of Alg. 1 that the previous step's count predicts, in parallel, then the
// decision, the SVD and the branch of Alg. 2.  Bit-identical results.
void launch_arsvd_wb_spec(const ArsvdJob& one, int* err, hipStream_t s);
// out = in permuted longest-first (from the tracks' descriptors), for a
// batched arSVD launch over out; n <= RZF_BATCH_MAX.
void launch_arsvd_order(const ArsvdJob* in, ArsvdJob* out, int n, hipStream_t s);
// Large tracks (KS < K <= KM): one workgroup per track, working set in the
// track's global workspace.
void launch_arsvd_big(const ArsvdJob& one, const ArsvdJob* many, int n, int* err, hipStream_t s);
void launch_inv64_big(const Inv64Job& one, const Inv64Job* many, int n, int* err, hipStream_t s);
void launch_inv32_big(const Inv32Job& one, const Inv32Job* many, int n, int* err, hipStream_t s);
size_t sum_rate_scratch_doubles(int K);
// A single track's launch may split the antenna sum over ns workgroups
// (sum_rate_splits; batch launches take ns = 1); its scratch then holds
// sum_rate_split_scratch_doubles().
size_t sum_rate_split_scratch_doubles();
int sum_rate_splits(int K, int N);
void launch_sum_rate(const RateJob& one, const RateJob* many, int n, int maxK, int ns, int* err, hipStream_t s);
// Hybrid front end: every codebook beam's response G (K x nx ny), then the
// beam choice and H_eff.
void launch_beam_resp(const float2* H, int ldh, int K, int nx, int ny, float2* G, hipStream_t s);
void launch_beam_select(const float2* G, int K, int N, int n_rf, int select, int* beams, float2* Heff,
                        int ld_eff, int* err, hipStream_t s);
void launch_debug_sketch(uint64_t seed, uint64_t track, int t, int it, int K, int d, float2* Omega,
                         uint64_t* words, hipStream_t s);
