/*
 * rzf.h -- C ABI of the MI355X (gfx950) WB-arSVD RZF precoding library.
 *
 * Method: Momani, Delamotte, Knopp, "Efficient Precoding for LEO Satellites: A
 * Low-Complexity Matrix Inversion Method via Woodbury Matrix Identity and
 * arSVD" (arXiv 2512.16543).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Complex numbers are interleaved single precision (rzf_c32, the layout of
 *    torch.complex64).
 *  - H is K x N, row-major, leading dimension ldh >= N: row n is the channel
 *    h_n^T of user n (Sec. II, eq. (1)).  K users, N transmit antennas; the
 *    analog combiner of eq. (4) is the identity (fully digital, N_RF = N),
 *    or H is the effective channel H~ F_RF made by rzf_beamspace (N = N_RF).
 *  - W is N x K, row-major, leading dimension ldw >= K: column n is the
 *    precoding vector of user n (eq. (5)).
 *  - Every matrix argument is a DEVICE pointer (e.g. a torch tensor's
 *    data_ptr()).  The caller owns H and W; the library owns the per-track
 *    state, which it places in the arena given to rzf_ctx_create.
 *  - Calls that launch work are asynchronous on the context's HIP stream.
 *    Device-side failures (a non-positive pivot, a non-finite input) are
 *    recorded on the device and returned by the next rzf_sync; info records
 *    requested with a host pointer are filled in by that rzf_sync.
 *  - Nothing throws across this boundary; errors are status codes.  A call
 *    that returns an error has launched nothing.
 *  - Supported sizes: 1 <= K <= RZF_KMAX, 1 <= N <= RZF_NMAX.  Tracks with
 *    K <= 64 run kernels whose working set sits in LDS; larger tracks run
 *    blocked kernels on a per-track workspace in the arena (rzf_track_bytes
 *    includes it).
 */
#ifndef RZF_H
#define RZF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RZF_KMAX 256
#define RZF_NMAX 4096

typedef struct { float re, im; } rzf_c32;

typedef struct rzf_ctx rzf_ctx;       /* device, stream, arena, error word */
typedef struct rzf_track rzf_track;   /* state of one channel track        */

typedef enum {
  RZF_OK = 0,
  RZF_E_INVALID = 1,    /* bad argument: NULL, alpha < 0, tol outside (0,1], ... */
  RZF_E_SHAPE = 2,      /* K, N or a leading dimension out of range            */
  RZF_E_NOMEM = 3,      /* the arena cannot hold the track (admission refused) */
  RZF_E_NOT_HPD = 4,    /* Gram matrix not Hermitian positive definite         */
  RZF_E_NONFINITE = 5,  /* NaN or Inf met in an input or a factorisation       */
  RZF_E_DEVICE = 6      /* a HIP runtime call failed                           */
} rzf_status;

/* Which branch of Alg. 2 an update took. */
typedef enum {
  RZF_PATH_NOOP = 0,          /* Delta A = 0: inverse kept                        */
  RZF_PATH_WB = 1,            /* k_est/K <= switch: Woodbury update, eq. (12)     */
  RZF_PATH_FULL_RANK = 2,     /* k_est/K > switch: direct inversion of A'         */
  RZF_PATH_FULL_SINGULAR = 3, /* capacitance singular (Sec. III): direct inversion */
  RZF_PATH_RESET = 4          /* periodic FP64 re-inversion (drift bound)          */
} rzf_path;

typedef enum { RZF_KINIT_FIXED = 0, RZF_KINIT_WARM = 1 } rzf_kinit_policy;

/* Operand format of the Gram (eqs. (7)-(9)) and precoder (eq. (5)) products;
 * inputs and outputs stay complex64, accumulation FP32.  BF16X3 splits each
 * operand into BF16 hi + lo and forms hi*hi + hi*lo + lo*hi. */
typedef enum { RZF_PREC_FP32 = 0, RZF_PREC_BF16 = 1, RZF_PREC_BF16X3 = 2 } rzf_precision;

/* Parameters of one track; rzf_params_default fills the paper's values. */
typedef struct {
  int k_init;           /* initial rank estimate of Alg. 1 (Table IV: 2);
                           1 <= k_init <= RZF_KMAX                                 */
  int p;                /* oversampling of Alg. 1 (Table IV: 1; workloads use 5);
                           0 <= p <= RZF_KMAX                                      */
  int i_max;            /* Alg. 1 iteration cap; 0 = smallest I with
                           k_init * 2^(I-1) + p >= K                               */
  double switch_ratio;  /* Alg. 2: Woodbury when k_est <= floor(switch_ratio K)
                           (0.5).  The Woodbury workspace holds min(K, max(32,
                           K/2)) ranks: rzf_init and rzf_track_import refuse
                           (RZF_E_INVALID) a ratio whose floor(switch_ratio K)
                           exceeds it, which 0.5 never does                       */
  int reset_period;     /* re-invert A' in FP64 once this many steps have passed
                           since the last FP64 inversion (init or reset), skipping
                           Alg. 1 on that step; 0 = never                         */
  double P;             /* total transmit power, ||W||_F^2 = P (Sec. II)          */
  uint64_t seed;        /* sketch key word 0                                       */
  uint64_t track_id;    /* sketch key word 1                                       */
  int kinit_policy;     /* RZF_KINIT_FIXED: k0 = k_init every step (Alg. 1);
                           RZF_KINIT_WARM: k0 = max(k_init, previous k_est)        */
  int early_fallback;   /* 0: Alg. 1 as printed.  1: an iteration whose d already
                           exceeds the Woodbury limit floor(switch_ratio K) and
                           misses the energy target ends Alg. 1;
                           the step inverts directly (path FULL_RANK, k_est = d)  */
  int precision;        /* rzf_precision of the Gram and precoder products (FP32) */
  int error_feedback;   /* 0: Alg. 2 as printed.  1: the track keeps R, A' minus
                           the Gram matrix whose inverse is stored (what earlier
                           truncated updates left out); Alg. 1 sketches
                           Delta A + R and a Woodbury step leaves R = Delta A + R
                           - U_r Sigma_r V_r^H; any direct inversion clears R    */
} rzf_params;

/* Outcome of one rzf_update. */
typedef struct {
  int r;            /* k_est of Alg. 1 (0 on NOOP and RESET)                     */
  int iters;        /* Alg. 1 iterations run                                      */
  int path;         /* rzf_path                                                   */
  int d;            /* subspace dimension of the last iteration                   */
  double dA_fro2;   /* ||Delta A||_F^2                                            */
  double captured;  /* sum_{j<=r} sigma_j^2 (the retained energy of eq. (14))     */
} rzf_update_info;

const char* rzf_status_string(rzf_status s);

/* Fill *p with k_init=2, p=5, i_max=0, switch_ratio=0.5, reset_period=0,
 * P=1, seed=0, track_id=0, kinit_policy=FIXED, early_fallback=0,
 * precision=FP32, error_feedback=0.
 * RZF_E_INVALID if p is NULL. */
rzf_status rzf_params_default(rzf_params* p);

/* Whether *p is a valid parameter set for a track of K users (the checks
 * rzf_init and rzf_track_import make, without a device): RZF_OK, RZF_E_SHAPE
 * for K outside [1, RZF_KMAX], else RZF_E_INVALID for a NULL p or any field
 * out of its range above (switch_ratio in (0, 1] within the Woodbury
 * workspace, k_init and p up to RZF_KMAX, i_max up to 64, P > 0, policy
 * flags 0 or 1, precision an rzf_precision). */
rzf_status rzf_params_check(const rzf_params* p, int K);

/* Bytes of arena one track of size K x N occupies (0 if out of range). */
size_t rzf_track_bytes(int K, int N);

/* Create a context on HIP device `device`, launching on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  `arena` is device memory of
 * `arena_bytes` bytes owned by the caller and kept alive until
 * rzf_ctx_destroy; track state is carved from it.  If arena is NULL the
 * library allocates arena_bytes itself and frees it in rzf_ctx_destroy. */
rzf_status rzf_ctx_create(int device, void* hip_stream, void* arena, size_t arena_bytes,
                          rzf_ctx** out);
rzf_status rzf_ctx_destroy(rzf_ctx* ctx);

/* Wait for all work on the context's stream, fill pending info records, and
 * return (then clear) the first device-side error recorded since the last
 * rzf_sync.  The synchronous calls (rzf_init, rzf_track_import,
 * rzf_tune_switch) return only errors of their own work and leave an earlier
 * one pending for rzf_sync; rzf_sum_rate with a host sum_rate pointer
 * synchronises like rzf_sync and returns (and clears) it. */
rzf_status rzf_sync(rzf_ctx* ctx);

/* Alg. 2, else-branch: build the state of a new track from its first snapshot.
 * A = H H^H + alpha I_K (eq. (5)) and A^-1 are formed in FP64 and A^-1 is
 * stored in FP32.  alpha >= 0 (eq. (5)).  Synchronous: returns RZF_E_NOT_HPD
 * if A is not positive definite, RZF_E_NONFINITE for non-finite H,
 * RZF_E_NOMEM if the arena is full. */
rzf_status rzf_init(rzf_ctx* ctx, int K, int N, const rzf_c32* H, int ldh, double alpha,
                    const rzf_params* params, rzf_track** out);

/* Alg. 2, if-branch, for the next snapshot H_t of the track:
 *   Delta A from eq. (9); Alg. 1 (arSVD) with energy threshold eta = tol
 *   (eq. (14)); Woodbury update of A^-1 by eq. (12) when k_est <= switch*K,
 *   else direct inversion of A'; then W = H_t^H A'^-1 with ||W||_F^2 = P.
 * tol in (0, 1].
 * A snapshot holding NaN or Inf makes the next rzf_sync return
 * RZF_E_NONFINITE; that step writes a non-finite W (info: path NOOP, r = 0,
 * dA_fro2 NaN) and leaves the track's inverse, previous snapshot, residual
 * and SVD basis as they were, so the next finite snapshot is taken relative
 * to the last finite one.  Only the step counters advance (a reset step that
 * fails this way still restarts the reset count).  The same holds for a reset
 * step whose FP64 re-inversion finds A' not positive definite
 * (RZF_E_NOT_HPD).  The Woodbury capacitance system is solved with its unknown
 * held in FP64 (FP64 Gauss-Jordan, or correction passes whose small product
 * E X is taken in FP32).
 * `info` (host pointer, may be NULL) is filled by the next rzf_sync.
 * For K <= 64 the iterations of Alg. 1 that the track's previous step
 * predicts (its iteration count plus one) are computed at once on otherwise
 * idle CUs before the decision; the results are bit-identical to the same
 * update through rzf_update_batch, which runs them one after another.
 * For K <= 64 an iteration whose sketch spans all K columns (d = K, Q
 * unitary, so the SVD of B gives the truncated SVD of Delta A for any Q)
 * starts its Jacobi SVD from the track's left singular basis of its last
 * such iteration instead of a fresh Q: the same result up to rounding,
 * reached in about half the Jacobi passes.  The basis is part of the track's
 * state (and of its checkpoint). */
rzf_status rzf_update(rzf_track* tr, const rzf_c32* H_t, int ldh, double tol,
                      rzf_c32* W, int ldw, rzf_update_info* info);

/* One entry of a batched update. */
typedef struct {
  rzf_track* track;        /* track to update (each track at most once per batch) */
  const rzf_c32* H;        /* device: next snapshot, K x N, leading dimension ldh  */
  int ldh;
  rzf_c32* W;              /* device: precoder output, N x K, leading dimension ldw */
  int ldw;
  rzf_update_info* info;   /* host: filled by the next rzf_sync, or NULL           */
} rzf_update_item;

#define RZF_BATCH_MAX 2048

/* rzf_update for n independent tracks of this context in one set of launches
 * (one workgroup per track and tile): the data-parallel form of Alg. 2 over
 * many channel tracks.  Same semantics per track as rzf_update, same eta for
 * all.  1 <= n <= RZF_BATCH_MAX; RZF_E_INVALID if a track is NULL, belongs to
 * another context or appears twice. */
rzf_status rzf_update_batch(rzf_ctx* ctx, int n, const rzf_update_item* items, double tol);

/* Conventional RZF (the baseline of Sec. V): W = H^H (H H^H + alpha I)^-1,
 * full FP32 inversion, scaled to ||W||_F^2 = P.  Asynchronous; a
 * non-positive-definite Gram matrix is reported as RZF_E_NOT_HPD by the next
 * rzf_sync. */
rzf_status rzf_full(rzf_ctx* ctx, int K, int N, const rzf_c32* H, int ldh, double alpha,
                    double P, rzf_c32* W, int ldw);

/* One entry of a batched full-inversion RZF. */
typedef struct {
  int K, N;
  const rzf_c32* H;        /* device, K x N, leading dimension ldh */
  int ldh;
  double alpha, P;
  rzf_c32* W;              /* device, N x K, leading dimension ldw */
  int ldw;
  int precision;           /* rzf_precision of the Gram and precoder products */
} rzf_full_item;

/* rzf_full for n independent snapshots in one set of launches (each item with
 * its own operand precision; rzf_full itself is FP32).  Scratch for
 * the Gram matrices comes from the arena (grown on demand, RZF_E_NOMEM if it
 * cannot).  1 <= n <= RZF_BATCH_MAX. */
rzf_status rzf_full_batch(rzf_ctx* ctx, int n, const rzf_full_item* items);

/* rzf_full for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same kernels and result, launched on `hip_stream` (a hipStream_t; NULL =
 * the null stream) of the calling thread's current device, with no context.
 * Its intermediate buffers live in a fixed device array of the library
 * (1,050,624 bytes per device, held until the process ends), so it calls no
 * allocator; the array's device address is resolved on the first call on
 * each device.  Every call on a device shares that array: calls that overlap
 * on one device (two streams, two threads) race and must be serialised by
 * the caller.  Nothing in it needs clearing between calls.
 *  - 1 <= K <= RZF_KMAX, 1 <= N <= RZF_NMAX, ldh >= N, ldw >= K, else
 *    RZF_E_SHAPE (the array is sized for the largest such call);
 *    alpha >= 0 and P > 0 finite, H and W not NULL, else RZF_E_INVALID.
 *  - err: device int, or NULL.  If the Gram matrix is not positive definite
 *    the kernels store 1 there (2 for a non-finite value), when it is still 0;
 *    the caller clears it.  W is then not meaningful.
 * Asynchronous; returns RZF_E_DEVICE if a launch fails. */
rzf_status rzf_full_noalloc(void* hip_stream, int K, int N, const rzf_c32* H, int ldh, double alpha,
                            double P, rzf_c32* W, int ldw, int* err);

/* Sum rate of eq. (15): W is first scaled to ||W||_F^2 = P, then E = H W,
 * SINR_n = |E_nn|^2 / (sum_{i != n} |E_ni|^2 + sigma2), rate_n = log2(1+SINR_n).
 * rates: device pointer to K floats, or NULL.  sum_rate: host pointer; if not
 * NULL the call synchronises the stream and stores the FP64 sum. */
rzf_status rzf_sum_rate(rzf_ctx* ctx, int K, int N, const rzf_c32* H, int ldh,
                        const rzf_c32* W, int ldw, double P, double sigma2,
                        float* rates, double* sum_rate);

/* One entry of a batched sum-rate evaluation. */
typedef struct {
  int K, N;
  const rzf_c32* H;        /* device, K x N, leading dimension ldh */
  int ldh;
  const rzf_c32* W;        /* device, N x K, leading dimension ldw */
  int ldw;
  float* rates;            /* device, K floats, or NULL            */
  double* sum_rate;        /* device, one double, or NULL          */
  double sigma2;           /* this item's noise power; a negative value
                              takes the sigma2 of the call           */
} rzf_rate_item;

/* rzf_sum_rate for n independent (H, W) pairs, results left in device
 * memory (asynchronous).  1 <= n <= RZF_BATCH_MAX. */
rzf_status rzf_sum_rate_batch(rzf_ctx* ctx, int n, const rzf_rate_item* items, double P,
                              double sigma2);

/* ------------------------------------------------------------ launch tuning
 * Launch shapes chosen per track size, e.g. from the table that the
 * library's autotuner writes (paper_2512_16543_amd/tuning.json).  Neither
 * choice changes any result bit: the precoder's partial norms are per 32
 * rows whatever its rows per workgroup, and the sum rate's antenna sum is
 * rounded by fixed partitions however they are spread over workgroups.
 *  - precoder_rows: rows of W per precoder workgroup of a single-track
 *    launch, 32, 64 or 256 (256 only for K <= 64, else 64; 0 = default 64);
 *    batch_precoder_rows: the same for a batched launch of 128 tracks or
 *    more, which takes the entry of its largest (K, N) (smaller batches take
 *    that entry's precoder_rows).
 *  - rate_splits: workgroups over which a single track's sum rate (K <= 64)
 *    spreads its antenna sum, 1..8 (0 = default: one per 64 antennas, at
 *    most 8).  Batched sum rates use one workgroup per track.
 * A launch takes the entry with its exact (K, N), else the nearest one in
 * |log2 K - log2 K'| + |log2 N - log2 N'| (the lower K, then N, on ties),
 * else the defaults. */
typedef struct {
  int K, N;
  int precoder_rows;
  int batch_precoder_rows;
  int rate_splits;
} rzf_tune_entry;

/* Replaces the context's table (n = 0 clears it).  Entries with K or N out
 * of range or a knob outside its values give RZF_E_INVALID (table unchanged).
 * At most 4096 entries. */
rzf_status rzf_tune_table(rzf_ctx* ctx, int n, const rzf_tune_entry* entries);

/* ------------------------------------------------ captured steps (HIP graphs)
 * One step of rzf_update / rzf_update_batch (or of rzf_full / rzf_full_batch),
 * optionally followed by the sum rate of eq. (15) (Sec. VI) of every item,
 * captured once into HIP graphs over fixed buffers and then run by one call
 * per step.  A replay launches the same kernels with the same arguments as
 * the eager call, so its results are bit-identical to it; the branches of
 * Alg. 2 (Woodbury, direct inversion, skip) stay decisions of the kernels.
 * The host keeps only the FP64 re-inversion schedule (Sec. IV): an update
 * graph holds a Woodbury-step graph and, when the tracks have a reset
 * period, a re-inversion graph, and rzf_graph_launch picks one per step.
 *
 * The items' H and W pointers (and rates / sums) are fixed for the graph's
 * life: the caller writes each step's snapshots into the same H buffers,
 * ordered before rzf_graph_launch on the context's stream (or synchronised),
 * and reads W after it.  A graph keeps its job arrays and scratch in the
 * context's arena (RZF_E_NOMEM if it cannot hold them).
 *
 * Update graphs: 1 <= n <= RZF_BATCH_MAX tracks of the context, each at most
 * once; n == 1 captures rzf_update (two-phase arSVD for K <= 64), n > 1
 * rzf_update_batch.  Every track must have the same reset period and the
 * same steps since its last re-inversion (RZF_E_INVALID otherwise, also at a
 * launch after a track was updated outside the graph and fell out of step).
 * A track cannot be destroyed while a graph updates it (RZF_E_INVALID).
 * Per-step info records are not copied out: rzf_track_query and the other
 * track queries read the state after a step.
 *
 * rate: NULL, or the sum rate of each item after its precoder with power P
 * and noise sigma2 into sums[i] (device, n doubles): the arithmetic of
 * rzf_sum_rate for n == 1, of rzf_sum_rate_batch for n > 1. */
typedef struct rzf_graph rzf_graph;
typedef struct {
  double P, sigma2;
  double* sums;            /* device, n doubles */
} rzf_graph_rate;

rzf_status rzf_graph_update(rzf_ctx* ctx, int n, const rzf_update_item* items, double tol,
                            const rzf_graph_rate* rate, rzf_graph** out);
rzf_status rzf_graph_full(rzf_ctx* ctx, int n, const rzf_full_item* items, const rzf_graph_rate* rate,
                          rzf_graph** out);
/* One step: asynchronous on the context's stream, no allocation; device
 * errors are reported by the next rzf_sync as for the eager calls. */
rzf_status rzf_graph_launch(rzf_graph* g);
/* Waits for the context's stream, frees the graph and its arena memory. */
rzf_status rzf_graph_destroy(rzf_graph* g);

/* Hybrid front end of eq. (4): H_eff = H~ F_RF with F_RF made of n_rf beams
 * of the DFT codebook of an nx x ny UPA (N = nx ny, element index m_y nx + m_x;
 * beam b = q nx + p has entries exp(+j 2 pi (p m_x / nx + q m_y / ny)) / sqrt(N),
 * so F_RF has orthonormal columns and ||F_RF F_BB||_F = ||F_BB||_F).
 *  - H: device, K x N, leading dimension ldh >= N (rows h~_n^T of eq. (4)).
 *  - select = 1: choose the beams by the best-power criterion (Sec. II; the
 *    rule it cites is not given, so: user n = 0 .. K-1 in turn takes the
 *    not-yet-taken beam of largest |h~_n^T f_b|^2, lowest index on ties; the
 *    other n_rf - K chains take the untaken beams of largest total power
 *    sum_n |h~_n^T f_b|^2) and write them to beams (device, n_rf ints, users'
 *    beams first).  Needs K <= n_rf <= N.
 *  - select = 0: beams (device, n_rf ints) is an input, e.g. the choice made
 *    on another channel; 1 <= n_rf <= N.  An index outside [0, N) gives a zero
 *    column and RZF_E_INVALID at the next rzf_sync.
 *  - H_eff: device, K x n_rf, leading dimension ld_eff >= n_rf.
 * Asynchronous; uses K N complex values of context scratch (RZF_E_NOMEM if the
 * arena cannot hold them).  1 <= K <= RZF_KMAX, N <= RZF_NMAX. */
rzf_status rzf_beamspace(rzf_ctx* ctx, int K, int nx, int ny, const rzf_c32* H, int ldh, int n_rf,
                         int select, int* beams, rzf_c32* H_eff, int ld_eff);

/* Adaptive Woodbury / direct-inversion breakpoint (the paper's future-work
 * item of choosing Alg. 2's switch from measured costs instead of 0.5).
 * Times, on this context's device, the part of an update that follows the
 * SVD (the rank rule and then Alg. 2's branch, from the kernel's cycle
 * counters) for a K x N track with the given precision: the direct inversion
 * once, and the Woodbury update at several ranks r (synthetic channels whose
 * small change gives Delta A rank r, eta = 1 - 1e-4; the capacitance then
 * takes the X <- M - E X passes, as for a slowly varying channel).  The Woodbury cost is fitted as
 * a + b r; *switch_ratio is the largest r/K (r a whole number) at which it is
 * not above the direct inversion's, 0 if none, capped at the Woodbury
 * workspace (min(K, max(32, K/2)) ranks), so rzf_init accepts it as
 * rzf_params.switch_ratio.  An error of earlier asynchronous work stays
 * pending for the next rzf_sync.
 * Optional outputs: *direct_cycles, *wb_cycles_a and *wb_cycles_b (the fit).
 * Synchronous; uses temporary tracks and 3 K N complex values of the arena.
 * 2 <= K <= RZF_KMAX, K <= N <= RZF_NMAX. */
rzf_status rzf_tune_switch(rzf_ctx* ctx, int K, int N, int precision, double* switch_ratio,
                           double* direct_cycles, double* wb_cycles_a, double* wb_cycles_b);

/* Copy the track's stored inverse (K x K, row-major, ld = K) to device memory
 * Ainv.  Asynchronous. */
rzf_status rzf_get_inverse(rzf_track* tr, rzf_c32* Ainv);

/* Host-side view of the track: sizes, step count, steps since the last FP64
 * inversion, previous k_est.  Synchronises the stream.  NULL outputs are
 * skipped. */
rzf_status rzf_track_query(rzf_track* tr, int* K, int* N, int* t, int* since_reset,
                           int* last_r);

/* Release the track's arena space (after its queued work has finished). */
rzf_status rzf_track_destroy(rzf_track* tr);

/* Checkpoint / resume of a track (the state Alg. 2 carries between
 * snapshots: A^-1 and the previous snapshot, plus the step counters, the
 * previous k_est, the width and iteration count of the last SVD, the
 * error-feedback residual, the full-width SVD basis and the last narrower
 * SVD's basis).  rzf_track_export
 * with buf == NULL stores the blob size in
 * *bytes; otherwise it synchronises the context's stream and writes the blob
 * (host memory, *bytes >= that size, else RZF_E_INVALID with the size in
 * *bytes).  rzf_track_import creates a new track in `ctx` from a blob written
 * by this library version (RZF_E_INVALID for a foreign or truncated blob,
 * RZF_E_NOMEM if the arena is full); its next rzf_update gives the same result
 * as the exported track's would.  Both are synchronous. */
rzf_status rzf_track_export(rzf_track* tr, void* buf, size_t* bytes);
rzf_status rzf_track_import(rzf_ctx* ctx, const void* buf, size_t bytes, rzf_track** out);

/* ------------------------------------------------------ request server
 * Serving loop over resident tracks, with continuous batching: requests
 * (track, H_t, W) are submitted from any thread and go to a lane by their
 * track's kernel family (K <= 64, or K > 64).  Each lane launches on a HIP
 * stream of its own (created by the server, default priority), so the two
 * families' batches overlap on the device.  A dispatcher thread launches a
 * lane's next batch as soon as the lane has one of its max_inflight slots
 * free and max_batch of its requests are pending or the oldest has waited
 * max_wait_us; requests that arrive while earlier batches run join the next
 * batch.  A batch holds at most one request per track, in submission order
 * per track (a track's later requests go to later batches of its lane, which
 * run in order).  A completion thread per lane records each request when its
 * batch has finished, with that batch's own status (RZF_E_NOT_HPD,
 * RZF_E_NONFINITE: a device-side failure of one of the batch's kernels).
 *   RZF_SERVE_UPDATE: each request is one rzf_update of its track (Alg. 2).
 *   RZF_SERVE_FULL:   each request computes the full-inversion RZF of H_t
 *                     with the track's alpha and P (the conventional
 *                     baseline on the same requests); it uses the track's own
 *                     Gram and partial-sum buffers as scratch and leaves its
 *                     state (inverse, previous snapshot) unchanged.  A track
 *                     is served by one server at a time.
 * The server's launches do not follow the context's stream: the caller makes
 * H_t ready before submitting it (e.g. synchronises the stream that wrote
 * it), keeps H_t and W alive until the request completes, and reads W after
 * the completion.  rzf_sync does not wait for served requests; use
 * rzf_server_drain. */
typedef struct rzf_server rzf_server;
typedef enum { RZF_SERVE_UPDATE = 0, RZF_SERVE_FULL = 1 } rzf_serve_mode;
typedef struct {
  int max_batch;        /* requests per launch, 1..RZF_BATCH_MAX (512)            */
  double max_wait_us;   /* longest wait of the oldest request for a fuller batch  */
  double tol;           /* eta of every update (0.999)                            */
  int mode;             /* rzf_serve_mode                                         */
  int max_inflight;     /* batches in flight per lane at once, 1..8 (2)            */
} rzf_server_params;
typedef struct {
  uint64_t tag;         /* as submitted                                           */
  int status;           /* rzf_status of the request's batch                      */
  int pad;
  rzf_update_info info; /* the update's outcome (RZF_SERVE_UPDATE)                */
  double t_submit_us, t_launch_us, t_done_us;   /* server clock                   */
} rzf_completion;
typedef struct {
  rzf_track* track;
  const rzf_c32* H;     /* device, K x N, leading dimension ldh                   */
  int ldh;
  rzf_c32* W;           /* device, N x K, leading dimension ldw                   */
  int ldw;
  uint64_t tag;
  double t_arrival_us;  /* offset from the start of rzf_server_replay, ascending  */
} rzf_serve_request;

rzf_status rzf_server_params_default(rzf_server_params* p);
rzf_status rzf_server_create(rzf_ctx* ctx, const rzf_server_params* p, rzf_server** out);
rzf_status rzf_server_submit(rzf_server* s, rzf_track* tr, const rzf_c32* H_t, int ldh, rzf_c32* W,
                             int ldw, uint64_t tag);
/* Submit n requests, each at its arrival time (blocks until the last one is
 * submitted); completions are collected with rzf_server_poll. */
rzf_status rzf_server_replay(rzf_server* s, int n, const rzf_serve_request* reqs);
/* Move up to `max` finished requests into out[], oldest first. */
rzf_status rzf_server_poll(rzf_server* s, rzf_completion* out, int max, int* n_out);
/* Block until every submitted request has completed. */
rzf_status rzf_server_drain(rzf_server* s);
double rzf_server_now_us(rzf_server* s);
/* Dispatch what is pending, wait for it, stop the threads, free the server. */
rzf_status rzf_server_destroy(rzf_server* s);

/* The Gaussian sketch Omega of Alg. 1 for (seed, track_id, step t, iteration
 * it), K x d, written column-major (entry (i, j) at Omega[j*K + i]) as FP32
 * complex, and the two Philox4x64-10 words behind each entry to words
 * (uint64, 2*K*d, entry-major; may be NULL).  Both device pointers.  For
 * checking the generator against an independent implementation. */
rzf_status rzf_debug_sketch(rzf_ctx* ctx, uint64_t seed, uint64_t track_id, int t, int it,
                            int K, int d, rzf_c32* Omega, uint64_t* words);

/* Work counters of the track's last update, for tuning: [0] Jacobi sweeps,
 * [1] Jacobi rounds, [2] Householder columns, [3..6] shader-clock cycles in
 * sketching, orthogonalisation, SVD and the Woodbury/inversion branch,
 * [7] constant-rate real-time ticks of the whole arSVD kernel.  Synchronises
 * the stream; copies min(n, 8) ints to the host array `out`. */
rzf_status rzf_debug_counters(rzf_track* tr, int* out, int n);

/* The sigma_j^2 of the last update's small SVD (Alg. 1, the SVD of B),
 * descending: copies min(n, d) values to the host array `out` and stores d
 * in *d_out (0 when the update ran no SVD).  Synchronises the stream. */
rzf_status rzf_debug_sigma2(rzf_track* tr, double* out, int n, int* d_out);

/* Per-kernel timing with HIP events on the context's stream (for measuring a
 * kernel's average duration; off by default).  rzf_profile(ctx, 1) clears the
 * counters and starts recording an event pair around every launch;
 * rzf_profile(ctx, 0) stops.  rzf_profile_read synchronises the stream and
 * fills up to `max` entries (kernel name, launches, summed milliseconds),
 * returning the number of entries in *n. */
typedef struct {
  char name[32];
  int count;
  double total_ms;
} rzf_profile_entry;
rzf_status rzf_profile(rzf_ctx* ctx, int enable);
rzf_status rzf_profile_read(rzf_ctx* ctx, rzf_profile_entry* out, int max, int* n);

#ifdef __cplusplus
}
#endif
#endif /* RZF_H */
