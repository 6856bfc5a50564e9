// Alg. 1 (adaptive randomized SVD of Delta A) followed by the branch of
// Alg. 2: Woodbury update of the stored inverse by eq. (12) when
// k_est <= switch * K, direct inversion of A' otherwise.
//
// One workgroup (16 wavefronts) per track; Delta A (K <= 64) and every
// sketch-sized factor live in LDS, so the data-dependent iteration count and
// the branch stay on the device.
//
// Per iteration i, with d = min(k0 + p, K):
//   Omega  K x d   CN(0,1) from the counter-based sketch generator
//   Y      = Delta A Omega                    (matrix cores)
//   Q      = orth(Y): Householder QR, Q formed explicitly
//   Z      = Delta A^H Q                      (matrix cores), so B = Q^H Delta A = Z^H
//   Some r meets the energy target of eq. (14) exactly when the total
//   sum_j sigma_j^2 = ||B||_F^2 = ||Z||_F^2 does, so a failing iteration needs
//   no SVD: k0 <- 2 k0 and the next iteration draws a new sketch.
//   On success: SVD of B by one-sided (Hestenes) Jacobi on the columns of Z:
//   Z J has orthogonal columns z_j = sigma_j v_j (V_hat = Z J Sigma^-1, and
//   U_hat = J).  r is the smallest count whose leading sigma_j^2 reach
//   eta ||Delta A||_F^2.  J itself is never formed: B V_hat = U_hat Sigma
//   gives the retained left vectors as U_r = Q U_hat_r = Q Q^H Delta A Z_r
//   Sigma_r^-2 (three small matrix-core products, only when the step takes
//   the Woodbury branch), so U_r Sigma_r V_r^H = sum_{j<=r} u_j z_j^H.
//   After I_max failing iterations r = d and U_r Sigma_r V_r^H = Q Z^H.
// Full width (d = K): Q is unitary, so B = Q^H Delta A has the singular
// values of Delta A whatever Q is, and U_r = Q Q^H Delta A Z_r Sigma_r^-2 is
// Delta A Z_r Sigma_r^-2 (one product).
//   Such an iteration takes as Q the track's basis from its previous
//   full-width SVD instead of a fresh Householder Q: the normalised columns
//   z_j / sigma_j of that SVD, the right singular vectors V_hat of B,
//   orthonormal to the Jacobi's tolerance.  For a Hermitian Delta A they are
//   its eigenvectors (up to signs and phases), and consecutive Delta A differ
//   little, so about half the passes suffice.
//
// Single-track updates run the kernel in two launches (PH = 1, 2 below): the
// iterations the previous step predicts are computed at once, one workgroup
// each, and the second launch takes the first that decides.  The workgroup
// of the first full-width iteration carries the whole step through when its
// energy test passes (into a staging area), so that when the second launch
// finds the earlier iterations failing it only commits those results.
//
// Woodbury (Sec. III-A, steps 1-5) in the equivalent scaled form with
// U = [u_j] (orthonormal), V~ = [z_j] (V~ = V_r Sigma_r):
//   P  = A^-1 U                (step 1)
//   C  = I_r + V~^H P          (step 2; Sigma_r (Sigma_r^-1 + V_r^H A^-1 U_r))
//   X  = C^-1 (V~^H A^-1)      (step 3, X in FP64: passes X <- M - E X when
//                               C = I + E is close to I, else FP64 Gauss-Jordan
//                               inversion with partial pivoting and the product)
//   A^-1 <- A^-1 - P X         (steps 4-5)
// C is nonsingular exactly when the capacitance of eq. (12) is; a pivot below
// the working precision of C's entries sends the step to direct inversion
// (path FULL_SINGULAR).
#include "dense_device.h"
#include "rzf_internal.h"

namespace {

constexpr int NTH = 1024;
// LDS leading dimension of the K x K buffers: one element of padding puts
// the 16 rows (or columns) read by one matrix-core operand load on distinct
// banks (a stride of 64 complex values maps them all to the same bank)
constexpr int LDK = KS + 1;
constexpr int NWV = NTH / 64;
constexpr int MAX_SWEEPS = 30;
// the next full-width starting basis normalises every column z_j of a
// full-width SVD; one with sigma_j^2 at or below this fraction of the largest
// (numerically zero: the Jacobi sweeps cannot have made it orthogonal to the
// others) leaves the track without a basis, and its next full-width step
// starts from a fresh Householder Q
constexpr double BASIS_MIN_REL = 1e-20;
// two-phase form: longest wait (constant-rate clock ticks, 100 MHz) of the
// full-width iteration's workgroup for the earlier iterations' energy tests
// before it starts its SVD
constexpr long long SPEC_WAIT_TICKS = 10000;
// capacitance C = I + E: with ||E||_F <= NEUMANN_MAX the system C X = M is
// solved by X <- M - E X, the error shrinking by ||E||_F per pass, until it
// is below 2^-NEUMANN_BITS of X (under the FP32 rounding X then takes),
// else by Gauss-Jordan with partial pivoting.  The passes take E X on the
// FP32 matrix cores and keep X in FP64: the product's rounding, about
// 2^-24 ||E|| ||X|| <= 2^-26 ||X|| per pass, stays below X's FP32 rounding.
constexpr double NEUMANN_MAX = 0.25;
// narrowest SVD that starts from the sketch's Q turned towards the last
// narrower SVD (warm_rotate): below it the rotation, one barrier per column,
// costs more than the Jacobi passes it saves (measured at c2: a gain at
// d = 37, a loss of 2-5 % of the step at d = 9 .. 21)
constexpr int WARM_ROTATE_MIN_D = 32;
constexpr int NEUMANN_BITS = 30;

static_assert(2 * WB_RMAX >= KS, "pm and tm together hold a K x K matrix");
constexpr double JACOBI_TOL = 2e-6;
// passes stop after one whose largest |z_p^H z_q| / (||z_p|| ||z_q||) is below
// JACOBI_QSTOP: near convergence a pass squares that measure, so the next
// one would only rotate pairs at about JACOBI_QSTOP^2, the FP32 noise level
constexpr double JACOBI_QSTOP = 1e-3;
// C = I + E is taken as singular when a Gauss-Jordan pivot's modulus is at
// most SING_TOL (1 + ||E||_F): C is formed from FP32 factors, so its entries
// are known only to about r 2^-24 (1 + ||E||) (r <= 32 here), and a smaller
// pivot leaves nothing of X = C^-1 M that those entries determine; the step
// then inverts A' directly (path FULL_SINGULAR)
constexpr double SING_TOL = 0x1.0p-14;
// An iteration whose d leading singular values of Delta A fall short of the
// energy target by at least this relative margin cannot meet it (below): far
// above the FP32 rounding of its ||Z||_F^2 and of those sigma_j^2 (~1e-6).
constexpr double KYFAN_MARGIN = 1e-4;


struct Shared {
  float2 b0[KS * LDK];           // Delta A (row-major, ld LDK); later A^-1 or A'
  float2 b1[KS * LDK];           // column-major K x d (ld LDK): Omega, then Q
  float2 b2[KS * LDK];           // column-major K x d (ld LDK): Y / reflectors, then Z
  float2 pm[WB_RMAX * LDK];      // U (after the SVD), column-major
  float2 tm[WB_RMAX * LDK];      // Q^H Delta A Z_r, then P = A^-1 U, column-major
  double s2[KS];                 // ||z_j||^2
  double is2[KS];                // 1 / sigma_j^2 of the retained columns, by rank
  double2 gjm[2][WB_RMAX];       // Gauss-Jordan: column j of step j (two steps in flight)
  double2 gjinv[2];              // Gauss-Jordan: 1 / pivot
  double red[NWV];
  double totv[SPEC_MAX];         // second phase: ||Z||_F^2 of the speculated iterations
  int order[KS];
  int gjperm[WB_RMAX];           // Gauss-Jordan: pivot row of step j
  int gjpr[2], gjsing[2];
  int nrot, r, found, bad;
  double cap;
  float bsc[KS];                 // 1 / sigma_j of a full-width SVD (its basis columns)
  int bok;                       // that SVD's columns can all be normalised
  // one-launch form, full-width iteration computed first: its sigma_j^2 and
  // order, and the energies of its leading columns (topk[d] = the d largest)
  double s2k[KS];
  int ordk[KS];
  double topk[KS + 1];
};

// Householder vector of column c (rows >= c) of the column-major matrix `a`
// from the column's values x held one row per lane; writes the unit vector
// w (zero above row c) over that column.  H = I - 2 w w^H maps x to
// beta e_c with beta = -e^{i arg x_c} ||x||.  Wave-level, all lanes active.
__device__ void reflector_from(float2 x, float2* a, int c, int K) {
  const int lane = threadIdx.x & 63;
  if (!(lane < K && lane >= c)) x = cz();
  const float s = wave_sumf(cabs2(x));
  const float ax = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x.x), c));
  const float ay = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x.y), c));
  float2 w = cz();
  if (s >= 1e-36f) {
    // x is scaled by 1/||x||; FP32 hardware square root / reciprocals are
    // enough for the working precision of the data (a column whose squared
    // norm is below the FP32 normal range is treated as zero: H = I keeps Q
    // orthonormal)
    const float inx = __builtin_amdgcn_rsqf(s);
    const float bx = ax * inx, by = ay * inx;                // x_c / ||x||
    const float aa = __builtin_amdgcn_sqrtf(bx * bx + by * by);
    float ph_r = 1.f, ph_i = 0.f;
    if (aa > 0.f) { const float ia = __builtin_amdgcn_rcpf(aa); ph_r = bx * ia; ph_i = by * ia; }
    const float iw = __builtin_amdgcn_rsqf(2.f * (1.f + aa));   // 1 / ||x - beta e_c|| (scaled)
    if (lane == c) {
      const float m = (aa + 1.f) * iw;
      w = make_float2(ph_r * m, ph_i * m);
    } else {
      const float m = inx * iw;
      w = make_float2(x.x * m, x.y * m);
    }
  }
  if (lane < K) a[c * LDK + lane] = (lane >= c) ? w : cz();
}

// Tiled complex product over LDS on the matrix cores.  Output M x Nc in
// 16x16 tiles, wave w takes tiles w, w+16, ...; store(i, j, value) is called
// for in-range entries only.
template <class LA, class LB, class ST>
__device__ __forceinline__ void lds_gemm(int M, int Nc, int Kd, const LA& la, const LB& lb, const ST& st) {
  const int wid = threadIdx.x >> 6;
  const int mt = (M + 15) / 16, nt = (Nc + 15) / 16;
  for (int t = wid; t < mt * nt; t += NWV) {
    const int ti = t / nt, tj = t - ti * nt;
    floatx4 dr = zero4(), di = zero4();
    auto a = [&](int rr, int k) { return la(ti * 16 + rr, k); };
    auto b = [&](int k, int cc) { return lb(k, tj * 16 + cc); };
    ctile16(a, b, 0, Kd, dr, di);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = ti * 16 + tile_row(v), j = tj * 16 + tile_col();
      if (i < M && j < Nc) st(i, j, make_float2(dr[v], di[v]));
    }
  }
}

// One-sided Jacobi on the d columns of Z (b2), in blocks of 4 columns that
// wavefronts hold in registers.  A 16-lane row of a wave (row group g) owns
// one column of a pair at a time, 4 rows of the matrix per lane.
// A pass (sweep) over all column pairs:
//   * own pairs: wave w takes blocks 2w and 2w+1 and rotates the 6 pairs
//     inside each block (3 rounds; the columns move through the wave's own
//     LDS columns, no workgroup barrier);
//   * cross pairs: nb - 1 super-rounds pair the blocks round-robin; wave w
//     loads its blocks A and B, row group g keeps column g of A and meets
//     the 4 columns of B in turn, which move one row group up after every
//     round by a lane permute; then both blocks go back to LDS (one barrier
//     per super-round).
// Pairs rotate when |z_p^H z_q| > JACOBI_TOL ||z_p|| ||z_q||; passes stop
// after one in which no pair had |z_p^H z_q| > JACOBI_QSTOP ||z_p|| ||z_q||
// (`moved`).  Columns d .. 4 nb - 1 are zero and never rotate.
// The norms and z_p^H z_q are summed in FP32 (rounding error a few 2^-24
// ||z_p|| ||z_q||, well under the threshold); the row sums are bit-identical
// in the 16 lanes, so they all take the same decision and the same rotation.
// With FRESH the squared norms are summed from the columns and returned in
// alt, bet; otherwise alt, bet carry them in from the previous rotation and
// leave updated by the rotation's exact effect on them: ||z_p||^2 - t |gamma|
// and ||z_q||^2 + t |gamma| (the pair's energy moves by t |gamma|).
template <bool FRESH>
__device__ __forceinline__ void jacobi_rotate(float2 zp[4], float2 zq[4], bool act, bool& moved, float& alt,
                                              float& bet) {
  float al = 0.f, be = 0.f, grf32 = 0.f, gif32 = 0.f;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    if constexpr (FRESH) {
      al += cabs2(zp[m]);
      be += cabs2(zq[m]);
    }
    grf32 = fmaf(zp[m].x, zq[m].x, fmaf(zp[m].y, zq[m].y, grf32));
    gif32 = fmaf(zp[m].x, zq[m].y, fmaf(-zp[m].y, zq[m].x, gif32));
  }
  if constexpr (FRESH) {
    al = row16_sumf(al);
    be = row16_sumf(be);
  } else {
    al = alt;
    be = bet;
  }
  const float gr = row16_sumf(grf32);
  const float gi = row16_sumf(gif32);
  const float mx = fmaxf(al, be);
  bool rot = act && mx > 0.f;
  float c = 1.f, s = 0.f;
  float2 e = make_float2(1.f, 0.f);
  if (rot) {
    // rotation parameters with hardware rsq/rcp on sums scaled by
    // 1/max(alpha, beta) so nothing underflows; a pair whose scaled
    // |gamma|^2 is below the FP32 normal range is already orthogonal to
    // working precision
    const float sc = __builtin_amdgcn_rcpf(mx);
    const float alf = al * sc, bef = be * sc;
    const float grf = gr * sc, gif = gi * sc;
    const float gg = grf * grf + gif * gif;
    rot = gg >= 1e-36f && gg > (float)(JACOBI_TOL * JACOBI_TOL) * alf * bef;
    moved = moved || gg > (float)(JACOBI_QSTOP * JACOBI_QSTOP) * alf * bef;
    const float ig = __builtin_amdgcn_rsqf(fmaxf(gg, 1e-36f));   // 1/|gamma|
    const float zeta = (bef - alf) * 0.5f * ig;
    const float az = fabsf(zeta);
    const float tmag = (az > 1e18f) ? 0.5f * __builtin_amdgcn_rcpf(az)
                                    : __builtin_amdgcn_rcpf(az + __builtin_amdgcn_sqrtf(1.f + az * az));
    const float tt = zeta >= 0.f ? tmag : -tmag;
    c = __builtin_amdgcn_rsqf(1.f + tt * tt);
    s = c * tt;
    e = make_float2(grf * ig, -gif * ig);   // conj(gamma)/|gamma|
    if (rot) {
      const float tg = tt * gg * ig * mx;   // t |gamma|
      al = fmaxf(al - tg, 0.f);
      be = be + tg;
    }
  }
  alt = al;
  bet = be;
  if (rot) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const float2 zq2 = cmul(e, zq[m]);
      const float2 np = csub(cscale(zp[m], c), cscale(zq2, s));
      zq[m] = cadd(cscale(zp[m], s), cscale(zq2, c));
      zp[m] = np;
    }
  }
}

__device__ void jacobi_svd(Shared& sm, int K, int d, int* sweeps_out, int* rounds_out) {
  float2* b2 = sm.b2;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int nb = ((d + 3) / 4 + 1) & ~1;   // blocks of 4 columns, an even number (<= 16)
  const int nw = nb / 2;                   // waves holding a block pair
  for (int e = threadIdx.x; e < (4 * nb - d) * LDK; e += NTH) b2[d * LDK + e] = cz();
  int sweeps = 0, rounds = 0;
  for (int sweep = 0; sweep < MAX_SWEEPS; ++sweep) {
    if (threadIdx.x == 0) sm.nrot = 0;
    __syncthreads();
    ++sweeps;
    bool moved = false;
    // own pairs of blocks 2w (row groups 0, 1) and 2w + 1 (row groups 2, 3)
    if (wid < nw) {
      const int c0 = 4 * (2 * wid + (g >> 1)), m = g & 1;
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        int p, q;
        rr_pair(t, m, 4, &p, &q);
        float2* zpc = b2 + (c0 + p) * LDK + li;
        float2* zqc = b2 + (c0 + q) * LDK + li;
        float2 zp[4], zq[4];
#pragma unroll
        for (int mm = 0; mm < 4; ++mm) {
          zp[mm] = zpc[16 * mm];
          zq[mm] = zqc[16 * mm];
        }
        float alt, bet;
        jacobi_rotate<true>(zp, zq, true, moved, alt, bet);
#pragma unroll
        for (int mm = 0; mm < 4; ++mm) {
          zpc[16 * mm] = zp[mm];
          zqc[16 * mm] = zq[mm];
        }
        wave_sync();
      }
    }
    rounds += 3;
    __syncthreads();
    // cross pairs, one super-round per round-robin pairing of the blocks
    for (int sr = 0; sr < nb - 1; ++sr) {
      if (wid < nw) {
        int A, B;
        rr_pair(sr, wid, nb, &A, &B);
        float2* zac = b2 + (4 * A + g) * LDK + li;
        float2* zbc = b2 + (4 * B + g) * LDK + li;
        float2 za[4], zb[4];
#pragma unroll
        for (int mm = 0; mm < 4; ++mm) {
          za[mm] = zac[16 * mm];
          zb[mm] = zbc[16 * mm];
        }
        const int up = (lane + 16) & 63;
        // the norms are summed at the first step of the super-round and
        // carried through the next three (B's move up with its columns)
        float alt, bet;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          // column 4A + g with column 4B + (g + t) % 4
          if (t == 0) jacobi_rotate<true>(za, zb, true, moved, alt, bet);
          else jacobi_rotate<false>(za, zb, true, moved, alt, bet);
#pragma unroll
          for (int mm = 0; mm < 4; ++mm) zb[mm] = make_float2(__shfl(zb[mm].x, up), __shfl(zb[mm].y, up));
          bet = __shfl(bet, up);
        }
#pragma unroll
        for (int mm = 0; mm < 4; ++mm) {
          zac[16 * mm] = za[mm];
          zbc[16 * mm] = zb[mm];
        }
      }
      rounds += 4;
      __syncthreads();
    }
    if (moved && li == 0) sm.nrot = 1;
    __syncthreads();
    const bool done = (sm.nrot == 0);
    __syncthreads();
    if (done) break;
  }
  *sweeps_out += sweeps;
  *rounds_out += rounds;
}

// Rotation within the sketch's subspace before a Jacobi SVD below full width
// (d < K).  Q (b1, K x d) is one orthonormal basis of range(Delta A Omega);
// for a d x d unitary W, QW spans the same subspace and Z W = Delta A^H (QW)
// has the same singular values, so the rank, U_r (formed through Q Q^H), the
// captured energy and the update are those of Q (up to rounding).  W is the
// unitary factor of the Householder QR of Q^H X, X the d leading columns of
// the track's last narrower SVD basis (Xd: its normalised columns by
// descending sigma), so that QW spans, column by column, the sketch's
// subspace lined up with the previous step's singular directions, and the
// Jacobi passes on Z W start close to convergence.  Householder's W is
// unitary to rounding whatever the conditioning of Q^H X.  The factorisation
// runs in pm/tm (d x d, column-major, ld LDK); W is formed in Xd, which the
// basis of this step's SVD replaces afterwards.
__device__ void warm_rotate(Shared& sm, float2* Xd, int K, int d) {
  float2* const b1 = sm.b1;
  float2* const b2 = sm.b2;
  float2* const g = sm.pm;   // pm and tm are contiguous: d <= KS columns of LDK
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  // G = Q^H X
  lds_gemm(d, d, K,
           [&](int i, int k) { return (i < d && k < K) ? cconj(b1[i * LDK + k]) : cz(); },
           [&](int k, int c) { return (k < K && c < d) ? Xd[(size_t)c * K + k] : cz(); },
           [&](int i, int c, float2 v) { g[c * LDK + i] = v; });
  __syncthreads();
  // Householder QR of G, as for the sketch (reflector j over column j; one
  // barrier per column), rows >= d masked
  if (wid == 0) reflector_from((lane < d) ? g[lane] : cz(), g, 0, d);
  for (int j = 0; j < d; ++j) {
    __syncthreads();
    const float2 w = (lane < d) ? g[j * LDK + lane] : cz();
    float2 y[KS / NWV];
    float dr[KS / NWV], di[KS / NWV];
#pragma unroll
    for (int q = 0; q < KS / NWV; ++q) {
      const int c = j + 1 + wid + NWV * q;
      y[q] = (c < d && lane < d) ? g[c * LDK + lane] : cz();
      dr[q] = w.x * y[q].x + w.y * y[q].y;     // conj(w) y
      di[q] = w.x * y[q].y - w.y * y[q].x;
    }
#pragma unroll
    for (int q = 0; q < KS / NWV; ++q) {
      const int c = j + 1 + wid + NWV * q;
      if (c >= d) break;
      const float fr = 2.f * wave_sumf(dr[q]), fi = 2.f * wave_sumf(di[q]);
      y[q].x -= w.x * fr - w.y * fi;
      y[q].y -= w.x * fi + w.y * fr;
      if (lane < d) g[c * LDK + lane] = y[q];
    }
    if (wid == 0 && j + 1 < d) reflector_from(y[0], g, j + 1, d);
  }
  __syncthreads();
  // W = H_0 ... H_{d-1} (square): column c is H_0 ... H_c e_c, formed by its
  // wave with no barrier, into Xd (ld K)
  {
    float2 y[KS / NWV];
    int cmax = -1;
#pragma unroll
    for (int q = 0; q < KS / NWV; ++q) {
      const int c = wid + NWV * q;
      y[q] = (lane == c) ? make_float2(1.f, 0.f) : cz();
      if (c < d) cmax = c;
    }
    for (int j = cmax; j >= 0; --j) {
      const float2 w = (lane < d) ? g[j * LDK + lane] : cz();
#pragma unroll
      for (int q = 0; q < KS / NWV; ++q) {
        const int c = wid + NWV * q;
        if (c >= d || c < j) continue;
        float dr = w.x * y[q].x + w.y * y[q].y;
        float di = w.x * y[q].y - w.y * y[q].x;
        dr = wave_sumf(dr);
        di = wave_sumf(di);
        const float fr = 2.f * dr, fi = 2.f * di;
        y[q].x -= w.x * fr - w.y * fi;
        y[q].y -= w.x * fi + w.y * fr;
      }
    }
#pragma unroll
    for (int q = 0; q < KS / NWV; ++q) {
      const int c = wid + NWV * q;
      if (c < d && lane < d) Xd[(size_t)c * K + lane] = y[q];
    }
  }
  __syncthreads();
  // Z <- Z W, each wave's tile held in registers until every wave has read Z
  const int kt = (K + 15) / 16, dt = (d + 15) / 16;
  floatx4 dr = zero4(), di = zero4();
  const int ti = wid / dt, tj = wid - (wid / dt) * dt;
  const bool mine = wid < kt * dt;
  if (mine)
    ctile16([&](int rr, int k) {
              const int i = ti * 16 + rr;
              return (i < K && k < d) ? b2[k * LDK + i] : cz();
            },
            [&](int k, int cc) {
              const int c = tj * 16 + cc;
              return (k < d && c < d) ? Xd[(size_t)c * K + k] : cz();
            },
            0, (d + 3) & ~3, dr, di);
  __syncthreads();
  if (mine) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = ti * 16 + tile_row(v), c = tj * 16 + tile_col();
      if (i < K && c < d) b2[c * LDK + i] = make_float2(dr[v], di[v]);
    }
  }
  __syncthreads();
}

// Squared norms of the d columns of Z (b2) into sm.s2, one 16-lane row per column.
__device__ void column_norms(Shared& sm, int K, int d) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int li = lane & 15, slot = wid * 4 + (lane >> 4);
  double v = 0.0;
  if (slot < d) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int i = li + 16 * m;
      if (i < K) v += (double)cabs2(sm.b2[slot * LDK + i]);
    }
  }
  v = row16_sum(v);
  if (slot < d && li == 0) sm.s2[slot] = v;
}

// After the SVD: sigma_j^2 = ||z_j||^2, their descending order (ties by
// index) in sm.order, the smallest r whose leading sigma_j^2 reach Et (all d
// if rounding keeps the sum just below it) and the retained energy.
__device__ void pick_rank(Shared& sm, int K, int d, double Et, int* r_out, double* cap_out,
                          double* td_sig2) {
  const int tid = threadIdx.x, lane = tid & 63;
  column_norms(sm, K, d);
  __syncthreads();
  if (tid < 64) {
    // wave 0, lane j holds sigma_j^2; its rank counts the larger values
    // (and the equal ones of lower index)
    // (the other values read from LDS, every lane the same address: the
    // loads issue back to back, unlike a chain of lane reads)
    const double v = lane < d ? sm.s2[lane] : -1.0;
    int rank = 0;
#pragma unroll 8
    for (int k = 0; k < d; ++k) {
      const double w = sm.s2[k];
      rank += (w > v) || (w == v && k < lane);
    }
    if (lane < d) sm.order[rank] = lane;
    wave_sync();
    const double sv = lane < d ? sm.s2[sm.order[lane]] : 0.0;   // descending
    // running sum in descending order, one term at a time
    double cs = 0.0;
    int rr = d;
    for (int m = 0; m < d; ++m) {
      cs += readlane_d(sv, m);
      if (cs >= Et) { rr = m + 1; break; }
    }
    if (lane == 0) {
      sm.r = rr;
      sm.cap = cs;
    }
    if (lane < d) td_sig2[lane] = sv;
  }
  __syncthreads();
  *r_out = sm.r;
  *cap_out = sm.cap;
  __syncthreads();
}

// In-place Gauss-Jordan inversion with partial pivoting of the r x r FP64
// capacitance C held in columns 0 .. r - 1 of aug (row-major, ld ldg),
// r <= WB_RMAX.  Rows are never exchanged: step j takes as pivot the not yet
// used row p_j with the largest |C[i, j]| (the lowest such row).  Run on the
// row-permuted matrix, the in-place steps leave S with S[p_j, c] =
// C^-1[j, p_c]; S is written back over C and p_j to sm.gjperm[j].
// Half-wave h = 2 wid + (lane >> 5) holds column h in registers, row
// lane & 31.  Half-wave j + 1 owns the next pivot column: after the barrier
// of step j it updates that column first, at raised wave priority, and
// publishes the next pivot (row, 1 / pivot and the column) in the other of
// two LDS slots, so a step costs one workgroup barrier.  Returns false
// (every thread alike) if a pivot's squared modulus is not above tol2 or is
// not finite.
__device__ bool gj_invert_small(Shared& sm, double2* aug, int r, int ldg, double tol2) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int row = lane & 31, hw = 2 * wid + (lane >> 5), base = lane & 32;
  double2 x = (hw < r && row < r) ? aug[row * ldg + hw] : dz();
  bool used = false;
  // pivot of column j (half-wave j, the only active half of its wave here),
  // published in slot j & 1
  auto publish = [&](int j) {
    const int b = j & 1;
    const int hb = __builtin_amdgcn_readfirstlane(base);
    const double mag = (!used && row < r) ? dabs2(x) : -1.0;
    double mx = mag;   // maximum over the 16-lane rows, then over the two rows
    mx = fmax(mx, dpp_d<DPP_QUAD_1032>(mx));
    mx = fmax(mx, dpp_d<DPP_QUAD_2301>(mx));
    mx = fmax(mx, dpp_d<DPP_ROW_HALF_MIRROR>(mx));
    mx = fmax(mx, dpp_d<DPP_ROW_MIRROR>(mx));
    mx = fmax(readlane_d(mx, hb), readlane_d(mx, hb + 16));
    const unsigned int hit = (unsigned int)(__ballot(mag == mx) >> hb);
    const int pr = __ffs((int)hit) - 1;   // -1: NaN column, no maximum
    const int pu = pr < 0 ? 0 : pr;
    const double2 p = lane_read(x, hb + pu);
    if (row < r) sm.gjm[b][row] = x;
    if (row == 0) {
      const bool sing = pr < 0 || !(mx > tol2) || !isfinite(mx);
      // 1 / |p|^2: hardware reciprocal and one Newton step
      const double a2 = sing ? 1.0 : dabs2(p);
      double id = __builtin_amdgcn_rcp(a2);
      id = fma(id, fma(-a2, id, 1.0), id);
      sm.gjinv[b] = make_double2(p.x * id, -p.y * id);
      sm.gjpr[b] = pu;
      sm.gjsing[b] = sing;
      sm.gjperm[j] = pu;
    }
  };
  if (hw == 0) publish(0);
  bool sing = false;
  for (int j = 0; j < r; ++j) {
    __syncthreads();
    const int b = j & 1;
    // the published step (a singular pivot only spoils values that are then
    // discarded, so it is checked once, after the loop)
    sing = sing || sm.gjsing[b] != 0;
    const int pr = __builtin_amdgcn_readfirstlane(sm.gjpr[b]);
    const double2 inv = sm.gjinv[b];
    const double2 m = (row < r) ? sm.gjm[b][row] : dz();   // column j before this step
    used = used || row == pr;
    const bool owner_wave = wid == ((j + 1) >> 1) && j + 1 < r;
    if (owner_wave) __builtin_amdgcn_s_setprio(2);
    if (hw == j) {
      // the pivot column becomes column j of the inverse: 1 / pivot at the
      // pivot row, -C[i, j] / pivot elsewhere
      const double2 v = dmul(m, inv);
      x = (row == pr) ? inv : make_double2(-v.x, -v.y);
    } else if (hw < r) {
      // this column's pivot-row entry, read from this half-wave's lanes
      const double2 lo = lane_read(x, pr), hi = lane_read(x, 32 + pr);
      const double2 u = dmul(base ? hi : lo, inv);
      x = (row == pr) ? u : dsub(x, dmul(m, u));
    }
    if (hw == j + 1 && j + 1 < r) publish(j + 1);
    if (owner_wave) __builtin_amdgcn_s_setprio(0);
  }
  const bool ok = !sing;
  if (ok && hw < r && row < r) aug[row * ldg + hw] = x;
  __syncthreads();
  return ok;
}

// PH = 0: the whole step (single track or batch).  Two-phase single-track
// form: PH = 1, one workgroup per speculated iteration (blockIdx.x + 1) up to
// the energy test, its Q, Z and ||Z||_F^2 written to jb.spec (the first
// full-width iteration, when it passes, goes on through the SVD and the
// branch into the staging area instead); PH = 2, the decision over those
// iterations in order (continuing one by one if none decides), then the SVD
// and the branch, or the commit of the staged results, exactly as PH = 0
// computes them.
template <bool MANY, int PH>
__global__ __launch_bounds__(NTH) void k_arsvd_wb(ArsvdJob one, const ArsvdJob* many, int* err) {
  __shared__ Shared sm;
  const ArsvdJob& jb = job_of<MANY>(one, many);
  GTrackDesc* __restrict__ td = (GTrackDesc*)jb.td;
  TrackDesc* const tdg = (TrackDesc*)td;    // the same, for whole-struct copies
  const int t = td->t_dev + 1, i_max = jb.i_max;
  const unsigned long long seq = td->seq_dev;
  const double eta = jb.eta;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int K = td->K;
  float2* b0 = sm.b0;
  float2* b1 = sm.b1;
  float2* b2 = sm.b2;

  // Z / reflector buffer cleared: its rows K..KS-1 stay zero for the whole
  // launch (the products and reflectors only write rows < K), which the
  // Jacobi sweeps rely on
  for (int e = tid; e < KS * LDK; e += NTH) b2[e] = cz();
  // Delta A -> LDS, returning E = ||Delta A||_F^2 in FP64 (every thread)
  const bool fb = td->error_feedback != 0;   // sketch Delta A + R
  auto load_dA = [&]() -> double {
    double part = 0.0;
    for (int e = tid; e < K * K; e += NTH) {
      const int i = e / K, j = e - i * K;
      float2 v = td->dA[e];
      if (fb) v = cadd(v, td->Rfb[e]);
      b0[i * LDK + j] = v;
      part += (double)v.x * v.x + (double)v.y * v.y;
    }
    return block_sum(part, sm.red);
  };
  // the second phase takes E from the first (the same sum of the same
  // values) and loads Delta A only when it goes on past a commit
  double* const spec_d = PH == 0 ? nullptr : reinterpret_cast<double*>(jb.spec + (size_t)2 * KS * KS * SPEC_MAX);
  // two-phase form: tags[i] = this launch's number once iteration i + 1 has
  // posted ||Z||_F^2, with bit 63 set when it meets the energy target (the
  // numbers stay below 2^63); tags[SPEC_MAX] once the first phase has written the
  // whole step to the track
  unsigned long long* const tags = PH == 0 ? nullptr : reinterpret_cast<unsigned long long*>(spec_d + SPEC_MAX + 1);
  bool dA_in = PH != 2;
  double E;
  if constexpr (PH == 2) {
    E = spec_d[SPEC_MAX];
    // the first phase may have completed the step already
    if (tid == 0) sm.found = tags[SPEC_MAX] == seq;
    __syncthreads();
    if (sm.found) return;
  } else {
    E = load_dA();
    if (PH == 1 && blockIdx.x == 0 && tid == 0) spec_d[SPEC_MAX] = E;
  }
  // a non-finite snapshot leaves the track's state as it was (the precoder
  // then keeps H_prev too)
  if (PH != 1 && tid == 0) td->hold = isfinite(E) ? 0 : 1;
  if (!isfinite(E) || E == 0.0) {
    if (PH == 1) return;                     // the second phase records the step
    if (fb && E == 0.0)                      // nothing to apply: the residual is zero
      for (int e = tid; e < K * K; e += NTH) td->Rfb[e] = cz();
    if (tid == 0) {
      if (!isfinite(E)) atomicCAS(err, 0, DEV_ERR_NONFINITE);
      td->info.r = 0; td->info.iters = 0; td->info.path = RZF_PATH_NOOP; td->info.d = 0;
      td->info.dA_fro2 = E; td->info.captured = 0.0;
      if (jb.out) *jb.out = tdg->info;
      if (E == 0.0) td->last_r = 0;
      td->dbg[0] = 0; td->dbg[1] = 0; td->dbg[2] = 0;
      td->nsig = 0;
    }
    return;
  }
  const double Et = eta * E;
  long long t_sk = 0, t_qr = 0, t_jac = 0, t_wb = 0;
  const long long c_begin = clock64(), r_begin = wall_clock64();
  long long c_mark = c_begin;
  int k0 = td->k_init;
  if (td->kinit_policy == RZF_KINIT_WARM && td->last_r > k0) k0 = td->last_r;
  const int p = td->p;
  const uint64_t seed = td->seed, trk = td->track_id;

  int d = 0, iters = 0, r = 0, sweeps = 0, rounds = 0, qrcols = 0;
  double captured = 0.0;
  bool found = false, rotated = false;
  // iterations computed ahead in the two-phase form: the last count plus one
  // (a track's first step, with no count yet, computes every iteration ahead)
  const int n_spec = PH == 0 ? 0
                             : min(min(i_max, SPEC_MAX), td->spec_hint > 0 ? td->spec_hint + 1 : i_max);
  // a full-width sketch (d = K) has a unitary Q, and the SVD of B = Q^H Delta A
  // then yields the truncated SVD of Delta A whatever Q is: such an iteration
  // starts from the track's basis of its last full-width SVD when it has one
  const bool warm_ok = td->warm != 0;
  // columns of the last narrower SVD's basis (Xd) that a Jacobi below full
  // width may start from (warm_rotate)
  const int dwarm = td->Xd != nullptr ? td->dwarm : 0;
  bool basis = false;   // the SVD ran at d = K
  // the first iteration whose sketch spans all K columns (0: none that the
  // step can reach: past i_max, or after the early-fallback policy's end)
  int kfull = 0;
  {
    int kk = k0;
    for (int it = 1; it <= i_max; ++it) {
      const int dd = min(kk + p, K);
      if (dd == K) { kfull = it; break; }
      if (td->early_fallback && dd > td->wb_limit) break;
      kk = min(2 * kk, K);
    }
  }
  // two-phase form: the first phase's workgroup of that iteration carries the
  // step through (its results to the staging area) when the test passes there
  const bool stage_ok = PH != 0 && kfull > 0 && kfull <= n_spec && jb.stage != nullptr;
  char* const stage = stage_ok ? jb.stage : nullptr;
  SpecStage* const st_h = reinterpret_cast<SpecStage*>(stage);
  double* const st_sig2 = reinterpret_cast<double*>(stage + sizeof(SpecStage));
  float2* const st_Ainv = reinterpret_cast<float2*>(stage + sizeof(SpecStage) + sizeof(double) * KS);
  float2* const st_R = st_Ainv + K * K;
  float2* const st_Xw = st_R + K * K;
  // where the step's results go: the track, or the staging area
  float2* o_Ainv = td->Ainv;
  float2* o_R = td->Rfb;
  float2* o_Xw = td->Xw;
  double* o_sig2 = tdg->sig2;
  bool staged = false;
  // one iteration of Alg. 1 up to the energy test: Omega, Y, Q (b1), Z (b2),
  // returning ||Z||_F^2
  auto sketch_iteration = [&](int itn, int d) -> double {
    if (d == K && warm_ok) {
    // the track's basis -> b1
    for (int e = tid; e < K * K; e += NTH) {
      const int j = e / K, i = e - j * K;
      b1[j * LDK + i] = td->Xw[e];
    }
    __syncthreads();
    t_sk += clock64() - c_mark; c_mark = clock64();
    } else {
    // Omega -> b1 (column-major), two rows per counter block
    const int Kh = (K + 1) >> 1;
    for (int e = tid; e < Kh * d; e += NTH) {
      const int j = e / Kh, h = e - j * Kh;
      float2 ev, od;
      sketch_pair(seed, trk, t, itn, h, j, &ev, &od);
      b1[j * LDK + 2 * h] = ev;
      if (2 * h + 1 < K) b1[j * LDK + 2 * h + 1] = od;
    }
    __syncthreads();
    // Y = Delta A Omega -> b2
    lds_gemm(K, d, K,
             [&](int i, int k) { return (i < K && k < K) ? b0[i * LDK + k] : cz(); },
             [&](int k, int j) { return (k < K && j < d) ? b1[j * LDK + k] : cz(); },
             [&](int i, int j, float2 v) { b2[j * LDK + i] = v; });
    __syncthreads();
    t_sk += clock64() - c_mark; c_mark = clock64();
    // Householder QR of Y (b2): reflector j lands in column j of b2.  Wave 0
    // updates column j+1 and immediately forms its reflector (one barrier per
    // column); the other waves update the remaining columns.
    // Each wave updates its (at most 4) columns c with H_j = I - 2 w w^H,
    // y <- y - 2 w (w^H y), all of them together so that their reductions
    // overlap.  Rows K..KS-1 of w and y are zero and stay zero.
    if (wid == 0) reflector_from((lane < K) ? b2[lane] : cz(), b2, 0, K);
    for (int j = 0; j < d; ++j) {
      __syncthreads();
      const float2 w = b2[j * LDK + lane];
      float2 y[KS / NWV];
      float dr[KS / NWV], di[KS / NWV];
#pragma unroll
      for (int q = 0; q < KS / NWV; ++q) {
        const int c = j + 1 + wid + NWV * q;
        y[q] = c < d ? b2[c * LDK + lane] : cz();
        dr[q] = w.x * y[q].x + w.y * y[q].y;     // conj(w) y
        di[q] = w.x * y[q].y - w.y * y[q].x;
      }
#pragma unroll
      for (int q = 0; q < KS / NWV; ++q) {
        const int c = j + 1 + wid + NWV * q;
        if (c >= d) break;
        const float fr = 2.f * wave_sumf(dr[q]), fi = 2.f * wave_sumf(di[q]);
        y[q].x -= w.x * fr - w.y * fi;
        y[q].y -= w.x * fi + w.y * fr;
        b2[c * LDK + lane] = y[q];
      }
      if (wid == 0 && j + 1 < d) reflector_from(y[0], b2, j + 1, K);
    }
    qrcols += d;
    // Q = H_0 ... H_{d-1} [I_d; 0] -> b1.  Column c is H_0 ... H_c e_c (H_j
    // leaves e_c alone for j > c: w_j is zero above row j), so every wave
    // forms its own columns c = wid, wid + 16, ... with no barrier, the
    // reflectors applied in the same order as to the whole of Q.
    {
      float2 y[KS / NWV];
      int cmax = -1;
#pragma unroll
      for (int q = 0; q < KS / NWV; ++q) {
        const int c = wid + NWV * q;
        y[q] = (lane == c) ? make_float2(1.f, 0.f) : cz();
        if (c < d) cmax = c;
      }
      for (int j = cmax; j >= 0; --j) {
        const float2 w = b2[j * LDK + lane];
#pragma unroll
        for (int q = 0; q < KS / NWV; ++q) {
          const int c = wid + NWV * q;
          if (c >= d || c < j) continue;          // no column, or H_j leaves it alone
          float dr = w.x * y[q].x + w.y * y[q].y;  // conj(w) y
          float di = w.x * y[q].y - w.y * y[q].x;
          dr = wave_sumf(dr);
          di = wave_sumf(di);
          const float fr = 2.f * dr, fi = 2.f * di;
          y[q].x -= w.x * fr - w.y * fi;
          y[q].y -= w.x * fi + w.y * fr;
        }
      }
#pragma unroll
      for (int q = 0; q < KS / NWV; ++q)
        if (wid + NWV * q < d) b1[(wid + NWV * q) * LDK + lane] = y[q];
    }
    __syncthreads();
    }
    // Z = Delta A^H Q = B^H -> b2 (Delta A is Hermitian unless error feedback
    // has added its residual, so the conjugate transpose is taken explicitly)
    lds_gemm(K, d, K,
             [&](int i, int k) { return (i < K && k < K) ? cconj(b0[k * LDK + i]) : cz(); },
             [&](int k, int j) { return (k < K && j < d) ? b1[j * LDK + k] : cz(); },
             [&](int i, int j, float2 v) { b2[j * LDK + i] = v; });
    __syncthreads();
    // ||B||_F^2 = ||Z||_F^2: does any r reach the target?
    double zp = 0.0;
    for (int e = tid; e < K * d; e += NTH) {
      const int j = e / K, i = e - j * K;
      zp += (double)cabs2(b2[j * LDK + i]);
    }
    const double tot = block_sum(zp, sm.red);
    t_qr += clock64() - c_mark; c_mark = clock64();
    return tot;
  };
  // the first phase carried the full-width iteration `it` through: copy its
  // results to the track
  auto commit_stage = [&](int it) {
    // every load is issued before the first store (the compiler cannot tell
    // the staging area from the track's buffers), so the copy waits on one
    // round trip to memory rather than one per element
    constexpr int PER = (KS * KS + NTH - 1) / NTH;
    float2* const Ai = td->Ainv;
    float2* const Xw = td->Xw;
    float2* const Rf = td->Rfb;
    float2 va[PER], vx[PER], vr[PER];
    double vs = 0.0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + q * NTH;
      if (e < K * K) {
        va[q] = st_Ainv[e];
        vx[q] = st_Xw[e];
        if (fb) vr[q] = st_R[e];
      }
    }
    if (tid < K) vs = st_sig2[tid];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + q * NTH;
      if (e < K * K) {
        Ai[e] = va[q];
        Xw[e] = vx[q];
        if (fb) Rf[e] = vr[q];
      }
    }
    if (tid < K) td->sig2[tid] = vs;
    if (tid == 0) {
      tdg->info = st_h->info;
      if (jb.out) *jb.out = st_h->info;
      td->last_r = st_h->info.r;
      td->spec_hint = it;
      td->warm = st_h->warm;
      for (int q = 0; q < 8; ++q) td->dbg[q] = st_h->dbg[q];
      td->dbg[2] = qrcols;
      td->nsig = st_h->nsig;
      if (st_h->err) atomicCAS(err, 0, st_h->err);
    }
  };
  int it0 = 1;
  bool decided = false;
  if constexpr (PH == 1) {
    const int itn = blockIdx.x + 1;
    if (itn > n_spec) return;
    int kk = k0;
    for (int m = 1; m < itn; ++m) kk = min(2 * kk, K);   // d depends on min(k0 + p, K) only
    const int dd = min(kk + p, K);
    const double tot = sketch_iteration(itn, dd);
    // the earlier iterations' posted energy tests (wave 0, lane j for
    // iteration j + 1, every lane returns the same): 2 if one of them meets
    // the target (it, not this one, decides the step), 1 if all are posted
    // and none does, 0 if some are still missing after the wait.  The
    // outcome is in the tag itself, so one relaxed load per poll, all lanes
    // at once, tells it (no fence: nothing else the other workgroups wrote
    // is read here).
    constexpr unsigned long long MEETS = 1ull << 63;
    auto poll_earlier = [&](bool wait) -> int {
      const long long t_end = wall_clock64() + (wait ? SPEC_WAIT_TICKS : 0);
      const bool mine = lane + 1 < kfull;
      bool seen = !mine;   // posted and missing the target, or no iteration
      for (;;) {
        const unsigned long long tg =
            seen ? 0ull : __hip_atomic_load(&tags[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__builtin_amdgcn_ballot_w64(!seen && tg == (seq | MEETS)) != 0) return 2;
        seen = seen || tg == seq;
        if (__builtin_amdgcn_ballot_w64(!seen) == 0) return 1;
        if (wall_clock64() >= t_end) return 0;
        __builtin_amdgcn_s_sleep(8);
      }
    };
    if (tid == 0) {
      // post ||Z||_F^2, then its tag (release: the value is visible first)
      spec_d[itn - 1] = tot;
      __hip_atomic_store(&tags[itn - 1], tot >= Et ? (seq | MEETS) : seq, __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    if (stage_ok && itn == kfull && tot >= Et && kfull > 1) {
      // the step needs this iteration only if no earlier one meets the energy
      // target: read the earlier iterations' posted tests (waiting, bounded,
      // when the last step ended before d = K or there was none), and leave
      // the step to the second phase if one of them decides
      if (wid == 0) {
        const int pr = poll_earlier(td->spec_hint < kfull);
        if (lane == 0) sm.found = pr == 2;
      }
      __syncthreads();
      if (sm.found) return;
    }
    if (!(stage_ok && itn == kfull && tot >= Et)) {
      float2* Qw = jb.spec + (size_t)(itn - 1) * 2 * KS * KS;
      float2* Zw = Qw + KS * KS;
      for (int e = tid; e < K * dd; e += NTH) {
        const int j = e / K, i = e - j * K;
        Qw[j * KS + i] = b1[j * LDK + i];
        Zw[j * KS + i] = b2[j * LDK + i];
      }
      return;
    }
    // the full-width iteration passes the test: the step goes on here, as
    // the second phase would take it from this iteration
    iters = itn;
    d = dd;
    found = true;
    basis = true;
    c_mark = clock64();
    jacobi_svd(sm, K, d, &sweeps, &rounds);
    t_jac += clock64() - c_mark; c_mark = clock64();
    // where its results go: straight to the track once every earlier
    // iteration is known to miss the target (the second phase then has
    // nothing left to do), else to the staging area for the second phase
    __syncthreads();
    if (wid == 0) {
      const int pr = kfull > 1 ? poll_earlier(true) : 1;
      if (lane == 0) sm.found = pr;
    }
    __syncthreads();
    const int mode = sm.found;
    if (mode == 2) return;
    staged = mode != 1;
    if (staged) {
      o_Ainv = st_Ainv; o_R = st_R; o_Xw = st_Xw; o_sig2 = st_sig2;
      if (tid == 0) st_h->err = 0;
    } else {
      // the earlier iterations' QR columns, as the second phase counts them
      int kk = k0;
      for (int m = 1; m < itn; ++m) {
        const int dm = min(kk + p, K);
        if (!(dm == K && warm_ok)) qrcols += dm;
        kk = min(2 * kk, K);
      }
    }
    rotated = true;
    pick_rank(sm, K, d, Et, &r, &captured, o_sig2);
    decided = true;
  }
  if constexpr (PH == 2) {
    // the speculated iterations' ||Z||_F^2, read in one round trip
    const double* totw = reinterpret_cast<const double*>(jb.spec + (size_t)2 * KS * KS * SPEC_MAX);
    if (tid < n_spec) sm.totv[tid] = totw[tid];
    __syncthreads();
    for (int it = 1; it <= n_spec; ++it) {
      iters = it;
      d = min(k0 + p, K);
      if (!(d == K && warm_ok)) qrcols += d;
      const double tot = sm.totv[it - 1];
      const bool hit = tot >= Et;
      if (hit || it == i_max || (td->early_fallback && d > td->wb_limit)) {
        if (hit && stage_ok && it == kfull) {
          commit_stage(it);
          return;
        }
        if (!dA_in) {
          load_dA();
          dA_in = true;
        }
        const float2* Qw = jb.spec + (size_t)(it - 1) * 2 * KS * KS;
        const float2* Zw = Qw + KS * KS;
        for (int e = tid; e < K * d; e += NTH) {
          const int j = e / K, i = e - j * K;
          b1[j * LDK + i] = Qw[j * KS + i];
          b2[j * LDK + i] = Zw[j * KS + i];
        }
        __syncthreads();
        c_mark = clock64();
        if (hit) {
          found = true;
          basis = d == K;
          if (d < K && d >= WARM_ROTATE_MIN_D && dwarm >= d) warm_rotate(sm, td->Xd, K, d);
          jacobi_svd(sm, K, d, &sweeps, &rounds);
          t_jac += clock64() - c_mark; c_mark = clock64();
          rotated = true;
          pick_rank(sm, K, d, Et, &r, &captured, o_sig2);
        } else {
          r = d;
          captured = tot;
        }
        decided = true;
        break;
      }
      k0 = min(2 * k0, K);   // d = min(k0 + p, K) is unchanged by the cap
    }
    it0 = n_spec + 1;
  }
  if (!decided) {
    if (!dA_in) {
      load_dA();
      dA_in = true;
    }
    // One-launch form, when the track's last step was decided at d = K (as
    // Alg. 1 at a high eta usually is): the full-width iteration first.  Its
    // SVD is the SVD of Delta A (its Q is unitary), and for any d orthonormal
    // columns Q_i, ||Q_i^H Delta A||_F^2 <= sigma_1^2 + ... + sigma_d^2 (Ky Fan).
    // So an earlier iteration whose d leading sigma_j^2 miss the target cannot
    // meet it: it is skipped, which leaves Alg. 1's outcome as it is (the
    // first iteration that meets the target decides, and its own Q and Z give
    // the step).  The others run in order as before; the full-width results
    // are kept aside (Z in pm/tm) for when none of them meets the target.
    bool pre = false;
    int rk = 0, sweeps_k = 0, rounds_k = 0;
    double capk = 0.0;
    if constexpr (PH == 0) {
      pre = kfull > 1 && kfull <= i_max && warm_ok && td->spec_hint == kfull && !td->early_fallback;
      if (pre) {
        const double totk = sketch_iteration(kfull, K);
        if (totk >= Et) {
          c_mark = clock64();
          jacobi_svd(sm, K, K, &sweeps_k, &rounds_k);
          t_jac += clock64() - c_mark; c_mark = clock64();
          pick_rank(sm, K, K, Et, &rk, &capk, o_sig2);
          float2* const zs = sm.pm;   // pm and tm hold K x K
          for (int e = tid; e < K * K; e += NTH) {
            const int j = e / K, i = e - j * K;
            zs[e] = b2[j * LDK + i];
          }
          if (tid < K) {
            sm.s2k[tid] = sm.s2[tid];
            sm.ordk[tid] = sm.order[tid];
          }
          if (tid == 0) {
            double c = 0.0;
            sm.topk[0] = 0.0;
            for (int j = 0; j < K; ++j) {
              c += sm.s2[sm.order[j]];
              sm.topk[j + 1] = c;
            }
          }
          __syncthreads();
        } else {
          pre = false;   // (eta = 1 within rounding) the iterations in order
        }
      }
    }
    for (int it = it0; it <= i_max; ++it) {
      iters = it;
      d = min(k0 + p, K);
      if (pre && it == kfull) {
        // no earlier iteration met the target: the full-width step
        const float2* zs = sm.pm;
        for (int e = tid; e < K * K; e += NTH) {
          const int j = e / K, i = e - j * K;
          b2[j * LDK + i] = zs[e];
        }
        if (tid < K) {
          sm.s2[tid] = sm.s2k[tid];
          sm.order[tid] = sm.ordk[tid];
          o_sig2[tid] = sm.s2k[sm.ordk[tid]];
        }
        __syncthreads();
        found = true;
        basis = true;
        rotated = true;
        r = rk;
        captured = capk;
        sweeps += sweeps_k;
        rounds += rounds_k;
        break;
      }
      if (pre && sm.topk[d] < Et * (1.0 - KYFAN_MARGIN)) {
        k0 = min(2 * k0, K);   // cannot meet the target
        continue;
      }
      const double tot = sketch_iteration(it, d);
      if (tot >= Et) {
        found = true;
        basis = d == K;
        if (d < K && d >= WARM_ROTATE_MIN_D && dwarm >= d) warm_rotate(sm, td->Xd, K, d);
        jacobi_svd(sm, K, d, &sweeps, &rounds);
        t_jac += clock64() - c_mark; c_mark = clock64();
        rotated = true;
        pick_rank(sm, K, d, Et, &r, &captured, o_sig2);
        break;
      }
      // after the last iteration, or (early-fallback policy) once d is past
      // the Woodbury limit: every component, k_est = d, and the step inverts
      if (it == i_max || (td->early_fallback && d > td->wb_limit)) {
        r = d;                 // every component: U_r Sigma_r V_r^H = Q Z^H
        captured = tot;
        break;
      }
      k0 = min(2 * k0, K);   // d = min(k0 + p, K) is unchanged by the cap
    }
  }
  if (!rotated) {
    if (tid < d) sm.order[tid] = tid;
    __syncthreads();
  }
  (void)found;

  // Alg. 2's switch k_est <= switch * K, within the Woodbury workspace
  bool use_wb = r <= td->wb_limit;
  int path = use_wb ? RZF_PATH_WB : RZF_PATH_FULL_RANK;
  float2* pm = sm.pm;
  float2* tm = sm.tm;
  // the full-width SVD's normalised columns z_j / sigma_j (V_hat): the next
  // full-width step's starting basis, unless a column is numerically zero
  bool basis_ok = false;
  if (basis) {
    if (tid < 64) {
      const double v = lane < K ? sm.s2[lane] : 0.0;
      double smax = v;
#pragma unroll 8
      for (int j = 0; j < K; ++j) smax = fmax(smax, sm.s2[j]);
      const bool ok = smax > 0.0 && __all(lane >= K || v > BASIS_MIN_REL * smax);
      sm.bsc[lane] = ok && lane < K ? (float)(1.0 / sqrt(v)) : 0.f;
      if (lane == 0) sm.bok = ok;
    }
    __syncthreads();
    basis_ok = sm.bok != 0;
    if (basis_ok)
      for (int e = tid; e < K * K; e += NTH) {
        const int j = e / K, i = e - j * K;
        o_Xw[e] = cscale(b2[j * LDK + i], sm.bsc[j]);
      }
  }
  if (rotated && d < K && d >= WARM_ROTATE_MIN_D && td->Xd != nullptr) {
    // this SVD's normalised columns z_j / sigma_j by descending sigma_j: the
    // start of the next narrower Jacobi (warm_rotate), unless a column is
    // numerically zero
    if (tid < 64) {
      const double v = lane < d ? sm.s2[lane] : 0.0;
      double smax = v;
#pragma unroll 8
      for (int j = 0; j < d; ++j) smax = fmax(smax, sm.s2[j]);
      const bool good = lane >= d || (smax > 0.0 && v > BASIS_MIN_REL * smax);
      if (lane == 0) sm.bok = __all(good) && smax > 0.0;
    }
    __syncthreads();
    const bool ok = sm.bok != 0;
    if (ok)
      for (int e = tid; e < K * d; e += NTH) {
        const int m = e / K, i = e - m * K, j = sm.order[m];
        td->Xd[e] = cscale(b2[j * LDK + i], (float)(1.0 / sqrt(sm.s2[j])));
      }
    if (tid == 0) td->dwarm = ok ? d : 0;
    __syncthreads();
  }
  if (rotated && use_wb) {
    if (tid < r) sm.is2[tid] = 1.0 / sm.s2[sm.order[tid]];
    __syncthreads();
  }
  if (rotated && use_wb && basis) {
    // U_r = Delta A Z_r Sigma_r^-2 (Q is unitary at d = K); every retained
    // sigma_j is positive
    const int* ord = sm.order;
    lds_gemm(K, r, K,
             [&](int i, int k) { return (i < K && k < K) ? b0[i * LDK + k] : cz(); },
             [&](int k, int c) { return (k < K && c < r) ? b2[ord[c] * LDK + k] : cz(); },
             [&](int i, int c, float2 v) {
               const double is2 = sm.is2[c];
               pm[c * LDK + i] = make_float2((float)(v.x * is2), (float)(v.y * is2));
             });
    __syncthreads();
  } else if (rotated && use_wb) {
    // U_r = Q U_hat_r = Q Q^H Delta A Z_r Sigma_r^-2 (B V_hat = U_hat Sigma with
    // V_hat = Z Sigma^-1); every retained sigma_j is positive
    const int* ord = sm.order;
    lds_gemm(K, r, K,
             [&](int i, int k) { return (i < K && k < K) ? b0[i * LDK + k] : cz(); },
             [&](int k, int c) { return (k < K && c < r) ? b2[ord[c] * LDK + k] : cz(); },
             [&](int i, int c, float2 v) { pm[c * LDK + i] = v; });
    __syncthreads();
    lds_gemm(d, r, K,
             [&](int j, int k) { return (j < d && k < K) ? cconj(b1[j * LDK + k]) : cz(); },
             [&](int k, int c) { return (k < K && c < r) ? pm[c * LDK + k] : cz(); },
             [&](int j, int c, float2 v) { tm[c * LDK + j] = v; });
    __syncthreads();
    lds_gemm(K, r, d,
             [&](int i, int j) { return (i < K && j < d) ? b1[j * LDK + i] : cz(); },
             [&](int j, int c) { return (j < d && c < r) ? tm[c * LDK + j] : cz(); },
             [&](int i, int c, float2 v) {
               const double is2 = sm.is2[c];
               pm[c * LDK + i] = make_float2((float)(v.x * is2), (float)(v.y * is2));
             });
    __syncthreads();
  }
  const float2* Ub = rotated ? pm : b1;   // column c of U at Ub[c * LDK]
  if (fb && use_wb) {
    // residual of the rank-r update: R = (Delta A + R) - U V~^H, read from b0
    // before the Woodbury step reuses it (a direct inversion clears R below)
    float2* R = o_R;
    const int* ord = sm.order;
    lds_gemm(K, K, r,
             [&](int i, int c) { return (i < K && c < r) ? Ub[c * LDK + i] : cz(); },
             [&](int c, int j) { return (c < r && j < K) ? cconj(b2[ord[c] * LDK + j]) : cz(); },
             [&](int i, int j, float2 v) { R[(size_t)i * K + j] = csub(b0[i * LDK + j], v); });
    __syncthreads();
  }

  if (use_wb) {
    // A^-1 -> b0
    for (int e = tid; e < K * K; e += NTH) {
      const int i = e / K, j = e - i * K;
      b0[i * LDK + j] = td->Ainv[e];
    }
    __syncthreads();
    const int* ord = sm.order;
    // step 1: P = A^-1 U
    lds_gemm(K, r, K,
             [&](int i, int k) { return (i < K && k < K) ? b0[i * LDK + k] : cz(); },
             [&](int k, int c) { return (k < K && c < r) ? Ub[c * LDK + k] : cz(); },
             [&](int i, int c, float2 v) { tm[c * LDK + i] = v; });
    __syncthreads();
    // step 2: C = I + V~^H P (r x r), and V~^H A^-1 (r x K); tiles held in
    // registers until every wave has finished reading U and V~
    const int rt = (r + 15) / 16, kt = (K + 15) / 16;
    const int nct = rt * rt, nqt = rt * kt;
    floatx4 dr = zero4(), di = zero4();
    int my_ti = -1, my_tj = -1, my_kind = -1;
    for (int tt = wid; tt < nct + nqt; tt += NWV) {   // at most one tile per wave
      const bool ct = tt < nct;
      const int u = ct ? tt : tt - nct;
      const int ncol = ct ? rt : kt;
      my_ti = u / ncol; my_tj = u - my_ti * ncol; my_kind = ct ? 0 : 1;
      auto la = [&](int rr, int k) {
        const int a = my_ti * 16 + rr;
        return (a < r && k < K) ? cconj(b2[ord[a] * LDK + k]) : cz();
      };
      auto lbc = [&](int k, int cc) {
        const int b = my_tj * 16 + cc;
        return (k < K && b < r) ? tm[b * LDK + k] : cz();
      };
      auto lbq = [&](int k, int cc) {
        const int j = my_tj * 16 + cc;
        return (k < K && j < K) ? b0[k * LDK + j] : cz();
      };
      if (ct) ctile16(la, lbc, 0, K, dr, di); else ctile16(la, lbq, 0, K, dr, di);
    }
    __syncthreads();
    const int ldg = r + K;
    double2* aug = reinterpret_cast<double2*>(b1);   // r x (r + K), spans b1 and b2
    if (my_kind >= 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = my_ti * 16 + tile_row(v), c = my_tj * 16 + tile_col();
        if (my_kind == 0) {
          if (a < r && c < r)
            aug[a * ldg + c] = make_double2((a == c ? 1.0 : 0.0) + (double)dr[v], (double)di[v]);
        } else {
          if (a < r && c < K) aug[a * ldg + r + c] = make_double2((double)dr[v], (double)di[v]);
        }
      }
    }
    __syncthreads();
    // step 3: X = C^-1 V~^H A^-1 in FP64 (M = V~^H A^-1 in columns r.. of
    // aug; X replaces it).  C = I + E with E = V~^H A^-1 U, and
    // ||E|| <= ||Delta A_r|| ||A^-1||, small for a small update: then X <- M - E X
    // from X = M (the error shrinks by ||E||_F per pass, down to the rounding
    // of the FP32 product E X);
    // otherwise C^-1 by Gauss-Jordan with partial pivoting, then
    // X = C^-1 M = S_p M_p (S_p[a, c] = S[p_a, c], M_p[c, :] = M[p_c, :]).
    double e2 = 0.0;
    for (int e = tid; e < r * r; e += NTH) {
      const int a = e / r, c = e - a * r;
      const double2 v = aug[a * ldg + c];
      const double re = v.x - (a == c ? 1.0 : 0.0);
      e2 += re * re + v.y * v.y;
    }
    const double eps2 = block_sum(e2, sm.red);
    const int xt = (r + 15) / 16, yt = (K + 15) / 16;
    const int ti = wid / yt, tj = wid - (wid / yt) * yt;
    const bool xtile = wid < xt * yt;   // one 16 x 16 tile of X per wave
    bool solved;
    if (eps2 <= NEUMANN_MAX * NEUMANN_MAX) {
      // passes for ||E||_F^n <= 2^-NEUMANN_BITS (at most 15 at ||E||_F = 1/4)
      const int nit = eps2 > 0.0 ? (int)ceil(-NEUMANN_BITS * 0.6931471805599453 / (0.5 * log(eps2))) : 1;
      double2 mreg[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = ti * 16 + tile_row(v), j = tj * 16 + tile_col();
        mreg[v] = (xtile && a < r && j < K) ? aug[a * ldg + r + j] : dz();
      }
      for (int a = tid; a < r; a += NTH) aug[a * ldg + a].x -= 1.0;   // C -> E
      __syncthreads();
      // this lane's matrix-core operand values of E (row ti 16 + lane % 16,
      // column 4 s + lane / 16 at step s), in FP32, held for every pass
      const int el = lane & 15, ek = lane >> 4;
      float2 ea[WB_RMAX / 4];
#pragma unroll
      for (int st = 0; st < WB_RMAX / 4; ++st) {
        const int a = ti * 16 + el, k = 4 * st + ek;
        ea[st] = (xtile && a < r && k < r) ? d2f(aug[a * ldg + k]) : cz();
      }
      for (int it = 0; it < nit; ++it) {
        double2 acc[4] = {mreg[0], mreg[1], mreg[2], mreg[3]};
        if (xtile) {
          // E X for this tile: the products of ctile16 with E's values from
          // registers, the four real products in independent accumulators
          floatx4 xx = zero4(), yy = zero4(), xy = zero4(), yx = zero4();
          const int j = tj * 16 + el;
#pragma unroll
          for (int st = 0; st < WB_RMAX / 4; ++st) {
            if (4 * st < r) {
              const int k = 4 * st + ek;
              const float2 b = (k < r && j < K) ? d2f(aug[k * ldg + r + j]) : cz();
              xx = mfma4(ea[st].x, b.x, xx);
              yy = mfma4(ea[st].y, b.y, yy);
              xy = mfma4(ea[st].x, b.y, xy);
              yx = mfma4(ea[st].y, b.x, yx);
            }
          }
          const floatx4 dr = xx - yy, di = xy + yx;
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[v] = make_double2(acc[v].x - (double)dr[v], acc[v].y - (double)di[v]);
        }
        __syncthreads();
        if (xtile) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int a = ti * 16 + tile_row(v), j = tj * 16 + tile_col();
            if (a < r && j < K) aug[a * ldg + r + j] = acc[v];
          }
        }
        __syncthreads();
      }
      solved = true;
    } else {
      const double stol = SING_TOL * (1.0 + sqrt(eps2));
      solved = gj_invert_small(sm, aug, r, ldg, stol * stol);
      if (solved) {
        const int* pv = sm.gjperm;
        double2 acc[4] = {dz(), dz(), dz(), dz()};
        if (xtile)
          dtile16([&](int i, int c) {
                    const int a = ti * 16 + i;
                    return (a < r && c < r) ? aug[pv[a] * ldg + c] : dz();
                  },
                  [&](int c, int j) {
                    const int jj = tj * 16 + j;
                    return (c < r && jj < K) ? aug[pv[c] * ldg + r + jj] : dz();
                  },
                  0, r, acc);
        __syncthreads();
        if (xtile) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int a = ti * 16 + tile_row(v), j = tj * 16 + tile_col();
            if (a < r && j < K) aug[a * ldg + r + j] = acc[v];
          }
        }
        __syncthreads();
      }
    }
    if (!solved) {
      use_wb = false;
      path = RZF_PATH_FULL_SINGULAR;
    } else {
      // steps 4-5: A^-1 <- A^-1 - P X
      float2* out = o_Ainv;
      lds_gemm(K, K, r,
               [&](int i, int a) { return (i < K && a < r) ? tm[a * LDK + i] : cz(); },
               [&](int a, int j) { return (a < r && j < K) ? d2f(aug[a * ldg + r + j]) : cz(); },
               [&](int i, int j, float2 v) { out[(size_t)i * K + j] = csub(b0[i * LDK + j], v); });
    }
    __syncthreads();
  }
  if (!use_wb) {
    // direct inversion of A' (FP32)
    if (fb)
      for (int e = tid; e < K * K; e += NTH) o_R[e] = cz();
    if (tid == 0) sm.bad = 0;
    for (int e = tid; e < K * K; e += NTH) {
      const int i = e / K, j = e - i * K;
      b0[i * LDK + j] = td->Anew[e];
    }
    __syncthreads();
    gj_inverse_hpd_mfma(b0, K, LDK, b1, b1 + 16 * KS, b1 + 32 * KS, &sm.bad);
    for (int e = tid; e < K * K; e += NTH) {
      const int i = e / K, j = e - i * K;
      o_Ainv[e] = b0[i * LDK + j];
    }
    if (tid == 0 && sm.bad) {
      const int code = sm.bad == 2 ? DEV_ERR_NONFINITE : DEV_ERR_NOT_HPD;
      if (staged) st_h->err = code;
      else atomicCAS(err, 0, code);
    }
  }
  if (tid == 0) {
    DevInfo inf;
    inf.r = r; inf.iters = iters; inf.path = path; inf.d = d;
    inf.dA_fro2 = E; inf.captured = captured;
    t_wb = clock64() - c_mark;
    int* dbg = staged ? st_h->dbg : tdg->dbg;
    dbg[0] = sweeps; dbg[1] = rounds; dbg[2] = qrcols;
    dbg[3] = (int)t_sk; dbg[4] = (int)t_qr; dbg[5] = (int)t_jac; dbg[6] = (int)t_wb;
    dbg[7] = (int)(wall_clock64() - r_begin);
    if (staged) {
      st_h->info = inf;
      st_h->warm = basis_ok ? 1 : 0;
      st_h->nsig = d;
    } else {
      tdg->info = inf;
      if (jb.out) *jb.out = inf;
      td->last_r = r;
      td->spec_hint = iters;
      if (basis) td->warm = basis_ok ? 1 : 0;
      td->nsig = rotated ? d : 0;
      if (PH == 1) {
        td->hold = 0;   // a finite step (the second phase, which would record it, returns at once)
        __hip_atomic_store(&tags[SPEC_MAX], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    (void)c_begin;
  }
}

// Longest-first order of a batch's arSVD jobs (out = in, permuted): the jobs
// expected to take longest start in the first wave of workgroups, so that a
// launch's time is not one slow track left for last on its CU.  Key 7 .. 0,
// stable within a key: a large track (K > KS) by its size (min(7, K / 32));
// a K <= KS track 1 when its next full-width iteration has no warm basis or
// its last SVD stopped below d = K (its step runs more of Alg. 1 or a cold
// Jacobi), else 0.  Reads only the descriptors as the previous step left
// them.  One workgroup; every track's results are what they are in any order.
__global__ __launch_bounds__(1024) void k_arsvd_order(const ArsvdJob* in, ArsvdJob* out, int n) {
  constexpr int NK = 8;
  __shared__ int cnt[NK], base[NK];
  __shared__ int wsum[NTH / 64][NK];
  __shared__ unsigned char keys[RZF_BATCH_MAX];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  auto key_of = [&](int t) -> int {
    const GTrackDesc* td = (const GTrackDesc*)in[t].td;
    const int K = td->K;
    if (K > KS) return min(NK - 1, K / 32);
    return (td->warm != 0 && td->nsig == K) ? 0 : 1;
  };
  if (tid < NK) cnt[tid] = 0;
  __syncthreads();
  for (int t = tid; t < n; t += NTH) {
    const int k = key_of(t);
    keys[t] = (unsigned char)k;
    atomicAdd(&cnt[k], 1);
  }
  __syncthreads();
  if (tid == 0) {
    int b = 0;
    for (int k = NK - 1; k >= 0; --k) {
      base[k] = b;
      b += cnt[k];
    }
  }
  __syncthreads();
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int c0 = 0; c0 < n; c0 += NTH) {
    const int t = c0 + tid;
    const int k = t < n ? (int)keys[t] : -1;
    unsigned long long mk = 0ull;
#pragma unroll
    for (int b = 0; b < NK; ++b) {
      const unsigned long long m = __ballot(k == b);
      if (lane == 0) wsum[wid][b] = __popcll(m);
      if (k == b) mk = m;
    }
    __syncthreads();
    if (k >= 0) {
      int off = base[k] + __popcll(mk & below);
      for (int w = 0; w < wid; ++w) off += wsum[w][k];
      out[off] = in[t];
    }
    __syncthreads();
    if (tid < NK) {
      int c = 0;
      for (int w = 0; w < NTH / 64; ++w) c += wsum[w][tid];
      base[tid] += c;
    }
    __syncthreads();
  }
}

__global__ void k_debug_sketch(uint64_t seed, uint64_t track, int t, int it, int K, int d,
                               float2* Omega, uint64_t* words) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K * d) return;
  const int j = e / K, i = e - j * K;
  uint64_t wa, wb;
  sketch_words(seed, track, t, it, i, j, &wa, &wb);
  if (Omega) Omega[e] = words_to_cn(wa, wb);
  if (words) {
    const int ent = i * d + j;
    words[2 * ent] = wa;
    words[2 * ent + 1] = wb;
  }
}

}  // namespace

void launch_arsvd_wb(const ArsvdJob& one, const ArsvdJob* many, int n, int* err, hipStream_t s) {
  if (many) k_arsvd_wb<true, 0><<<dim3(1, n), NTH, 0, s>>>(one, many, err);
  else k_arsvd_wb<false, 0><<<1, NTH, 0, s>>>(one, many, err);
}

void launch_arsvd_order(const ArsvdJob* in, ArsvdJob* out, int n, hipStream_t s) {
  k_arsvd_order<<<1, NTH, 0, s>>>(in, out, n);
}

void launch_arsvd_wb_spec(const ArsvdJob& one, int* err, hipStream_t s) {
  k_arsvd_wb<false, 1><<<SPEC_MAX, NTH, 0, s>>>(one, nullptr, err);
  k_arsvd_wb<false, 2><<<1, NTH, 0, s>>>(one, nullptr, err);
}

void launch_debug_sketch(uint64_t seed, uint64_t track, int t, int it, int K, int d, float2* Omega,
                         uint64_t* words, hipStream_t s) {
  const int n = K * d;
  k_debug_sketch<<<(n + 255) / 256, 256, 0, s>>>(seed, track, t, it, K, d, Omega, words);
}
