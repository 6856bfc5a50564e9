// Alg. 1 + Alg. 2 for the large tracks (64 < K <= 256), and their direct
// inverses.
//
// Same computation and the same order as k_arsvd_wb (arsvd.hip): per
// iteration Omega -> Y = Delta A Omega -> Q = orth(Y) (Householder) ->
// Z = Delta A^H Q, the ||Z||_F^2 test of eq. (14), on success a one-sided
// Jacobi SVD of B = Z^H, the rank rule, U_r rebuilt as Q Q^H Delta A Z_r
// Sigma_r^-2, then the Woodbury update of eq. (12) in the scaled form (U_r,
// V~ = Z columns) or direct inversion of A'.
//
// What changes with K: the K x d factors no longer fit in LDS, so each track
// keeps them in its own global workspace (column-major Y, Q, Z; row-major
// FP64 capacitance system), which stays resident in L2 while the single
// workgroup of the track works on it, and the algorithms are blocked so that
// every pass streams a matrix once:
//   * Householder QR in 16-column panels: the panel is factored in LDS, its
//     compact WY form H_0..H_15 = I - V T V^H is applied to the trailing
//     columns with three 16-wide products on the matrix cores, and Q is
//     formed by the same blocks in reverse order;
//   * one-sided Jacobi in column blocks: block pairs of Z are staged in LDS
//     and every column pair is rotated once per pass (d <= 2b: all columns
//     in LDS, plain cyclic sweeps);
//   * Gauss-Jordan with partial pivoting on [C | V~^H A^-1] in 32-column
//     panels: the panel is eliminated in LDS, recording its pivots and
//     multipliers, then every other column replays them;
//   * 16 x 16 block Gauss-Jordan for the HPD inverses (gj_inverse_hpd_blocked).
#include "dense_device.h"
#include "rzf_internal.h"

namespace {

constexpr int NTH = 1024;
constexpr int NWV = NTH / 64;
constexpr int MAX_SWEEPS = 30;      // Jacobi passes
constexpr double JACOBI_TOL = 2e-6;
constexpr double JACOBI_QSTOP = 1e-3;   // passes stop after one with no pair above it
// a full-width SVD leaves its normalised columns z_j / sigma_j as the next
// full-width iteration's starting basis; a column with sigma_j^2 at or below
// this fraction of the largest (numerically zero, so not made orthogonal to
// the others) leaves the track without one
constexpr double BASIS_MIN_REL = 1e-20;
// margin on Ky Fan's bound (below) for the rounding of the full-width sigma_j^2
constexpr double KYFAN_MARGIN = 1e-4;
// C = I + E is taken as singular when a pivot's modulus is at most
// SING_TOL (1 + ||E||_F): its entries come from FP32 factors and are known
// only to about r 2^-24 (1 + ||E||) (r <= 128 here), so a smaller pivot leaves
// nothing of C^-1 M that they determine (path FULL_SINGULAR)
constexpr double SING_TOL = 0x1.0p-14;
constexpr int JOB_ELEMS = KM * 32;  // LDS entries of one job matrix
constexpr int GJ_W = 32;            // panel width of the capacitance solve
constexpr int RB = KM / 2;          // largest Woodbury rank of a large track

struct BigShared {
  union {
    struct {
      float2 pan[KM * 16];            // panel (column-major, ld K)
      float2 tf[(KM / 16) * 256];     // T of every panel (row-major 16 x 16)
      float2 ws[NWV * 256];           // per-wave 16 x 16 scratch
    } qr;
    struct {
      float2 z[2 * JOB_ELEMS];        // job columns of Z (column-major, ld K)
    } jac;
    struct {
      double2 pan[RB * GJ_W];         // capacitance panel (row-major, ld GJ_W)
      double2 ustash[GJ_W];
    } gj;
    struct {
      float2 xs[16 * KM];
      float2 cs[KM * 16];
      float2 pb[2 * 256];
    } inv;
    float2 om[KM * 16];               // one 16-column tile of Omega
  } u;
  double s2[KM];
  // full-width iteration computed first: its sigma_j^2 and order, and the
  // energies of its leading columns (topk[d] = the d largest)
  double s2k[KM];
  int ordk[KM];
  double topk[KM + 1];
  double red[NWV];
  double2 pivv[GJ_W];
  int order[KM];
  int pivrow[GJ_W];
  int nrot, r, singular, bad;
  double cap;
};

__device__ __forceinline__ int up4(int k) { return (k + 3) & ~3; }

// ---------------------------------------------------------------- QR
// Householder vector of panel column c from the column values x[m] (row
// lane + 64 m), pivot row pr: H = I - 2 w w^H maps x to beta e_pr.  Written
// over panel column c, zero above pr.  Wave-level, all lanes active.
__device__ __forceinline__ void reflector_big(const float2 x[4], float2* pan, int c, int pr, int K) {
  const int lane = threadIdx.x & 63;
  float sp = 0.f;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int i = lane + 64 * m;
    if (i < K && i >= pr) sp += cabs2(x[m]);
  }
  const float s = wave_sumf(sp);
  const int ms = pr >> 6, ls = pr & 63;
  float2 xp = x[0];
#pragma unroll
  for (int m = 1; m < 4; ++m) if (m == ms) xp = x[m];
  const float ax = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(xp.x), ls));
  const float ay = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(xp.y), ls));
  float2 w[4] = {cz(), cz(), cz(), cz()};
  if (s >= 1e-36f) {
    const float inx = __builtin_amdgcn_rsqf(s);
    const float bx = ax * inx, by = ay * inx;
    const float aa = __builtin_amdgcn_sqrtf(bx * bx + by * by);
    float ph_r = 1.f, ph_i = 0.f;
    if (aa > 0.f) { const float ia = __builtin_amdgcn_rcpf(aa); ph_r = bx * ia; ph_i = by * ia; }
    const float iw = __builtin_amdgcn_rsqf(2.f * (1.f + aa));
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int i = lane + 64 * m;
      if (i == pr) {
        const float mm = (aa + 1.f) * iw;
        w[m] = make_float2(ph_r * mm, ph_i * mm);
      } else if (i > pr) {
        const float mm = inx * iw;
        w[m] = make_float2(x[m].x * mm, x[m].y * mm);
      }
    }
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int i = lane + 64 * m;
    if (i < K) pan[c * K + i] = w[m];
  }
}

// Column c of the panel <- (I - 2 w w^H) column c, w = panel column wc.
__device__ __forceinline__ void apply_reflector_big(float2* pan, int wc, int c, int K, float2 y[4]) {
  const int lane = threadIdx.x & 63;
  float2 w[4];
  float dr = 0.f, di = 0.f;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int i = lane + 64 * m;
    w[m] = (i < K) ? pan[wc * K + i] : cz();
    y[m] = (i < K) ? pan[c * K + i] : cz();
    dr += w[m].x * y[m].x + w[m].y * y[m].y;
    di += w[m].x * y[m].y - w[m].y * y[m].x;
  }
  dr = wave_sumf(dr);
  di = wave_sumf(di);
  const float fr = 2.f * dr, fi = 2.f * di;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int i = lane + 64 * m;
    y[m].x -= w[m].x * fr - w[m].y * fi;
    y[m].y -= w[m].x * fi + w[m].y * fr;
    if (i < K) pan[c * K + i] = y[m];
  }
}

// Block of 16 reflectors (panel V, factor T) applied to the 16 columns
// cc0..cc0+15 (< d) of the column-major K x d matrix M, rows >= r0:
//   M <- M - V op(T) (V^H M),  op(T) = T^H when `adj`, else T.
__device__ __forceinline__ void apply_block(const float2* pan, const float2* T, float2* ws, float2* M, int K, int d,
                            int r0, int cc0, bool adj) {
  floatx4 dr = zero4(), di = zero4();
  ctile16([&](int i, int k) { return (k < K) ? cconj(pan[i * K + k]) : cz(); },
          [&](int k, int j) {
            const int c = cc0 + j;
            return (k < K && c < d) ? M[(size_t)c * K + k] : cz();
          },
          r0 & ~3, up4(K), dr, di);
#pragma unroll
  for (int v = 0; v < 4; ++v) ws[tile_row(v) * 16 + tile_col()] = make_float2(dr[v], di[v]);
  wave_sync();
  dr = zero4(); di = zero4();
  if (adj)
    ctile16([&](int i, int k) { return cconj(T[k * 16 + i]); }, [&](int k, int j) { return ws[k * 16 + j]; },
            0, 16, dr, di);
  else
    ctile16([&](int i, int k) { return T[i * 16 + k]; }, [&](int k, int j) { return ws[k * 16 + j]; },
            0, 16, dr, di);
  wave_sync();
#pragma unroll
  for (int v = 0; v < 4; ++v) ws[tile_row(v) * 16 + tile_col()] = make_float2(dr[v], di[v]);
  wave_sync();
  for (int rc = r0 >> 4; rc * 16 < K; ++rc) {
    floatx4 er = zero4(), ei = zero4();
    ctile16([&](int i, int k) {
              const int row = rc * 16 + i;
              return (row < K) ? pan[k * K + row] : cz();
            },
            [&](int k, int j) { return ws[k * 16 + j]; }, 0, 16, er, ei);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = rc * 16 + tile_row(v), c = cc0 + tile_col();
      if (row < K && c < d) {
        float2* p = M + (size_t)c * K + row;
        *p = csub(*p, make_float2(er[v], ei[v]));
      }
    }
  }
  wave_sync();
}

// Householder QR of Y (K x d, in Ym) by 16-column panels: the reflectors
// replace Y, the T factors stay in LDS, and Q = H_0 ... H_{d-1} [I_d; 0] is
// formed in Qm.
__device__ __forceinline__ void qr_big(BigShared& sm, float2* Ym, float2* Qm, int K, int d) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  float2* pan = sm.u.qr.pan;
  float2* ws = sm.u.qr.ws + wid * 256;
  const int np = (d + 15) / 16;
  for (int p = 0; p < np; ++p) {
    const int c0 = 16 * p, nc = min(16, d - c0);
    float2* T = sm.u.qr.tf + p * 256;
    for (int e = tid; e < 16 * K; e += NTH) {
      const int c = e / K, i = e - c * K;
      pan[e] = (c < nc) ? Ym[(size_t)(c0 + c) * K + i] : cz();
    }
    __syncthreads();
    if (wid == 0) {
      float2 x[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int i = lane + 64 * m;
        x[m] = (i < K) ? pan[i] : cz();
      }
      reflector_big(x, pan, 0, c0, K);
    }
    for (int j = 0; j < nc; ++j) {
      __syncthreads();
      for (int c = j + 1 + wid; c < nc; c += NWV) {
        float2 y[4];
        apply_reflector_big(pan, j, c, K, y);
        if (c == j + 1) reflector_big(y, pan, c, c0 + c, K);
      }
    }
    __syncthreads();
    if (wid == 0) {
      // S = V^H V, then T (upper triangular) of H_0 ... H_15 = I - V T V^H:
      // T_jj = 2, T[0:j, j] = -2 T[0:j, 0:j] S[0:j, j]
      floatx4 dr = zero4(), di = zero4();
      ctile16([&](int i, int k) { return (k < K) ? cconj(pan[i * K + k]) : cz(); },
              [&](int k, int j) { return (k < K) ? pan[j * K + k] : cz(); }, c0, up4(K), dr, di);
#pragma unroll
      for (int v = 0; v < 4; ++v) ws[tile_row(v) * 16 + tile_col()] = make_float2(dr[v], di[v]);
      for (int e = lane; e < 256; e += 64) T[e] = cz();
      wave_sync();
      for (int j = 0; j < 16; ++j) {
        if (lane < 16) {
          const int i = lane;
          float2 val = cz();
          if (j < nc) {
            if (i == j) {
              val = make_float2(2.f, 0.f);
            } else if (i < j) {
              float2 acc = cz();
              for (int k = i; k < j; ++k) acc = cadd(acc, cmul(T[i * 16 + k], ws[k * 16 + j]));
              val = make_float2(-2.f * acc.x, -2.f * acc.y);
            }
          }
          T[i * 16 + j] = val;
        }
      }
      wave_sync();
    }
    for (int e = tid; e < nc * K; e += NTH) {
      const int c = e / K, i = e - c * K;
      Ym[(size_t)(c0 + c) * K + i] = pan[e];
    }
    __syncthreads();
    // trailing columns: C <- (I - V T^H V^H) C
    const int cs0 = c0 + 16;
    const int nt = (d > cs0) ? (d - cs0 + 15) / 16 : 0;
    for (int t = wid; t < nt; t += NWV) apply_block(pan, T, ws, Ym, K, d, c0, cs0 + 16 * t, true);
    __syncthreads();
  }
  for (int e = tid; e < K * d; e += NTH) {
    const int j = e / K, i = e - j * K;
    Qm[e] = (i == j) ? make_float2(1.f, 0.f) : cz();
  }
  __syncthreads();
  for (int p = np - 1; p >= 0; --p) {
    const int c0 = 16 * p, nc = min(16, d - c0);
    for (int e = tid; e < 16 * K; e += NTH) {
      const int c = e / K, i = e - c * K;
      pan[e] = (c < nc) ? Ym[(size_t)(c0 + c) * K + i] : cz();
    }
    __syncthreads();
    const int nt = (d - c0 + 15) / 16;
    for (int t = wid; t < nt; t += NWV)
      apply_block(pan, sm.u.qr.tf + p * 256, ws, Qm, K, d, c0, c0 + 16 * t, false);
    __syncthreads();
  }
}

// ------------------------------------------------------------ Jacobi
template <int G>
__device__ __forceinline__ float gsumf(float v) {
  v = row16_sumf(v);
  if constexpr (G == 16) return v;
  return v + __shfl_xor(v, 16);
}

// Rotation of the job column pair (pp, qq) of Z held in LDS (sm.u.jac.z,
// column c at c*K) by the calling group of G lanes (rows gl + G m, m < JR):
// the one-sided Jacobi step that makes z_p and z_q orthogonal.  ||z_p||^2
// and ||z_q||^2 are sums of non-negative FP32 terms.  The inner product
// z_p^H z_q cancels as the columns become orthogonal: each lane forms its
// share in FP32 and the G shares are added in FP32 too (rounding error at
// most about 13 x 2^-24 ||z_p|| ||z_q||, under half the rotation threshold);
// every lane of the group forms the same bits, so the group applies one
// rotation.  A pair already orthogonal to JACOBI_TOL is left alone.  Sets
// sm.nrot when |z_p^H z_q| > JACOBI_QSTOP ||z_p|| ||z_q||: near convergence a
// pass squares that measure, so after a pass with no such pair the next one
// would rotate at the FP32 noise level only, and the passes stop.
// Every lane of the wave calls it (act = false for an idle group).
constexpr int JR = 8;   // rows per lane: G = 16 covers K <= 128, G = 32 K <= 256
template <int G>
__device__ __forceinline__ void jacobi_pair(BigShared& sm, int K, int pp, int qq, bool act) {
  float2* zb = sm.u.jac.z;
  const int gl = threadIdx.x & (G - 1);
  float2 zp[JR], zq[JR];
  float al = 0.f, be = 0.f, grs = 0.f, gis = 0.f;
#pragma unroll
  for (int m = 0; m < JR; ++m) {
    const int i = gl + G * m;
    const bool ok = act && i < K;
    zp[m] = ok ? zb[pp * K + i] : cz();
    zq[m] = ok ? zb[qq * K + i] : cz();
  }
#pragma unroll
  for (int m = 0; m < JR; ++m) {
    al += cabs2(zp[m]);
    be += cabs2(zq[m]);
    grs = fmaf(zp[m].x, zq[m].x, fmaf(zp[m].y, zq[m].y, grs));
    gis = fmaf(zp[m].x, zq[m].y, fmaf(-zp[m].y, zq[m].x, gis));
  }
  al = gsumf<G>(al);
  be = gsumf<G>(be);
  const float gr = gsumf<G>(grs);
  const float gi = gsumf<G>(gis);
  const float mx = fmaxf(al, be);
  bool rot = act && mx > 0.f;
  float c = 1.f, s = 0.f;
  float2 e = make_float2(1.f, 0.f);
  if (rot) {
    // same rotation as the LDS kernel: sums scaled by 1/max(alpha, beta)
    const float sc = __builtin_amdgcn_rcpf(mx);
    const float alf = al * sc, bef = be * sc;
    const float grf = gr * sc, gif = gi * sc;
    const float gg = grf * grf + gif * gif;
    rot = gg >= 1e-36f && gg > (float)(JACOBI_TOL * JACOBI_TOL) * alf * bef;
    if (gg > (float)(JACOBI_QSTOP * JACOBI_QSTOP) * alf * bef && gl == 0) sm.nrot = 1;
    const float ig = __builtin_amdgcn_rsqf(fmaxf(gg, 1e-36f));
    const float zeta = (bef - alf) * 0.5f * ig;
    const float az = fabsf(zeta);
    const float tmag = (az > 1e18f) ? 0.5f * __builtin_amdgcn_rcpf(az)
                                    : __builtin_amdgcn_rcpf(az + __builtin_amdgcn_sqrtf(1.f + az * az));
    const float tt = zeta >= 0.f ? tmag : -tmag;
    c = __builtin_amdgcn_rsqf(1.f + tt * tt);
    s = c * tt;
    e = make_float2(grf * ig, -gif * ig);
  }
  if (rot) {
#pragma unroll
    for (int m = 0; m < JR; ++m) {
      const int i = gl + G * m;
      if (i >= K) continue;
      const float2 zq2 = cmul(e, zq[m]);
      zb[pp * K + i] = csub(cscale(zp[m], c), cscale(zq2, s));
      zb[qq * K + i] = cadd(cscale(zp[m], s), cscale(zq2, c));
    }
  }
}

// One sweep of the cyclic (round-robin) ordering over the job columns
// c0 .. c0+nc-1: nc-1 rounds (nc even, else nc), a barrier after each.
template <int G>
__device__ __forceinline__ void jacobi_sweep(BigShared& sm, int K, int c0, int nc, int* rounds) {
  const int wid = threadIdx.x >> 6, slot = threadIdx.x / G;
  const int n = nc + (nc & 1);
  for (int k = 0; k < n - 1; ++k) {
    ++*rounds;
    if (wid * (64 / G) < n / 2) {
      int pp = 0, qq = 0;
      bool act = slot < n / 2;
      if (act) {
        rr_pair(k, slot, n, &pp, &qq);
        act = pp < nc && qq < nc;
      }
      jacobi_pair<G>(sm, K, c0 + pp, c0 + qq, act);
    }
    __syncthreads();
  }
}

// One-sided Jacobi SVD of B = Z^H (Z rotated in place; the rotations are
// not accumulated); every pass rotates each column pair once, and the passes
// stop after one with no pair above JACOBI_QSTOP (or after MAX_SWEEPS).  A round pairs up to
// NTH / G columns; LDS holds NCMAX = 2 NTH / G columns (NCMAX K <= 2 JOB_ELEMS).
//   d <= NCMAX: all d columns sit in LDS; a pass is one cyclic sweep.
//   d > NCMAX: blocks of b = NCMAX/2 columns.  For each block A in turn,
//     A is loaded, its own pairs take one cyclic sweep, then every later
//     block B is streamed through: b rounds whose round s pairs column i of
//     A with column (i + s) mod b of B, so every pair (A_i, B_j) meets once.
//     A ordering of the cyclic kind, pass by pass like the single-block one.
template <int G>
__device__ __forceinline__ void jacobi_big(BigShared& sm, float2* Zm, int K, int d, int* sweeps, int* rounds) {
  constexpr int NCMAX = 2 * NTH / G;   // 128 columns (G = 16, K <= 128) or 64 (G = 32)
  static_assert(NCMAX * (G * JR) <= 2 * JOB_ELEMS, "job columns exceed the LDS buffer");
  const int tid = threadIdx.x, wid = tid >> 6, slot = tid / G;
  float2* zb = sm.u.jac.z;
  if (d <= NCMAX) {
    for (int e = tid; e < d * K; e += NTH) zb[e] = Zm[e];
    for (int pass = 0; pass < MAX_SWEEPS; ++pass) {
      if (tid == 0) sm.nrot = 0;
      __syncthreads();
      ++*sweeps;
      jacobi_sweep<G>(sm, K, 0, d, rounds);
      const bool done = sm.nrot == 0;
      __syncthreads();
      if (done) break;
    }
    for (int e = tid; e < d * K; e += NTH) Zm[e] = zb[e];
    __syncthreads();
    return;
  }
  const int b = NCMAX / 2;
  const int nblk = (d + b - 1) / b;
  for (int pass = 0; pass < MAX_SWEEPS; ++pass) {
    if (tid == 0) sm.nrot = 0;
    ++*sweeps;
    for (int A = 0; A < nblk; ++A) {
      const int na = min(b, d - A * b);
      const size_t ga = (size_t)A * b * K;
      for (int e = tid; e < na * K; e += NTH) zb[e] = Zm[ga + e];
      __syncthreads();
      jacobi_sweep<G>(sm, K, 0, na, rounds);
      for (int B = A + 1; B < nblk; ++B) {
        const int nb = min(b, d - B * b);
        const size_t gb = (size_t)B * b * K;
        for (int e = tid; e < nb * K; e += NTH) zb[b * K + e] = Zm[gb + e];
        __syncthreads();
        for (int s = 0; s < b; ++s) {
          ++*rounds;
          if (wid * (64 / G) < b) {
            const int qi = (slot + s) % b;
            const bool act = slot < na && qi < nb;
            jacobi_pair<G>(sm, K, slot, b + qi, act);
          }
          __syncthreads();
        }
        for (int e = tid; e < nb * K; e += NTH) Zm[gb + e] = zb[b * K + e];
        __syncthreads();
      }
      for (int e = tid; e < na * K; e += NTH) Zm[ga + e] = zb[e];
      __syncthreads();
    }
    const bool done = sm.nrot == 0;
    __syncthreads();
    if (done) break;
  }
}

// sigma_j^2 = ||z_j||^2 (FP64), their descending order, the smallest r whose
// leading sigma_j^2 reach Et (all d if rounding keeps the sum below it).
__device__ __forceinline__ void pick_rank_big(BigShared& sm, const float2* Zm, int K, int d, double Et, int* r_out,
                              double* cap_out, double* td_sig2) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int c = wid; c < d; c += NWV) {
    double v = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int i = lane + 64 * m;
      if (i < K) v += (double)cabs2(Zm[(size_t)c * K + i]);
    }
    v = wave_sum(v);
    if (lane == 0) sm.s2[c] = v;
  }
  __syncthreads();
  if (tid < d) {
    const double v = sm.s2[tid];
    int rank = 0;
    for (int k = 0; k < d; ++k) {
      const double w = sm.s2[k];
      rank += (w > v) || (w == v && k < tid);
    }
    sm.order[rank] = tid;
  }
  __syncthreads();
  if (tid == 0) {
    double cs = 0.0;
    int rr = d;
    for (int m = 0; m < d; ++m) {
      cs += sm.s2[sm.order[m]];
      if (cs >= Et) { rr = m + 1; break; }
    }
    sm.r = rr;
    sm.cap = cs;
  }
  __syncthreads();
  if (tid < d) td_sig2[tid] = sm.s2[sm.order[tid]];
  *r_out = sm.r;
  *cap_out = sm.cap;
  __syncthreads();
}

// ---------------------------------------------------- capacitance solve
// Gauss-Jordan with partial pivoting on the r x (r + K) FP64 system
// aug = [C | M] (row-major, ld ldg) so that its last K columns become
// C^-1 M.  Returns false (and leaves aug partly eliminated) if a pivot's
// modulus is not above SING_TOL (1 + ||C - I||_F) or is not finite.
__device__ __forceinline__ bool solve_capacitance(BigShared& sm, double2* aug, int r, int ldg) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  double2* gp = sm.u.gj.pan;
  double e2 = 0.0;
  for (int e = tid; e < r * r; e += NTH) {
    const int a = e / r, c = e - a * r;
    const double2 v = aug[(size_t)a * ldg + c];
    const double re = v.x - (a == c ? 1.0 : 0.0);
    e2 += re * re + v.y * v.y;
  }
  const double stol = SING_TOL * (1.0 + sqrt(block_sum(e2, sm.red)));
  if (tid == 0) sm.singular = 0;
  for (int j0 = 0; j0 < r; j0 += GJ_W) {
    const int nc = min(GJ_W, r - j0);
    for (int e = tid; e < r * GJ_W; e += NTH) {
      const int i = e / GJ_W, c = e - i * GJ_W;
      gp[e] = (c < nc) ? aug[(size_t)i * ldg + j0 + c] : dz();
    }
    __syncthreads();
    for (int k = 0; k < nc; ++k) {
      const int j = j0 + k;
      if (wid == 0) {
        // rows lane and lane + 64; the smallest row index holding the maximum modulus
        const double2 v0 = (lane < r) ? gp[lane * GJ_W + k] : dz();
        const double2 v1 = (lane + 64 < r) ? gp[(lane + 64) * GJ_W + k] : dz();
        const double m0 = (lane >= j && lane < r) ? dabs2(v0) : -1.0;
        const double m1 = (lane + 64 >= j && lane + 64 < r) ? dabs2(v1) : -1.0;
        double mx = fmax(m0, m1);
        mx = fmax(mx, dpp_d<DPP_QUAD_1032>(mx));
        mx = fmax(mx, dpp_d<DPP_QUAD_2301>(mx));
        mx = fmax(mx, dpp_d<DPP_ROW_ROR4>(mx));
        mx = fmax(mx, dpp_d<DPP_ROW_ROR8>(mx));
        mx = fmax(fmax(readlane_d(mx, 0), readlane_d(mx, 16)), fmax(readlane_d(mx, 32), readlane_d(mx, 48)));
        const unsigned long long h0 = __ballot(m0 == mx);
        const unsigned long long h1 = __ballot(m1 == mx);
        int prow = -1;
        if (h0) prow = __ffsll((long long)h0) - 1;
        else if (h1) prow = 64 + __ffsll((long long)h1) - 1;
        if (lane == 0) {
          if (prow < 0) {
            sm.pivrow[k] = j;
            sm.singular = 1;
          } else {
            sm.pivrow[k] = prow;
            if (!(sqrt(mx) > stol) || !isfinite(mx)) sm.singular = 1;
          }
        }
        if (prow >= 0) {
          const double2 pv = (prow < 64) ? v0 : v1;
          if (lane == (prow & 63)) sm.pivv[k] = pv;
        }
      }
      __syncthreads();
      if (sm.singular) return false;
      const int pr = sm.pivrow[k];
      const double2 piv = sm.pivv[k];
      // row exchange j <-> pr in panel columns k.., the normalised pivot row;
      // column k keeps the multipliers (row j: 1 / pivot)
      if (tid < nc - k) {
        const int c = k + tid;
        const double2 a = gp[j * GJ_W + c], bb = gp[pr * GJ_W + c];
        if (c == k) {
          gp[pr * GJ_W + k] = a;
          gp[j * GJ_W + k] = ddiv(make_double2(1.0, 0.0), piv);
        } else {
          const double2 u = ddiv(bb, piv);
          gp[pr * GJ_W + c] = a;
          gp[j * GJ_W + c] = u;
          sm.u.gj.ustash[c] = u;
        }
      }
      __syncthreads();
      const int w = nc - k - 1;
      for (int e = tid; e < r * w; e += NTH) {
        const int i = e / w, c = k + 1 + (e - i * w);
        if (i == j) continue;
        gp[i * GJ_W + c] = dsub(gp[i * GJ_W + c], dmul(gp[i * GJ_W + k], sm.u.gj.ustash[c]));
      }
      __syncthreads();
    }
    // replay the panel's exchanges and eliminations on every later column
    for (int c = j0 + nc + wid; c < ldg; c += NWV) {
      double2 x0 = (lane < r) ? aug[(size_t)lane * ldg + c] : dz();
      double2 x1 = (lane + 64 < r) ? aug[(size_t)(lane + 64) * ldg + c] : dz();
      for (int k = 0; k < nc; ++k) {
        const int j = j0 + k, pr = sm.pivrow[k];
        const double2 sj = (j < 64) ? x0 : x1;
        const double2 sp = (pr < 64) ? x0 : x1;
        const double2 vj = make_double2(readlane_d(sj.x, j & 63), readlane_d(sj.y, j & 63));
        const double2 vp = make_double2(readlane_d(sp.x, pr & 63), readlane_d(sp.y, pr & 63));
        const double2 u = dmul(vp, gp[j * GJ_W + k]);
        // row pr takes the old row j (then is eliminated like any other row)
        if (pr != j) {
          if (pr < 64) { if (lane == pr) x0 = vj; } else { if (lane == pr - 64) x1 = vj; }
        }
        if (lane < r) x0 = (lane == j) ? u : dsub(x0, dmul(gp[lane * GJ_W + k], u));
        if (lane + 64 < r) x1 = (lane + 64 == j) ? u : dsub(x1, dmul(gp[(lane + 64) * GJ_W + k], u));
      }
      if (lane < r) aug[(size_t)lane * ldg + c] = x0;
      if (lane + 64 < r) aug[(size_t)(lane + 64) * ldg + c] = x1;
    }
    __syncthreads();
  }
  return true;
}

template <bool MANY>
__global__ __launch_bounds__(NTH) void k_arsvd_big(ArsvdJob one, const ArsvdJob* many, int* err) {
  __shared__ BigShared sm;
  const ArsvdJob& jb = job_of<MANY>(one, many);
  GTrackDesc* __restrict__ td = (GTrackDesc*)jb.td;
  TrackDesc* const tdg = (TrackDesc*)td;    // the same, for whole-struct copies
  const int t = td->t_dev + 1, i_max = jb.i_max;
  const double eta = jb.eta;
  const int tid = threadIdx.x, wid = tid >> 6;
  const int K = td->K;
  float2* dA = td->dA;       // Delta A (+ R under error feedback, formed in place below)
  float2* Ym = td->Ym;
  float2* Qm = td->Qm;
  float2* Zm = td->Zm;

  const bool fb = td->error_feedback != 0;   // sketch Delta A + R
  double part = 0.0;
  for (int e = tid; e < K * K; e += NTH) {
    float2 v = dA[e];
    if (fb) {
      v = cadd(v, td->Rfb[e]);
      dA[e] = v;
    }
    part += (double)v.x * v.x + (double)v.y * v.y;
  }
  const double E = block_sum(part, sm.red);
  // a non-finite snapshot leaves the track's state as it was (the precoder
  // then keeps H_prev too)
  if (tid == 0) td->hold = isfinite(E) ? 0 : 1;
  if (!isfinite(E) || E == 0.0) {
    if (fb && E == 0.0)
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
  const long long r_begin = wall_clock64();
  long long c_mark = clock64();
  int k0 = td->k_init;
  if (td->kinit_policy == RZF_KINIT_WARM && td->last_r > k0) k0 = td->last_r;
  const int p = td->p;
  const uint64_t seed = td->seed, trk = td->track_id;
  const int ktl = (K + 15) / 16;

  int d = 0, iters = 0, r = 0, sweeps = 0, rounds = 0, qrcols = 0;
  double captured = 0.0;
  bool rotated = false;
  // the basis of the track's last full-width SVD, if it left one
  const bool warm_in = td->warm != 0;
  // Alg. 1's iteration `it` at width d: Q in Qm and Z = Delta A^H Q in Zm;
  // returns ||Z||_F^2
  auto sketch_iteration = [&](int it, int d) -> double {
    if (d == K && warm_in) {
      // At full width every unitary Q gives the same B = Q^H Delta A up to a
      // unitary factor, hence the same SVD, captured energy and U_r.  The
      // previous full-width basis replaces the sketch and its QR; it is close
      // to Delta A's singular vectors, so the Jacobi passes start nearly done.
      for (int e = tid; e < K * K; e += NTH) Qm[e] = td->Xw[e];
      __syncthreads();
      t_sk += clock64() - c_mark; c_mark = clock64();
    } else {
      // Y = Delta A Omega, one 16-column tile of Omega at a time
      for (int ct = 0; ct * 16 < d; ++ct) {
        const int j0 = 16 * ct;
        for (int e = tid; e < 16 * K; e += NTH) {
          const int jj = e / K, i = e - jj * K;
          sm.u.om[e] = (j0 + jj < d) ? sketch_entry(seed, trk, t, it, i, j0 + jj) : cz();
        }
        __syncthreads();
        for (int rt = wid; rt < ktl; rt += NWV) {
          floatx4 dr = zero4(), di = zero4();
          ctile16([&](int i, int k) {
                    const int row = rt * 16 + i;
                    return (row < K && k < K) ? dA[(size_t)row * K + k] : cz();
                  },
                  [&](int k, int jj) { return (k < K) ? sm.u.om[jj * K + k] : cz(); }, 0, up4(K), dr, di);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = rt * 16 + tile_row(v), c = j0 + tile_col();
            if (row < K && c < d) Ym[(size_t)c * K + row] = make_float2(dr[v], di[v]);
          }
        }
        __syncthreads();
      }
      t_sk += clock64() - c_mark; c_mark = clock64();
      qr_big(sm, Ym, Qm, K, d);
      qrcols += d;
    }
    // Z = Delta A^H Q = B^H and ||Z||_F^2 (Delta A + R need not be Hermitian)
    double zp = 0.0;
    const int dtl = (d + 15) / 16;
    for (int tt = wid; tt < ktl * dtl; tt += NWV) {
      const int ti = tt / dtl, tj = tt - ti * dtl;
      floatx4 dr = zero4(), di = zero4();
      ctile16([&](int i, int k) {
                const int row = ti * 16 + i;
                return (row < K && k < K) ? cconj(dA[(size_t)k * K + row]) : cz();
              },
              [&](int k, int jj) {
                const int c = tj * 16 + jj;
                return (k < K && c < d) ? Qm[(size_t)c * K + k] : cz();
              },
              0, up4(K), dr, di);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = ti * 16 + tile_row(v), c = tj * 16 + tile_col();
        if (row < K && c < d) {
          Zm[(size_t)c * K + row] = make_float2(dr[v], di[v]);
          zp += (double)dr[v] * dr[v] + (double)di[v] * di[v];
        }
      }
    }
    const double tot = block_sum(zp, sm.red);
    t_qr += clock64() - c_mark; c_mark = clock64();
    return tot;
  };
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
  // When the track's last step ended at d = K and left its basis, the
  // full-width iteration runs first.  Its sigma_1^2 >= ... >= sigma_K^2 are
  // Delta A's, and for any d orthonormal columns Q, ||Q^H Delta A||_F^2 <=
  // sigma_1^2 + ... + sigma_d^2 (Ky Fan).  So an earlier iteration whose d
  // leading sigma_j^2 miss the target cannot meet it: it is skipped, which
  // leaves Alg. 1's outcome as it is (the first iteration that meets the
  // target decides, with its own Q and Z).  The others run in order as
  // before; the full-width Z is kept aside (in the capacitance workspace,
  // unused until the branch) for when none of them meets the target.
  bool pre = kfull > 1 && warm_in && td->nsig == K && !td->early_fallback;
  int rk = 0, sweeps_k = 0, rounds_k = 0;
  double capk = 0.0;
  float2* const zstash = reinterpret_cast<float2*>(td->Aug);   // K x K fits in (K/2) x (3K/2) double2
  if (pre) {
    const double totk = sketch_iteration(kfull, K);
    if (totk >= Et) {
      if (K <= 128) jacobi_big<16>(sm, Zm, K, K, &sweeps_k, &rounds_k);
      else jacobi_big<32>(sm, Zm, K, K, &sweeps_k, &rounds_k);
      t_jac += clock64() - c_mark; c_mark = clock64();
      pick_rank_big(sm, Zm, K, K, Et, &rk, &capk, tdg->sig2);
      for (int e = tid; e < K * K; e += NTH) zstash[e] = Zm[e];
      if (tid < K) {
        sm.s2k[tid] = sm.s2[tid];
        sm.ordk[tid] = sm.order[tid];
      }
      if (tid == 0) {
        double c = 0.0;
        sm.topk[0] = 0.0;
        for (int jj = 0; jj < K; ++jj) {
          c += sm.s2[sm.order[jj]];
          sm.topk[jj + 1] = c;
        }
      }
      __syncthreads();
    } else {
      pre = false;   // (eta = 1 within rounding) the iterations in order
    }
  }
  for (int it = 1; it <= i_max; ++it) {
    iters = it;
    d = min(k0 + p, K);
    if (pre && it == kfull) {
      // no earlier iteration met the target: the full-width step (its Q is
      // the stored basis)
      for (int e = tid; e < K * K; e += NTH) {
        Zm[e] = zstash[e];
        Qm[e] = td->Xw[e];
      }
      if (tid < K) {
        sm.s2[tid] = sm.s2k[tid];
        sm.order[tid] = sm.ordk[tid];
        tdg->sig2[tid] = sm.s2k[sm.ordk[tid]];
      }
      __syncthreads();
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
      if (K <= 128) jacobi_big<16>(sm, Zm, K, d, &sweeps, &rounds);
      else jacobi_big<32>(sm, Zm, K, d, &sweeps, &rounds);
      t_jac += clock64() - c_mark; c_mark = clock64();
      rotated = true;
      pick_rank_big(sm, Zm, K, d, Et, &r, &captured, tdg->sig2);
      break;
    }
    // after the last iteration, or (early-fallback policy) once d is past
    // the Woodbury limit: every component, k_est = d, and the step inverts
    if (it == i_max || (td->early_fallback && d > td->wb_limit)) {
      r = d;
      captured = tot;
      break;
    }
    k0 = min(2 * k0, K);   // d = min(k0 + p, K) is unchanged by the cap
  }
  if (rotated && d == K) {
    // this full-width SVD's normalised columns z_j / sigma_j (norms in
    // sm.s2): the next full-width step's starting basis
    double smax = 0.0;
    for (int c = 0; c < K; ++c) smax = fmax(smax, sm.s2[c]);
    bool ok = smax > 0.0;
    for (int c = 0; c < K; ++c) ok = ok && sm.s2[c] > BASIS_MIN_REL * smax;
    __syncthreads();   // every read of the stored basis above is done
    if (ok)
      for (int e = tid; e < K * K; e += NTH) td->Xw[e] = cscale(Zm[e], (float)(1.0 / sqrt(sm.s2[e / K])));
    if (tid == 0) td->warm = ok ? 1 : 0;
  }
  if (!rotated) {
    if (tid < d) sm.order[tid] = tid;
    __syncthreads();
  }

  // Alg. 2's switch k_est <= switch * K, within the Woodbury workspace
  bool use_wb = r <= td->wb_limit;
  int path = use_wb ? RZF_PATH_WB : RZF_PATH_FULL_RANK;
  float2* Ainv = td->Ainv;
  float2* Pm = td->Pm;
  if (rotated && use_wb) {
    // U_r = Q U_hat_r = Q Q^H Delta A Z_r Sigma_r^-2 (B V_hat = U_hat Sigma
    // with V_hat = Z Sigma^-1): T1 = Delta A Z_r -> Pm, T2 = Q^H T1 -> Ym (the
    // reflectors are no longer needed), U -> Pm; every retained sigma_j > 0
    const int* ord = sm.order;
    const int rtl = (r + 15) / 16, dtl = (d + 15) / 16;
    for (int tt = wid; tt < ktl * rtl; tt += NWV) {
      const int ti = tt / rtl, tj = tt - ti * rtl;
      floatx4 dr = zero4(), di = zero4();
      ctile16([&](int i, int k) {
                const int row = ti * 16 + i;
                return (row < K && k < K) ? dA[(size_t)row * K + k] : cz();
              },
              [&](int k, int c) {
                const int cc = tj * 16 + c;
                return (k < K && cc < r) ? Zm[(size_t)ord[cc] * K + k] : cz();
              },
              0, up4(K), dr, di);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = ti * 16 + tile_row(v), c = tj * 16 + tile_col();
        if (row < K && c < r) Pm[(size_t)c * K + row] = make_float2(dr[v], di[v]);
      }
    }
    __syncthreads();
    for (int tt = wid; tt < dtl * rtl; tt += NWV) {
      const int ti = tt / rtl, tj = tt - ti * rtl;
      floatx4 dr = zero4(), di = zero4();
      ctile16([&](int i, int k) {
                const int j = ti * 16 + i;
                return (j < d && k < K) ? cconj(Qm[(size_t)j * K + k]) : cz();
              },
              [&](int k, int c) {
                const int cc = tj * 16 + c;
                return (k < K && cc < r) ? Pm[(size_t)cc * K + k] : cz();
              },
              0, up4(K), dr, di);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = ti * 16 + tile_row(v), c = tj * 16 + tile_col();
        if (j < d && c < r) Ym[(size_t)c * K + j] = make_float2(dr[v], di[v]);
      }
    }
    __syncthreads();
    for (int tt = wid; tt < ktl * rtl; tt += NWV) {
      const int ti = tt / rtl, tj = tt - ti * rtl;
      floatx4 dr = zero4(), di = zero4();
      ctile16([&](int i, int j) {
                const int row = ti * 16 + i;
                return (row < K && j < d) ? Qm[(size_t)j * K + row] : cz();
              },
              [&](int j, int c) {
                const int cc = tj * 16 + c;
                return (j < d && cc < r) ? Ym[(size_t)cc * K + j] : cz();
              },
              0, up4(d), dr, di);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = ti * 16 + tile_row(v), c = tj * 16 + tile_col();
        if (row < K && c < r) {
          const double s2 = sm.s2[ord[c]];
          Pm[(size_t)c * K + row] = make_float2((float)(dr[v] / s2), (float)(di[v] / s2));
        }
      }
    }
    __syncthreads();
  }
  // column c of U at Ub[c * K]: the rebuilt vectors, or Q itself (unrotated,
  // sm.order is the identity); P = A^-1 U goes to Ym
  const float2* Ub = rotated ? Pm : Qm;
  float2* Pw = Ym;
  if (fb && use_wb) {
    // residual of the rank-r update: R = (Delta A + R) - U V~^H (a direct
    // inversion clears R below)
    const int* ord = sm.order;
    float2* R = td->Rfb;
    for (int tt = wid; tt < ktl * ktl; tt += NWV) {
      const int ti = tt / ktl, tj = tt - ti * ktl;
      floatx4 dr = zero4(), di = zero4();
      ctile16([&](int i, int c) {
                const int row = ti * 16 + i;
                return (row < K && c < r) ? Ub[(size_t)c * K + row] : cz();
              },
              [&](int c, int j) {
                const int col = tj * 16 + j;
                return (c < r && col < K) ? cconj(Zm[(size_t)ord[c] * K + col]) : cz();
              },
              0, up4(r), dr, di);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = ti * 16 + tile_row(v), col = tj * 16 + tile_col();
        if (row < K && col < K)
          R[(size_t)row * K + col] = csub(dA[(size_t)row * K + col], make_float2(dr[v], di[v]));
      }
    }
    __syncthreads();
  }
  if (use_wb) {
    const int* ord = sm.order;
    double2* aug = td->Aug;
    const int rtl = (r + 15) / 16;
    // step 1: P = A^-1 U
    for (int tt = wid; tt < ktl * rtl; tt += NWV) {
      const int ti = tt / rtl, tj = tt - ti * rtl;
      floatx4 dr = zero4(), di = zero4();
      ctile16([&](int i, int k) {
                const int row = ti * 16 + i;
                return (row < K && k < K) ? Ainv[(size_t)row * K + k] : cz();
              },
              [&](int k, int c) {
                const int cc = tj * 16 + c;
                return (k < K && cc < r) ? Ub[(size_t)cc * K + k] : cz();
              },
              0, up4(K), dr, di);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = ti * 16 + tile_row(v), c = tj * 16 + tile_col();
        if (row < K && c < r) Pw[(size_t)c * K + row] = make_float2(dr[v], di[v]);
      }
    }
    __syncthreads();
    // step 2: [C | M] = [I + V~^H P | V~^H A^-1] in FP64
    const int ldg = r + K;
    for (int tt = wid; tt < rtl * (rtl + ktl); tt += NWV) {
      const int ti = tt / (rtl + ktl), tj = tt - ti * (rtl + ktl);
      const bool ct = tj < rtl;
      floatx4 dr = zero4(), di = zero4();
      auto la = [&](int i, int k) {
        const int a = ti * 16 + i;
        return (a < r && k < K) ? cconj(Zm[(size_t)ord[a] * K + k]) : cz();
      };
      if (ct)
        ctile16(la, [&](int k, int c) {
                  const int b = tj * 16 + c;
                  return (k < K && b < r) ? Pw[(size_t)b * K + k] : cz();
                }, 0, up4(K), dr, di);
      else
        ctile16(la, [&](int k, int c) {
                  const int j = (tj - rtl) * 16 + c;
                  return (k < K && j < K) ? Ainv[(size_t)k * K + j] : cz();
                }, 0, up4(K), dr, di);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = ti * 16 + tile_row(v);
        if (a >= r) continue;
        if (ct) {
          const int c = tj * 16 + tile_col();
          if (c < r) aug[(size_t)a * ldg + c] = make_double2((a == c ? 1.0 : 0.0) + (double)dr[v], (double)di[v]);
        } else {
          const int j = (tj - rtl) * 16 + tile_col();
          if (j < K) aug[(size_t)a * ldg + r + j] = make_double2((double)dr[v], (double)di[v]);
        }
      }
    }
    __syncthreads();
    // step 3: X = C^-1 (V~^H A^-1)
    if (!solve_capacitance(sm, aug, r, ldg)) {
      use_wb = false;
      path = RZF_PATH_FULL_SINGULAR;
    } else {
      // steps 4-5: A^-1 <- A^-1 - P X (each wave rewrites its own tiles)
      for (int tt = wid; tt < ktl * ktl; tt += NWV) {
        const int ti = tt / ktl, tj = tt - ti * ktl;
        floatx4 dr = zero4(), di = zero4();
        ctile16([&](int i, int a) {
                  const int row = ti * 16 + i;
                  return (row < K && a < r) ? Pw[(size_t)a * K + row] : cz();
                },
                [&](int a, int c) {
                  const int j = tj * 16 + c;
                  return (a < r && j < K) ? d2f(aug[(size_t)a * ldg + r + j]) : cz();
                },
                0, up4(r), dr, di);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = ti * 16 + tile_row(v), j = tj * 16 + tile_col();
          if (row < K && j < K) {
            float2* q = Ainv + (size_t)row * K + j;
            *q = csub(*q, make_float2(dr[v], di[v]));
          }
        }
      }
    }
    __syncthreads();
  }
  if (!use_wb) {
    if (tid == 0) sm.bad = 0;
    if (fb)
      for (int e = tid; e < K * K; e += NTH) td->Rfb[e] = cz();
    for (int e = tid; e < K * K; e += NTH) Ainv[e] = td->Anew[e];
    __syncthreads();
    gj_inverse_hpd_blocked<float2>(Ainv, K, K, sm.u.inv.xs, sm.u.inv.cs, sm.u.inv.pb, &sm.bad);
    if (tid == 0 && sm.bad) atomicCAS(err, 0, sm.bad == 2 ? DEV_ERR_NONFINITE : DEV_ERR_NOT_HPD);
  }
  if (tid == 0) {
    td->info.r = r; td->info.iters = iters; td->info.path = path; td->info.d = d;
    td->info.dA_fro2 = E; td->info.captured = captured;
    if (jb.out) *jb.out = tdg->info;
    td->last_r = r;
    td->dbg[0] = sweeps; td->dbg[1] = rounds; td->dbg[2] = qrcols;
    td->nsig = rotated ? d : 0;
    t_wb = clock64() - c_mark;
    td->dbg[3] = (int)t_sk; td->dbg[4] = (int)t_qr; td->dbg[5] = (int)t_jac; td->dbg[6] = (int)t_wb;
    td->dbg[7] = (int)(wall_clock64() - r_begin);
  }
}

// FP64 inverse of the init / reset Gram matrix for a large track, in place
// in the FP64 buffer, rounded to the FP32 state.
template <bool MANY>
__global__ __launch_bounds__(NTH) void k_inv64_big(Inv64Job one, const Inv64Job* many, int* err) {
  __shared__ double2 xs[16 * KM], cs[KM * 16], pb[2 * 256];
  __shared__ int bad;
  const Inv64Job& jb = job_of<MANY>(one, many);
  const int K = jb.K;
  double2* A = const_cast<double2*>(jb.A);
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  gj_inverse_hpd_blocked<double2>(A, K, K, xs, cs, pb, &bad);
  // a reset that fails keeps the track's state (rzf_init discards the track)
  const bool keep = bad && jb.hold;
  if (!keep)
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
      jb.Ainv[e] = d2f(A[e]);
      if (jb.zero) jb.zero[e] = cz();
    }
  if (threadIdx.x == 0) {
    if (bad) atomicCAS(err, 0, bad == 2 ? DEV_ERR_NONFINITE : DEV_ERR_NOT_HPD);
    if (jb.hold) *jb.hold = bad ? 1 : 0;
    DevInfo rec;
    rec.r = 0; rec.iters = 0; rec.path = keep ? RZF_PATH_NOOP : RZF_PATH_RESET; rec.d = 0;
    rec.dA_fro2 = keep ? __builtin_nan("") : 0.0; rec.captured = 0.0;
    if (jb.info) *jb.info = rec;
    if (jb.out) *jb.out = rec;
  }
}

// FP32 inverse for rzf_full on a large track: A is copied to Ainv (unless
// they alias) and inverted there in place.
template <bool MANY>
__global__ __launch_bounds__(NTH) void k_inv32_big(Inv32Job one, const Inv32Job* many, int* err) {
  __shared__ float2 xs[16 * KM], cs[KM * 16], pb[2 * 256];
  __shared__ int bad;
  const Inv32Job& jb = job_of<MANY>(one, many);
  const int K = jb.K;
  float2* Ainv = jb.Ainv;
  if (threadIdx.x == 0) bad = 0;
  if (jb.A != Ainv)
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) Ainv[e] = jb.A[e];
  __syncthreads();
  gj_inverse_hpd_blocked<float2>(Ainv, K, K, xs, cs, pb, &bad);
  if (threadIdx.x == 0 && bad && err) atomicCAS(err, 0, bad == 2 ? DEV_ERR_NONFINITE : DEV_ERR_NOT_HPD);
}

}  // namespace

void launch_arsvd_big(const ArsvdJob& one, const ArsvdJob* many, int n, int* err, hipStream_t s) {
  if (many) k_arsvd_big<true><<<dim3(1, n), NTH, 0, s>>>(one, many, err);
  else k_arsvd_big<false><<<1, NTH, 0, s>>>(one, many, err);
}

void launch_inv64_big(const Inv64Job& one, const Inv64Job* many, int n, int* err, hipStream_t s) {
  if (many) k_inv64_big<true><<<dim3(1, n), NTH, 0, s>>>(one, many, err);
  else k_inv64_big<false><<<1, NTH, 0, s>>>(one, many, err);
}

void launch_inv32_big(const Inv32Job& one, const Inv32Job* many, int n, int* err, hipStream_t s) {
  if (many) k_inv32_big<true><<<dim3(1, n), NTH, 0, s>>>(one, many, err);
  else k_inv32_big<false><<<1, NTH, 0, s>>>(one, many, err);
}
