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
//   Z      = Delta A Q                        (matrix cores)
//   SVD    B = Q^H Delta A = Z^H by one-sided (Hestenes) Jacobi on the
//          columns of Z; every rotation is applied to the columns of Q as
//          well, so at convergence z_j = sigma_j v_j and q_j = (Q U_hat)_j.
//          Hence U_r Sigma_r V_r^H = sum_{j<=r} q_j z_j^H needs no division
//          by sigma.
//   r      smallest with sum_{j<=r} sigma_j^2 >= eta ||Delta A||_F^2 (eq. (14));
//          none: k0 <- 2 k0 and repeat; after I_max iterations r = d.
//
// Woodbury (Sec. III-A, steps 1-5) in the equivalent scaled form with
// U = [q_j], V~ = [z_j] (V~ = V_r Sigma_r):
//   P  = A^-1 U                (step 1)
//   C  = I_r + V~^H P          (step 2; Sigma_r (Sigma_r^-1 + V_r^H A^-1 U_r))
//   X  = C^-1 (V~^H A^-1)      (step 3, FP64 Gauss-Jordan with partial pivoting)
//   A^-1 <- A^-1 - P X         (steps 4-5)
// C is nonsingular exactly when the capacitance of eq. (12) is; a pivot below
// SING_TOL sends the step to direct inversion (path FULL_SINGULAR).
#include "dense_device.h"
#include "rzf_internal.h"

namespace {

constexpr int NTH = 1024;
constexpr int NWV = NTH / 64;
constexpr int MAX_SWEEPS = 30;
constexpr double JACOBI_TOL = 2e-6;
constexpr double SING_TOL = 1e-12;

struct Shared {
  float2 b0[KM * KM];            // Delta A (row-major, ld KM); later A^-1 or A'
  float2 b1[KM * KM];            // column-major K x d: Omega, then Q
  float2 b2[KM * KM];            // column-major K x d: Y / reflectors, then Z
  float2 pm[KM * WB_RMAX];       // P = A^-1 U, column-major
  double s2[KM];                 // ||z_j||^2
  double colj[WB_RMAX];          // Gauss-Jordan: column j before the swap
  double2 ustash[WB_RMAX + KM];  // Gauss-Jordan: normalised pivot row
  double red[NWV];
  int order[KM];
  int nrot, r, found, piv_row, singular, bad;
  double pivr, pivi;
};

// Column pair (p, q) of round k, slot m, of the round-robin ordering over n
// (even) columns: every pair meets once in n-1 rounds.
__device__ __forceinline__ void rr_pair(int k, int m, int n, int* p, int* q) {
  if (m == 0) { *p = k; *q = n - 1; return; }
  const int n1 = n - 1;
  *p = (k + m) % n1;
  *q = (k - m + n1) % n1;
}

// Wave-level Householder vector of column c (rows >= c) of the column-major
// matrix `a`; writes the unit vector w (zero above row c) over that column.
__device__ void reflector(float2* a, int c, int K) {
  const int lane = threadIdx.x & 63;
  float2 x = (lane < K && lane >= c) ? a[c * KM + lane] : cz();
  const double s = wave_sum((double)cabs2(x));
  const float ax = __shfl(x.x, c, 64), ay = __shfl(x.y, c, 64);
  float2 w = cz();
  if (s > 0.0) {
    const double nx = sqrt(s);
    const double aa = sqrt((double)ax * ax + (double)ay * ay);
    double ph_r = 1.0, ph_i = 0.0;
    if (aa > 0.0) { ph_r = ax / aa; ph_i = ay / aa; }
    const double wn = sqrt(2.0 * nx * (nx + aa));       // ||x - beta e_c||
    if (lane == c) {
      w = make_float2((float)(ph_r * (aa + nx) / wn), (float)(ph_i * (aa + nx) / wn));
    } else {
      w = make_float2((float)(x.x / wn), (float)(x.y / wn));
    }
  }
  if (lane < K) a[c * KM + lane] = (lane >= c) ? w : cz();
}

// y <- (I - 2 w w^H) y for column y of `a` and reflector column wc of `wsrc`.
__device__ __forceinline__ void apply_reflector(const float2* wsrc, int wc, float2* a, int c, int K) {
  const int lane = threadIdx.x & 63;
  const float2 w = (lane < K) ? wsrc[wc * KM + lane] : cz();
  float2 y = (lane < K) ? a[c * KM + lane] : cz();
  double dr = (double)w.x * y.x + (double)w.y * y.y;     // conj(w) y
  double di = (double)w.x * y.y - (double)w.y * y.x;
  dr = wave_sum(dr);
  di = wave_sum(di);
  const float fr = (float)(2.0 * dr), fi = (float)(2.0 * di);
  y.x -= w.x * fr - w.y * fi;
  y.y -= w.x * fi + w.y * fr;
  if (lane < K) a[c * KM + lane] = y;
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

__global__ __launch_bounds__(NTH) void k_arsvd_wb(TrackDesc* __restrict__ td, int t, double eta,
                                                  int i_max, int* err) {
  __shared__ Shared sm;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int K = td->K;
  float2* b0 = sm.b0;
  float2* b1 = sm.b1;
  float2* b2 = sm.b2;

  // Delta A -> LDS, E = ||Delta A||_F^2 in FP64
  double part = 0.0;
  for (int e = tid; e < K * K; e += NTH) {
    const int i = e / K, j = e - i * K;
    const float2 v = td->dA[e];
    b0[i * KM + j] = v;
    part += (double)v.x * v.x + (double)v.y * v.y;
  }
  const double E = block_sum(part, sm.red);
  if (!isfinite(E)) {
    if (tid == 0) {
      atomicCAS(err, 0, DEV_ERR_NONFINITE);
      td->info.r = 0; td->info.iters = 0; td->info.path = RZF_PATH_NOOP; td->info.d = 0;
      td->info.dA_fro2 = E; td->info.captured = 0.0;
    }
    return;
  }
  if (E == 0.0) {
    if (tid == 0) {
      td->info.r = 0; td->info.iters = 0; td->info.path = RZF_PATH_NOOP; td->info.d = 0;
      td->info.dA_fro2 = 0.0; td->info.captured = 0.0;
      td->last_r = 0;
    }
    return;
  }
  const double Et = eta * E;
  int k0 = td->k_init;
  if (td->kinit_policy == RZF_KINIT_WARM && td->last_r > k0) k0 = td->last_r;
  const int p = td->p;
  const uint64_t seed = td->seed, trk = td->track_id;

  int d = 0, iters = 0, r = 0;
  double captured = 0.0;
  bool found = false;
  for (int it = 1; it <= i_max; ++it) {
    iters = it;
    d = min(k0 + p, K);
    // Omega -> b1 (column-major)
    for (int e = tid; e < K * d; e += NTH) {
      const int j = e / K, i = e - j * K;
      b1[j * KM + i] = sketch_entry(seed, trk, t, it, i, j);
    }
    __syncthreads();
    // Y = Delta A Omega -> b2
    lds_gemm(K, d, K,
             [&](int i, int k) { return (i < K && k < K) ? b0[i * KM + k] : cz(); },
             [&](int k, int j) { return (k < K && j < d) ? b1[j * KM + k] : cz(); },
             [&](int i, int j, float2 v) { b2[j * KM + i] = v; });
    __syncthreads();
    // Householder QR of Y (b2): reflector j lands in column j of b2
    if (wid == 0) reflector(b2, 0, K);
    for (int j = 0; j < d; ++j) {
      __syncthreads();
      for (int c = j + 1 + wid; c < d; c += NWV) {
        apply_reflector(b2, j, b2, c, K);
        if (c == j + 1) reflector(b2, c, K);
      }
    }
    // Q = H_0 ... H_{d-1} [I_d; 0] -> b1
    for (int e = tid; e < d * KM; e += NTH) {
      const int j = e / KM, i = e - j * KM;
      b1[e] = (i == j) ? make_float2(1.f, 0.f) : cz();
    }
    for (int j = d - 1; j >= 0; --j) {
      __syncthreads();
      for (int c = j + wid; c < d; c += NWV) apply_reflector(b2, j, b1, c, K);
    }
    __syncthreads();
    // Z = Delta A Q -> b2
    lds_gemm(K, d, K,
             [&](int i, int k) { return (i < K && k < K) ? b0[i * KM + k] : cz(); },
             [&](int k, int j) { return (k < K && j < d) ? b1[j * KM + k] : cz(); },
             [&](int i, int j, float2 v) { b2[j * KM + i] = v; });
    // One-sided Jacobi on the columns of Z, rotating Q alongside
    const int n = d + (d & 1);
    for (int sweep = 0; sweep < MAX_SWEEPS; ++sweep) {
      if (tid == 0) sm.nrot = 0;
      __syncthreads();
      for (int k = 0; k < n - 1; ++k) {
        for (int m = wid; m < n / 2; m += NWV) {
          int pp, qq;
          rr_pair(k, m, n, &pp, &qq);
          if (pp >= d || qq >= d) continue;
          float2 zp = (lane < K) ? b2[pp * KM + lane] : cz();
          float2 zq = (lane < K) ? b2[qq * KM + lane] : cz();
          const double al = wave_sum((double)cabs2(zp));
          const double be = wave_sum((double)cabs2(zq));
          const double gr = wave_sum((double)zp.x * zq.x + (double)zp.y * zq.y);
          const double gi = wave_sum((double)zp.x * zq.y - (double)zp.y * zq.x);
          const double g = sqrt(gr * gr + gi * gi);
          if (g > 0.0 && g > JACOBI_TOL * sqrt(al * be)) {
            const double zeta = (be - al) / (2.0 * g);
            const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double cs = 1.0 / sqrt(1.0 + tt * tt);
            const float c = (float)cs, s = (float)(cs * tt);
            const float2 e = make_float2((float)(gr / g), (float)(-gi / g));   // conj(gamma)/|gamma|
            float2 qp = (lane < K) ? b1[pp * KM + lane] : cz();
            float2 qv = (lane < K) ? b1[qq * KM + lane] : cz();
            const float2 zq2 = cmul(e, zq), qv2 = cmul(e, qv);
            const float2 nzp = csub(cscale(zp, c), cscale(zq2, s));
            const float2 nzq = cadd(cscale(zp, s), cscale(zq2, c));
            const float2 nqp = csub(cscale(qp, c), cscale(qv2, s));
            const float2 nqq = cadd(cscale(qp, s), cscale(qv2, c));
            if (lane < K) {
              b2[pp * KM + lane] = nzp; b2[qq * KM + lane] = nzq;
              b1[pp * KM + lane] = nqp; b1[qq * KM + lane] = nqq;
            }
            if (lane == 0) sm.nrot = 1;
          }
        }
        __syncthreads();
      }
      const bool done = (sm.nrot == 0);
      __syncthreads();
      if (done) break;
    }
    // sigma_j^2 = ||z_j||^2, descending order, smallest r meeting the target
    for (int j = wid; j < d; j += NWV) {
      const float2 z = (lane < K) ? b2[j * KM + lane] : cz();
      const double v = wave_sum((double)cabs2(z));
      if (lane == 0) sm.s2[j] = v;
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
      int rr = 0;
      for (int m = 0; m < d; ++m) {
        cs += sm.s2[sm.order[m]];
        if (cs >= Et) { rr = m + 1; break; }
      }
      sm.found = rr > 0;
      sm.r = rr > 0 ? rr : d;
      // retained energy of the returned components
      double cap = 0.0;
      for (int m = 0; m < sm.r; ++m) cap += sm.s2[sm.order[m]];
      sm.red[0] = cap;
    }
    __syncthreads();
    found = sm.found != 0;
    r = sm.r;
    captured = sm.red[0];
    __syncthreads();
    if (found) break;
    k0 *= 2;
  }

  int rmax = (int)floor(td->switch_ratio * (double)K);
  bool use_wb = r <= rmax && r <= WB_RMAX;
  int path = use_wb ? RZF_PATH_WB : RZF_PATH_FULL_RANK;

  if (use_wb) {
    // A^-1 -> b0
    for (int e = tid; e < K * K; e += NTH) {
      const int i = e / K, j = e - i * K;
      b0[i * KM + j] = td->Ainv[e];
    }
    __syncthreads();
    const int* ord = sm.order;
    float2* pm = sm.pm;
    // step 1: P = A^-1 U
    lds_gemm(K, r, K,
             [&](int i, int k) { return (i < K && k < K) ? b0[i * KM + k] : cz(); },
             [&](int k, int c) { return (k < K && c < r) ? b1[ord[c] * KM + k] : cz(); },
             [&](int i, int c, float2 v) { pm[c * KM + i] = v; });
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
        return (a < r && k < K) ? cconj(b2[ord[a] * KM + k]) : cz();
      };
      auto lbc = [&](int k, int cc) {
        const int b = my_tj * 16 + cc;
        return (k < K && b < r) ? pm[b * KM + k] : cz();
      };
      auto lbq = [&](int k, int cc) {
        const int j = my_tj * 16 + cc;
        return (k < K && j < K) ? b0[k * KM + j] : cz();
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
    if (tid == 0) sm.singular = 0;
    __syncthreads();
    // step 3: Gauss-Jordan with partial pivoting on [C | V~^H A^-1]
    for (int j = 0; j < r; ++j) {
      if (wid == 0) {
        const double2 v = (lane < r) ? aug[lane * ldg + j] : dz();
        double mag = (lane >= j && lane < r) ? dabs2(v) : -1.0;
        int idx = lane;
        for (int off = 32; off > 0; off >>= 1) {
          const double om = __shfl_xor(mag, off, 64);
          const int oi = __shfl_xor(idx, off, 64);
          if (om > mag || (om == mag && oi < idx)) { mag = om; idx = oi; }
        }
        if (lane < r) sm.colj[lane] = 0.0;   // placeholder, real values below
        if (lane == 0) {
          sm.piv_row = idx;
          if (!(sqrt(mag) > SING_TOL) || !isfinite(mag)) sm.singular = 1;
        }
        if (lane == idx) { sm.pivr = v.x; sm.pivi = v.y; }
      }
      __syncthreads();
      if (sm.singular) break;
      const int pr = sm.piv_row;
      const double2 piv = make_double2(sm.pivr, sm.pivi);
      // multipliers of the rows after the swap, from the column before it
      double2 fj = dz();
      if (tid < r) {
        const int src = (tid == j) ? pr : (tid == pr ? j : tid);
        fj = aug[src * ldg + j];
      }
      __syncthreads();
      double2* fcol = reinterpret_cast<double2*>(sm.s2);   // r <= 32 entries
      if (tid < r) fcol[tid] = fj;
      for (int c = j + tid; c < ldg; c += NTH) {
        const double2 a = aug[j * ldg + c], b = aug[pr * ldg + c];
        const double2 u = ddiv(b, piv);
        aug[pr * ldg + c] = a;
        aug[j * ldg + c] = u;
        sm.ustash[c] = u;
      }
      __syncthreads();
      const int w = ldg - j - 1;
      for (int e = tid; e < r * w; e += NTH) {
        const int i = e / w, c = j + 1 + (e - i * w);
        if (i == j) continue;
        aug[i * ldg + c] = dsub(aug[i * ldg + c], dmul(fcol[i], sm.ustash[c]));
      }
      __syncthreads();
    }
    if (sm.singular) {
      use_wb = false;
      path = RZF_PATH_FULL_SINGULAR;
    } else {
      // steps 4-5: A^-1 <- A^-1 - P X
      float2* out = td->Ainv;
      lds_gemm(K, K, r,
               [&](int i, int a) { return (i < K && a < r) ? pm[a * KM + i] : cz(); },
               [&](int a, int j) { return (a < r && j < K) ? d2f(aug[a * ldg + r + j]) : cz(); },
               [&](int i, int j, float2 v) { out[(size_t)i * K + j] = csub(b0[i * KM + j], v); });
    }
    __syncthreads();
  }
  if (!use_wb) {
    // direct inversion of A' (FP32)
    if (tid == 0) sm.bad = 0;
    for (int e = tid; e < K * K; e += NTH) {
      const int i = e / K, j = e - i * K;
      b0[i * KM + j] = td->Anew[e];
    }
    __syncthreads();
    float2* res = gj_inverse_hpd<float2>(b0, b1, K, KM, &sm.bad);
    for (int e = tid; e < K * K; e += NTH) {
      const int i = e / K, j = e - i * K;
      td->Ainv[e] = res[i * KM + j];
    }
    if (tid == 0 && sm.bad) atomicCAS(err, 0, sm.bad == 2 ? DEV_ERR_NONFINITE : DEV_ERR_NOT_HPD);
  }
  if (tid == 0) {
    td->info.r = r; td->info.iters = iters; td->info.path = path; td->info.d = d;
    td->info.dA_fro2 = E; td->info.captured = captured;
    td->last_r = r;
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

void launch_arsvd_wb(TrackDesc* td, int K, int t, double eta, int i_max, int* err, hipStream_t s) {
  (void)K;
  k_arsvd_wb<<<1, NTH, 0, s>>>(td, t, eta, i_max, err);
}

void launch_debug_sketch(uint64_t seed, uint64_t track, int t, int it, int K, int d, float2* Omega,
                         uint64_t* words, hipStream_t s) {
  const int n = K * d;
  k_debug_sketch<<<(n + 255) / 256, 256, 0, s>>>(seed, track, t, it, K, d, Omega, words);
}
