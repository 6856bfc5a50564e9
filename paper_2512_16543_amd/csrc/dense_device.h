// Workgroup-level dense kernels: Gauss-Jordan inverses of HPD matrices and
// the round-robin pair ordering of the Jacobi sweeps.
#pragma once

#include "rzf_device.h"

// Column pair (p, q) of round k, slot m, of the round-robin ordering over n
// (even) columns: every pair meets once in n-1 rounds.
// With 0 <= k < n-1 and 0 < m < n/2 both sums stay within one period, so a
// conditional add or subtract replaces the modulo (an integer division is
// dozens of VALU instructions).
__device__ __forceinline__ void rr_pair(int k, int m, int n, int* p, int* q) {
  if (m == 0) { *p = k; *q = n - 1; return; }
  const int n1 = n - 1;
  int a = k + m, b = k - m;
  if (a >= n1) a -= n1;
  if (b < 0) b += n1;
  *p = a;
  *q = b;
}

template <class T> struct CX;
template <> struct CX<float2> {
  static __device__ __forceinline__ float2 zero() { return make_float2(0.f, 0.f); }
  static __device__ __forceinline__ float2 one() { return make_float2(1.f, 0.f); }
  static __device__ __forceinline__ float2 add(float2 a, float2 b) { return cadd(a, b); }
  static __device__ __forceinline__ float2 mul(float2 a, float2 b) { return cmul(a, b); }
  static __device__ __forceinline__ float2 sub(float2 a, float2 b) { return csub(a, b); }
  static __device__ __forceinline__ float2 neg(float2 a) { return make_float2(-a.x, -a.y); }
  static __device__ __forceinline__ float2 inv(float2 a) {
    const float d = 1.0f / (a.x * a.x + a.y * a.y);
    return make_float2(a.x * d, -a.y * d);
  }
  static __device__ __forceinline__ double re(float2 a) { return (double)a.x; }
  static __device__ __forceinline__ bool finite(float2 a) { return isfinite(a.x) && isfinite(a.y); }
};
template <> struct CX<double2> {
  static __device__ __forceinline__ double2 zero() { return make_double2(0.0, 0.0); }
  static __device__ __forceinline__ double2 one() { return make_double2(1.0, 0.0); }
  static __device__ __forceinline__ double2 add(double2 a, double2 b) { return dadd(a, b); }
  static __device__ __forceinline__ double2 mul(double2 a, double2 b) { return dmul(a, b); }
  static __device__ __forceinline__ double2 sub(double2 a, double2 b) { return dsub(a, b); }
  static __device__ __forceinline__ double2 neg(double2 a) { return make_double2(-a.x, -a.y); }
  static __device__ __forceinline__ double2 inv(double2 a) {
    const double d = 1.0 / (a.x * a.x + a.y * a.y);
    return make_double2(a.x * d, -a.y * d);
  }
  static __device__ __forceinline__ double re(double2 a) { return a.x; }
  static __device__ __forceinline__ bool finite(double2 a) { return isfinite(a.x) && isfinite(a.y); }
};

// Inverse of a Hermitian positive definite K x K matrix (K <= 64) by
// Gauss-Jordan exchange steps on BS x BS pivot blocks, without pivoting: the
// principal blocks of an HPD matrix and of its Schur complements are HPD.
// With P the pivot block and R the remaining indices one step maps
//   a_PP -> P^-1,  a_PR -> P^-1 a_PR,  a_RP -> -a_RP P^-1,
//   a_RR -> a_RR - a_RP P^-1 a_PR,
// and after sweeping every block the matrix holds A^-1.  P^-1 is formed in
// registers by every thread (scalar exchange steps), so a step costs
// one barrier: it reads buffer `a` and writes buffer `b`.  Thread layout: the
// thread owns column j = tid % 64 and rows tid/64 + 16 m, m = 0..3; the block
// must have 1024 threads.  `a` holds A on entry (leading dimension ld).
// Returns the buffer holding A^-1.  *bad (LDS) becomes nonzero if a scalar
// pivot is not a positive finite number (1: not HPD, 2: non-finite).
template <class T, int BS = 4>
__device__ T* gj_inverse_hpd(T* a, T* b, int K, int ld, int* bad) {
  typedef CX<T> C;
  const int j = threadIdx.x & 63, r0 = threadIdx.x >> 6;
  for (int k0 = 0; k0 < K; k0 += BS) {
    const int bs = min(BS, K - k0);
    T p[BS][BS];
#pragma unroll
    for (int u = 0; u < BS; ++u)
#pragma unroll
      for (int v = 0; v < BS; ++v)
        p[u][v] = (u < bs && v < bs) ? a[(k0 + u) * ld + k0 + v] : (u == v ? C::one() : C::zero());
    bool ok = true, fin = true;
#pragma unroll
    for (int q = 0; q < BS; ++q) {
      const T piv = p[q][q];
      fin = fin && C::finite(piv);
      ok = ok && (C::re(piv) > 0.0);
      const T ip = C::inv(piv);
      // in place: trailing entries first (they read the old row/column q)
#pragma unroll
      for (int u = 0; u < BS; ++u)
#pragma unroll
        for (int v = 0; v < BS; ++v)
          if (u != q && v != q) p[u][v] = C::sub(p[u][v], C::mul(C::mul(p[u][q], ip), p[q][v]));
#pragma unroll
      for (int v = 0; v < BS; ++v)
        if (v != q) p[q][v] = C::mul(p[q][v], ip);
#pragma unroll
      for (int u = 0; u < BS; ++u)
        if (u != q) p[u][q] = C::neg(C::mul(p[u][q], ip));
      p[q][q] = ip;
    }
    if (threadIdx.x == 0) {
      if (!fin) *bad = 2;
      else if (!ok && *bad == 0) *bad = 1;
    }
    if (j < K) {
      const bool jP = j >= k0 && j < k0 + bs;
      const int jj = j - k0;
      // x = P^-1 a_Pj for a column outside the block; for a column inside it,
      // pc = column jj of P^-1 (selects keep the arrays in registers)
      T x[BS], pc[BS];
#pragma unroll
      for (int u = 0; u < BS; ++u) {
        T c = C::zero();
#pragma unroll
        for (int v = 0; v < BS; ++v)
          if (v == jj) c = p[u][v];
        pc[u] = c;
      }
      {
        T col[BS];
#pragma unroll
        for (int u = 0; u < BS; ++u) col[u] = (!jP && u < bs) ? a[(k0 + u) * ld + j] : C::zero();
#pragma unroll
        for (int u = 0; u < BS; ++u) {
          T s = C::zero();
#pragma unroll
          for (int v = 0; v < BS; ++v) s = C::add(s, C::mul(p[u][v], col[v]));
          x[u] = s;
        }
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int i = r0 + 16 * m;
        if (i >= K) continue;
        const bool iP = i >= k0 && i < k0 + bs;
        const int ii = i - k0;
        T v;
        if (iP) {
          T sel = C::zero();
#pragma unroll
          for (int u = 0; u < BS; ++u)
            if (u == ii) sel = jP ? pc[u] : x[u];
          v = sel;
        } else {
          T row[BS];
#pragma unroll
          for (int u = 0; u < BS; ++u) row[u] = (u < bs) ? a[i * ld + k0 + u] : C::zero();
          if (jP) {
            T s = C::zero();
#pragma unroll
            for (int u = 0; u < BS; ++u) s = C::add(s, C::mul(row[u], pc[u]));
            v = C::neg(s);
          } else {
            T s = a[i * ld + j];
#pragma unroll
            for (int u = 0; u < BS; ++u) s = C::sub(s, C::mul(row[u], x[u]));
            v = s;
          }
        }
        b[i * ld + j] = v;
      }
    }
    __syncthreads();
    T* t = a; a = b; b = t;
  }
  return a;
}

// Lane moves of one complex value (FP32 or FP64 parts).
__device__ __forceinline__ float2 lane_read(float2 v, int l) {
  return make_float2(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.x), l)),
                     __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.y), l)));
}
__device__ __forceinline__ double2 lane_read(double2 v, int l) {
  return make_double2(readlane_d(v.x, l), readlane_d(v.y, l));
}
__device__ __forceinline__ float2 lane_shfl(float2 v, int src) {
  return make_float2(__shfl(v.x, src), __shfl(v.y, src));
}
__device__ __forceinline__ double2 lane_shfl(double2 v, int src) {
  return make_double2(__shfl(v.x, src), __shfl(v.y, src));
}
// value of quad lane k (0..3) to every lane of its quad
template <int K4>
__device__ __forceinline__ float2 quad_bcast(float2 v) {
  constexpr int c = K4 | (K4 << 2) | (K4 << 4) | (K4 << 6);
  return make_float2(dpp_f<c>(v.x), dpp_f<c>(v.y));
}
template <int K4>
__device__ __forceinline__ double2 quad_bcast(double2 v) {
  constexpr int c = K4 | (K4 << 2) | (K4 << 4) | (K4 << 6);
  return make_double2(dpp_d<c>(v.x), dpp_d<c>(v.y));
}
template <class T>
__device__ __forceinline__ T quad_bcast_any(T v, int k) {
  switch (k) {
    case 0: return quad_bcast<0>(v);
    case 1: return quad_bcast<1>(v);
    case 2: return quad_bcast<2>(v);
    default: return quad_bcast<3>(v);
  }
}

// 16 x 16 pivot-block inverse by scalar exchange steps in one wavefront,
// held in registers: lane l keeps row r = l / 4, columns 4 (l % 4) .. +3 (so
// a row is one quad).  Step q reads the pivot from its lane, x[r][q] from the
// quad and the pivot row x[q][:] by a lane permute.  ld(r, c) loads the
// block; the inverse is left in pb[0..255] (row-major).
template <class T, class LD>
__device__ __forceinline__ void pivot_inverse16(const LD& ld, T* pb, int* bad) {
  typedef CX<T> C;
  const int lane = threadIdx.x & 63;
  const int r = lane >> 2, c0 = (lane & 3) * 4;
  T x[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) x[u] = ld(r, c0 + u);
  bool ok = true, fin = true;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int qu = q & 3;
    const T piv = lane_read(x[qu], 4 * q + (q >> 2));
    fin = fin && C::finite(piv);
    ok = ok && C::re(piv) > 0.0;
    const T ip = C::inv(piv);
    const T xrq = quad_bcast_any(x[qu], q >> 2);          // x[r][q]
    T xq[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) xq[u] = lane_shfl(x[u], 4 * q + (lane & 3));   // x[q][c0 + u]
    const T f = C::mul(xrq, ip);
    const T nf = C::neg(f);
    const bool rq = r == q;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool cq = c0 + u == q;
      const T row = C::mul(xq[u], ip);               // pivot row
      const T rest = C::sub(x[u], C::mul(f, xq[u]));
      const T a = rq ? ip : nf;                      // pivot column
      const T b = rq ? row : rest;
      x[u] = cq ? a : b;
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) pb[r * 16 + c0 + u] = x[u];
  wave_sync();
  if (lane == 0) {
    if (!fin) *bad = 2;
    else if (!ok && *bad == 0) *bad = 1;
  }
}

// Inverse of a Hermitian positive definite K x K matrix (K <= 64) by
// Gauss-Jordan exchange steps on 16 x 16 pivot blocks, with the block
// products on the FP32 matrix cores.  With P the pivot block and R the rest,
// one step maps (same exchange as above)
//   a_PP -> P^-1,  a_PR -> X = P^-1 a_PR,  a_RP -> -Y, Y = a_RP P^-1,
//   a_RR -> a_RR - a_RP X.
// P^-1 comes from scalar exchange steps by one wavefront (no pivoting: the
// pivot block of an HPD matrix is HPD).  The matrix is padded to a multiple
// of 16 with the identity, whose inverse leaves A^-1 in the leading block.
// `a` (leading dimension ld >= 64) holds A on entry and A^-1 on return;
// `xs` must hold 16*64 complex values, `ys` 64*16, `pb` 2*16*16.  All 1024
// threads of the block call it.  *bad (LDS) becomes nonzero if a scalar pivot
// is not a positive finite number (1: not HPD, 2: non-finite).
__device__ void gj_inverse_hpd_mfma(float2* a, int K, int ld, float2* xs, float2* ys, float2* pb,
                                    int* bad) {
  const int tid = threadIdx.x, wid = tid >> 6;
  const int KP = (K + 15) & ~15, nb = KP / 16;
  for (int e = tid; e < KP * KP; e += blockDim.x) {
    const int i = e / KP, j = e - i * KP;
    if (i >= K || j >= K) a[i * ld + j] = (i == j) ? make_float2(1.f, 0.f) : cz();
  }
  __syncthreads();
  for (int s = 0; s < nb; ++s) {
    const int p0 = 16 * s;
    if (wid == 0) pivot_inverse16<float2>([&](int r, int c) { return a[(p0 + r) * ld + p0 + c]; }, pb, bad);
    __syncthreads();
    const float2* pinv = pb;
    // X = P^-1 a_P,:  (16 x KP, waves 0..nb-1) and Y = a_:,P P^-1 (KP x 16, waves 8..8+nb-1)
    if (wid < nb) {
      floatx4 dr = zero4(), di = zero4();
      const int j0 = 16 * wid;
      ctile16([&](int i, int k) { return pinv[i * 16 + k]; },
              [&](int k, int j) { return a[(p0 + k) * ld + j0 + j]; }, 0, 16, dr, di);
#pragma unroll
      for (int v = 0; v < 4; ++v) xs[tile_row(v) * 64 + j0 + tile_col()] = make_float2(dr[v], di[v]);
    } else if (wid >= 8 && wid < 8 + nb) {
      floatx4 dr = zero4(), di = zero4();
      const int i0 = 16 * (wid - 8);
      ctile16([&](int i, int k) { return a[(i0 + i) * ld + p0 + k]; },
              [&](int k, int j) { return pinv[k * 16 + j]; }, 0, 16, dr, di);
#pragma unroll
      for (int v = 0; v < 4; ++v) ys[(i0 + tile_row(v)) * 16 + tile_col()] = make_float2(dr[v], di[v]);
    }
    __syncthreads();
    // every tile of the new matrix; values stay in registers until all reads are done
    float2 nv[4];
    const int ti = wid / 4, tj = wid % 4;
    const bool mine = ti < nb && tj < nb;
    if (mine) {
      const int i0 = 16 * ti, j0 = 16 * tj;
      if (ti == s && tj == s) {
#pragma unroll
        for (int v = 0; v < 4; ++v) nv[v] = pinv[tile_row(v) * 16 + tile_col()];
      } else if (ti == s) {
#pragma unroll
        for (int v = 0; v < 4; ++v) nv[v] = xs[tile_row(v) * 64 + j0 + tile_col()];
      } else if (tj == s) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float2 y = ys[(i0 + tile_row(v)) * 16 + tile_col()];
          nv[v] = make_float2(-y.x, -y.y);
        }
      } else {
        floatx4 dr = zero4(), di = zero4();
        ctile16([&](int i, int k) { return a[(i0 + i) * ld + p0 + k]; },
                [&](int k, int j) { return xs[k * 64 + j0 + j]; }, 0, 16, dr, di);
#pragma unroll
        for (int v = 0; v < 4; ++v)
          nv[v] = csub(a[(i0 + tile_row(v)) * ld + j0 + tile_col()], make_float2(dr[v], di[v]));
      }
    }
    __syncthreads();
    if (mine) {
#pragma unroll
      for (int v = 0; v < 4; ++v) a[(16 * ti + tile_row(v)) * ld + 16 * tj + tile_col()] = nv[v];
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------
// Inverse of a Hermitian positive definite K x K matrix for any K (the large
// tracks, 64 < K <= 256), in place, by the same Gauss-Jordan exchange on
// 16 x 16 pivot blocks as gj_inverse_hpd_mfma.  The matrix may sit in global
// memory (it then stays in L2 between steps) or in LDS; only the strips of
// the current step are staged in LDS:
//   xs (16 x KP)  X = P^-1 a_P,:         (new pivot block row)
//   cs (KP x 16)  a_:,P before the step  (old pivot block column)
// so every 16 x 16 tile is read and rewritten by the wavefront that owns it:
//   a_PP -> P^-1,  a_PR -> X_R,  a_RP -> -a_RP P^-1,  a_RR -> a_RR - a_RP X_R.
// T = float2 multiplies on the FP32 matrix cores, T = double2 on the FP64
// vector units.  Indices past K read as the identity and are never written.
// All threads of the block (a multiple of 64, at most 1024) call it; pb holds
// 2 * 256 values.  *bad (LDS) becomes 1 (pivot not positive) or 2 (not finite).
template <class T, class LA, class LB>
__device__ __forceinline__ void tile16_any(const LA& la, const LB& lb, int k0, int k1, T acc[4]) {
  if constexpr (sizeof(T) == sizeof(float2)) {
    floatx4 dr = zero4(), di = zero4();
    ctile16(la, lb, k0, k1, dr, di);
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = make_float2(dr[v], di[v]);
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = dz();
    dtile16(la, lb, k0, k1, acc);
  }
}

template <class T>
__device__ __forceinline__ void gj_inverse_hpd_blocked(T* a, int K, int ld, T* xs, T* cs, T* pb, int* bad) {
  typedef CX<T> C;
  const int tid = threadIdx.x, wid = tid >> 6, nwv = blockDim.x >> 6;
  const int KP = (K + 15) & ~15, nb = KP / 16;
  auto at = [&](int i, int j) -> T {
    return (i < K && j < K) ? a[(size_t)i * ld + j] : (i == j ? C::one() : C::zero());
  };
  for (int s = 0; s < nb; ++s) {
    const int p0 = 16 * s;
    if (wid == 0) pivot_inverse16<T>([&](int r, int c) { return at(p0 + r, p0 + c); }, pb, bad);
    __syncthreads();
    const T* pinv = pb;
    // strips: X_j = P^-1 a_P,j (tiles 0..nb-1) and a copy of a_:,P (tiles nb..2nb-1)
    for (int t = wid; t < 2 * nb; t += nwv) {
      if (t < nb) {
        const int j0 = 16 * t;
        T acc[4];
        tile16_any<T>([&](int i, int k) { return pinv[i * 16 + k]; },
                      [&](int k, int j) { return at(p0 + k, j0 + j); }, 0, 16, acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) xs[tile_row(v) * KP + j0 + tile_col()] = acc[v];
      } else {
        const int i0 = 16 * (t - nb);
#pragma unroll
        for (int v = 0; v < 4; ++v)
          cs[(i0 + tile_row(v)) * 16 + tile_col()] = at(i0 + tile_row(v), p0 + tile_col());
      }
    }
    __syncthreads();
    for (int t = wid; t < nb * nb; t += nwv) {
      const int ti = t / nb, tj = t - ti * nb;
      const int i0 = 16 * ti, j0 = 16 * tj;
      T nv[4];
      if (ti == s && tj == s) {
#pragma unroll
        for (int v = 0; v < 4; ++v) nv[v] = pinv[tile_row(v) * 16 + tile_col()];
      } else if (ti == s) {
#pragma unroll
        for (int v = 0; v < 4; ++v) nv[v] = xs[tile_row(v) * KP + j0 + tile_col()];
      } else if (tj == s) {
        T acc[4];
        tile16_any<T>([&](int i, int k) { return cs[(i0 + i) * 16 + k]; },
                      [&](int k, int j) { return pinv[k * 16 + j]; }, 0, 16, acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) nv[v] = C::neg(acc[v]);
      } else {
        T acc[4];
        tile16_any<T>([&](int i, int k) { return cs[(i0 + i) * 16 + k]; },
                      [&](int k, int j) { return xs[k * KP + j0 + j]; }, 0, 16, acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) nv[v] = C::sub(at(i0 + tile_row(v), j0 + tile_col()), acc[v]);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + tile_row(v), j = j0 + tile_col();
        if (i < K && j < K) a[(size_t)i * ld + j] = nv[v];
      }
    }
    __syncthreads();
  }
}
