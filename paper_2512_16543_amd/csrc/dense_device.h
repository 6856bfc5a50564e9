// Workgroup-level dense kernels on matrices held in LDS.
#pragma once

#include "rzf_device.h"

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
