// Workgroup-level dense kernels on matrices held in LDS.
#pragma once

#include "rzf_device.h"

template <class T> struct CX;
template <> struct CX<float2> {
  typedef float R;
  static __device__ __forceinline__ float2 mul(float2 a, float2 b) { return cmul(a, b); }
  static __device__ __forceinline__ float2 sub(float2 a, float2 b) { return csub(a, b); }
  static __device__ __forceinline__ float2 neg(float2 a) { return make_float2(-a.x, -a.y); }
  static __device__ __forceinline__ float2 inv(float2 a) {
    const double2 r = ddiv(make_double2(1.0, 0.0), f2d(a));
    return d2f(r);
  }
};
template <> struct CX<double2> {
  typedef double R;
  static __device__ __forceinline__ double2 mul(double2 a, double2 b) { return dmul(a, b); }
  static __device__ __forceinline__ double2 sub(double2 a, double2 b) { return dsub(a, b); }
  static __device__ __forceinline__ double2 neg(double2 a) { return make_double2(-a.x, -a.y); }
  static __device__ __forceinline__ double2 inv(double2 a) { return ddiv(make_double2(1.0, 0.0), a); }
};

// Inverse of a Hermitian positive definite K x K matrix by Gauss-Jordan
// exchange steps without pivoting (the pivots of an HPD matrix are the
// positive diagonal entries of its successive Schur complements).  Step k maps
//   a_kk -> 1/p,  a_kj -> a_kj/p,  a_ik -> -a_ik/p,  a_ij -> a_ij - a_ik a_kj/p
// with p = a_kk; after K steps the matrix holds A^-1.  Each step reads one
// buffer and writes the other, so one barrier per step suffices.
// `a` holds A on entry (leading dimension ld); `b` is scratch of the same
// shape.  Returns the buffer holding A^-1.  *bad (LDS) becomes nonzero if a
// pivot is not a positive finite number (1: not HPD, 2: non-finite).
template <class T>
__device__ T* gj_inverse_hpd(T* a, T* b, int K, int ld, int* bad) {
  typedef CX<T> C;
  const int n = K * K;
  for (int k = 0; k < K; ++k) {
    const T piv = a[k * ld + k];
    if (threadIdx.x == 0) {
      if (!isfinite(piv.x) || !isfinite(piv.y)) *bad = 2;
      else if (!(piv.x > 0)) { if (*bad == 0) *bad = 1; }
    }
    const T ip = C::inv(piv);
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
      const int i = e / K, j = e - i * K;
      T v;
      if (i == k) {
        v = (j == k) ? ip : C::mul(a[k * ld + j], ip);
      } else if (j == k) {
        v = C::neg(C::mul(a[i * ld + k], ip));
      } else {
        v = C::sub(a[i * ld + j], C::mul(C::mul(a[i * ld + k], ip), a[k * ld + j]));
      }
      b[i * ld + j] = v;
    }
    __syncthreads();
    T* t = a; a = b; b = t;
  }
  return a;
}
