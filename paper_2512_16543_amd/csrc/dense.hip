// Direct inversion of the Gram matrix (Alg. 2, "direct matrix inversion").
//
//   k_inv32: FP32, for the conventional full-inversion RZF of rzf_full
//            (16 x 16 pivot blocks, block products on the matrix cores).
//   k_inv64: FP64, for the initial inverse of rzf_init and the periodic
//            drift reset; the result is rounded to the FP32 state.  On a
//            reset step it also records the step's outcome (path RESET).
// One workgroup holds the K x K matrix (two buffers) in LDS.
#include "dense_device.h"
#include "rzf_internal.h"

namespace {

template <bool MANY>
__global__ __launch_bounds__(1024) void k_inv32(Inv32Job one, const Inv32Job* many, int* err) {
  __shared__ float2 b0[KS * KS], xs[16 * KS], ys[KS * 16], pb[2 * 256];
  __shared__ int bad;
  const Inv32Job& jb = job_of<MANY>(one, many);
  const int K = jb.K;
  const float2* A = jb.A;
  float2* Ainv = jb.Ainv;
  if (threadIdx.x == 0) bad = 0;
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
    const int i = e / K, j = e - i * K;
    b0[i * KS + j] = A[e];
  }
  __syncthreads();
  gj_inverse_hpd_mfma(b0, K, KS, xs, ys, pb, &bad);
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
    const int i = e / K, j = e - i * K;
    Ainv[e] = b0[i * KS + j];
  }
  if (threadIdx.x == 0 && bad && err) atomicCAS(err, 0, bad == 2 ? DEV_ERR_NONFINITE : DEV_ERR_NOT_HPD);
}

template <bool MANY>
__global__ __launch_bounds__(1024) void k_inv64(Inv64Job one, const Inv64Job* many, int* err) {
  __shared__ double2 b0[KS * KS], b1[KS * KS];
  __shared__ int bad;
  const Inv64Job& jb = job_of<MANY>(one, many);
  const int K = jb.K;
  const double2* __restrict__ A = jb.A;
  float2* __restrict__ Ainv = jb.Ainv;
  DevInfo* info = jb.info;
  if (threadIdx.x == 0) bad = 0;
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) b0[e] = A[e];
  __syncthreads();
  double2* res = gj_inverse_hpd<double2, 2>(b0, b1, K, K, &bad);
  // a reset that fails keeps the track's state (rzf_init discards the track)
  const bool keep = bad && jb.hold;
  if (!keep)
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
      Ainv[e] = d2f(res[e]);
      if (jb.zero) jb.zero[e] = cz();
    }
  if (threadIdx.x == 0) {
    if (bad) atomicCAS(err, 0, bad == 2 ? DEV_ERR_NONFINITE : DEV_ERR_NOT_HPD);
    if (jb.hold) *jb.hold = bad ? 1 : 0;
    DevInfo rec;
    rec.r = 0; rec.iters = 0; rec.path = keep ? RZF_PATH_NOOP : RZF_PATH_RESET; rec.d = 0;
    rec.dA_fro2 = keep ? __builtin_nan("") : 0.0; rec.captured = 0.0;
    if (info) *info = rec;
    if (jb.out) *jb.out = rec;
  }
}

}  // namespace

void launch_inv32(const Inv32Job& one, const Inv32Job* many, int n, int* err, hipStream_t s) {
  if (many) k_inv32<true><<<dim3(1, n), 1024, 0, s>>>(one, many, err);
  else k_inv32<false><<<1, 1024, 0, s>>>(one, many, err);
}

void launch_inv64(const Inv64Job& one, const Inv64Job* many, int n, int* err, hipStream_t s) {
  if (many) k_inv64<true><<<dim3(1, n), 1024, 0, s>>>(one, many, err);
  else k_inv64<false><<<1, 1024, 0, s>>>(one, many, err);
}
