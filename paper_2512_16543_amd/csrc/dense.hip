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

__global__ __launch_bounds__(1024) void k_inv32(int K, const float2* __restrict__ A,
                                                float2* __restrict__ Ainv, int* err) {
  __shared__ float2 b0[KM * KM], xs[16 * KM], ys[KM * 16], pb[2 * 256];
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
    const int i = e / K, j = e - i * K;
    b0[i * KM + j] = A[e];
  }
  __syncthreads();
  gj_inverse_hpd_mfma(b0, K, KM, xs, ys, pb, &bad);
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
    const int i = e / K, j = e - i * K;
    Ainv[e] = b0[i * KM + j];
  }
  if (threadIdx.x == 0 && bad) atomicCAS(err, 0, bad == 2 ? DEV_ERR_NONFINITE : DEV_ERR_NOT_HPD);
}

__global__ __launch_bounds__(1024) void k_inv64(int K, const double2* __restrict__ A,
                                                float2* __restrict__ Ainv, int* err, DevInfo* info) {
  __shared__ double2 b0[KM * KM], b1[KM * KM];
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) b0[e] = A[e];
  __syncthreads();
  double2* res = gj_inverse_hpd<double2, 2>(b0, b1, K, K, &bad);
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) Ainv[e] = d2f(res[e]);
  if (threadIdx.x == 0) {
    if (bad) atomicCAS(err, 0, bad == 2 ? DEV_ERR_NONFINITE : DEV_ERR_NOT_HPD);
    if (info) {
      info->r = 0; info->iters = 0; info->path = RZF_PATH_RESET; info->d = 0;
      info->dA_fro2 = 0.0; info->captured = 0.0;
    }
  }
}

}  // namespace

void launch_inv32(int K, const float2* A, float2* Ainv, int* err, hipStream_t s) {
  k_inv32<<<1, 1024, 0, s>>>(K, A, Ainv, err);
}

void launch_inv64(int K, const double2* A64, float2* Ainv, int* err, DevInfo* info, hipStream_t s) {
  k_inv64<<<1, 1024, 0, s>>>(K, A64, Ainv, err, info);
}
