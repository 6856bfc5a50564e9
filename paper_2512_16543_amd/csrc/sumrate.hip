// Per-user SINR and sum rate of eq. (15).
//
// W is first scaled to ||W||_F^2 = P, then E = H W (K x K, on the matrix
// cores), SINR_n = |E_nn|^2 / (sum_{i != n} |E_ni|^2 + sigma^2) and
// R = sum_n log2(1 + SINR_n) (the row-n channel of eq. (15) is row n of H).
// One workgroup of 16 wavefronts; the K x K product sits in LDS.
#include "rzf_device.h"
#include "rzf_internal.h"

namespace {

__global__ __launch_bounds__(1024) void k_sum_rate(int K, int N, const float2* __restrict__ H,
                                                   int ldh, const float2* __restrict__ W, int ldw,
                                                   double P, double sigma2, float* rates,
                                                   double* sum_out, int* err) {
  __shared__ float2 e[KM * KM];
  __shared__ double red[16];
  const int tid = threadIdx.x, wid = tid >> 6;
  double part = 0.0;
  for (int x = tid; x < N * K; x += blockDim.x) {
    const int n = x / K, k = x - n * K;
    part += (double)cabs2(W[(size_t)n * ldw + k]);
  }
  const double wn = block_sum(part, red);
  const double s2 = (wn > 0.0) ? P / wn : 0.0;      // |scale|^2
  const int kt = (K + 15) / 16;
  for (int t = wid; t < kt * kt; t += 16) {
    const int ti = t / kt, tj = t - ti * kt;
    floatx4 dr = zero4(), di = zero4();
    auto la = [&](int rr, int j) {
      const int n = ti * 16 + rr;
      return (n < K && j < N) ? H[(size_t)n * ldh + j] : cz();
    };
    auto lb = [&](int j, int cc) {
      const int m = tj * 16 + cc;
      return (j < N && m < K) ? W[(size_t)j * ldw + m] : cz();
    };
    ctile16(la, lb, 0, N, dr, di);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = ti * 16 + tile_row(v), j = tj * 16 + tile_col();
      if (i < K && j < K) e[i * KM + j] = make_float2(dr[v], di[v]);
    }
  }
  __syncthreads();
  double rate = 0.0;
  if (tid < K) {
    double sig = 0.0, intf = 0.0;
    for (int i = 0; i < K; ++i) {
      const double a = (double)cabs2(e[tid * KM + i]) * s2;
      if (i == tid) sig = a; else intf += a;
    }
    rate = log2(1.0 + sig / (intf + sigma2));
    if (rates) rates[tid] = (float)rate;
    if (!isfinite(rate)) atomicCAS(err, 0, DEV_ERR_NONFINITE);
  }
  const double tot = block_sum(rate, red);
  if (tid == 0 && sum_out) *sum_out = tot;
}

}  // namespace

void launch_sum_rate(int K, int N, const float2* H, int ldh, const float2* W, int ldw, double P,
                     double sigma2, float* rates, double* sum_out, int* err, hipStream_t s) {
  k_sum_rate<<<1, 1024, 0, s>>>(K, N, H, ldh, W, ldw, P, sigma2, rates, sum_out, err);
}
