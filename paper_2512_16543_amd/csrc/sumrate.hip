// Per-user SINR and sum rate of eq. (15).
//
// W is first scaled to ||W||_F^2 = P, then E = H W (K x K), SINR_n =
// |E_nn|^2 / (sum_{i != n} |E_ni|^2 + sigma^2) and R = sum_n log2(1 + SINR_n)
// (the row-n channel of eq. (15) is row n of H).
//
// k_sr_tiles: one workgroup per 16x16 tile of E (four wavefronts split the
//   length-N reduction on the matrix cores).  For each row of its tile it
//   writes the tile's share of the signal (diagonal tile only) and of the
//   interference; the workgroups of the first tile row also write the squared
//   norm of their 16 columns of W.
// k_sr_final: one workgroup adds the shares in a fixed order, applies the
//   power scaling and sums the rates in FP64.
#include "rzf_device.h"
#include "rzf_internal.h"

namespace {

template <bool MANY>
__global__ __launch_bounds__(256) void k_sr_tiles(RateJob one, const RateJob* many) {
  __shared__ float red[4][8][64];
  __shared__ double wred[4];
  const RateJob& jb = job_of<MANY>(one, many);
  const int K = jb.K, N = jb.N, ldh = jb.ldh, ldw = jb.ldw;
  const float2* __restrict__ H = jb.H;
  const float2* __restrict__ W = jb.W;
  double* __restrict__ part = jb.part;
  const int kt = (K + 15) / 16;
  if ((int)blockIdx.x >= kt * kt) return;
  const int ti = blockIdx.x / kt, tj = blockIdx.x - ti * kt;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int n0 = ti * 16, m0 = tj * 16;
  floatx4 dr = zero4(), di = zero4();
  double wn = 0.0;
  for (int j0 = wid * 16; j0 < N; j0 += 64) {
    ctile16([&](int rr, int j) { const int n = n0 + rr; return (n < K && j < N) ? H[(size_t)n * ldh + j] : cz(); },
            [&](int j, int cc) {
              const int m = m0 + cc;
              return (j < N && m < K) ? W[(size_t)j * ldw + m] : cz();
            },
            j0, j0 + 16, dr, di);
    if (ti == 0) {
      // |W|^2 over rows j0..j0+15 and this tile's 16 columns
      for (int e = lane; e < 256; e += 64) {
        const int j = j0 + (e >> 4), m = m0 + (e & 15);
        if (j < N && m < K) wn += (double)cabs2(W[(size_t)j * ldw + m]);
      }
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    red[wid][v][lane] = dr[v];
    red[wid][4 + v][lane] = di[v];
  }
  if (ti == 0) {
    wn = wave_sum(wn);
    if (lane == 0) wred[wid] = wn;
  }
  __syncthreads();
  if (wid != 0) return;
  // per row of the tile: signal share and interference share
  float sig[4], intf[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    float re = 0.f, im = 0.f;
    for (int w = 0; w < 4; ++w) { re += red[w][v][lane]; im += red[w][4 + v][lane]; }
    const int n = n0 + tile_row(v), m = m0 + tile_col();
    const float e2 = (n < K && m < K) ? re * re + im * im : 0.f;
    sig[v] = (n == m) ? e2 : 0.f;
    intf[v] = (n == m) ? 0.f : e2;
  }
  // sum over the 16 columns of the tile (lanes of one 16-lane row)
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double s = row16_sum((double)sig[v]);
    const double f = row16_sum((double)intf[v]);
    const int n = n0 + tile_row(v);
    if ((lane & 15) == 0 && n < K) {
      part[(size_t)(n * kt + tj) * 2] = s;
      part[(size_t)(n * kt + tj) * 2 + 1] = f;
    }
  }
  if (ti == 0 && lane == 0) part[(size_t)K * kt * 2 + tj] = wred[0] + wred[1] + wred[2] + wred[3];
}

template <bool MANY>
__global__ __launch_bounds__(64) void k_sr_final(RateJob one, const RateJob* many, int* err) {
  const RateJob& jb = job_of<MANY>(one, many);
  const int K = jb.K;
  const double P = jb.P, sigma2 = jb.sigma2;
  const double* __restrict__ part = jb.part;
  float* rates = jb.rates;
  double* sum_out = jb.sum;
  const int kt = (K + 15) / 16;
  double wn = 0.0;
  for (int t = 0; t < kt; ++t) wn += part[(size_t)K * kt * 2 + t];
  const double s2 = (wn > 0.0) ? P / wn : 0.0;      // |scale|^2
  double acc = 0.0;
  for (int n = threadIdx.x; n < K; n += 64) {
    double sig = 0.0, intf = 0.0;
    for (int t = 0; t < kt; ++t) {
      sig += part[(size_t)(n * kt + t) * 2];
      intf += part[(size_t)(n * kt + t) * 2 + 1];
    }
    const double rate = log2(1.0 + (s2 * sig) / (s2 * intf + sigma2));
    if (rates) rates[n] = (float)rate;
    if (!isfinite(rate)) atomicCAS(err, 0, DEV_ERR_NONFINITE);
    acc += rate;
  }
  acc = wave_sum(acc);
  if (threadIdx.x == 0 && sum_out) *sum_out = acc;
}

}  // namespace

size_t sum_rate_scratch_doubles(int K) {
  const int kt = (K + 15) / 16;
  return (size_t)K * kt * 2 + kt;
}

void launch_sum_rate(const RateJob& one, const RateJob* many, int n, int maxK, int* err, hipStream_t s) {
  const int kt = (maxK + 15) / 16;
  if (many) {
    k_sr_tiles<true><<<dim3(kt * kt, n), 256, 0, s>>>(one, many);
    k_sr_final<true><<<dim3(1, n), 64, 0, s>>>(one, many, err);
  } else {
    k_sr_tiles<false><<<kt * kt, 256, 0, s>>>(one, many);
    k_sr_final<false><<<1, 64, 0, s>>>(one, many, err);
  }
}
