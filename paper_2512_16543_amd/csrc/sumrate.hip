// Per-user SINR and sum rate of eq. (15).
//
// W is first scaled to ||W||_F^2 = P, then E = H W (K x K), SINR_n =
// |E_nn|^2 / (sum_{i != n} |E_ni|^2 + sigma^2) and R = sum_n log2(1 + SINR_n)
// (the row-n channel of eq. (15) is row n of H).
//
// k_sr_tiles: one workgroup per 16x16 tile of E.  The length-N reduction is
//   cut into 16 slices (slice s: antennas 16 s + 256 j + [0, 16)), each
//   summed from zero on the matrix cores, and the slice sums are added as
//   (s0 + s4 + s8 + s12) + (s1 + s5 + ...) + ....  A single-track launch
//   gives every slice its own wavefront (16 wavefronts: each issues its few
//   loads at once); a batch launch, where many workgroups share each CU, gives
//   each of four wavefronts the slices w, w + 4, w + 8, w + 12 in turn.  Both
//   forms add the same numbers in the same order.  For each row of its tile
//   the workgroup writes its share of the signal (diagonal tile only) and of
//   the interference; the workgroups of the first tile row also write the
//   squared norm of their 16 columns of W.
// k_sr_final: one workgroup adds the shares in a fixed order, applies the
//   power scaling and sums the rates in FP64.
#include "rzf_device.h"
#include "rzf_internal.h"

namespace {

constexpr int SR_SLICES = 16;
template <bool MANY> constexpr int sr_waves() { return MANY ? 4 : SR_SLICES; }

template <bool MANY>
__global__ __launch_bounds__(64 * sr_waves<MANY>()) void k_sr_tiles(RateJob one, const RateJob* many) {
  constexpr int NW = sr_waves<MANY>(), PER = SR_SLICES / NW;   // waves, slices per wave
  __shared__ float red[NW][8][64];
  __shared__ double wred[NW];
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
  floatx4 tr = zero4(), tim = zero4();   // this wave's slices, added in order
  double twn = 0.0;
  for (int q = 0; q < PER; ++q) {
    const int sl = wid + NW * q;
    floatx4 dr = zero4(), di = zero4();
    double wn = 0.0;
    for (int j0 = sl * 16; j0 < N; j0 += 16 * SR_SLICES) {
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
    if (q == 0) {
      tr = dr; tim = di;
    } else {
      tr += dr; tim += di;
    }
    if (ti == 0) {
      const double ws = wave_sum(wn);
      twn = q == 0 ? ws : twn + ws;
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    red[wid][v][lane] = tr[v];
    red[wid][4 + v][lane] = tim[v];
  }
  if (ti == 0 && lane == 0) wred[wid] = twn;
  __syncthreads();
  // wave v (< 4): signal and interference shares of the tile's rows 4 kq + v
  if (wid >= 4) return;
  {
    const int v = wid;
    float re = 0.f, im = 0.f;
    for (int w = 0; w < 4; ++w) {
      // slice sums of group w (slices w, w + 4, ...), added in order
      float gr = red[w][v][lane], gi = red[w][4 + v][lane];
      for (int q = 1; q < SR_SLICES / 4 / PER; ++q) {
        gr += red[w + 4 * q][v][lane];
        gi += red[w + 4 * q][4 + v][lane];
      }
      re += gr;
      im += gi;
    }
    const int n = n0 + tile_row(v), m = m0 + tile_col();
    const float e2 = (n < K && m < K) ? re * re + im * im : 0.f;
    // sum over the 16 columns of the tile (lanes of one 16-lane row)
    const double s = row16_sum((double)((n == m) ? e2 : 0.f));
    const double f = row16_sum((double)((n == m) ? 0.f : e2));
    if ((lane & 15) == 0 && n < K) {
      part[(size_t)(n * kt + tj) * 2] = s;
      part[(size_t)(n * kt + tj) * 2 + 1] = f;
    }
  }
  if (ti == 0 && threadIdx.x == 0) {
    double w = 0.0;
    for (int g = 0; g < 4; ++g) {
      double gw = wred[g];
      for (int q = 1; q < SR_SLICES / 4 / PER; ++q) gw += wred[g + 4 * q];
      w += gw;
    }
    part[(size_t)K * kt * 2 + tj] = w;
  }
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
    k_sr_tiles<true><<<dim3(kt * kt, n), 64 * sr_waves<true>(), 0, s>>>(one, many);
    k_sr_final<true><<<dim3(1, n), 64, 0, s>>>(one, many, err);
  } else {
    k_sr_tiles<false><<<kt * kt, 64 * sr_waves<false>(), 0, s>>>(one, many);
    k_sr_final<false><<<1, 64, 0, s>>>(one, many, err);
  }
}
