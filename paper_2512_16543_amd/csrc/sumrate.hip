// Per-user SINR and sum rate of eq. (15).
//
// W is first scaled to ||W||_F^2 = P, then E = H W (K x K), SINR_n =
// |E_nn|^2 / (sum_{i != n} |E_ni|^2 + sigma^2) and R = sum_n log2(1 + SINR_n)
// (the row-n channel of eq. (15) is row n of H).
//
// One launch.  A workgroup of 16 wavefronts owns a 64 x 64 block of E (users
// rb*64.. by users cb*64..) of one track; wave w computes its 16x16 tile on the
// FP32 matrix cores.  The length-N reduction runs over chunks of 64 antennas:
// the chunk's 64 x 64 block of H and 64 x 64 block of W are staged in LDS
// (the next chunk's loads in flight while this one is multiplied).  For each
// of its rows the workgroup writes its share of the signal (diagonal block
// only) and of the interference; the workgroups of the first block row also
// add the squared norm of their 64 columns of W.  With K <= 64 the track's one
// workgroup then applies the power scaling and sums the rates in FP64 from
// LDS.  Otherwise the shares go to scratch and the track's last workgroup to
// finish (a completion count per item, zero between launches) adds them in a
// fixed order; only the wave that wrote them fences before counting, since an
// agent-scope fence writes back the XCD's L2.
//
// A single track with K <= 64 and N > 64 (no batch to fill the chip) splits
// the antenna sum over ns workgroups, each taking whole chunks: they write
// their partial 64 x 64 blocks of E and partial ||W||^2 to scratch, and the
// last to finish adds the partials in split order before the steps above.
// A batch launch keeps one workgroup per block, so a split track's rates
// agree with its batched ones to FP32 rounding, not bit for bit.
#include "rzf_device.h"
#include "rzf_internal.h"

namespace {

constexpr int SB = 64;          // users per block side
constexpr int SC = 64;          // antennas per reduction chunk
constexpr int SNT = 1024;
constexpr int SNW = SNT / 64;
constexpr int SLD = SC + 4;     // LDS row stride of the H chunk (64 users x 64 antennas)
constexpr int WLD = SB + 4;     // LDS row stride of the W chunk (64 antennas x 64 users)
constexpr int SPER = SB * SC / SNT;   // values of each chunk a thread stages (4)

// Scratch layout of one item (doubles): the shares [n][cb][2] (signal,
// interference), then the column blocks' ||W||^2 [cb].  The completion count
// (one per item) is zero before the launch and is left at zero.
__host__ __device__ constexpr int sr_blocks(int K) { return (K + SB - 1) / SB; }
constexpr int SR_SPLIT_MAX = 8;

template <bool MANY>
__global__ __launch_bounds__(SNT) void k_sum_rate(RateJob one, const RateJob* many, int ns, int* err) {
  __shared__ float2 hs[SB * SLD], ws[SC * WLD];
  __shared__ double rs[4][SB], rf[4][SB];
  __shared__ double red[SNW];
  __shared__ int last;
  const RateJob& jb = job_of<MANY>(one, many);
  const int K = jb.K, N = jb.N, ldh = jb.ldh, ldw = jb.ldw;
  const float2* __restrict__ H = jb.H;
  const float2* __restrict__ W = jb.W;
  unsigned* const count = jb.count;
  double* __restrict__ part = jb.part;
  const int kb = sr_blocks(K);
  if ((int)blockIdx.x >= kb * kb * ns) return;
  const int blk = blockIdx.x / ns, sp = blockIdx.x - blk * ns;   // ns > 1 only with kb == 1
  const int rb = blk / kb, cb = blk - rb * kb;
  // this workgroup's antennas: whole chunks [cbeg, cend)
  const int cps = ((N + SC - 1) / SC + ns - 1) / ns;
  const int cbeg = sp * cps * SC, cend = min(N, (sp + 1) * cps * SC);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int nt = wid >> 2, ct = wid & 3;          // this wave's tile in the block
  const int r0 = rb * SB, m0 = cb * SB;
  floatx4 dr = zero4(), di = zero4();
  double wn = 0.0;                                // |W|^2 of the staged values (rb == 0)
  float2 ph[SPER], pw[SPER];
  auto fetch = [&](int c0) {
#pragma unroll
    for (int e = 0; e < SPER; ++e) {
      const int idx = tid + SNT * e;
      const int a = idx / SC, b = idx % SC;     // H: user a, antenna b;  W: antenna a, user b
      const int n = r0 + a, j = c0 + b;
      ph[e] = (n < K && j < N) ? H[(size_t)n * ldh + j] : cz();
      const int jw = c0 + a, m = m0 + b;
      pw[e] = (jw < N && m < K) ? W[(size_t)jw * ldw + m] : cz();
    }
  };
  if (cbeg < cend) fetch(cbeg);
  for (int c0 = cbeg; c0 < cend; c0 += SC) {
#pragma unroll
    for (int e = 0; e < SPER; ++e) {
      const int idx = tid + SNT * e;
      const int a = idx / SC, b = idx % SC;
      hs[a * SLD + b] = ph[e];
      ws[a * WLD + b] = pw[e];
      if (rb == 0) wn += (double)cabs2(pw[e]);
    }
    __syncthreads();
    if (c0 + SC < cend) fetch(c0 + SC);
    const int jc = min(SC, cend - c0);
    // E(n, m) += sum_j H[n][j] W[j][m]
    ctile16([&](int rr, int j) { return hs[(nt * 16 + rr) * SLD + j]; },
            [&](int j, int cc) { return ws[j * WLD + ct * 16 + cc]; }, 0, (jc + 3) & ~3, dr, di);
    __syncthreads();
  }
  wn = wave_sum(wn);
  if (lane == 0) red[wid] = wn;
  double wt = 0.0;   // ||W||^2 of the block's columns (kb == 1: all of W)
  if (ns > 1) {
    // partial E and ||W||^2 to scratch; the last split adds them up
    float2* const pe = reinterpret_cast<float2*>(part);   // [ns][SB * SB]
    double* const pw = part + (size_t)ns * SB * SB;      // [ns]
#pragma unroll
    for (int v = 0; v < 4; ++v)
      pe[(size_t)sp * SB * SB + (nt * 16 + tile_row(v)) * SB + ct * 16 + tile_col()] = make_float2(dr[v], di[v]);
    __syncthreads();
    if (tid == 0) {
      double w = 0.0;
      for (int q = 0; q < SNW; ++q) w += red[q];
      pw[sp] = w;
      __threadfence();   // after the barrier: the workgroup's stores before the count
      last = atomicAdd(count, 1u) == (unsigned)(ns - 1);
    }
    __syncthreads();
    if (!last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const size_t o = (nt * 16 + tile_row(v)) * SB + ct * 16 + tile_col();
      float er = 0.f, ei = 0.f;
      for (int q = 0; q < ns; ++q) {
        const float2 x = pe[(size_t)q * SB * SB + o];
        er += x.x;
        ei += x.y;
      }
      dr[v] = er;
      di[v] = ei;
    }
    for (int q = 0; q < ns; ++q) wt += pw[q];
  }
  // the block's signal and interference shares of each row, over its columns
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = nt * 16 + tile_row(v);
    const int n = r0 + i, m = m0 + ct * 16 + tile_col();
    const float e2 = (n < K && m < K) ? dr[v] * dr[v] + di[v] * di[v] : 0.f;
    const double s = row16_sum((double)((n == m) ? e2 : 0.f));
    const double f = row16_sum((double)((n == m) ? 0.f : e2));
    if ((lane & 15) == 0) {
      rs[ct][i] = s;
      rf[ct][i] = f;
    }
  }
  __syncthreads();
  double acc = 0.0;
  if (kb == 1) {
    // one workgroup owns the track: the rates straight from its shares
    if (tid < K) {
      if (ns == 1)
        for (int q = 0; q < SNW; ++q) wt += red[q];
      const double s2 = (wt > 0.0) ? jb.P / wt : 0.0;   // |scale|^2
      const double sig = ((rs[0][tid] + rs[1][tid]) + rs[2][tid]) + rs[3][tid];
      const double intf = ((rf[0][tid] + rf[1][tid]) + rf[2][tid]) + rf[3][tid];
      const double rate = log2(1.0 + (s2 * sig) / (s2 * intf + jb.sigma2));
      if (jb.rates) jb.rates[tid] = (float)rate;
      if (!isfinite(rate)) atomicCAS(err, 0, DEV_ERR_NONFINITE);
      acc = rate;
    }
  } else {
    // the shares (written by wave 0 alone) go to memory for the track's last block
    if (tid < SB && r0 + tid < K) {
      const double s = ((rs[0][tid] + rs[1][tid]) + rs[2][tid]) + rs[3][tid];
      const double f = ((rf[0][tid] + rf[1][tid]) + rf[2][tid]) + rf[3][tid];
      part[((size_t)(r0 + tid) * kb + cb) * 2] = s;
      part[((size_t)(r0 + tid) * kb + cb) * 2 + 1] = f;
    }
    double* const wnorm = part + (size_t)2 * K * kb;
    if (wid == 0) {
      if (tid == 0 && rb == 0) {
        double w = 0.0;
        for (int q = 0; q < SNW; ++q) w += red[q];
        wnorm[cb] = w;
      }
      __threadfence();   // the wave's stores before the block counts itself done
      if (tid == 0) last = atomicAdd(count, 1u) == (unsigned)(kb * kb - 1);
    }
    __syncthreads();
    if (!last) return;
    // the track's last block: every share is visible
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    for (int c = 0; c < kb; ++c) wt += wnorm[c];
    const double s2 = (wt > 0.0) ? jb.P / wt : 0.0;
    for (int n = tid; n < K; n += SNT) {
      double sig = 0.0, intf = 0.0;
      for (int c = 0; c < kb; ++c) {
        sig += part[((size_t)n * kb + c) * 2];
        intf += part[((size_t)n * kb + c) * 2 + 1];
      }
      const double rate = log2(1.0 + (s2 * sig) / (s2 * intf + jb.sigma2));
      if (jb.rates) jb.rates[n] = (float)rate;
      if (!isfinite(rate)) atomicCAS(err, 0, DEV_ERR_NONFINITE);
      acc += rate;
    }
  }
  acc = wave_sum(acc);
  __syncthreads();   // every read of red above is done
  if (lane == 0) red[wid] = acc;
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    for (int q = 0; q < SNW; ++q) tot += red[q];
    if (jb.sum) *jb.sum = tot;
    if (kb > 1 || ns > 1) *count = 0u;
  }
}

}  // namespace

size_t sum_rate_scratch_doubles(int K) {
  const int kb = sr_blocks(K);
  return (size_t)2 * K * kb + kb;
}

size_t sum_rate_split_scratch_doubles() { return (size_t)SR_SPLIT_MAX * SB * SB + SR_SPLIT_MAX; }

int sum_rate_splits(int K, int N) {
  if (sr_blocks(K) > 1) return 1;
  return std::max(1, std::min(SR_SPLIT_MAX, (N + SC - 1) / SC));
}

void launch_sum_rate(const RateJob& one, const RateJob* many, int n, int maxK, int ns, int* err, hipStream_t s) {
  const int kb = sr_blocks(maxK);
  if (many) k_sum_rate<true><<<dim3(kb * kb, n), SNT, 0, s>>>(one, many, 1, err);
  else k_sum_rate<false><<<kb * kb * ns, SNT, 0, s>>>(one, many, ns, err);
}
