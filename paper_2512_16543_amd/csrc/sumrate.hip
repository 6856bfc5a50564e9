// Per-user SINR and sum rate of eq. (15).
//
// W is first scaled to ||W||_F^2 = P, then E = H W (K x K), SINR_n =
// |E_nn|^2 / (sum_{i != n} |E_ni|^2 + sigma^2) and R = sum_n log2(1 + SINR_n)
// (the row-n channel of eq. (15) is row n of H).
//
// One launch.  A workgroup of 16 wavefronts owns a 64 x 64 block of E (users
// rb*64.. by users cb*64..) of one track; wave w computes its 16x16 tile on the
// FP32 matrix cores.  The length-N reduction runs over chunks of 64 antennas
// (the chunk's 64 x 64 block of H and 64 x 64 block of W staged in LDS, the
// next chunk's loads in flight while this one is multiplied).  The chunks
// fall into SR_NP fixed partitions (contiguous runs of ceil(chunks / SR_NP));
// each chunk's product is formed from zero and added to its partition's
// accumulator, and E is the sum of the partitions in order, starting from
// zero.  ||W||^2 (over the W values that the first block row stages) is summed
// the same way: per thread over a partition's values, per partition over the
// waves in order, then over the partitions in order.  The partitions, not the launch, fix every rounding: a single
// track with K <= 64 may spread its partitions over ns workgroups (partition q
// to workgroup q mod ns), which write their partitions' E blocks and norms to
// scratch for the last of them to add up, and gives bit for bit what one
// workgroup (ns = 1, as in a batch) gives.
//
// For each of its rows the workgroup then forms its share of the signal
// (diagonal block only) and of the interference.  With K <= 64 the track's
// one block applies the power scaling and sums the rates in FP64 from LDS.
// Otherwise the shares go to scratch and the track's last workgroup to finish
// (a completion count per item, zero between launches) adds them in a fixed
// order; only the wave that wrote them fences before counting, since an
// agent-scope fence writes back the XCD's L2.
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
constexpr int SR_NP = 8;        // fixed partitions of the antenna chunks (and the largest split)

// Scratch layout of one item (doubles): the shares [n][cb][2] (signal,
// interference), then the column blocks' ||W||^2 [cb].  The completion count
// (one per item) is zero before the launch and is left at zero.  A split
// launch uses [SR_NP][SB * SB] complex partition blocks of E, then SR_NP
// partition norms.
__host__ __device__ constexpr int sr_blocks(int K) { return (K + SB - 1) / SB; }

template <bool MANY>
__global__ __launch_bounds__(SNT) void k_sum_rate(RateJob one, const RateJob* many, int ns, int* err) {
  __shared__ float2 hs[SB * SLD], ws[SC * WLD];
  __shared__ double rs[4][SB], rf[4][SB];
  __shared__ double red[SNW];
  __shared__ double wq[SR_NP][SNW];   // per partition and wave: |W|^2
  __shared__ int last;
  const GridPos gp = grid_pos<MANY>();
  const RateJob& jb = job_at<MANY>(one, many, gp.item);
  const int K = jb.K, N = jb.N, ldh = jb.ldh, ldw = jb.ldw;
  const float2* __restrict__ H = jb.H;
  const float2* __restrict__ W = jb.W;
  unsigned* const count = jb.count;
  double* __restrict__ part = jb.part;
  const int kb = sr_blocks(K);
  if (gp.x >= kb * kb * ns) return;
  const int blk = gp.x / ns, sp = gp.x - blk * ns;   // ns > 1 only with kb == 1
  const int rb = blk / kb, cb = blk - rb * kb;
  const int nch = (N + SC - 1) / SC;
  const int cpp = (nch + SR_NP - 1) / SR_NP;      // chunks per partition
  auto owned = [&](int c) { return (c / cpp) % ns == sp; };
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int nt = wid >> 2, ct = wid & 3;          // this wave's tile in the block
  const int r0 = rb * SB, m0 = cb * SB;
  const bool live = r0 + nt * 16 < K && m0 + ct * 16 < K;   // the wave's tile holds users
  // E of the completed partitions (ns == 1) and of the current one; |W|^2 of
  // the current partition's staged values (rb == 0)
  floatx4 Er = zero4(), Ei = zero4(), pr = zero4(), pi = zero4();
  double wcur = 0.0;
  float2* const pe = reinterpret_cast<float2*>(part);   // split: [SR_NP][SB * SB] partition blocks of E
  double* const pw2 = part + (size_t)SR_NP * SB * SB;   // split: [SR_NP] partition norms
  float2 ph[SPER], pw[SPER];
  auto fetch = [&](int c0) {
#pragma unroll
    for (int e = 0; e < SPER; ++e) {
      const int idx = tid + SNT * e;
      const int a = idx / SC, b = idx % SC;     // H: user a, antenna b;  W: antenna a, user b
      const int n = r0 + a, j = c0 + b;
      ph[e] = (n < K && j < N) ? gld(H, (size_t)n * ldh + j) : cz();
      const int jw = c0 + a, m = m0 + b;
      pw[e] = (jw < N && m < K) ? gld(W, (size_t)jw * ldw + m) : cz();
    }
  };
  int c = 0;
  while (c < nch && !owned(c)) ++c;
  if (c < nch) fetch(c * SC);
  while (c < nch) {
    const int q = c / cpp;
#pragma unroll
    for (int e = 0; e < SPER; ++e) {
      const int idx = tid + SNT * e;
      const int a = idx / SC, b = idx % SC;
      hs[a * SLD + b] = ph[e];
      ws[a * WLD + b] = pw[e];
      if (rb == 0) wcur += (double)cabs2(pw[e]);
    }
    __syncthreads();
    int cn = c + 1;
    while (cn < nch && !owned(cn)) ++cn;
    if (cn < nch) fetch(cn * SC);
    const int jc = min(SC, N - c * SC);
    // this chunk's E(n, m) = sum_j H[n][j] W[j][m], added to its partition (a
    // tile wholly past the track's K users has zero operands: it stays zero)
    floatx4 dr = zero4(), di = zero4();
    if (live)
      ctile16([&](int rr, int j) { return hs[(nt * 16 + rr) * SLD + j]; },
              [&](int j, int cc) { return ws[j * WLD + ct * 16 + cc]; }, 0, (jc + 3) & ~3, dr, di);
#pragma unroll
    for (int v = 0; v < 4; ++v) { pr[v] += dr[v]; pi[v] += di[v]; }
    if (cn >= nch || cn / cpp != q) {
      // partition q is complete
      if (ns == 1) {
#pragma unroll
        for (int v = 0; v < 4; ++v) { Er[v] += pr[v]; Ei[v] += pi[v]; }
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          pe[(size_t)q * SB * SB + (nt * 16 + tile_row(v)) * SB + ct * 16 + tile_col()] =
              make_float2(pr[v], pi[v]);
      }
      pr = zero4();
      pi = zero4();
      const double w = wave_sum(wcur);
      if (lane == 0) wq[q][wid] = w;
      wcur = 0.0;
    }
    __syncthreads();
    c = cn;
  }
  // |W|^2 per completed partition of this workgroup: its waves in order
  const int npart = (nch + cpp - 1) / cpp;        // partitions that hold a chunk
  floatx4 dr = zero4(), di = zero4();
  double wt = 0.0;   // ||W||^2 of the block's columns (kb == 1: all of W)
  if (ns > 1) {
    // the last workgroup adds every partition in order
    if (tid < npart && tid % ns == sp) {
      double w = 0.0;
      for (int k = 0; k < SNW; ++k) w += wq[tid][k];
      pw2[tid] = w;
    }
    __syncthreads();
    if (tid == 0) {
      __threadfence();   // after the barrier: the workgroup's stores before the count
      last = atomicAdd(count, 1u) == (unsigned)(ns - 1);
    }
    __syncthreads();
    if (!last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    for (int q = 0; q < npart; ++q) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float2 x = pe[(size_t)q * SB * SB + (nt * 16 + tile_row(v)) * SB + ct * 16 + tile_col()];
        dr[v] += x.x;
        di[v] += x.y;
      }
      wt += pw2[q];
    }
  } else {
    dr = Er;
    di = Ei;
    for (int q = 0; q < npart; ++q) {
      double w = 0.0;
      for (int k = 0; k < SNW; ++k) w += wq[q][k];
      wt += w;
    }
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
      if (tid == 0 && rb == 0) wnorm[cb] = wt;
      __threadfence();   // the wave's stores before the block counts itself done
      if (tid == 0) last = atomicAdd(count, 1u) == (unsigned)(kb * kb - 1);
    }
    __syncthreads();
    if (!last) return;
    // the track's last block: every share is visible
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    double wtot = 0.0;
    for (int c = 0; c < kb; ++c) wtot += wnorm[c];
    const double s2 = (wtot > 0.0) ? jb.P / wtot : 0.0;
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

size_t sum_rate_split_scratch_doubles() { return (size_t)SR_NP * SB * SB + SR_NP; }

int sum_rate_splits(int K, int N) {
  if (sr_blocks(K) > 1) return 1;
  return std::max(1, std::min(SR_NP, (N + SC - 1) / SC));
}

void launch_sum_rate(const RateJob& one, const RateJob* many, int n, int maxK, int ns, int* err, hipStream_t s) {
  const int kb = sr_blocks(maxK);
  if (many || kb > 1) ns = 1;
  ns = std::max(1, std::min(SR_NP, ns));
  if (many) k_sum_rate<true><<<dim3(kb * kb, n), SNT, 0, s>>>(one, many, 1, err);
  else k_sum_rate<false><<<kb * kb * ns, SNT, 0, s>>>(one, many, ns, err);
}
