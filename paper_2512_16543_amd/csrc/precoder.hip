// Precoder W = H^H X with its power normalisation ||W||_F^2 = P (Sec. II,
// eq. (5)), where X is the stored inverse of the Gram matrix.
//
// With the BF16 precision options the product takes BF16 operands (or BF16
// hi/lo splits, three products each) with FP32 accumulation.
//
// W is N x K (row-major).  A workgroup of four wavefronts owns 16 rows of W
// (16 antennas); wave w computes the 16x16 tiles w, w+4, ... along K with a
// length-K reduction on the FP32 matrix cores.  The FP32 path reads the
// block's 16 columns of H_t into LDS once (all of its tiles share them).  The
// block also writes its partial sum of |W|^2 (FP64) and, for rzf_update,
// copies the 16 columns of H_t it has read into the track's H_prev.  A second kernel scales W once
// every partial sum is known (partials are added in a fixed order).
#include "rzf_device.h"
#include "rzf_internal.h"

namespace {

template <bool MANY>
__global__ __launch_bounds__(256) void k_precoder(PrecJob one, const PrecJob* many) {
  __shared__ double red[4];
  __shared__ float2 hs[KM * 16];   // FP32 path: H[i][n0 + c] at hs[16 i + c]
  const PrecJob& jb = job_of<MANY>(one, many);
  const int K = jb.K, N = jb.N, ldh = jb.ldh, ldw = jb.ldw;
  const float2* __restrict__ H = jb.H;
  const float2* __restrict__ X = jb.X;
  float2* __restrict__ W = jb.W;
  double* __restrict__ wpart = jb.wpart;
  float2* __restrict__ Hcopy = jb.Hcopy;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int n0 = blockIdx.x * 16;
  if (n0 >= N) return;
  double acc = 0.0;
  const bool fp32 = jb.prec == RZF_PREC_FP32;
  if (fp32) {
    // the block's 16 columns of H, read once (and copied to H_prev here)
    for (int e = threadIdx.x; e < K * 16; e += blockDim.x) {
      const int i = e >> 4, n = n0 + (e & 15);
      const float2 v = n < N ? H[(size_t)i * ldh + n] : cz();
      hs[e] = v;
      if (Hcopy && n < N) Hcopy[(size_t)i * N + n] = v;
    }
    __syncthreads();
  }
  for (int kt = wid; kt * 16 < K; kt += 4) {
    const int k0 = kt * 16;
    floatx4 dr = zero4(), di = zero4();
    if (fp32) {
      // A(n, i) = conj(H[i][n]) from LDS;  B(i, k) = X[i][k]
      const int col = k0 + (lane & 15);
      const bool okc = col < K;
      const float2* xc = X + col;
      ctile16([&](int rr, int i) { return i < K ? cconj(hs[i * 16 + rr]) : cz(); },
              [&](int i, int) { return (i < K && okc) ? xc[(size_t)i * K] : cz(); }, 0, K, dr, di);
    } else {
      // BF16 operands, 32 users of the reduction per product
      const bool x3 = jb.prec == RZF_PREC_BF16X3;
      const int rr = lane & 15, kq = lane >> 4;
      const int n = n0 + rr, k = k0 + rr;
      for (int i0 = 0; i0 < K; i0 += 32) {
        float2 a[8], b[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int i = i0 + 8 * kq + e;
          a[e] = (n < N && i < K) ? H[(size_t)i * ldh + n] : cz();
          b[e] = (i < K && k < K) ? X[(size_t)i * K + k] : cz();
        }
        cmac8_bf16(a, b, true, false, x3, dr, di);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int n = n0 + tile_row(v), k = k0 + tile_col();
      if (n < N && k < K) {
        W[(size_t)n * ldw + k] = make_float2(dr[v], di[v]);
        acc += (double)dr[v] * dr[v] + (double)di[v] * di[v];
      }
    }
  }
  acc = wave_sum(acc);
  if (lane == 0) red[wid] = acc;
  if (Hcopy && !fp32) {
    // the 16 columns n0..n0+15 of every row of H_t
    for (int e = threadIdx.x; e < K * 16; e += blockDim.x) {
      const int i = e >> 4, n = n0 + (e & 15);
      if (n < N) Hcopy[(size_t)i * N + n] = H[(size_t)i * ldh + n];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) wpart[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Blocks stride over the N x K entries of W (SCALE_BLOCKS per track at most),
// so a batch of small and large tracks launches few empty blocks.
constexpr int SCALE_BLOCKS = 32;

template <bool MANY>
__global__ __launch_bounds__(256) void k_scale(ScaleJob one, const ScaleJob* many) {
  const ScaleJob& jb = job_of<MANY>(one, many);
  const int K = jb.K, N = jb.N, ldw = jb.ldw, nparts = jb.nparts;
  float2* __restrict__ W = jb.W;
  const double* __restrict__ wpart = jb.wpart;
  const double P = jb.P;
  const int NK = N * K;
  if ((int)(blockIdx.x * blockDim.x) >= NK) return;
  double tot = 0.0;
  for (int b = 0; b < nparts; ++b) tot += wpart[b];
  const float s = (tot > 0.0) ? (float)sqrt(P / tot) : 0.f;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < NK; e += gridDim.x * blockDim.x) {
    const int n = e / K, k = e - n * K;
    float2* w = W + (size_t)n * ldw + k;
    *w = cscale(*w, s);
  }
}

}  // namespace

int precoder_blocks(int N) { return (N + 15) / 16; }

void launch_precoder(const PrecJob& one, const PrecJob* many, int n, int maxN, hipStream_t s) {
  const dim3 grid(precoder_blocks(maxN), many ? n : 1);
  if (many) k_precoder<true><<<grid, 256, 0, s>>>(one, many);
  else k_precoder<false><<<grid, 256, 0, s>>>(one, many);
}

void launch_scale(const ScaleJob& one, const ScaleJob* many, int n, int maxNK, hipStream_t s) {
  const int blocks = (maxNK + 255) / 256 < SCALE_BLOCKS ? (maxNK + 255) / 256 : SCALE_BLOCKS;
  const dim3 grid(blocks, many ? n : 1);
  if (many) k_scale<true><<<grid, 256, 0, s>>>(one, many);
  else k_scale<false><<<grid, 256, 0, s>>>(one, many);
}
