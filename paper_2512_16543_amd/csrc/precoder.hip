// Precoder W = H^H X with its power normalisation ||W||_F^2 = P (Sec. II,
// eq. (5)), where X is the stored inverse of the Gram matrix.
//
// With the BF16 precision options the product takes BF16 operands (or BF16
// hi/lo splits, three products each) with FP32 accumulation.
//
// W is N x K (row-major).  A workgroup owns 16 rows of W (16 antennas) and
// computes their 16x16 tiles along K (tile slot s: tiles s, s + 4, ...) with
// a length-K reduction on the FP32 matrix cores.  The FP32 path reads the
// block's 16 columns of H_t into LDS once (all of its tiles share them).  The
// block also writes its partial sum of |W|^2 (FP64) and, for rzf_update,
// copies the 16 columns of H_t it has read into the track's H_prev.  A second kernel scales W once
// every partial sum is known (partials are added in a fixed order).
#include "rzf_device.h"
#include "rzf_internal.h"

namespace {

// The length-K reduction of each tile is cut into four slices, each summed
// from zero and then added in slice order.  A single-track launch gives every
// (tile slot, slice) pair its own wavefront (16 wavefronts, slices added
// through LDS); a batch launch, where many workgroups share each CU, gives
// each of four wavefronts a tile slot and its four slices in turn.  Both forms
// add the same numbers in the same order.
template <bool MANY> constexpr int prec_waves() { return MANY ? 4 : 16; }

template <bool MANY>
__global__ __launch_bounds__(64 * prec_waves<MANY>()) void k_precoder(PrecJob one, const PrecJob* many) {
  constexpr int NW = prec_waves<MANY>(), PER = 16 / NW;   // waves; slices per wave
  __shared__ double red[NW];
  __shared__ float part[NW == 16 ? 16 : 1][8][64];   // 16-wave form: the slices' partial tiles
  __shared__ float2 hs[KM * 16];   // FP32 path: H[i][n0 + c] at hs[16 i + c]
  const PrecJob& jb = job_of<MANY>(one, many);
  const int K = jb.K, N = jb.N, ldh = jb.ldh, ldw = jb.ldw;
  const float2* __restrict__ H = jb.H;
  const float2* __restrict__ X = jb.X;
  float2* __restrict__ W = jb.W;
  double* __restrict__ wpart = jb.wpart;
  // a step that met a non-finite snapshot keeps the track's previous one
  float2* __restrict__ Hcopy = (jb.hold && *jb.hold) ? nullptr : jb.Hcopy;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int slot = wid & 3;
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
  // slice ks: users [ks kc, ks kc + kc), kc a multiple of 4 (FP32 tiles) or
  // of 32 (BF16 products)
  const int kc = fp32 ? ((K + 15) / 16) * 4 : ((K + 127) / 128) * 32;
  // every wave runs the same number of passes (the 16-wave form has barriers)
  for (int base = 0; base * 16 < K; base += 4) {
    const int kt = base + slot, k0 = kt * 16;
    const bool active = k0 < K;
    floatx4 tre = zero4(), tim = zero4();
    if (active) {
      for (int q = 0; q < PER; ++q) {
        const int ks = (wid >> 2) + q;
        const int i0 = ks * kc, i1 = min(K, i0 + kc);
        floatx4 dr = zero4(), di = zero4();
        if (fp32) {
          // A(n, i) = conj(H[i][n]) from LDS;  B(i, k) = X[i][k]
          const int col = k0 + (lane & 15);
          const bool okc = col < K;
          const float2* xc = X + col;
          ctile16([&](int rr, int i) { return i < K ? cconj(hs[i * 16 + rr]) : cz(); },
                  [&](int i, int) { return (i < K && okc) ? xc[(size_t)i * K] : cz(); }, i0, i1, dr, di);
        } else {
          // BF16 operands, 32 users of the reduction per product
          const bool x3 = jb.prec == RZF_PREC_BF16X3;
          const int rr = lane & 15, kq = lane >> 4;
          const int n = n0 + rr, k = k0 + rr;
          for (int j0 = i0; j0 < i1; j0 += 32) {
            float2 a[8], b[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const int i = j0 + 8 * kq + e;
              a[e] = (n < N && i < K) ? H[(size_t)i * ldh + n] : cz();
              b[e] = (i < K && k < K) ? X[(size_t)i * K + k] : cz();
            }
            cmac8_bf16(a, b, true, false, x3, dr, di);
          }
        }
        tre += dr;
        tim += di;
      }
    }
    bool own = active;   // this wave writes the tile
    if constexpr (NW == 16) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        part[wid][v][lane] = tre[v];
        part[wid][4 + v][lane] = tim[v];
      }
      __syncthreads();
      own = active && wid < 4;
      if (own) {
        tre = zero4();
        tim = zero4();
        for (int q = 0; q < 4; ++q) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            tre[v] += part[slot + 4 * q][v][lane];
            tim[v] += part[slot + 4 * q][4 + v][lane];
          }
        }
      }
      __syncthreads();
    }
    if (own) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int n = n0 + tile_row(v), k = k0 + tile_col();
        if (n < N && k < K) {
          W[(size_t)n * ldw + k] = make_float2(tre[v], tim[v]);
          acc += (double)tre[v] * tre[v] + (double)tim[v] * tim[v];
        }
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
  if (threadIdx.x == 0) {
    // waves 4.. of the 16-wave form hold zero
    double w = red[0] + red[1] + red[2] + red[3];
    wpart[blockIdx.x] = w;
  }
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
  if (many) k_precoder<true><<<grid, 64 * prec_waves<true>(), 0, s>>>(one, many);
  else k_precoder<false><<<grid, 64 * prec_waves<false>(), 0, s>>>(one, many);
}

void launch_scale(const ScaleJob& one, const ScaleJob* many, int n, int maxNK, hipStream_t s) {
  const int blocks = (maxNK + 255) / 256 < SCALE_BLOCKS ? (maxNK + 255) / 256 : SCALE_BLOCKS;
  const dim3 grid(blocks, many ? n : 1);
  if (many) k_scale<true><<<grid, 256, 0, s>>>(one, many);
  else k_scale<false><<<grid, 256, 0, s>>>(one, many);
}
