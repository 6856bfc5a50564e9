// Precoder W = H^H X with its power normalisation ||W||_F^2 = P (Sec. II,
// eq. (5)), where X is the stored inverse of the Gram matrix.
//
// W is N x K (row-major).  A workgroup of 16 wavefronts owns PB rows of W (PB
// antennas, 32 or 64, or 256 when every track has K <= 64: a launch choice) of one track and computes their
// 16x16 tiles (PB/16 x ceil(K/16) of them, wave w taking tiles w, w + 16, ...)
// on the FP32 matrix cores.  The length-K reduction runs over chunks of 32
// users: the chunk's 32 x PB block of H and its 32 x K rows of X are staged in
// LDS (the next chunk's loads in flight while this one is multiplied), so H
// and X are read from memory once per workgroup.  For rzf_update the staged H
// is also copied into the track's H_prev.
//
// Every workgroup writes its rows of W and, per group of 32 rows, the FP64
// sum of their |w|^2 (each 16x16 tile summed by its wave, the tiles of a
// group added in a fixed order): the same partial sums whatever PB is, so
// the choice of PB never changes a result.  A second kernel then adds the
// partial sums in order and rescales W by sqrt(P / ||W||_F^2), with 16-byte
// loads and stores.  The two launches meet at a kernel boundary, which makes
// the partial sums visible to every XCD's L2 without a fence per workgroup.
//
// With the BF16 precision options the products take BF16 operands (or BF16
// hi/lo splits, three products each), read per tile from memory, with FP32
// accumulation.
#include "rzf_device.h"
#include "rzf_internal.h"

namespace {

constexpr int PG = 32;          // rows of W per partial sum of |w|^2
constexpr int PIC = 32;         // users per reduction chunk
constexpr int PNT = 1024;       // threads per workgroup
constexpr int PNW = PNT / 64;

// Dynamic LDS of a launch with PB rows per workgroup for tracks up to maxK
// users: the H chunk (row stride PB + 4), then the X chunk (row stride maxK + 4).
size_t prec_lds_bytes(int pb, int maxK) { return sizeof(float2) * (size_t)PIC * (pb + 4 + maxK + 4); }

// KMX: the largest K of the launch's tracks the kernel is built for (64 or KM).
template <bool MANY, int PB, int KMX>
__global__ __launch_bounds__(PNT) void k_precoder(PrecJob one, const PrecJob* many, int xld) {
  constexpr int HLD = PB + 4;                 // LDS row stride of the staged H chunk (float2)
  constexpr int HPER = PIC * PB / PNT;        // H values a thread stages per chunk
  constexpr int XPER = (PIC * KMX + PNT - 1) / PNT;  // X values a thread stages per chunk, at most
  extern __shared__ float2 dyn[];
  float2* hs = dyn;                       // [PIC][HLD]: H[i0 + ii][n0 + c] at hs[ii * HLD + c]
  float2* xs = dyn + PIC * HLD;           // [PIC][xld]: X[i0 + ii][k] at xs[ii * xld + k]
  __shared__ double tsum[PB / 16][KMX / 16];  // |w|^2 of each 16x16 tile
  const GridPos gp = grid_pos<MANY>();
  const PrecJob& jb = job_at<MANY>(one, many, gp.item);
  const int K = jb.K, N = jb.N, ldh = jb.ldh, ldw = jb.ldw;
  const float2* __restrict__ H = jb.H;
  const float2* __restrict__ X = jb.X;
  float2* __restrict__ W = jb.W;
  double* __restrict__ wpart = jb.wpart;
  // a step that met a non-finite snapshot keeps the track's previous one
  float2* __restrict__ Hcopy = (jb.hold && *jb.hold) ? nullptr : jb.Hcopy;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int n0 = gp.x * PB;
  if (n0 >= N) return;
  const int kt = (K + 15) / 16;
  const int ntile = (PB / 16) * kt;
  constexpr int TPW = (PB / 16) * (KMX / 16) / PNW;  // tiles per wave, at most
  floatx4 tre[TPW], tim[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) { tre[q] = zero4(); tim[q] = zero4(); }
  const bool fp32 = jb.prec == RZF_PREC_FP32;
  if (fp32) {
    float2 ph[HPER], px[XPER];
    auto fetch = [&](int i0) {
#pragma unroll
      for (int e = 0; e < HPER; ++e) {
        const int idx = tid + PNT * e;          // 32 users x 64 antennas
        const int i = i0 + idx / PB, n = n0 + idx % PB;
        ph[e] = (i < K && n < N) ? H[(size_t)i * ldh + n] : cz();
      }
#pragma unroll
      for (int e = 0; e < XPER; ++e) {
        const int idx = tid + PNT * e;          // 32 users x K
        const int ii = idx / K, k = idx - ii * K;
        px[e] = (ii < PIC && i0 + ii < K) ? X[(size_t)(i0 + ii) * K + k] : cz();
      }
    };
    fetch(0);
    for (int i0 = 0; i0 < K; i0 += PIC) {
#pragma unroll
      for (int e = 0; e < HPER; ++e) {
        const int idx = tid + PNT * e;
        const int ii = idx / PB, c = idx % PB;
        hs[ii * HLD + c] = ph[e];
        if (Hcopy && i0 + ii < K && n0 + c < N) Hcopy[(size_t)(i0 + ii) * N + n0 + c] = ph[e];
      }
#pragma unroll
      for (int e = 0; e < XPER; ++e) {
        const int idx = tid + PNT * e;
        const int ii = idx / K, k = idx - ii * K;
        if (ii < PIC) xs[ii * xld + k] = px[e];
      }
      __syncthreads();
      if (i0 + PIC < K) fetch(i0 + PIC);
      const int ic = min(PIC, K - i0);   // users of this chunk (the rest of LDS holds zeros)
#pragma unroll
      for (int q = 0; q < TPW; ++q) {
        const int t = wid + PNW * q;
        if (t >= ntile) break;
        const int nt = t % (PB / 16), ct = t / (PB / 16);
        const int col = ct * 16 + (lane & 15);
        const bool okc = col < K;
        // A(n, i) = conj(H[i][n]);  B(i, k) = X[i][k]
        ctile16([&](int rr, int i) { return cconj(hs[i * HLD + nt * 16 + rr]); },
                [&](int i, int) { return okc ? xs[i * xld + col] : cz(); }, 0, (ic + 3) & ~3, tre[q], tim[q]);
      }
      __syncthreads();
    }
  } else {
    // BF16 operands, 32 users of the reduction per product
    const bool x3 = jb.prec == RZF_PREC_BF16X3;
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int t = wid + PNW * q;
      if (t >= ntile) break;
      const int nt = t % (PB / 16), ct = t / (PB / 16);
      const int rr = lane & 15, kq = lane >> 4;
      const int n = n0 + nt * 16 + rr, k = ct * 16 + rr;
      for (int j0 = 0; j0 < K; j0 += 32) {
        float2 a[8], b[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int i = j0 + 8 * kq + e;
          a[e] = (n < N && i < K) ? H[(size_t)i * ldh + n] : cz();
          b[e] = (i < K && k < K) ? X[(size_t)i * K + k] : cz();
        }
        cmac8_bf16(a, b, true, false, x3, tre[q], tim[q]);
      }
    }
    if (Hcopy)
      for (int e = tid; e < K * PB; e += PNT) {
        const int i = e / PB, n = n0 + e % PB;
        if (n < N) Hcopy[(size_t)i * N + n] = H[(size_t)i * ldh + n];
      }
  }
  // the block's rows of W (unscaled) and each tile's sum of |w|^2
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    const int t = wid + PNW * q;
    if (t >= ntile) break;
    const int nt = t % (PB / 16), ct = t / (PB / 16);
    double acc = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int n = n0 + nt * 16 + tile_row(v), k = ct * 16 + tile_col();
      if (n < N && k < K) {
        W[(size_t)n * ldw + k] = make_float2(tre[q][v], tim[q][v]);
        acc += (double)tre[q][v] * tre[q][v] + (double)tim[q][v] * tim[q][v];
      }
    }
    acc = wave_sum(acc);
    if (lane == 0) tsum[nt][ct] = acc;
  }
  __syncthreads();
  // one partial per 32 rows: its two row tiles, column tiles in order
  if (tid < PB / PG) {
    const int g = tid;
    if (n0 + g * PG < N) {
      double w = 0.0;
      for (int ct = 0; ct < kt; ++ct) w += tsum[2 * g][ct] + tsum[2 * g + 1][ct];
      wpart[n0 / PG + g] = w;
    }
  }
}

// Power normalisation: blocks of SCT threads stride over a track's N x K
// entries of W (at most SCB blocks per track); each first adds the partial
// sums in block order.  Rows of W are scaled two entries per 16-byte access
// when ldw and K are even (the row starts are then 16-byte aligned).
constexpr int SCT = 256, SCB = 64;

template <bool MANY>
__global__ __launch_bounds__(SCT) void k_scale(ScaleJob one, const ScaleJob* many) {
  const ScaleJob& jb = job_of<MANY>(one, many);
  const int K = jb.K, N = jb.N, ldw = jb.ldw, nparts = jb.nparts;
  float2* __restrict__ W = jb.W;
  const int per = (N * K + 2 * SCT - 1) / (2 * SCT);   // blocks a track needs at two entries per thread
  if ((int)blockIdx.x >= min(per, SCB)) return;
  __shared__ float sc;
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int b = 0; b < nparts; ++b) tot += jb.wpart[b];
    sc = tot > 0.0 ? (float)sqrt(jb.P / tot) : 0.f;
  }
  __syncthreads();
  const float s = sc;
  if (jb.adv && blockIdx.x == 0 && threadIdx.x == 0) {
    // the track's step is complete: its next one takes the next index and tag
    jb.adv->t_dev += 1;
    jb.adv->seq_dev += 1;
  }
  const int stride = min(per, SCB) * SCT;
  if ((K & 1) == 0 && (ldw & 1) == 0 && (reinterpret_cast<uintptr_t>(W) & 15) == 0) {
    const int K2 = K >> 1;
    for (int e = blockIdx.x * SCT + threadIdx.x; e < N * K2; e += stride) {
      const int n = e / K2, k2 = e - n * K2;
      float4* w = reinterpret_cast<float4*>(W + (size_t)n * ldw) + k2;
      float4 v = *w;
      v.x *= s; v.y *= s; v.z *= s; v.w *= s;
      *w = v;
    }
  } else {
    for (int e = blockIdx.x * SCT + threadIdx.x; e < N * K; e += stride) {
      const int n = e / K, k = e - n * K;
      float2* w = W + (size_t)n * ldw + k;
      *w = cscale(*w, s);
    }
  }
}

}  // namespace

int precoder_blocks(int N) { return (N + PG - 1) / PG; }

void launch_scale(const ScaleJob& one, const ScaleJob* many, int n, int maxNK, hipStream_t s) {
  const int blocks = std::min((maxNK + 2 * SCT - 1) / (2 * SCT), SCB);
  const dim3 grid(blocks, many ? n : 1);
  if (many) k_scale<true><<<grid, SCT, 0, s>>>(one, many);
  else k_scale<false><<<grid, SCT, 0, s>>>(one, many);
}

int precoder_scratch(int N) { return precoder_blocks(N); }

template <int PB, int KMX>
void launch_precoder_pb(const PrecJob& one, const PrecJob* many, int n, int maxN, int maxK, hipStream_t s) {
  const dim3 grid((maxN + PB - 1) / PB, many ? n : 1);
  const size_t lds = prec_lds_bytes(PB, maxK);
  const int xld = maxK + 4;
  if (many) k_precoder<true, PB, KMX><<<grid, PNT, lds, s>>>(one, many, xld);
  else k_precoder<false, PB, KMX><<<grid, PNT, lds, s>>>(one, many, xld);
}

void launch_precoder(const PrecJob& one, const PrecJob* many, int n, int maxN, int maxK, int pb, hipStream_t s) {
  if (pb == 256 && maxK <= 64) launch_precoder_pb<256, 64>(one, many, n, maxN, maxK, s);
  else if (pb == 32) launch_precoder_pb<32, KM>(one, many, n, maxN, maxK, s);
  else launch_precoder_pb<64, KM>(one, many, n, maxN, maxK, s);
}
