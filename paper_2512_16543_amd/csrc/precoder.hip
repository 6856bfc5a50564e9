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

// LDS row stride of the staged X chunk for tracks up to maxK users: the
// columns of whole 16-column tiles, plus 4.
int prec_xld(int maxK) { return ((maxK + 15) & ~15) + 4; }

// Dynamic LDS of a launch with PB rows per workgroup for tracks up to maxK
// users: the H chunk (row stride PB + 4), then the X chunk (row stride prec_xld).
size_t prec_lds_bytes(int pb, int maxK) { return sizeof(float2) * (size_t)PIC * (pb + 4 + prec_xld(maxK)); }

// KMX: the largest K of the launch's tracks the kernel is built for (64 or KM);
// PNT: threads per workgroup.  FUSE (a launch whose workgroups each hold a
// whole track, N <= PB): the workgroup also does k_scale's work for its
// track (same partial sums, added in the same order, same scale factor), so
// W is written once, already scaled.
template <bool MANY, int PB, int KMX, int PNT, bool FUSE>
__global__ __launch_bounds__(PNT) void k_precoder(PrecJob one, const PrecJob* many, ScaleJob sone,
                                                  const ScaleJob* smany, int xld) {
  constexpr int PNW = PNT / 64;
  static_assert((PIC * PB) % PNT == 0 && ((PB / 16) * (KMX / 16)) % PNW == 0, "launch shape");
  constexpr int HLD = PB + 4;                 // LDS row stride of the staged H chunk (float2)
  constexpr int HPER = PIC * PB / PNT;        // H values a thread stages per chunk
  constexpr int XPER = (PIC * KMX + PNT - 1) / PNT;  // X values a thread stages per chunk, at most
  extern __shared__ float2 dyn[];
  float2* hs = dyn;                       // [PIC][HLD]: H[i0 + ii][n0 + c] at hs[ii * HLD + c]
  float2* xs = dyn + PIC * HLD;           // [PIC][xld]: X[i0 + ii][k] at xs[ii * xld + k],
                                          // zeros past K up to the last column tile
  __shared__ double tsum[PB / 16][KMX / 16];  // |w|^2 of each 16x16 tile
  const GridPos gp = grid_pos<MANY>();
  const PrecJob& jb = job_at<MANY>(one, many, gp.item);
  const int K = jb.K, N = jb.N, ldh = jb.ldh, ldw = jb.ldw;
  const float2* __restrict__ H = jb.H;
  const float2* __restrict__ X = jb.X;
  float2* __restrict__ W = jb.W;
  double* __restrict__ wpart = jb.wpart;
  // a step that met a non-finite snapshot keeps the track's previous one
  float2* __restrict__ Hcopy = (jb.hold && gld(jb.hold, 0)) ? nullptr : jb.Hcopy;
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
    static_assert(PNW % (PB / 16) == 0, "a wave's tiles share their rows of W");
    const int nt = wid % (PB / 16), rr = lane & 15, kk = lane >> 4;
    int nq = 0;   // the wave's tiles inside the track (wave-uniform)
#pragma unroll
    for (int q = 0; q < TPW; ++q) nq += __builtin_amdgcn_readfirstlane(wid) + PNW * q < ntile ? 1 : 0;
    const int K16 = kt * 16;   // columns of whole tiles (X staged with zeros past K)
    int colc[TPW];             // the tile's column of X for this lane (a tile past the
                               // track reads, unused, the last staged column)
#pragma unroll
    for (int q = 0; q < TPW; ++q) colc[q] = min(((wid + PNW * q) / (PB / 16)) * 16 + rr, K16 - 1);
    float2 ph[HPER], px[XPER];
    auto fetch = [&](int i0) {
#pragma unroll
      for (int e = 0; e < HPER; ++e) {
        const int idx = tid + PNT * e;          // 32 users x 64 antennas
        const int i = i0 + idx / PB, n = n0 + idx % PB;
        ph[e] = (i < K && n < N) ? gld(H, (size_t)i * ldh + n) : cz();
      }
#pragma unroll
      for (int e = 0; e < XPER; ++e) {
        const int idx = tid + PNT * e;          // 32 users x K
        const int ii = idx / K16, k = idx - ii * K16;
        px[e] = (ii < PIC && i0 + ii < K && k < K) ? gld(X, (size_t)(i0 + ii) * K + k) : cz();
      }
    };
    fetch(0);
    for (int i0 = 0; i0 < K; i0 += PIC) {
#pragma unroll
      for (int e = 0; e < HPER; ++e) {
        const int idx = tid + PNT * e;
        const int ii = idx / PB, c = idx % PB;
        hs[ii * HLD + c] = ph[e];
        if (Hcopy && i0 + ii < K && n0 + c < N) gst(Hcopy, (size_t)(i0 + ii) * N + n0 + c, ph[e]);
      }
#pragma unroll
      for (int e = 0; e < XPER; ++e) {
        const int idx = tid + PNT * e;
        const int ii = idx / K16, k = idx - ii * K16;
        if (ii < PIC) xs[ii * xld + k] = px[e];
      }
      __syncthreads();
      if (i0 + PIC < K) fetch(i0 + PIC);
      const int steps = (min(PIC, K - i0) + 3) / 4;   // 4 users per product (past K: zeros in LDS)
      // A(n, i) = conj(H[i][n]);  B(i, k) = X[i][k].  The wave's tiles share
      // their rows of W, so a step reads the H operand once for all of them,
      // and the next step's operands are read while this one's products run.
      // Every tile's products are those of ctile16, in its order.
      auto operands = [&](int st, float2& av, float2 (&bv)[TPW]) {
        const int i = min(4 * st + kk, PIC - 1);   // a step past the chunk reads, unused, its last row
        av = hs[i * HLD + nt * 16 + rr];   // conjugated in the products below
#pragma unroll
        for (int q = 0; q < TPW; ++q) bv[q] = xs[i * xld + colc[q]];
      };
      auto products = [&](const float2& av, const float2 (&bv)[TPW]) {
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
          if (q >= nq) break;
          tre[q] = mfma4(av.x, bv[q].x, tre[q]);
          tre[q] = mfma4(av.y, bv[q].y, tre[q]);
          tim[q] = mfma4(av.x, bv[q].y, tim[q]);
          tim[q] = mfma4(-av.y, bv[q].x, tim[q]);
        }
      };
      // two operand buffers in turn: a step's products run while the next
      // step's operands are read
      float2 a0, b0[TPW], a1, b1[TPW];
      operands(0, a0, b0);
      for (int st = 0; st < steps; st += 2) {
        operands(st + 1, a1, b1);
        products(a0, b0);
        operands(st + 2, a0, b0);
        if (st + 1 < steps) products(a1, b1);
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
          a[e] = (n < N && i < K) ? gld(H, (size_t)i * ldh + n) : cz();
          b[e] = (i < K && k < K) ? gld(X, (size_t)i * K + k) : cz();
        }
        cmac8_bf16(a, b, true, false, x3, tre[q], tim[q]);
      }
    }
    if (Hcopy)
      for (int e = tid; e < K * PB; e += PNT) {
        const int i = e / PB, n = n0 + e % PB;
        if (n < N) gst(Hcopy, (size_t)i * N + n, gld(H, (size_t)i * ldh + n));
      }
  }
  // the block's rows of W (unscaled, unless FUSE) and each tile's sum of |w|^2
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
        if (!FUSE) gst(W, (size_t)n * ldw + k, make_float2(tre[q][v], tim[q][v]));
        acc += (double)tre[q][v] * tre[q][v] + (double)tim[q][v] * tim[q][v];
      }
    }
    acc = wave_sum(acc);
    if (lane == 0) tsum[nt][ct] = acc;
  }
  __syncthreads();
  if (FUSE) {
    // the track's partials (those of the 32-row groups) added in order, then
    // W = sqrt(P / ||W||^2) W, as k_scale does
    __shared__ float sc;
    const ScaleJob& sj = job_at<MANY>(sone, smany, gp.item);
    if (tid == 0) {
      double tot = 0.0;
      for (int g = 0; g * PG < N; ++g) {
        double w = 0.0;
        for (int ct = 0; ct < kt; ++ct) w += tsum[2 * g][ct] + tsum[2 * g + 1][ct];
        tot += w;
      }
      sc = tot > 0.0 ? (float)sqrt(sj.P / tot) : 0.f;
      if (sj.adv) {
        // the track's step is complete: its next one takes the next index and tag
        sj.adv->t_dev += 1;
        sj.adv->seq_dev += 1;
      }
    }
    __syncthreads();
    const float s = sc;
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int t = wid + PNW * q;
      if (t >= ntile) break;
      const int nt = t % (PB / 16), ct = t / (PB / 16);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int n = n0 + nt * 16 + tile_row(v), k = ct * 16 + tile_col();
        if (n < N && k < K) gst(W, (size_t)n * ldw + k, make_float2(tre[q][v] * s, tim[q][v] * s));
      }
    }
    return;
  }
  // one partial per 32 rows: its two row tiles, column tiles in order
  if (tid < PB / PG) {
    const int g = tid;
    if (n0 + g * PG < N) {
      double w = 0.0;
      for (int ct = 0; ct < kt; ++ct) w += tsum[2 * g][ct] + tsum[2 * g + 1][ct];
      gst(wpart, (size_t)(n0 / PG + g), w);
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

template <int PB, int KMX, int PNT = 1024>
bool launch_precoder_pb(const PrecJob& one, const PrecJob* many, const ScaleJob& sone, const ScaleJob* smany,
                        int n, int maxN, int maxK, hipStream_t s) {
  const int nb = (maxN + PB - 1) / PB;
  const dim3 grid(nb, many ? n : 1);
  const size_t lds = prec_lds_bytes(PB, maxK);
  const int xld = prec_xld(maxK);
  if (nb == 1) {
    if (many) k_precoder<true, PB, KMX, PNT, true><<<grid, PNT, lds, s>>>(one, many, sone, smany, xld);
    else k_precoder<false, PB, KMX, PNT, true><<<grid, PNT, lds, s>>>(one, many, sone, smany, xld);
    return true;
  }
  if (many) k_precoder<true, PB, KMX, PNT, false><<<grid, PNT, lds, s>>>(one, many, sone, smany, xld);
  else k_precoder<false, PB, KMX, PNT, false><<<grid, PNT, lds, s>>>(one, many, sone, smany, xld);
  return false;
}

bool launch_precoder(const PrecJob& one, const PrecJob* many, const ScaleJob& sone, const ScaleJob* smany, int n,
                     int maxN, int maxK, int pb, hipStream_t s) {
  if (pb == 256 && maxK <= 64) return launch_precoder_pb<256, 64>(one, many, sone, smany, n, maxN, maxK, s);
  if (pb == 32) return launch_precoder_pb<32, KM>(one, many, sone, smany, n, maxN, maxK, s);
  return launch_precoder_pb<64, KM>(one, many, sone, smany, n, maxN, maxK, s);
}
