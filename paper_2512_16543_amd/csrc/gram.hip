// Gram matrix and its per-step correction on the FP32 matrix cores.
//
//   A'      = H_t H_t^H + alpha I_K                      (Sec. II, eq. (5); eq. (7))
//   Delta A = H_{t-1} dH^H + dH H_t^H,  dH = H_t - H_{t-1}
//
// The second line is eq. (9), H dH^H + dH H^H + dH dH^H, with the last two
// terms grouped as dH (H + dH)^H.  Forming Delta A from dH keeps its rounding
// error proportional to ||Delta A|| rather than to ||A'||, which the
// difference A' - A would not (the per-step change is ~1e-4 of A).
//
// With the BF16 precision options the products take BF16 operands (or
// BF16 hi/lo splits, three products each) with FP32 accumulation.
//
// Both outputs are Hermitian, so only the lower 16x16 tiles are computed and
// mirrored.  A workgroup of four wavefronts owns one output tile and splits
// the length-N reduction between its waves; the partial tiles are summed in
// a fixed order (deterministic).
#include "rzf_device.h"
#include "rzf_internal.h"

namespace {

__device__ __forceinline__ void mac_conj(float2 x, float2 y, floatx4& dr, floatx4& di) {
  // D += x * conj(y)
  dr = mfma4(x.x, y.x, dr);
  dr = mfma4(x.y, y.y, dr);
  di = mfma4(x.y, y.x, di);
  di = mfma4(-x.x, y.y, di);
}

template <bool DELTA, bool MANY>
__global__ __launch_bounds__(256) void k_gram(GramJob one, const GramJob* many) {
  // FP32 path: chunks of GC antennas staged through LDS (rows i0.. and j0.. of
  // H_t, then of H_{t-1}).  An operand read takes one antenna of 16 rows per
  // 16 lanes: the odd row stride GLD (130 dwords, 2 mod 32) puts those rows
  // in distinct bank pairs (a stride of 68 put four rows on each pair).  The
  // partial tiles reuse the same memory afterwards.
  constexpr int GC = 64, GLD = GC + 1;
  __shared__ float2 st[4][16][GLD];
  float (*red)[16][64] = reinterpret_cast<float (*)[16][64]>(&st[0][0][0]);
  const GridPos gp = grid_pos<MANY>();
  const GramJob& jb = job_at<MANY>(one, many, gp.item);
  const int K = jb.K, N = jb.N, ldh = jb.ldh, ldp = jb.ldp;
  const float2* __restrict__ Ht = jb.Ht;
  const float2* __restrict__ Hp = jb.Hp;
  float2* __restrict__ Anew = jb.Anew;
  float2* __restrict__ dA = jb.dA;
  const float alpha = jb.alpha;
  const int ktl = (K + 15) / 16;
  // lower-triangular tile index -> (bi, bj), bi >= bj
  const int tix = gp.x;
  if (tix >= ktl * (ktl + 1) / 2) return;
  int bi = (int)((sqrtf(8.0f * tix + 1.0f) - 1.0f) * 0.5f);
  while ((bi + 1) * (bi + 2) / 2 <= tix) ++bi;
  while (bi * (bi + 1) / 2 > tix) --bi;
  const int bj = tix - bi * (bi + 1) / 2;
  const int i0 = bi * 16, j0 = bj * 16;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int r = lane & 15, kq = lane >> 4;
  const int ri = i0 + r, rj = j0 + r;
  const bool oki = ri < K, okj = rj < K;

  floatx4 ar = zero4(), ai = zero4(), gr = zero4(), gi = zero4();
  if (jb.prec == RZF_PREC_FP32) {
    // A wavefront's load reads 64 consecutive antennas of one row (four cache
    // lines instead of sixteen).  Wave w takes antennas 16 w .. 16 w + 15 of
    // every chunk, four per product step, in increasing order; the next
    // chunk's loads are in flight while this one is multiplied.
    constexpr int NM = DELTA ? 4 : 2;
    float2 pre[NM][4];
    auto fetch = [&](int c0) {
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        const float2* src = m < 2 ? Ht : Hp;
        const int ld = m < 2 ? ldh : ldp;
        const int rb = (m & 1) ? j0 : i0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int idx = threadIdx.x + 256 * e;   // 16 rows x 64 antennas
          const int row = rb + (idx >> 6), n = c0 + (idx & 63);
          pre[m][e] = (row < K && n < N) ? gld(src, (size_t)row * ld + n) : cz();
        }
      }
    };
    fetch(0);
    for (int c0 = 0; c0 < N; c0 += GC) {
#pragma unroll
      for (int m = 0; m < NM; ++m)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int idx = threadIdx.x + 256 * e;
          st[m][idx >> 6][idx & 63] = pre[m][e];
        }
      __syncthreads();
      if (c0 + GC < N) fetch(c0 + GC);
#pragma unroll
      for (int k = 0; k < 16; k += 4) {
        const int nn = wid * 16 + k + kq;
        const float2 ti = st[0][r][nn];
        const float2 tj = st[1][r][nn];
        mac_conj(ti, tj, ar, ai);                         // H_t H_t^H
        if (DELTA) {
          const float2 pi = st[2][r][nn];
          const float2 pj = st[3][r][nn];
          const float2 di = csub(ti, pi), dj = csub(tj, pj);
          mac_conj(pi, dj, gr, gi);                       // H_{t-1} dH^H
          mac_conj(di, tj, gr, gi);                       // dH H_t^H
        }
      }
      __syncthreads();
    }
  } else {
    // BF16 operands, 32 antennas per product; dH is formed in FP32 before
    // rounding, so the correction keeps its error relative to ||Delta A||
    const bool x3 = jb.prec == RZF_PREC_BF16X3;
    for (int n0 = wid * 32; n0 < N; n0 += 128) {
      const int nb = n0 + 8 * kq;
      float2 ti[8], tj[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int n = nb + e;
        const bool okn = n < N;
        ti[e] = (oki && okn) ? gld(Ht, (size_t)ri * ldh + n) : cz();
        tj[e] = (okj && okn) ? gld(Ht, (size_t)rj * ldh + n) : cz();
      }
      cmac8_bf16(ti, tj, false, true, x3, ar, ai);       // H_t H_t^H
      if (DELTA) {
        float2 pi[8], dj[8], di[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int n = nb + e;
          const bool okn = n < N;
          pi[e] = (oki && okn) ? gld(Hp, (size_t)ri * ldp + n) : cz();
          const float2 pj = (okj && okn) ? gld(Hp, (size_t)rj * ldp + n) : cz();
          di[e] = csub(ti[e], pi[e]);
          dj[e] = csub(tj[e], pj);
        }
        cmac8_bf16(pi, dj, false, true, x3, gr, gi);     // H_{t-1} dH^H
        cmac8_bf16(di, tj, false, true, x3, gr, gi);     // dH H_t^H
      }
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    red[wid][v][lane] = ar[v];
    red[wid][4 + v][lane] = ai[v];
    red[wid][8 + v][lane] = gr[v];
    red[wid][12 + v][lane] = gi[v];
  }
  __syncthreads();
  if (wid != 0) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    float s[4] = {0.f, 0.f, 0.f, 0.f};
    for (int w = 0; w < 4; ++w) {
      s[0] += red[w][v][lane];
      s[1] += red[w][4 + v][lane];
      s[2] += red[w][8 + v][lane];
      s[3] += red[w][12 + v][lane];
    }
    const int i = i0 + tile_row(v), j = j0 + tile_col();
    if (i >= K || j >= K) continue;
    if (bi == bj && i < j) continue;   // the diagonal tile is mirrored from below
    float2 a = make_float2(s[0], s[1]);
    float2 g = make_float2(s[2], s[3]);
    if (i == j) {
      a = make_float2(a.x + alpha, 0.f);
      g.y = 0.f;
    }
    gst(Anew, (size_t)i * K + j, a);
    if (i != j) gst(Anew, (size_t)j * K + i, cconj(a));
    if (DELTA) {
      gst(dA, (size_t)i * K + j, g);
      if (i != j) gst(dA, (size_t)j * K + i, cconj(g));
    }
  }
}

// Lower 16x16 tile t of a K x K Hermitian output -> block coordinates (bi >= bj).
__device__ __forceinline__ void lower_tile(int t, int* bi, int* bj) {
  int i = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  *bi = i;
  *bj = t - i * (i + 1) / 2;
}

// Batched Gram of FP32 tracks with K <= 64: one 16-wave workgroup per track,
// which stages each chunk of 64 antennas of H_t (and H_{t-1}) once for all of
// the track's lower tiles instead of once per tile.  A work unit (tile,
// slice) is exactly what wave `slice` of k_gram computes for that tile
// (antennas 16 slice .. 16 slice + 15 of every chunk, four per product step,
// in increasing order, in its own accumulators), unit u = 4 tile + slice runs
// on wave u mod 16, and the four slices of a tile are added in k_gram's
// order: a track's A' and Delta A are bit-identical to k_gram's.
template <bool DELTA>
__global__ __launch_bounds__(1024) void k_gram_track(const GramJob* many) {
  constexpr int GC = 64, GLD = GC + 1, KT = 64, NM = DELTA ? 2 : 1;   // GLD: as in k_gram
  __shared__ float2 st[2][KT][GLD];   // [H_t, H_{t-1}][row][antenna of the chunk]
  // after the last chunk: one 16 x 64 float block per wave (the tile partials)
  float (*red)[16][64] = reinterpret_cast<float (*)[16][64]>(&st[0][0][0]);
  const GridPos gp = xcd_grid_pos();
  const GramJob& jb = many[gp.item];
  const int K = jb.K, N = jb.N, ldh = jb.ldh, ldp = jb.ldp;
  const float2* __restrict__ Ht = jb.Ht;
  const float2* __restrict__ Hp = jb.Hp;
  float2* __restrict__ Anew = jb.Anew;
  float2* __restrict__ dA = jb.dA;
  const float alpha = jb.alpha;
  const int ktl = (K + 15) / 16;
  const int nunit = 2 * ktl * (ktl + 1);        // 4 slices x the lower tiles
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int r = lane & 15, kq = lane >> 4;
  floatx4 acc[3][4];                             // units wid, wid + 16, wid + 32
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[q][c] = zero4();
  float2 pre[NM][4];
  auto fetch = [&](int c0) {
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      const float2* src = m == 0 ? Ht : Hp;
      const int ld = m == 0 ? ldh : ldp;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int idx = threadIdx.x + 1024 * e;   // 64 rows x 64 antennas
        const int row = idx >> 6, n = c0 + (idx & 63);
        pre[m][e] = (row < K && n < N) ? gld(src, (size_t)row * ld + n) : cz();
      }
    }
  };
  fetch(0);
  for (int c0 = 0; c0 < N; c0 += GC) {
#pragma unroll
    for (int m = 0; m < NM; ++m)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int idx = threadIdx.x + 1024 * e;
        st[m][idx >> 6][idx & 63] = pre[m][e];
      }
    __syncthreads();
    if (c0 + GC < N) fetch(c0 + GC);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int u = wid + 16 * q;
      if (u >= nunit) break;
      int bi, bj;
      lower_tile(u >> 2, &bi, &bj);
      const int sl = u & 3;
#pragma unroll
      for (int k = 0; k < 16; k += 4) {
        const int nn = sl * 16 + k + kq;
        const float2 ti = st[0][bi * 16 + r][nn];
        const float2 tj = st[0][bj * 16 + r][nn];
        mac_conj(ti, tj, acc[q][0], acc[q][1]);          // H_t H_t^H
        if (DELTA) {
          const float2 pi = st[1][bi * 16 + r][nn];
          const float2 pj = st[1][bj * 16 + r][nn];
          const float2 di = csub(ti, pi), dj = csub(tj, pj);
          mac_conj(pi, dj, acc[q][2], acc[q][3]);        // H_{t-1} dH^H
          mac_conj(di, tj, acc[q][2], acc[q][3]);        // dH H_t^H
        }
      }
    }
    __syncthreads();
  }
  // one round per unit slot q: every wave posts its unit, and the wave of a
  // tile's slice 0 adds the four slices (waves wid .. wid + 3) in order
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    if (16 * q >= nunit) break;
    const int u = wid + 16 * q;
    if (u < nunit) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        red[wid][v][lane] = acc[q][0][v];
        red[wid][4 + v][lane] = acc[q][1][v];
        red[wid][8 + v][lane] = acc[q][2][v];
        red[wid][12 + v][lane] = acc[q][3][v];
      }
    }
    __syncthreads();
    if (u < nunit && (u & 3) == 0) {
      int bi, bj;
      lower_tile(u >> 2, &bi, &bj);
      const int i0 = bi * 16, j0 = bj * 16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float sm[4] = {0.f, 0.f, 0.f, 0.f};
        for (int w = 0; w < 4; ++w) {
          sm[0] += red[wid + w][v][lane];
          sm[1] += red[wid + w][4 + v][lane];
          sm[2] += red[wid + w][8 + v][lane];
          sm[3] += red[wid + w][12 + v][lane];
        }
        const int i = i0 + tile_row(v), j = j0 + tile_col();
        if (i >= K || j >= K) continue;
        if (bi == bj && i < j) continue;   // the diagonal tile is mirrored from below
        float2 a = make_float2(sm[0], sm[1]);
        float2 g = make_float2(sm[2], sm[3]);
        if (i == j) {
          a = make_float2(a.x + alpha, 0.f);
          g.y = 0.f;
        }
        gst(Anew, (size_t)i * K + j, a);
        if (i != j) gst(Anew, (size_t)j * K + i, cconj(a));
        if (DELTA) {
          gst(dA, (size_t)i * K + j, g);
          if (i != j) gst(dA, (size_t)j * K + i, cconj(g));
        }
      }
    }
    __syncthreads();
  }
}

// FP64 Gram for the exact (re-)inversions: one thread per lower element.
template <bool MANY>
__global__ __launch_bounds__(256) void k_gram64(Gram64Job one, const Gram64Job* many) {
  const Gram64Job& jb = job_of<MANY>(one, many);
  const int K = jb.K, N = jb.N, ldh = jb.ldh;
  const float2* __restrict__ H = jb.H;
  double2* __restrict__ A = jb.A;
  const double alpha = jb.alpha;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int nl = K * (K + 1) / 2;
  if (e >= nl) return;
  int i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= e) ++i;
  while (i * (i + 1) / 2 > e) --i;
  const int j = e - i * (i + 1) / 2;
  const float2* hi = H + (size_t)i * ldh;
  const float2* hj = H + (size_t)j * ldh;
  double re = 0.0, im = 0.0;
  for (int n = 0; n < N; ++n) {
    const double2 a = f2d(hi[n]), b = f2d(hj[n]);
    re += a.x * b.x + a.y * b.y;
    im += a.y * b.x - a.x * b.y;
  }
  if (i == j) {
    A[(size_t)i * K + i] = make_double2(re + alpha, 0.0);
  } else {
    A[(size_t)i * K + j] = make_double2(re, im);
    A[(size_t)j * K + i] = make_double2(re, -im);
  }
}

}  // namespace

void launch_gram(const GramJob& one, const GramJob* many, int n, int maxK, bool per_track, hipStream_t s) {
  if (many && per_track && maxK <= 64) {
    if (one.Hp != nullptr) k_gram_track<true><<<dim3(1, n), 1024, 0, s>>>(many);
    else k_gram_track<false><<<dim3(1, n), 1024, 0, s>>>(many);
    return;
  }
  const int kt = (maxK + 15) / 16;
  const dim3 grid(kt * (kt + 1) / 2, many ? n : 1);
  const bool delta = one.Hp != nullptr;   // a batch passes its mode in `one`
  if (delta) {
    if (many) k_gram<true, true><<<grid, 256, 0, s>>>(one, many);
    else k_gram<true, false><<<grid, 256, 0, s>>>(one, many);
  } else {
    if (many) k_gram<false, true><<<grid, 256, 0, s>>>(one, many);
    else k_gram<false, false><<<grid, 256, 0, s>>>(one, many);
  }
}

void launch_gram64(const Gram64Job& one, const Gram64Job* many, int n, int maxK, hipStream_t s) {
  const int nl = maxK * (maxK + 1) / 2;
  const dim3 grid((nl + 255) / 256, many ? n : 1);
  if (many) k_gram64<true><<<grid, 256, 0, s>>>(one, many);
  else k_gram64<false><<<grid, 256, 0, s>>>(one, many);
}
