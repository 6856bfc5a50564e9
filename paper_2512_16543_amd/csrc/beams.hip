// Hybrid front end of eq. (4): analog beams from the DFT codebook of the
// UPA and the effective channel H_eff = H F_RF.
//
// Codebook (nx x ny UPA, element m = m_y nx + m_x, N = nx ny): beam
// b = q nx + p has entries exp(+j 2 pi (p m_x / nx + q m_y / ny)) / sqrt(N);
// distinct beams are orthonormal.
//
// k_beam_resp: one workgroup per user row n computes G[n, b] = sum_m H[n, m]
//   f_b[m] for every beam, as two separable DFT passes staged in LDS (along
//   x, then along y).  Twiddles come from LDS tables exp(+j 2 pi k / nx) and
//   exp(+j 2 pi k / ny), indexed by the exact reduced phase (p m_x mod nx).
// k_beam_select: one workgroup.  Best-power rule: user n in turn takes the
//   untaken beam maximising |G[n, b]|^2 (lowest index on ties), then the
//   remaining chains take the untaken beams of largest total power
//   sum_n |G[n, b]|^2 (a NaN power ranks below every number and raises
//   DEV_ERR_NONFINITE).  N <= 4096 = 64 lanes x 64 mask bits.  With select = 0 the caller's beams are kept (an index
//   outside [0, N) zeroes its column and raises DEV_ERR_BEAM).  Either way
//   H_eff[n, c] = G[n, beams[c]].
#include "rzf_device.h"
#include "rzf_internal.h"

namespace {

constexpr int RESP_THREADS = 256;
constexpr int SEL_THREADS = 1024;
static_assert(RZF_NMAX <= 64 * 64, "the taken set is 64 lanes x 64 mask bits");

__global__ __launch_bounds__(RESP_THREADS) void k_beam_resp(const float2* H, int ldh, int nx, int ny,
                                                            float2* G) {
  __shared__ float2 h[RZF_NMAX], tx[RZF_NMAX], tw[RZF_NMAX + 1];
  const int n = blockIdx.x, N = nx * ny;
  float2* twx = tw;        // exp(+j 2 pi k / nx), k < nx
  float2* twy = tw + nx;   // exp(+j 2 pi k / ny), k < ny
  for (int k = threadIdx.x; k < nx + ny; k += RESP_THREADS) {
    const int num = k < nx ? k : k - nx, den = k < nx ? nx : ny;
    float s, c;
    sincospif(2.0f * (float)num / (float)den, &s, &c);
    tw[k] = make_float2(c, s);
  }
  const float2* row = H + (size_t)n * ldh;
  for (int m = threadIdx.x; m < N; m += RESP_THREADS) h[m] = row[m];
  __syncthreads();
  // along x: tx[m_y][p] = sum_{m_x} h[m_y][m_x] e^{+j 2 pi p m_x / nx}
  for (int e = threadIdx.x; e < N; e += RESP_THREADS) {
    const int my = e / nx, p = e - my * nx;
    const float2* hr = h + my * nx;
    float2 acc = cz();
    int k = 0;   // p m_x mod nx
    for (int mx = 0; mx < nx; ++mx) {
      acc = cadd(acc, cmul(hr[mx], twx[k]));
      k += p;
      if (k >= nx) k -= nx;
    }
    tx[e] = acc;
  }
  __syncthreads();
  // along y: G[q nx + p] = sum_{m_y} tx[m_y][p] e^{+j 2 pi q m_y / ny} / sqrt(N)
  const float sc = rsqrtf((float)N);
  for (int e = threadIdx.x; e < N; e += RESP_THREADS) {
    const int q = e / nx, p = e - q * nx;
    float2 acc = cz();
    int k = 0;   // q m_y mod ny
    for (int my = 0; my < ny; ++my) {
      acc = cadd(acc, cmul(tx[my * nx + p], twy[k]));
      k += q;
      if (k >= ny) k -= ny;
    }
    G[(size_t)n * N + e] = cscale(acc, sc);
  }
}

// Largest value over the wavefront, lowest index among equals; every lane
// ends with the winner.
__device__ __forceinline__ void wave_argmax(float& v, int& idx) {
  for (int off = 32; off > 0; off >>= 1) {
    const float ov = __shfl_xor(v, off);
    const int oi = __shfl_xor(idx, off);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
}

// Power of a candidate: a NaN ranks below every number (and is reported).
__device__ __forceinline__ float rank_power(float v, bool& bad) {
  if (v != v) {
    bad = true;
    return -0.5f;
  }
  return v;
}

// Best untaken beam of one row of powers (row = G row c, or tot when row is
// null), scanned by one wavefront: lane l owns beams l + 64 j and bit j of
// its own taken mask tk.
__device__ __forceinline__ int wave_pick(const float2* grow, const float* tot, int N, unsigned long long tk,
                                         bool& bad) {
  const int lane = threadIdx.x & 63;
  float best = -1.f;
  int bi = N;
  for (int j = 0, b = lane; b < N; ++j, b += 64) {   // ascending b: the first maximum is kept
    float v = rank_power(grow ? cabs2(grow[b]) : tot[b], bad);
    if ((tk >> j) & 1ull) v = -1.f;
    if (v > best) {
      best = v;
      bi = b;
    }
  }
  wave_argmax(best, bi);
  return bi;
}

// Phase 1, all waves: each user's strongest beam over the whole codebook
// (first[c]) and, when chains outnumber users, every beam's total power.
// Phase 2, wave 0 alone, in the greedy order: user c keeps first[c] unless an
// earlier chain took it (the best untaken beam is then the overall best, as
// the overall best has the lowest index among the maxima); otherwise, and for
// the extra chains, the wave rescans.  The taken set lives in the lanes'
// masks, so the sequential phase needs no barrier.
__global__ __launch_bounds__(SEL_THREADS) void k_beam_select(const float2* G, int K, int N, int n_rf,
                                                             int select, int* beams, float2* Heff,
                                                             int ld_eff, int* err) {
  __shared__ float tot[RZF_NMAX];
  __shared__ int sel[RZF_NMAX];
  __shared__ int first[KM];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  bool bad = false;
  if (select) {
    for (int c = wid; c < K; c += SEL_THREADS / 64) {
      const int b = wave_pick(G + (size_t)c * N, nullptr, N, 0ull, bad);
      if (lane == 0) first[c] = b;
    }
    if (n_rf > K)
      for (int b = tid; b < N; b += SEL_THREADS) {
        float v = 0.f;
        for (int u = 0; u < K; ++u) v += cabs2(G[(size_t)u * N + b]);
        tot[b] = v;
      }
    __syncthreads();
    if (wid == 0) {
      unsigned long long tk = 0;   // bit j: beam lane + 64 j taken
      for (int c = 0; c < n_rf; ++c) {
        int w;
        if (c < K) {
          w = first[c];
          const unsigned long long owner = __shfl(tk, w & 63);
          if ((owner >> (w >> 6)) & 1ull) w = wave_pick(G + (size_t)c * N, nullptr, N, tk, bad);
        } else {
          w = wave_pick(nullptr, tot, N, tk, bad);
        }
        if (lane == (w & 63)) tk |= 1ull << (w >> 6);
        if (lane == 0) {
          sel[c] = w;
          beams[c] = w;
        }
      }
    }
    if (bad) atomicCAS(err, 0, DEV_ERR_NONFINITE);
  } else {
    for (int c = tid; c < n_rf; c += SEL_THREADS) {
      const int b = beams[c];
      const bool ok = b >= 0 && b < N;
      if (!ok) atomicCAS(err, 0, DEV_ERR_BEAM);
      sel[c] = ok ? b : -1;
    }
  }
  __syncthreads();
  for (int e = tid; e < K * n_rf; e += SEL_THREADS) {
    const int n = e / n_rf, c = e - n * n_rf;
    const int b = sel[c];
    Heff[(size_t)n * ld_eff + c] = b >= 0 ? G[(size_t)n * N + b] : cz();
  }
}

}  // namespace

void launch_beam_resp(const float2* H, int ldh, int K, int nx, int ny, float2* G, hipStream_t s) {
  k_beam_resp<<<K, RESP_THREADS, 0, s>>>(H, ldh, nx, ny, G);
}

void launch_beam_select(const float2* G, int K, int N, int n_rf, int select, int* beams, float2* Heff,
                        int ld_eff, int* err, hipStream_t s) {
  k_beam_select<<<1, SEL_THREADS, 0, s>>>(G, K, N, n_rf, select, beams, Heff, ld_eff, err);
}
