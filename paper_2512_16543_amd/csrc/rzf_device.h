// Device-side helpers shared by the gfx950 kernels: complex arithmetic on
// interleaved float2/double2, wavefront reductions, the Philox4x64-10 sketch
// generator and a 16x16 complex tile product on the FP32 matrix cores.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Global-memory loads and stores through a device pointer.  A pointer read
// from a job array in memory is generic to the compiler, so plain accesses
// through it become flat instructions, which count against the LDS wait
// counter as well: every wait for an LDS read then also waits for the
// global loads in flight.  These go through the global address space.
typedef float gf2_t __attribute__((ext_vector_type(2)));
#define RZF_GLOBAL __attribute__((address_space(1)))
__device__ __forceinline__ float2 gld(const float2* p, size_t i) {
  const gf2_t v = ((const RZF_GLOBAL gf2_t*)p)[i];
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void gst(float2* p, size_t i, float2 v) {
  gf2_t w;
  w.x = v.x;
  w.y = v.y;
  ((RZF_GLOBAL gf2_t*)p)[i] = w;
}
template <class T>
__device__ __forceinline__ T gld(const T* p, size_t i) { return ((const RZF_GLOBAL T*)p)[i]; }
template <class T>
__device__ __forceinline__ void gst(T* p, size_t i, T v) { ((RZF_GLOBAL T*)p)[i] = v; }

#define RZF_WAVE 64

// ------------------------------------------------------------ complex float
__device__ __forceinline__ float2 cz() { return make_float2(0.f, 0.f); }
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }

__device__ __forceinline__ double2 dz() { return make_double2(0.0, 0.0); }
__device__ __forceinline__ double2 dadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 dsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 dconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 dmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double dabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ double2 ddiv(double2 a, double2 b) {
  // Smith's algorithm keeps the intermediate products in range.
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, den = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / den, (a.y - a.x * r) / den);
  } else {
    double r = b.x / b.y, den = b.x * r + b.y;
    return make_double2((a.x * r + a.y) / den, (a.y * r - a.x) / den);
  }
}
__device__ __forceinline__ double2 f2d(float2 a) { return make_double2((double)a.x, (double)a.y); }
__device__ __forceinline__ float2 d2f(double2 a) { return make_float2((float)a.x, (float)a.y); }

// --------------------------------------------------------- wave reductions
// Cross-lane sums with DPP row operations (quad permutations and mirrors
// inside each 16-lane row, row broadcasts across rows).  Each step adds a
// lane's value to its partner's under a pairing that is its own inverse, so
// both partners form the same sum (a + b == b + a) and every lane of a row
// ends with bit-identical results, in FP32 too.  All 64 lanes must be active
// when these are called.
#define DPP_QUAD_1032 0xB1        // quad_perm [1,0,3,2]
#define DPP_QUAD_2301 0x4E        // quad_perm [2,3,0,1]
#define DPP_ROW_ROR4 0x124
#define DPP_ROW_ROR8 0x128
#define DPP_ROW_MIRROR 0x140      // lane i <-> 15 - i within the row
#define DPP_ROW_HALF_MIRROR 0x141 // lane i <-> 7 - i within each half-row
#define DPP_ROW_BCAST15 0x142     // lane 15 of row k to every lane of row k + 1
#define DPP_ROW_BCAST31 0x143     // lane 31 to every lane of rows 2 and 3

// Lanes whose DPP source is out of range read zero (bound_ctrl), so no
// "old" value has to be set up first; the permutations used here (quad
// permutes, row rotates and mirrors) have no such lanes anyway.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// A row broadcast written only to the rows in ROWS (a 4-bit row mask); the
// other lanes read zero.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_rows_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_rows_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// Sum over the 16 lanes of each row; every lane of the row gets the row sum
// ((q0 + q1) + (q2 + q3) over the quad sums q).
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_d<DPP_QUAD_1032>(v);
  v += dpp_d<DPP_QUAD_2301>(v);
  v += dpp_d<DPP_ROW_HALF_MIRROR>(v);
  v += dpp_d<DPP_ROW_MIRROR>(v);
  return v;
}
__device__ __forceinline__ float row16_sumf(float v) {
  v += dpp_f<DPP_QUAD_1032>(v);
  v += dpp_f<DPP_QUAD_2301>(v);
  v += dpp_f<DPP_ROW_HALF_MIRROR>(v);
  v += dpp_f<DPP_ROW_MIRROR>(v);
  return v;
}
__device__ __forceinline__ float row16_sum(float v) { return row16_sumf(v); }
// Sum over each 8-lane half-row (quad permutations, then the half-row mirror).
__device__ __forceinline__ double row8_sum(double v) {
  v += dpp_d<DPP_QUAD_1032>(v);
  v += dpp_d<DPP_QUAD_2301>(v);
  v += dpp_d<DPP_ROW_HALF_MIRROR>(v);
  return v;
}
__device__ __forceinline__ float row8_sum(float v) {
  v += dpp_f<DPP_QUAD_1032>(v);
  v += dpp_f<DPP_QUAD_2301>(v);
  v += dpp_f<DPP_ROW_HALF_MIRROR>(v);
  return v;
}
__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// Sum over all 64 lanes, (r3 + r2) + (r1 + r0) over the row sums r: the row
// broadcasts fold rows 0 into 1 and 2 into 3, then rows 0-1 into 3; lane 63
// holds the total and every lane returns it.
__device__ __forceinline__ double wave_sum(double v) {
  v = row16_sum(v);
  v += dpp_rows_d<DPP_ROW_BCAST15, 0xA>(v);
  v += dpp_rows_d<DPP_ROW_BCAST31, 0xC>(v);
  return readlane_d(v, 63);
}
__device__ __forceinline__ float wave_sumf(float v) {
  v = row16_sumf(v);
  v += dpp_rows_f<DPP_ROW_BCAST15, 0xA>(v);
  v += dpp_rows_f<DPP_ROW_BCAST31, 0xC>(v);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Sum over the whole workgroup; `red` holds one double per wave.  Every
// thread returns the total.  Contains two barriers.
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += red[w];   // same order in every thread
  __syncthreads();
  return s;
}

// ------------------------------------------------ Philox4x64-10 (SC'11)
// Counter-based generator of Salmon, Moraes, Dror and Shaw; round constants
// and Weyl increments from that paper.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    const uint64_t lo0 = M0 * c[0], hi0 = __umul64hi(M0, c[0]);
    const uint64_t lo1 = M1 * c[2], hi1 = __umul64hi(M1, c[2]);
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
}

// Sketch entry (row i, column j) of iteration `it` at step `t`: the counter
// block (q, it, t, 0) with q = (1024 j + i) >> 1 under key (seed, track);
// words 0,1 serve even rows, words 2,3 odd rows.  Box-Muller in FP64 turns
// the two 53-bit uniforms into a CN(0,1) sample.
__device__ __forceinline__ void sketch_words(uint64_t seed, uint64_t track, int t, int it, int i,
                                             int j, uint64_t* wa, uint64_t* wb) {
  uint64_t c[4];
  c[0] = ((uint64_t)j * 1024ull + (uint64_t)i) >> 1;
  c[1] = (uint64_t)it;
  c[2] = (uint64_t)t;
  c[3] = 0ull;
  philox4x64_10(c, seed, track);
  if (i & 1) { *wa = c[2]; *wb = c[3]; } else { *wa = c[0]; *wb = c[1]; }
}

__device__ __forceinline__ float2 words_to_cn(uint64_t wa, uint64_t wb) {
  const double ua = ((double)(wa >> 11) + 0.5) * 0x1.0p-53;
  const double ub = ((double)(wb >> 11) + 0.5) * 0x1.0p-53;
  const double rad = sqrt(-2.0 * log(ua)) / sqrt(2.0);
  const double ang = 2.0 * 3.141592653589793 * ub;
  double s, c;
  sincos(ang, &s, &c);
  return make_float2((float)(rad * c), (float)(rad * s));
}

__device__ __forceinline__ float2 sketch_entry(uint64_t seed, uint64_t track, int t, int it, int i, int j) {
  uint64_t wa, wb;
  sketch_words(seed, track, t, it, i, j, &wa, &wb);
  return words_to_cn(wa, wb);
}

// Rows 2h and 2h + 1 of column j from their one shared counter block.
__device__ __forceinline__ void sketch_pair(uint64_t seed, uint64_t track, int t, int it, int h, int j,
                                            float2* even, float2* odd) {
  uint64_t c[4];
  c[0] = (uint64_t)j * 512ull + (uint64_t)h;
  c[1] = (uint64_t)it;
  c[2] = (uint64_t)t;
  c[3] = 0ull;
  philox4x64_10(c, seed, track);
  *even = words_to_cn(c[0], c[1]);
  *odd = words_to_cn(c[2], c[3]);
}

// ------------------------------------------------- complex MFMA 16x16 tile
// One wavefront accumulates D(16x16) += A(16 x k) * B(k x 16) in FP32 on the
// matrix cores with v_mfma_f32_16x16x4_f32.  Operand lane layout of that
// instruction: lane l holds A[l%16][l/16] and B[l/16][l%16] of a 16x4 / 4x16
// slab; the result lane l holds D[4*(l/16)+v][l%16] in register v.
// la(i, k) and lb(k, j) return the complex operands (zero outside the matrix;
// conjugation is the loader's business).  Real and imaginary parts take four
// real products.
__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <class LA, class LB>
__device__ __forceinline__ void ctile16(const LA& la, const LB& lb, int k0, int k1, floatx4& dr,
                                        floatx4& di) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, kk = lane >> 4;
  for (int k = k0; k < k1; k += 4) {
    const float2 a = la(r, k + kk);
    const float2 b = lb(k + kk, r);
    dr = mfma4(a.x, b.x, dr);
    dr = mfma4(-a.y, b.y, dr);
    di = mfma4(a.x, b.y, di);
    di = mfma4(a.y, b.x, di);
  }
}

__device__ __forceinline__ floatx4 zero4() { floatx4 z = {0.f, 0.f, 0.f, 0.f}; return z; }

// FP64 counterpart of ctile16 on the vector units, with the same result
// layout: acc[v] += sum_k la(tile_row(v), k) lb(k, tile_col()).
template <class LA, class LB>
__device__ __forceinline__ void dtile16(const LA& la, const LB& lb, int k0, int k1, double2 acc[4]) {
  const int lane = threadIdx.x & 63;
  const int c = lane & 15, rb = 4 * (lane >> 4);
  for (int k = k0; k < k1; ++k) {
    const double2 b = lb(k, c);
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = dadd(acc[v], dmul(la(rb + v, k), b));
  }
}

// Orders the LDS accesses of one wavefront around a point where its lanes
// exchange data through LDS.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Row / column of result register v in the calling lane.
__device__ __forceinline__ int tile_row(int v) { return 4 * ((threadIdx.x & 63) >> 4) + v; }
__device__ __forceinline__ int tile_col() { return threadIdx.x & 15; }

// ------------------------------------------- BF16 operands (precision option)
// v_mfma_f32_16x16x32_bf16: lane l supplies A[l%16][8*(l/16)+e] and
// B[8*(l/16)+e][l%16], e = 0..7, and receives D[4*(l/16)+v][l%16] (the FP32
// instruction's result layout).  FP32 operands are rounded to BF16 (one
// product per real product), or split x = hi + lo with hi = bf16(x) and
// lo = bf16(x - hi) and multiplied as hi*hi + hi*lo + lo*hi (three products),
// which carries about 16 significant bits per operand.  Accumulation is FP32.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

struct Bf16Pair { bf16x8 h, l; };

__device__ __forceinline__ Bf16Pair bf16_split8(const float v[8], bool x3) {
  Bf16Pair p;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = (__bf16)v[e];
    p.h[e] = h;
    p.l[e] = x3 ? (__bf16)(v[e] - (float)h) : (__bf16)0.0f;
  }
  return p;
}

__device__ __forceinline__ floatx4 mfma_bf16x(const Bf16Pair& a, const Bf16Pair& b, floatx4 c, bool x3) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.h, c, 0, 0, 0);
  if (x3) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.l, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.l, b.h, c, 0, 0, 0);
  }
  return c;
}

// D += op(A) op(B) for the calling lane's 8-element slices a[e] = A[row][k+e]
// and b[e] = B[k+e][col] of a complex 16 x 32 by 32 x 16 product; op
// conjugates when the flag is set.
__device__ __forceinline__ void cmac8_bf16(const float2 a[8], const float2 b[8], bool conja, bool conjb,
                                           bool x3, floatx4& dr, floatx4& di) {
  float ar[8], ai[8], nai[8], br[8], bi[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    ar[e] = a[e].x;
    ai[e] = conja ? -a[e].y : a[e].y;
    nai[e] = -ai[e];
    br[e] = b[e].x;
    bi[e] = conjb ? -b[e].y : b[e].y;
  }
  const Bf16Pair Ar = bf16_split8(ar, x3), Ai = bf16_split8(ai, x3), nAi = bf16_split8(nai, x3);
  const Bf16Pair Br = bf16_split8(br, x3), Bi = bf16_split8(bi, x3);
  dr = mfma_bf16x(Ar, Br, dr, x3);
  dr = mfma_bf16x(nAi, Bi, dr, x3);
  di = mfma_bf16x(Ar, Bi, di, x3);
  di = mfma_bf16x(Ai, Br, di, x3);
}
