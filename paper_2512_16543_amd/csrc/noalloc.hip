// rzf_full_noalloc: the conventional full-inversion RZF of rzf_full for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid allocation).  Its intermediate
// buffers (the Gram matrix, its inverse and the partial power sums) live in a
// fixed device array of this file instead of a context's arena, so the call
// needs no context and allocates nothing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "rzf_internal.h"

namespace {

// Largest intermediate set of one call: A and A^-1 (RZF_KMAX^2 complex64
// each) and the precoder's partial sums (fewer than one double per 16
// antennas of RZF_NMAX), each region on a 256-byte boundary.
constexpr size_t NA_ALIGN = 256;
constexpr size_t na_up(size_t x) { return (x + NA_ALIGN - 1) & ~(NA_ALIGN - 1); }
constexpr size_t NA_MAT = na_up(sizeof(float2) * (size_t)RZF_KMAX * RZF_KMAX);
constexpr size_t NA_PART = na_up(sizeof(double) * ((RZF_NMAX + 15) / 16));
constexpr size_t NA_BYTES = 2 * NA_MAT + NA_PART;   // 1,050,624 bytes

// The scratch of every rzf_full_noalloc call on a device (each device holds
// its own copy until the process ends).  Host code never uses this name as an
// address: it takes the device address from hipGetSymbolAddress below.
static __device__ __align__(256) char scratch[NA_BYTES];

constexpr int NA_MAX_DEVICES = 64;
std::mutex na_mu;
char* na_ptr[NA_MAX_DEVICES] = {};   // device address of `scratch`, per device

// The device address of this device's scratch, resolved once per device with
// that device current; nullptr if the runtime cannot give it.
char* scratch_on(int device) {
  std::lock_guard<std::mutex> lk(na_mu);
  if (!na_ptr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    na_ptr[device] = static_cast<char*>(p);
  }
  return na_ptr[device];
}

}  // namespace

extern "C" rzf_status rzf_full_noalloc(void* hip_stream, int K, int N, const rzf_c32* H, int ldh,
                                       double alpha, double P, rzf_c32* W, int ldw, int* err) {
  if (!H || !W) return RZF_E_INVALID;
  if (K < 1 || K > RZF_KMAX || N < 1 || N > RZF_NMAX || ldh < N || ldw < K) return RZF_E_SHAPE;
  if (!std::isfinite(alpha) || alpha < 0.0 || !std::isfinite(P) || P <= 0.0) return RZF_E_INVALID;
  int device = -1;
  if (hipGetDevice(&device) != hipSuccess || device < 0 || device >= NA_MAX_DEVICES) return RZF_E_DEVICE;
  char* base = scratch_on(device);
  if (!base) return RZF_E_DEVICE;
  // sizes within RZF_KMAX x RZF_NMAX always fit the three regions
  float2* A = reinterpret_cast<float2*>(base);
  float2* Ainv = reinterpret_cast<float2*>(base + NA_MAT);
  double* wpart = reinterpret_cast<double*>(base + 2 * NA_MAT);
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  const float2* Hf = reinterpret_cast<const float2*>(H);
  float2* Wf = reinterpret_cast<float2*>(W);
  // the launches of rzf_full, on the scratch above
  const GramJob gj{Hf, nullptr, A, nullptr, K, N, ldh, 0, (float)alpha, RZF_PREC_FP32};
  const Inv32Job vj{A, Ainv, K};
  const PrecJob pj{Hf, Ainv, Wf, wpart, nullptr, K, N, ldh, ldw, RZF_PREC_FP32, nullptr};
  const ScaleJob sj{Wf, wpart, P, K, N, ldw, precoder_blocks(N), nullptr};
  launch_gram(gj, nullptr, 1, K, false, s);
  if (K > KS) launch_inv32_big(vj, nullptr, 1, err, s);
  else launch_inv32(vj, nullptr, 1, err, s);
  if (!launch_precoder(pj, nullptr, sj, nullptr, 1, N, K, 64, s)) launch_scale(sj, nullptr, 1, N * K, s);
  return hipGetLastError() == hipSuccess ? RZF_OK : RZF_E_DEVICE;
}
