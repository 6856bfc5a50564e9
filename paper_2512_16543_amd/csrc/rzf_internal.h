// Host/device shared definitions of the HIP implementation behind rzf.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rzf.h"

#define KM RZF_KMAX     // largest K held in one workgroup's LDS
#define WB_RMAX 32      // largest Woodbury rank handled in LDS (= KM / 2)

// Device-side error codes (first one wins; rzf_sync maps them to rzf_status).
#define DEV_ERR_NOT_HPD 1
#define DEV_ERR_NONFINITE 2

// Per-update outcome, same layout as rzf_update_info.
struct DevInfo {
  int r, iters, path, d;
  double dA_fro2, captured;
};

// One track, resident in device memory (in the context arena).
struct TrackDesc {
  int K, N;
  double alpha, P, switch_ratio;
  int k_init, p, i_max, kinit_policy;
  uint64_t seed, track_id;
  float2* Ainv;    // K x K, ld K: stored inverse
  float2* Hprev;   // K x N, ld N: previous snapshot
  float2* Anew;    // K x K, ld K: A' of the current step (FP32)
  float2* dA;      // K x K, ld K: Delta A of the current step
  double2* A64;    // K x K, ld K: FP64 Gram for init / reset
  double* wpart;   // partial ||W||^2 of the precoder blocks
  // written by the device
  int last_r;
  int pad_;
  DevInfo info;
  int dbg[8];      // last update: [0] Jacobi sweeps, [1] Jacobi rounds, [2] QR columns
  int nsig;        // number of sigma^2 below (d of the last SVD, 0 if none)
  int pad2_;
  double sig2[KM]; // last SVD: sigma_j^2, descending
};

// Launchers (defined next to their kernels).
void launch_gram(int K, int N, const float2* Ht, int ldh, const float2* Hp, int ldp, float2* Anew,
                 float2* dA, double alpha, hipStream_t s);
void launch_gram64(int K, int N, const float2* H, int ldh, double alpha, double2* A64, hipStream_t s);
void launch_inv64(int K, const double2* A64, float2* Ainv, int* err, DevInfo* info, hipStream_t s);
void launch_inv32(int K, const float2* A, float2* Ainv, int* err, hipStream_t s);
int precoder_blocks(int N);
void launch_precoder(int K, int N, const float2* H, int ldh, const float2* X, float2* W, int ldw,
                     double* wpart, float2* Hcopy, hipStream_t s);
void launch_scale(int K, int N, float2* W, int ldw, const double* wpart, int nparts, double P,
                  hipStream_t s);
void launch_arsvd_wb(TrackDesc* td, int K, int t, double eta, int i_max, int* err, hipStream_t s);
size_t sum_rate_scratch_doubles(int K);
void launch_sum_rate(int K, int N, const float2* H, int ldh, const float2* W, int ldw, double P,
                     double sigma2, float* rates, double* sum_out, double* part, int* err,
                     hipStream_t s);
void launch_debug_sketch(uint64_t seed, uint64_t track, int t, int it, int K, int d, float2* Omega,
                         uint64_t* words, hipStream_t s);
