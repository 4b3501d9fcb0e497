// Launchers of the warm-start network kernels (mlp.hip), used by mlp_api.cpp.
#pragma once

#include "common.h"

namespace vemb {

constexpr float kAdamB1 = 0.9f, kAdamB2 = 0.999f, kAdamEps = 1e-8f;
constexpr float kStdFloor = 1e-6f;

enum { kEpiPlain = 0, kEpiSilu = 1, kEpiSiluGrad = 2 };

// C(i, j) = sum_k A(i, k) B(k, j) (+ bias_j), M x N x K, FP32 accumulation.
// A(i, k) = A[i*sai + k*sak] (FP32); B(k, j) = B[k*sbk + j*sbj], FP32 or bfloat16.
// Epilogues: kEpiPlain C = acc (+ bias); kEpiSilu C = z, C2 = silu(z) with
// z = acc + bias; kEpiSiluGrad C = acc * silu'(Z[i*ldz + j]).  C row-major (ldc).
// Skinny products with a long K (few output tiles) are split along K over
// `splits` workgroup slices writing partial tiles to ws (splits x M x N floats),
// then summed in a fixed order and finished by the same epilogue.
struct GemmArgs {
  int M, N, K;
  const float* A;
  long sai, sak;
  const void* B;
  long sbk, sbj;
  float* C;
  long ldc;
  const float* bias;
  int epi;
  float* C2;
  const float* Z;
  long ldz;
  float* ws;       // split-K workspace (may be null: no split)
  long ws_floats;
  int splits;      // set by launch_gemm
  int kchunk;      // set by launch_gemm
};

hipError_t launch_gemm(const GemmArgs& g, bool b_is_bf16, hipStream_t st);
// dY = 2 (Y - (T - mean)/std) / (B O); *loss = mean squared residual (FP64), via
// `partial` (max_partials doubles) -- all on the device.
hipError_t launch_loss_grad(const float* Y, const float* T, const float* mean, const float* stdv, int B, int O,
                            float* dY, double* partial, int max_partials, double* loss, hipStream_t st);
hipError_t launch_colsum(const float* dZ, int B, int N, float* db, hipStream_t st);
// c1 = 1/(1 - b1^t), c2 = 1/(1 - b2^t) (bias corrections of step t).
hipError_t launch_adam(float* theta, float* m, float* v, const float* g, uint16_t* wbf, long n, float lr, float c1,
                       float c2, hipStream_t st);
hipError_t launch_to_bf16(const float* theta, uint16_t* wbf, long n, hipStream_t st);
// mean / std per column; std floored at max(floor_abs, rel * largest std).
hipError_t launch_colstats(const float* T, int count, int O, float* mean, float* stdv, float floor_abs, float rel,
                           hipStream_t st);
hipError_t launch_denorm(const float* Y, const float* mean, const float* stdv, int B, int O, float* out,
                         hipStream_t st);
// dst(b, :) = X(rows[b], :); rows outside 0..count-1 give zero rows.
hipError_t launch_gather_rows(const float* X, int count, const int* rows, int B, int d, float* dst, hipStream_t st);

}  // namespace vemb
