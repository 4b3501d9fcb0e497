// Batched PSD projections of 256 x 256 blocks by the matrix sign function on matrix cores
// (sign_batched.hip), FP64: the pair and momentum projections of 4-site clusters.
#pragma once

#include "kernels.h"

namespace vemb {

constexpr int kSignMax = 256;  // block size handled (a multiple of 64, at most this)

// Scratch per block: 4 n^2 scalars (doubles for pairs, complex doubles for momentum blocks; half for
// FP32), sized here for FP64, which covers both precisions.
inline size_t sign_work_bytes(int n, int count, bool cplx) {
  return (size_t)count * 4 * n * n * (cplx ? 16 : 8);
}

// precision: VEMB_FP64 computes in FP64; any other mode in FP32 (matrix cores in FP32, state in FP64).
// Pair step 3 + Lambda update (as launch_pair_projection) for P blocks of size n.
hipError_t launch_pair_projection_sign(const double* rho, double* Lam, double* rho_t, double* feas, int n, int P,
                                       double mu, int* sweeps, void* work, hipStream_t st, int precision = VEMB_FP64);
// Step 8 in place (as launch_momentum_projection) for K complex blocks of size n_op.
hipError_t launch_momentum_projection_sign(double* Xh, int n_op, int K, int* sweeps, void* work, hipStream_t st,
                                           int precision = VEMB_FP64);
// Optional callback around each product launch of a sign projection (timing): phase 0 before the
// launch, 1 after it, on the launch's stream.  Null = none.
struct LaunchHook {
  void (*fn)(void* ctx, int phase, hipStream_t st);
  void* ctx;
};

// A batch size class (kind 0 pairs, 1 momentum blocks) through the batched policies.
hipError_t launch_projection_group_sign(int kind, int n, int count, const int2* item, const void* ptrs, void* work,
                                        hipStream_t st, const LaunchHook* hook = nullptr, int precision = VEMB_FP64);

// Smallest eigenvalue of `count` symmetric n x n matrices K (row-major, contiguous; n a multiple of 64,
// at most kSignMax) by one pass of spectral slicing: sigma_d from x_d (the Rayleigh quotient of the last
// Ritz vector, or the smallest diagonal entry where x_d = 0), sign(sigma_d I - K_d) by the sign-function
// products in `precision` in `work` (sign_work_bytes(n, count, false)), then the FP64 Rayleigh-Ritz value
// of K_d on x_d and kSliceCols - 1 projected columns into lmin[d] and its Ritz vector into x_d.
// flags[d] = 1 where more than kSliceCols - 2 eigenvalues lay below sigma_d (or no column survived): the
// value is then only an upper estimate and another pass (starting from the new x_d) is needed; *nflag
// counts the flagged blocks.  x: count x n, sigma: count, all device memory.
constexpr int kSliceCols = 16;
hipError_t launch_lambda_min_slice(const double* K, double* x, double* sigma, double* lmin, int* flags, int* nflag,
                                   int n, int count, void* work, hipStream_t st, int precision);

// Kernel launches of one sign-function projection (load, scale, the products, store, finish) in a precision.
int sign_launches(int precision);

// Real flops of one product launch over `count` blocks of size n: the upper-triangle 64 x 64 tiles
// of each block, 2 flops per multiply-add, four real products per complex one.
inline double sign_gemm_flops(int n, int count, bool cplx) {
  const double t = n / 64;
  return (cplx ? 4.0 : 1.0) * count * (t * (t + 1) / 2) * 64.0 * 64.0 * n * 2.0;
}

}  // namespace vemb
