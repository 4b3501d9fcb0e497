// PSD projections of many 256 x 256 blocks (pair blocks of 4-site clusters, real; momentum blocks,
// complex Hermitian) through the matrix sign function on matrix cores, FP64.
//
// Pi(A) = (A + A sign(A)) / 2 with sign(A) from the scaled Newton-Schulz schedule of polar.hip
// (X_0 = A / (1.01 ||A||_F), 38 steps X <- (a/2) X (3I - a^2 X^2), every eigenvalue above
// 1e-14 ||A||_F resolved).  A one-sided Jacobi solve of one 256 x 256 block runs on one workgroup
// with its columns streamed through L2; here every step is a batched product over all blocks, one
// workgroup per upper-triangle 64 x 64 tile per block, so the chip is filled by tiles.  The blocks
// are read and written through the eigensolver's policies (pair: C = rho - Lambda/mu in, rho~ and the
// Lambda update and ||rho - rho~||^2 out; momentum: in place), so single problems and batches share
// these kernels.  Products of Hermitian polynomials in A are Hermitian; each is written exactly
// Hermitian (tile and conjugate mirror, symmetrised diagonal tiles), because the products read
// P(i, k) as conj(P(k, i)).
#include "jacobi_common.h"
#include "mfma_tile.h"
#include "polar.h"
#include "sign_batched.h"

namespace vemb {
namespace {

constexpr int kSignThreads = 256;

template <typename S> __device__ inline S herm_part(S a, S at);
template <> __device__ inline double herm_part<double>(double a, double at) { return 0.5 * (a + at); }
template <> __device__ inline cplx<double> herm_part<cplx<double>>(cplx<double> a, cplx<double> at) {
  return {0.5 * (a.re + at.re), 0.5 * (a.im - at.im)};
}
__device__ inline double scale_s(double s, double a) { return s * a; }
__device__ inline cplx<double> scale_s(double s, cplx<double> a) { return {s * a.re, s * a.im}; }

// Per block: A = Hermitian part of the policy's input, X = A / (1.01 ||A||_F).  One workgroup per block.
template <typename S, typename Policy>
__global__ void __launch_bounds__(kSignThreads) sign_load_kernel(Policy pol, int n, S* work) {
  const int mat = blockIdx.x;
  const size_t nn = (size_t)n * n;
  S* A = work + (size_t)mat * 4 * nn;
  S* X = A + nn;
  __shared__ double red[kSignThreads];
  double acc = 0.0;
  for (size_t e = threadIdx.x; e < nn; e += kSignThreads) {
    const int i = (int)(e / n), j = (int)(e % n);
    const S a = herm_part<S>(pol.template load<S>(mat, i, j), pol.template load<S>(mat, j, i));
    A[e] = a;
    acc += abs2(a);
  }
  const double s2 = block_sum(acc, red);
  const double inv = s2 > 0.0 ? 1.0 / (1.01 * sqrt(s2)) : 1.0;
  for (size_t e = threadIdx.x; e < nn; e += kSignThreads) X[e] = scale_s(inv, A[e]);
}

// Per block: out(i, j) = c0 E(i, j) + c1 (P Q)(i, j) over the upper-triangle 64 x 64 tiles
// (blockIdx.x) of block blockIdx.y; P, Q, E, out are offsets (in scalars) inside the block's 4 n^2
// work area.  Sixteen wavefronts, one 16 x 16 sub-tile each; the reduction runs in chunks of 32:
// the 32 x 64 slices P(k0.., i-range) and Q(k0.., j-range) are staged in LDS with coalesced row
// reads (P(i, k) = conj(P(k, i)) read as rows of P), so every operand is read from memory once per
// 64 x 64 tile instead of once per 16 x 16 tile.  The finished tile passes through the same LDS to
// be written (with its conjugate mirror, or its Hermitian part on the diagonal) row by row.
template <typename S>
__global__ void __launch_bounds__(1024) sign_gemm_kernel(S* work, int n, int p_off, int q_off, int e_off, int o_off,
                                                         double c0, double c1) {
  constexpr int TB = 64, KC = 32;
  const int tiles = n / TB;
  if ((int)blockIdx.x >= tiles * (tiles + 1) / 2) return;
  int ti = 0, rem = blockIdx.x;
  while (rem >= tiles - ti) {
    rem -= tiles - ti;
    ++ti;
  }
  const int tj = ti + rem;
  S* base = work + (size_t)blockIdx.y * 4 * n * n;
  const S* P = base + p_off;
  const S* Q = base + q_off;
  const S* E = e_off >= 0 ? base + e_off : nullptr;
  S* out = base + o_off;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int r16 = l & 15, kk = l >> 4;
  const int sr = w >> 2, sc = w & 3;  // sub-tile of this wavefront
  // staging: Ps[k][i] = P(k0 + k, ti*64 + i), Qs[k][j] = Q(k0 + k, tj*64 + j); later the result tile
  __shared__ S lds[2 * KC * TB];
  S* Ps = lds;
  S* Qs = lds + KC * TB;
  mf_d4 re = {0.0, 0.0, 0.0, 0.0}, im = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < n; k0 += KC) {
    for (int e = tid; e < KC * TB; e += 1024) {
      const int k = e / TB, c = e % TB;
      Ps[e] = P[(size_t)(k0 + k) * n + ti * TB + c];
      Qs[e] = Q[(size_t)(k0 + k) * n + tj * TB + c];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < KC / 4; ++u) {
      const S av = Ps[(4 * u + kk) * TB + sr * 16 + r16];  // A(i, k) = conj(av)
      const S bv = Qs[(4 * u + kk) * TB + sc * 16 + r16];  // B(k, j)
      if constexpr (scalar_traits<S>::is_complex) {
        re = mfma_k4(av.re, bv.re, re);
        re = mfma_k4(av.im, bv.im, re);
        im = mfma_k4(av.re, bv.im, im);
        im = mfma_k4(-av.im, bv.re, im);
      } else {
        re = mfma_k4(av, bv, re);
      }
    }
    __syncthreads();
  }
  // the finished 64 x 64 tile into LDS: Ts[r][c]
  S* Ts = lds;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int r = sr * 16 + mfma_row<double>(l, g), c = sc * 16 + r16;
    if constexpr (scalar_traits<S>::is_complex)
      Ts[r * TB + c] = S{re[g], im[g]};
    else
      Ts[r * TB + c] = re[g];
  }
  __syncthreads();
  for (int e = tid; e < TB * TB; e += 1024) {
    const int r = e / TB, c = e % TB;
    S v = Ts[e];
    if (ti == tj) v = herm_part<S>(v, Ts[c * TB + r]);
    S val = scale_s(c1, v);
    const size_t o = (size_t)(ti * TB + r) * n + tj * TB + c;
    if (E) val = val + scale_s(c0, E[o]);
    out[o] = val;
    if (ti != tj) out[(size_t)(tj * TB + c) * n + ti * TB + r] = conjugate(val);
  }
}

// Per block: Pi(A) (at offset pi_off of the block's work area) through the policy's store;
// feasibility and the step count recorded.
template <typename S, typename Policy>
__global__ void __launch_bounds__(kSignThreads) sign_store_kernel(Policy pol, int n, const S* work, int pi_off,
                                                                  int steps) {
  const int mat = blockIdx.x;
  const size_t nn = (size_t)n * n;
  const S* Pi = work + (size_t)mat * 4 * nn + pi_off;
  __shared__ double red[kSignThreads];
  double part = 0.0;
  for (size_t e = threadIdx.x; e < nn; e += kSignThreads) part += pol.store(mat, (int)(e / n), (int)(e % n), Pi[e]);
  const double tot = block_sum(part, red);
  if (threadIdx.x == 0) {
    pol.finish(mat, tot);
    pol.record_sweeps(mat, steps);
  }
}

template <typename S>
void gemm(S* work, int n, int count, int p, int q, int e, int o, double c0, double c1, hipStream_t st,
          const LaunchHook* hook) {
  const int tiles = n / 64;
  if (hook) hook->fn(hook->ctx, 0, st);
  hipLaunchKernelGGL((sign_gemm_kernel<S>), dim3(tiles * (tiles + 1) / 2, count), dim3(1024), 0, st, work, n, p, q,
                     e, o, c0, c1);
  if (hook) hook->fn(hook->ctx, 1, st);
}

template <typename S, typename Policy>
hipError_t sign_project(const Policy& pol, int n, int count, void* work_raw, hipStream_t st,
                        const LaunchHook* hook = nullptr) {
  if (count <= 0) return hipSuccess;
  if (n % 64 || n > kSignMax) return hipErrorInvalidValue;
  S* work = static_cast<S*>(work_raw);
  static const std::vector<double> sched = ns_schedule(kNsResolved);
  const int nn = n * n;
  const int A = 0;
  const int Y = 2 * nn;
  int X = nn, T = 3 * nn;
  hipLaunchKernelGGL((sign_load_kernel<S, Policy>), dim3(count), dim3(kSignThreads), 0, st, pol, n, work);
  for (double a : sched) {
    gemm<S>(work, n, count, X, X, -1, Y, 0.0, 1.0, st, hook);
    gemm<S>(work, n, count, X, Y, X, T, 1.5 * a, -0.5 * a * a * a, st, hook);
    std::swap(X, T);
  }
  // Pi(A) = (A + A S) / 2 into the slot of X^2, free after the last step
  gemm<S>(work, n, count, A, X, A, Y, 0.5, 0.5, st, hook);
  hipLaunchKernelGGL((sign_store_kernel<S, Policy>), dim3(count), dim3(kSignThreads), 0, st, pol, n, work, Y,
                     (int)sched.size());
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pair_projection_sign(const double* rho, double* Lam, double* rho_t, double* feas, int n, int P,
                                       double mu, int* sweeps, void* work, hipStream_t st) {
  PairPolicy pol{rho, Lam, rho_t, feas, sweeps, n, mu};
  return sign_project<double>(pol, n, P, work, st);
}

hipError_t launch_momentum_projection_sign(double* Xh, int n_op, int K, int* sweeps, void* work, hipStream_t st) {
  MomentumPolicy pol{Xh, sweeps, n_op};
  return sign_project<cplx<double>>(pol, n_op, K, work, st);
}

hipError_t launch_projection_group_sign(int kind, int n, int count, const int2* item, const void* ptrs, void* work,
                                        hipStream_t st, const LaunchHook* hook) {
  if (kind == 0) {
    BatchedPairPolicy pol{item, static_cast<const PairPtrs*>(ptrs), n, 1};
    return sign_project<double>(pol, n, count, work, st, hook);
  }
  BatchedMomentumPolicy pol{item, static_cast<const MomPtrs*>(ptrs), n, 1};
  return sign_project<cplx<double>>(pol, n, count, work, st, hook);
}

}  // namespace vemb
