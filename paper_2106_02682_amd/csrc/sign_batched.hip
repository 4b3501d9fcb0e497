// PSD projections of many 256 x 256 blocks (pair blocks of 4-site clusters, real; momentum blocks,
// complex Hermitian) through the matrix sign function on matrix cores, in FP64 or FP32.
//
// Pi(A) = (A + A sign(A)) / 2 with sign(A) from the scaled Newton-Schulz schedule of polar.hip
// (X_0 = A / (1.01 ||A||_F), steps X <- (a/2) X (3I - a^2 X^2)): FP64 resolves every eigenvalue above
// 1e-14 ||A||_F (38 steps), FP32 every eigenvalue above 1e-6 ||A||_F, about its own rounding level
// (v_mfma_f32_16x16x4_f32, twice the FP64 rate, half the bytes, and fewer steps).  A one-sided Jacobi solve of one 256 x 256 block runs on one workgroup
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
#include "tile_map.h"

namespace vemb {
namespace {

constexpr int kSignThreads = 256;

template <typename R> __device__ inline R herm_part(R a, R at) { return R(0.5) * (a + at); }
template <typename R> __device__ inline cplx<R> herm_part(cplx<R> a, cplx<R> at) {
  return {R(0.5) * (a.re + at.re), R(0.5) * (a.im - at.im)};
}
template <typename R> __device__ inline R scale_s(double s, R a) { return R(s) * a; }
template <typename R> __device__ inline cplx<R> scale_s(double s, cplx<R> a) { return {R(s) * a.re, R(s) * a.im}; }

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
    const S a = herm_part(pol.template load<S>(mat, i, j), pol.template load<S>(mat, j, i));
    A[e] = a;
    acc += (double)abs2(a);
  }
  const double s2 = block_sum(acc, red);
  const double inv = s2 > 0.0 ? 1.0 / (1.01 * sqrt(s2)) : 1.0;
  for (size_t e = threadIdx.x; e < nn; e += kSignThreads) X[e] = scale_s(inv, A[e]);
}

// Per block: out(i, j) = c0 E(i, j) + c1 (P Q)(i, j) over the upper-triangle 64 x 64 tiles (blockIdx.x)
// of block blockIdx.y; P, Q, E, out are offsets (in scalars) inside the block's 4 n^2 work area.  The
// reduction runs in chunks of KC: the KC x 64 slices P(k0.., i-range) and Q(k0.., j-range) are staged in
// LDS with coalesced row reads (P(i, k) = conj(P(k, i)) read as rows of P).  Sixteen wavefronts, one
// 16 x 16 matrix-core sub-tile each; a complex product takes four real ones.  (Measured on the batched
// sweep, where the real pair blocks and the complex momentum blocks run concurrently on two streams:
// 2 x 2 sub-tiles per wavefront on four wavefronts make the real products alone 30 % faster but the
// step 10 % slower; three-product (Gauss) complex products are no faster; giving all tiles of a block to
// one XCD is 14 % slower.  The products wait on operand traffic more than on the matrix cores.)
// The finished tile passes through LDS (rows padded by one element) and is written row by row, and an
// off-diagonal tile's conjugate mirror row by row too: the mirror's rows are the tile's columns, read
// across the padded rows, and E's mirror entries are the conjugates of E's entries at the mirror
// position (E is Hermitian), so every global write and read is coalesced (the column-wise mirror writes
// of the first version cost 8 % of the step).  A diagonal tile stores its Hermitian part.
template <typename S> struct GemmShape { static constexpr int NT = 1024, KC = 32, SUB = 1; };  // real
template <typename R> struct GemmShape<cplx<R>> { static constexpr int NT = 1024, KC = 32, SUB = 1; };

template <typename S>
__global__ void __launch_bounds__(GemmShape<S>::NT) sign_gemm_kernel(S* work, int n, int count, int p_off, int q_off,
                                                                     int e_off, int o_off, double c0, double c1) {
  constexpr bool CPLX = scalar_traits<S>::is_complex;
  using R = typename scalar_traits<S>::real;
  using Acc = typename MfmaAcc<R>::T;
  constexpr int TB = 64, LDT = TB + 1;
  constexpr int NT = GemmShape<S>::NT, KC = GemmShape<S>::KC, SUB = GemmShape<S>::SUB;
  constexpr int STAGE = 2 * KC * TB, TILE = TB * LDT;
  constexpr int NACC = CPLX ? 2 : 1;
  constexpr int WSIDE = TB / (16 * SUB);  // wavefronts along a tile side
  const int tiles = n / TB;
  int blk = 0, ti = 0, tj = 0;
  if (!batched_tile_of((int)blockIdx.x, (int)blockIdx.y, count, tiles, &blk, &ti, &tj)) return;  // whole workgroup
  S* base = work + (size_t)blk * 4 * n * n;
  const S* P = base + p_off;
  const S* Q = base + q_off;
  const S* E = e_off >= 0 ? base + e_off : nullptr;
  S* out = base + o_off;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int r16 = l & 15, kk = l >> 4;
  const int wr = (w / WSIDE) * 16 * SUB, wc = (w % WSIDE) * 16 * SUB;  // this wavefront's corner in the tile
  // staging: Ps[k][i] = P(k0 + k, ti*64 + i), Qs[k][j] = Q(k0 + k, tj*64 + j); later the result tile
  __shared__ S lds[STAGE > TILE ? STAGE : TILE];
  S* Ps = lds;
  S* Qs = lds + KC * TB;
  Acc acc[NACC][SUB][SUB];
#pragma unroll
  for (int q = 0; q < NACC; ++q)
#pragma unroll
    for (int a = 0; a < SUB; ++a)
#pragma unroll
      for (int b = 0; b < SUB; ++b) acc[q][a][b] = Acc{R(0), R(0), R(0), R(0)};
  for (int k0 = 0; k0 < n; k0 += KC) {
    for (int e = tid; e < KC * TB; e += NT) {
      const int k = e / TB, c = e % TB;
      Ps[e] = P[(size_t)(k0 + k) * n + ti * TB + c];
      Qs[e] = Q[(size_t)(k0 + k) * n + tj * TB + c];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < KC / 4; ++u) {
      S av[SUB], bv[SUB];
#pragma unroll
      for (int a = 0; a < SUB; ++a) av[a] = Ps[(4 * u + kk) * TB + wr + a * 16 + r16];  // A(i, k) = conj(av)
#pragma unroll
      for (int b = 0; b < SUB; ++b) bv[b] = Qs[(4 * u + kk) * TB + wc + b * 16 + r16];  // B(k, j)
#pragma unroll
      for (int a = 0; a < SUB; ++a)
#pragma unroll
        for (int b = 0; b < SUB; ++b) {
          if constexpr (CPLX) {  // conj(a) b: real a_r b_r + a_i b_i, imaginary a_r b_i - a_i b_r
            acc[0][a][b] = mfma_k4(av[a].re, bv[b].re, acc[0][a][b]);
            acc[0][a][b] = mfma_k4(av[a].im, bv[b].im, acc[0][a][b]);
            acc[1][a][b] = mfma_k4(av[a].re, bv[b].im, acc[1][a][b]);
            acc[1][a][b] = mfma_k4(-av[a].im, bv[b].re, acc[1][a][b]);
          } else {
            acc[0][a][b] = mfma_k4(av[a], bv[b], acc[0][a][b]);
          }
        }
    }
    __syncthreads();
  }
  // the finished 64 x 64 tile into LDS: Ts[r][c] with padded rows
  S* Ts = lds;
#pragma unroll
  for (int a = 0; a < SUB; ++a)
#pragma unroll
    for (int b = 0; b < SUB; ++b)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int r = wr + a * 16 + mfma_row<R>(l, g), c = wc + b * 16 + r16;
        if constexpr (CPLX) {
          Ts[r * LDT + c] = S{acc[0][a][b][g], acc[1][a][b][g]};
        } else {
          Ts[r * LDT + c] = acc[0][a][b][g];
        }
      }
  __syncthreads();
  // the tile, row by row: out(ti*64 + r, tj*64 + c)
  for (int e = tid; e < TB * TB; e += NT) {
    const int r = e / TB, c = e % TB;
    S v = Ts[r * LDT + c];
    if (ti == tj) v = herm_part(v, Ts[c * LDT + r]);
    S val = scale_s(c1, v);
    const size_t o = (size_t)(ti * TB + r) * n + tj * TB + c;
    if (E) val = val + scale_s(c0, E[o]);
    out[o] = val;
  }
  if (ti == tj) return;
  // the conjugate mirror, row by row: out(tj*64 + r, ti*64 + c) = conj(value at (ti*64 + c, tj*64 + r))
  for (int e = tid; e < TB * TB; e += NT) {
    const int r = e / TB, c = e % TB;
    const size_t o = (size_t)(tj * TB + r) * n + ti * TB + c;
    S val = scale_s(c1, conjugate(Ts[c * LDT + r]));
    if (E) val = val + scale_s(c0, E[o]);  // conj(E(ti*64 + c, tj*64 + r)) = E(o)
    out[o] = val;
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
  hipLaunchKernelGGL((sign_gemm_kernel<S>), dim3(upper_tile_count(tiles), count), dim3(GemmShape<S>::NT), 0, st, work,
                     n, count, p, q, e, o, c0, c1);
  if (hook) hook->fn(hook->ctx, 1, st);
}

template <typename S, typename Policy>
hipError_t sign_project(const Policy& pol, int n, int count, void* work_raw, hipStream_t st,
                        const LaunchHook* hook = nullptr) {
  if (count <= 0) return hipSuccess;
  if (n % 64 || n > kSignMax) return hipErrorInvalidValue;
  S* work = static_cast<S*>(work_raw);
  constexpr bool F32 = sizeof(typename scalar_traits<S>::real) == 4;
  static const std::vector<double> sched =
      F32 ? ns_schedule(kNsResolved32, kNsStop32) : ns_schedule(kNsResolved, kNsStop);
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

int sign_launches(int precision) {
  const double l0 = precision == VEMB_FP64 ? kNsResolved : kNsResolved32;
  const double stop = precision == VEMB_FP64 ? kNsStop : kNsStop32;
  return 2 * (int)ns_schedule(l0, stop).size() + 3;
}

hipError_t launch_pair_projection_sign(const double* rho, double* Lam, double* rho_t, double* feas, int n, int P,
                                       double mu, int* sweeps, void* work, hipStream_t st, int precision) {
  PairPolicy pol{rho, Lam, rho_t, feas, sweeps, n, mu};
  return precision == VEMB_FP64 ? sign_project<double>(pol, n, P, work, st) : sign_project<float>(pol, n, P, work, st);
}

hipError_t launch_momentum_projection_sign(double* Xh, int n_op, int K, int* sweeps, void* work, hipStream_t st,
                                           int precision) {
  MomentumPolicy pol{Xh, sweeps, n_op};
  return precision == VEMB_FP64 ? sign_project<cplx<double>>(pol, n_op, K, work, st)
                                : sign_project<cplx<float>>(pol, n_op, K, work, st);
}

hipError_t launch_projection_group_sign(int kind, int n, int count, const int2* item, const void* ptrs, void* work,
                                        hipStream_t st, const LaunchHook* hook, int precision) {
  const bool f64 = precision == VEMB_FP64;
  if (kind == 0) {
    BatchedPairPolicy pol{item, static_cast<const PairPtrs*>(ptrs), n, 1};
    return f64 ? sign_project<double>(pol, n, count, work, st, hook) : sign_project<float>(pol, n, count, work, st, hook);
  }
  BatchedMomentumPolicy pol{item, static_cast<const MomPtrs*>(ptrs), n, 1};
  return f64 ? sign_project<cplx<double>>(pol, n, count, work, st, hook)
             : sign_project<cplx<float>>(pol, n, count, work, st, hook);
}

}  // namespace vemb
