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
#include <algorithm>

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

// A = Hermitian part of the policy's input, X = A / (1.01 ||A||_F), over `parts` workgroups per block
// (blockIdx.y; one for batches of many blocks, more for a single problem's few blocks, so that the
// chip is filled).  The input is read as pairs of 32 x 32 tiles, (i-range, j-range) and its transpose
// position, each with row-wise (coalesced) reads staged in LDS, so the transposed entry that the
// Hermitian part needs costs no cache line of its own (entry-wise column reads fetched 17x the block's
// bytes from HBM); A's tile and its conjugate mirror are written row by row.  Workgroup g of a block
// takes the tile pairs g, g + parts, ... and leaves its share of ||A||_F^2 in the block's T slot (free
// until the products); sign_scale_kernel then sums the shares in order and writes X.
constexpr int kLoadTile = 32;

template <typename S, typename Policy>
__global__ void __launch_bounds__(kSignThreads) sign_load_kernel(Policy pol, int n, S* work) {
  constexpr int TB = kLoadTile, LDT = TB + 1, TT = TB * TB;
  const int mat = blockIdx.x, part = blockIdx.y, parts = gridDim.y, tid = threadIdx.x;
  if (!policy_active(pol, mat)) return;  // a masked batch instance: its products run on stale data, unused
  const size_t nn = (size_t)n * n;
  S* A = work + (size_t)mat * 4 * nn;
  double* share = reinterpret_cast<double*>(A + 3 * nn);  // the T slot
  __shared__ S t1[TB * LDT], t2[TB * LDT];
  __shared__ double red[kSignThreads];
  const int tiles = n / TB, pairs = upper_tile_count(tiles);
  double acc = 0.0;
  for (int idx = part; idx < pairs; idx += parts) {
    int ti = 0, tj = 0;
    upper_tile(idx, tiles, &ti, &tj);
    const int i0 = ti * TB, j0 = tj * TB;
    for (int e = tid; e < TT; e += kSignThreads) {
      const int r = e / TB, c = e % TB;
      t1[r * LDT + c] = pol.template load<S>(mat, i0 + r, j0 + c);
      t2[r * LDT + c] = pol.template load<S>(mat, j0 + r, i0 + c);
    }
    __syncthreads();
    for (int e = tid; e < TT; e += kSignThreads) {
      const int r = e / TB, c = e % TB;
      const S a = herm_part(t1[r * LDT + c], t2[c * LDT + r]);  // from M(i0+r, j0+c) and M(j0+c, i0+r)
      A[(size_t)(i0 + r) * n + j0 + c] = a;
      acc += (double)abs2(a);
      if (ti != tj) {
        const S b = herm_part(t2[r * LDT + c], t1[c * LDT + r]);  // A(j0+r, i0+c), the mirror's row r
        A[(size_t)(j0 + r) * n + i0 + c] = b;
        acc += (double)abs2(b);
      }
    }
    __syncthreads();
  }
  const double s2 = block_sum(acc, red);
  if (tid == 0) share[part] = s2;
}

// X = A / (1.01 ||A||_F) over the same workgroups and tile pairs as sign_load_kernel, the norm from its
// shares summed in workgroup order.  A squared norm that overflows (entries beyond ~1e150: a diverged
// iterate) scales by NaN, so the failure shows in every result instead of a silently wrong projection.
template <typename S, typename Policy>
__global__ void __launch_bounds__(kSignThreads) sign_scale_kernel(Policy pol, int n, S* work) {
  constexpr int TB = kLoadTile, TT = TB * TB;
  const int mat = blockIdx.x, part = blockIdx.y, parts = gridDim.y, tid = threadIdx.x;
  if (!policy_active(pol, mat)) return;
  const size_t nn = (size_t)n * n;
  S* A = work + (size_t)mat * 4 * nn;
  S* X = A + nn;
  const double* share = reinterpret_cast<const double*>(A + 3 * nn);
  double s2 = 0.0;
  for (int g = 0; g < parts; ++g) s2 += share[g];
  const double inv = s2 > 0.0 ? (s2 < INFINITY ? 1.0 / (1.01 * sqrt(s2)) : NAN) : 1.0;
  const int tiles = n / TB, pairs = upper_tile_count(tiles);
  for (int idx = part; idx < pairs; idx += parts) {
    int ti = 0, tj = 0;
    upper_tile(idx, tiles, &ti, &tj);
    const int i0 = ti * TB, j0 = tj * TB;
    for (int e = tid; e < TT; e += kSignThreads) {
      const int r = e / TB, c = e % TB;
      const size_t o = (size_t)(i0 + r) * n + j0 + c;
      X[o] = scale_s(inv, A[o]);
      if (ti != tj) {
        const size_t m = (size_t)(j0 + r) * n + i0 + c;
        X[m] = scale_s(inv, A[m]);
      }
    }
  }
}

// Per block: out(i, j) = c0 E(i, j) + c1 (P Q)(i, j) over the upper-triangle 64 x 64 tiles (blockIdx.x)
// of block blockIdx.y; P, Q, E, out are offsets (in scalars) inside the block's 4 n^2 work area.  The
// reduction runs in chunks of KC: the KC x 64 slices P(k0.., i-range) and Q(k0.., j-range) are staged in
// LDS with coalesced row reads (P(i, k) = conj(P(k, i)) read as rows of P).  Sixteen wavefronts, one
// 16 x 16 matrix-core sub-tile each; a complex product takes four real ones; the next chunk's slices are
// loaded into registers while the current chunk's products run.  (Measured on the batched
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
  // prefetch of the next chunk into registers (as real words: a complex entry is two); complex blocks
  // prefetch the Q slice only
  constexpr int NC = CPLX ? 2 : 1;
  constexpr int ROWW = TB * NC, PERW = KC * ROWW / NT, PER = KC * TB / NT;
  static_assert(PERW * NT == KC * ROWW && PER * NT == KC * TB, "the staging covers whole slices");
  const R* Pw = reinterpret_cast<const R*>(P);
  const R* Qw = reinterpret_cast<const R*>(Q);
  R* Psw = reinterpret_cast<R*>(Ps);
  R* Qsw = reinterpret_cast<R*>(Qs);
  const size_t ldw = (size_t)n * NC;
  R pre_p[CPLX ? 1 : PERW], pre_q[PERW];
#pragma unroll
  for (int x = 0; x < PERW; ++x) {
    const int e = tid + x * NT, k = e / ROWW, c = e % ROWW;
    if constexpr (!CPLX) pre_p[x] = Pw[(size_t)k * ldw + ti * ROWW + c];
    pre_q[x] = Qw[(size_t)k * ldw + tj * ROWW + c];
  }
  for (int k0 = 0; k0 < n; k0 += KC) {
    if constexpr (CPLX) {
#pragma unroll
      for (int x = 0; x < PER; ++x) {
        const int e = tid + x * NT, k = e / TB, c = e % TB;
        Ps[e] = P[(size_t)(k0 + k) * n + ti * TB + c];
      }
    }
#pragma unroll
    for (int x = 0; x < PERW; ++x) {
      if constexpr (!CPLX) Psw[tid + x * NT] = pre_p[x];
      Qsw[tid + x * NT] = pre_q[x];
    }
    __syncthreads();
    if (k0 + KC < n) {
#pragma unroll
      for (int x = 0; x < PERW; ++x) {
        const int e = tid + x * NT, k = e / ROWW, c = e % ROWW;
        if constexpr (!CPLX) pre_p[x] = Pw[(size_t)(k0 + KC + k) * ldw + ti * ROWW + c];
        pre_q[x] = Qw[(size_t)(k0 + KC + k) * ldw + tj * ROWW + c];
      }
    }
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

// Pi(A) (at offset pi_off of the block's work area) through the policy's store, over `parts` workgroups
// per block (blockIdx.y, contiguous ranges of rows); each leaves its share of ||rho - rho~||^2 in the
// block's X slot (free after the last product), and sign_finish_kernel sums the shares in order.
template <typename S, typename Policy>
__global__ void __launch_bounds__(kSignThreads) sign_store_kernel(Policy pol, int n, S* work, int pi_off) {
  const int mat = blockIdx.x, part = blockIdx.y, parts = gridDim.y;
  if (!policy_active(pol, mat)) return;
  const size_t nn = (size_t)n * n;
  S* base = work + (size_t)mat * 4 * nn;
  const S* Pi = base + pi_off;
  double* share = reinterpret_cast<double*>(base + nn);  // the X slot
  __shared__ double red[kSignThreads];
  const size_t e0 = nn * part / parts, e1 = nn * (part + 1) / parts;
  double acc = 0.0;
  for (size_t e = e0 + threadIdx.x; e < e1; e += kSignThreads) acc += pol.store(mat, (int)(e / n), (int)(e % n), Pi[e]);
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) share[part] = tot;
}

template <typename S, typename Policy>
__global__ void __launch_bounds__(64) sign_finish_kernel(Policy pol, int n, const S* work, int parts, int steps,
                                                         int count) {
  const int mat = blockIdx.x * 64 + threadIdx.x;
  if (mat >= count || !policy_active(pol, mat)) return;
  const size_t nn = (size_t)n * n;
  const double* share = reinterpret_cast<const double*>(work + (size_t)mat * 4 * nn + nn);
  double tot = 0.0;
  for (int g = 0; g < parts; ++g) tot += share[g];
  pol.finish(mat, tot);
  pol.record_sweeps(mat, steps);
}

// Workgroups per block of the load, scale and store passes: enough to give the chip ~512 workgroups.
inline int pass_parts(int count) { return std::max(1, std::min(8, (512 + count - 1) / count)); }

template <typename S>
void gemm(S* work, int n, int count, int p, int q, int e, int o, double c0, double c1, hipStream_t st,
          const LaunchHook* hook) {
  const int tiles = n / 64;
  if (hook) hook->fn(hook->ctx, 0, st);
  hipLaunchKernelGGL((sign_gemm_kernel<S>), dim3(upper_tile_count(tiles), count), dim3(GemmShape<S>::NT), 0, st, work,
                     n, count, p, q, e, o, c0, c1);
  if (hook) hook->fn(hook->ctx, 1, st);
}

// sign(A) of every block by the scaled Newton-Schulz schedule (polar.hip) after the policy's load; on
// return *x_off is the slot (offset in scalars inside a block's 4 n^2 work area) that holds sign(A),
// slot 0 holds A, and the slot 2 n^2 is free.
template <typename S, typename Policy>
hipError_t sign_function(const Policy& pol, int n, int count, S* work, hipStream_t st, const LaunchHook* hook,
                         int* x_off, int* steps) {
  if (n % 64 || n > kSignMax) return hipErrorInvalidValue;
  constexpr bool F32 = sizeof(typename scalar_traits<S>::real) == 4;
  static const std::vector<double> sched =
      F32 ? ns_schedule(kNsResolved32, kNsStop32) : ns_schedule(kNsResolved, kNsStop);
  const int nn = n * n;
  const int Y = 2 * nn;
  int X = nn, T = 3 * nn;
  const int parts = pass_parts(count);
  hipLaunchKernelGGL((sign_load_kernel<S, Policy>), dim3(count, parts), dim3(kSignThreads), 0, st, pol, n, work);
  hipLaunchKernelGGL((sign_scale_kernel<S, Policy>), dim3(count, parts), dim3(kSignThreads), 0, st, pol, n, work);
  for (double a : sched) {
    gemm<S>(work, n, count, X, X, -1, Y, 0.0, 1.0, st, hook);
    gemm<S>(work, n, count, X, Y, X, T, 1.5 * a, -0.5 * a * a * a, st, hook);
    std::swap(X, T);
  }
  *x_off = X;
  *steps = (int)sched.size();
  return hipSuccess;
}

template <typename S, typename Policy>
hipError_t sign_project(const Policy& pol, int n, int count, void* work_raw, hipStream_t st,
                        const LaunchHook* hook = nullptr) {
  if (count <= 0) return hipSuccess;
  S* work = static_cast<S*>(work_raw);
  int X = 0, steps = 0;
  const hipError_t e = sign_function<S>(pol, n, count, work, st, hook, &X, &steps);
  if (e != hipSuccess) return e;
  const int A = 0, Y = 2 * n * n;
  // Pi(A) = (A + A S) / 2 into the slot of X^2, free after the last step
  gemm<S>(work, n, count, A, X, A, Y, 0.5, 0.5, st, hook);
  const int parts = pass_parts(count);
  hipLaunchKernelGGL((sign_store_kernel<S, Policy>), dim3(count, parts), dim3(kSignThreads), 0, st, pol, n, work, Y);
  hipLaunchKernelGGL((sign_finish_kernel<S, Policy>), dim3((count + 63) / 64), dim3(64), 0, st, pol, n, work, parts,
                     steps, count);
  return hipGetLastError();
}

// ----- Smallest eigenvalue by spectral slicing (the bound's 256 x 256 matrices) -----
//
// For a shift sigma, P = (I + sign(sigma I - K)) / 2 projects onto the eigenvectors of K with eigenvalues
// below sigma (one within the schedule's resolution of sigma enters with a weight in (0, 1)).  If sigma
// is at least lambda_min(K) and at most kSliceCols - 2 eigenvalues lie below it, the span of x and P z_c
// (c = 1 .. kSliceCols - 1, fixed pseudo-random +-1 columns) contains the lowest eigenvector, and the
// smallest Rayleigh-Ritz value of K on that span, computed in FP64 from K itself, is lambda_min to
// rounding (Ritz values are never below lambda_min, and extra directions do not move the smallest).
// sigma is the Rayleigh quotient of x, the Ritz vector of the previous evaluation (an upper bound of
// lambda_min), or the smallest diagonal entry on the first; a block with more eigenvalues below sigma
// is flagged, and the next pass starts from its Ritz vector, whose Rayleigh quotient lies lower.

struct ShiftPolicy {  // A = sigma_d I - K_d
  const double* K;
  const double* sigma;
  int n;
  template <typename S> __device__ S load(int mat, int i, int j) const {
    double v = -K[(size_t)mat * n * n + (size_t)i * n + j];
    if (i == j) v += sigma[mat];
    return from_double<S>(v);
  }
};

// sigma_d = x^T K x / x^T x, or, for x = 0, the smallest diagonal entry with x = its unit vector.
__global__ void __launch_bounds__(kSignThreads) slice_shift_kernel(const double* K, double* x, double* sigma,
                                                                   int* nflag, int n) {
  const int mat = blockIdx.x, tid = threadIdx.x;
  const double* Km = K + (size_t)mat * n * n;
  double* xm = x + (size_t)mat * n;
  __shared__ double red[kSignThreads];
  __shared__ int ridx[kSignThreads];
  __shared__ double xs[kSignMax];
  if (mat == 0 && tid == 0) *nflag = 0;
  double x2 = 0.0;
  for (int i = tid; i < n; i += kSignThreads) {
    xs[i] = xm[i];
    x2 += xs[i] * xs[i];
  }
  const double nx = block_sum(x2, red);
  if (nx > 0.5) {
    double q = 0.0;
    for (int i = tid; i < n; i += kSignThreads) {
      double y = 0.0;
      for (int j = 0; j < n; ++j) y += Km[(size_t)j * n + i] * xs[j];  // K symmetric: coalesced over i
      q += xs[i] * y;
    }
    const double num = block_sum(q, red);
    if (tid == 0) sigma[mat] = num / nx;
    return;
  }
  double best = INFINITY;
  int bi = n;
  for (int i = tid; i < n; i += kSignThreads) {
    const double v = Km[(size_t)i * n + i];
    if (v < best) {
      best = v;
      bi = i;
    }
  }
  red[tid] = best;
  ridx[tid] = bi;
  __syncthreads();
  for (int s = kSignThreads / 2; s > 0; s >>= 1) {
    if (tid < s) {
      const double o = red[tid + s];
      const int oi = ridx[tid + s];
      if (o < red[tid] || (o == red[tid] && oi < ridx[tid])) {
        red[tid] = o;
        ridx[tid] = oi;
      }
    }
    __syncthreads();
  }
  const int k = ridx[0];  // n when the diagonal holds no number: x stays 0 and sigma is not finite
  for (int i = tid; i < n; i += kSignThreads) xm[i] = i == k ? 1.0 : 0.0;
  if (tid == 0) sigma[mat] = red[0];
}

__device__ inline double slice_sign(int c, int i) {
  unsigned h = (unsigned)c * 0x9E3779B9u ^ ((unsigned)i + 0x7F4A7C15u) * 0x85EBCA6Bu;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  return (h & 1u) ? 1.0 : -1.0;
}

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

template <typename S>
__global__ void __launch_bounds__(kSignThreads) slice_ritz_kernel(const double* K, const S* work, int s_off,
                                                                  double* x, double* lmin, int* flags, int* nflag,
                                                                  int n) {
  constexpr int R = kSliceCols, NT = kSignThreads, RH = R / 2;
  static_assert(NT == R * R, "one thread per entry of the Ritz matrix");
  const int mat = blockIdx.x, tid = threadIdx.x;
  const size_t nn = (size_t)n * n;
  const double* Km = K + (size_t)mat * nn;
  const S* Sm = work + (size_t)mat * 4 * nn + s_off;
  double* xm = x + (size_t)mat * n;
  __shared__ double Z[kSignMax * R];  // start columns, then the orthonormal basis Q (row i at Z + i R)
  __shared__ double Y[kSignMax * R];  // P Z, then K Q
  __shared__ double T[R * R], V[R * R];
  __shared__ double red[NT];
  __shared__ double rc[RH], rs[RH];
  __shared__ int rp[RH], rq[RH];
  __shared__ unsigned kept_mask;
  __shared__ int best_idx;

  // 1. trace of sign(A) (eigenvalues of K below sigma: (n + tr) / 2) and the start columns
  double tr = 0.0;
  for (int i = tid; i < n; i += NT) tr += (double)Sm[(size_t)i * n + i];
  const double rs_n = 1.0 / sqrt((double)n);
  for (int e = tid; e < n * R; e += NT) {
    const int i = e / R, c = e % R;
    Z[e] = c == 0 ? xm[i] : slice_sign(c, i) * rs_n;
  }
  const double below = 0.5 * ((double)n + block_sum(tr, red));

  // 2. Y = [x, P z_1, ..., P z_{R-1}], P = (I + S) / 2 (S symmetric: column reads coalesced over rows)
  for (int i = tid; i < n; i += NT) {
    double acc[R];
#pragma unroll
    for (int c = 0; c < R; ++c) acc[c] = Z[i * R + c];
    for (int j = 0; j < n; ++j) {
      const double sv = (double)Sm[(size_t)j * n + i];
#pragma unroll
      for (int c = 1; c < R; ++c) acc[c] += sv * Z[j * R + c];
    }
    Y[i * R] = acc[0];
#pragma unroll
    for (int c = 1; c < R; ++c) Y[i * R + c] = 0.5 * acc[c];
  }
  __syncthreads();

  // 3. orthonormal basis by classical Gram-Schmidt applied twice, on the first wavefront (lane l holds
  //    rows l, l + 64, ...; each lane reads back only its own rows); negligible columns are dropped
  if (tid < 64) {
    const int rows = n / 64;
    unsigned mask = 0u;
    for (int c = 0; c < R; ++c) {
      double v[kSignMax / 64];
      double n0 = 0.0;
      for (int t = 0; t < rows; ++t) {
        v[t] = Y[(tid + 64 * t) * R + c];
        n0 += v[t] * v[t];
      }
      n0 = wave_sum(n0);
      for (int pass = 0; pass < 2; ++pass)
        for (int k = 0; k < c; ++k) {
          if (!(mask >> k & 1u)) continue;
          double h = 0.0;
          for (int t = 0; t < rows; ++t) h += Z[(tid + 64 * t) * R + k] * v[t];
          h = wave_sum(h);
          for (int t = 0; t < rows; ++t) v[t] -= h * Z[(tid + 64 * t) * R + k];
        }
      double n1 = 0.0;
      for (int t = 0; t < rows; ++t) n1 += v[t] * v[t];
      n1 = wave_sum(n1);
      const bool keep = n0 > 0.0 && n1 > 1e-24 * n0 && n1 < INFINITY;
      const double inv = keep ? 1.0 / sqrt(n1) : 0.0;
      for (int t = 0; t < rows; ++t) Z[(tid + 64 * t) * R + c] = v[t] * inv;
      if (keep) mask |= 1u << c;
    }
    if (tid == 0) kept_mask = mask;
  }
  __syncthreads();
  const unsigned mask = kept_mask;

  // 4. W = K Q (into Y), T = Q^T W, symmetrised; V = I
  for (int i = tid; i < n; i += NT) {
    double acc[R];
#pragma unroll
    for (int c = 0; c < R; ++c) acc[c] = 0.0;
    for (int j = 0; j < n; ++j) {
      const double kv = Km[(size_t)j * n + i];
#pragma unroll
      for (int c = 0; c < R; ++c) acc[c] += kv * Z[j * R + c];
    }
#pragma unroll
    for (int c = 0; c < R; ++c) Y[i * R + c] = acc[c];
  }
  __syncthreads();
  {
    const int a = tid / R, b = tid % R;
    double t = 0.0;
    for (int i = 0; i < n; ++i) t += Z[i * R + a] * Y[i * R + b];
    red[tid] = t;
    V[tid] = a == b ? 1.0 : 0.0;
  }
  __syncthreads();
  {
    const int a = tid / R, b = tid % R;
    const bool on = (mask >> a & 1u) && (mask >> b & 1u);
    T[tid] = on ? 0.5 * (red[a * R + b] + red[b * R + a]) : 0.0;  // dropped columns decoupled
  }
  __syncthreads();

  // 5. two-sided cyclic Jacobi on T (round-robin ordering, R/2 disjoint rotations per round)
  for (int sweep = 0; sweep < 40; ++sweep) {
    const int a = tid / R, b = tid % R;
    const double v = T[tid];
    const double off = block_sum(a != b ? v * v : 0.0, red);
    const double dia = block_sum(a == b ? v * v : 0.0, red);
    if (!(off > 1e-32 * dia)) break;  // also ends on a non-finite T
    for (int round = 0; round < R - 1; ++round) {
      if (tid < RH) {
        int p, q;
        if (tid == 0) {
          p = R - 1;
          q = round;
        } else {
          p = (round + tid) % (R - 1);
          q = (round - tid + R - 1) % (R - 1);
        }
        const double app = T[p * R + p], aqq = T[q * R + q], apq = T[p * R + q];
        double c = 1.0, s = 0.0;
        if (apq != 0.0) {
          const double tau = (aqq - app) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
        }
        rc[tid] = c;
        rs[tid] = s;
        rp[tid] = p;
        rq[tid] = q;
      }
      __syncthreads();
      if (tid < RH * R) {  // rows p, q of T
        const int g = tid / R, j = tid % R, p = rp[g], q = rq[g];
        const double c = rc[g], s = rs[g], tp = T[p * R + j], tq = T[q * R + j];
        T[p * R + j] = c * tp - s * tq;
        T[q * R + j] = s * tp + c * tq;
      }
      __syncthreads();
      {  // columns p, q of T (first half of the threads) and of V (second half)
        const int g = (tid / R) % RH, i = tid % R, p = rp[g], q = rq[g];
        double* Mx = tid < RH * R ? T : V;
        const double c = rc[g], s = rs[g], tp = Mx[i * R + p], tq = Mx[i * R + q];
        Mx[i * R + p] = c * tp - s * tq;
        Mx[i * R + q] = s * tp + c * tq;
      }
      __syncthreads();
    }
  }

  // 6. smallest Ritz value over the kept columns, its Ritz vector as the next start
  if (tid == 0) {
    int bi = -1;
    double bv = INFINITY;
    for (int a = 0; a < R; ++a)
      if ((mask >> a & 1u) && T[a * R + a] < bv) {
        bv = T[a * R + a];
        bi = a;
      }
    best_idx = bi;
    lmin[mat] = bi >= 0 ? bv : NAN;
    const bool bad = bi < 0 || !(below <= R - 1.5);
    flags[mat] = bad ? 1 : 0;
    if (bad) atomicAdd(nflag, 1);
  }
  __syncthreads();
  const int bi = best_idx;
  if (bi >= 0)
    for (int i = tid; i < n; i += NT) {
      double v = 0.0;
#pragma unroll
      for (int c = 0; c < R; ++c) v += Z[i * R + c] * V[c * R + bi];
      xm[i] = v;
    }
}

template <typename S>
hipError_t slice_pass(const double* K, double* x, double* sigma, double* lmin, int* flags, int* nflag, int n,
                      int count, void* work_raw, hipStream_t st) {
  S* work = static_cast<S*>(work_raw);
  hipLaunchKernelGGL(slice_shift_kernel, dim3(count), dim3(kSignThreads), 0, st, K, x, sigma, nflag, n);
  int X = 0, steps = 0;
  const hipError_t e = sign_function<S>(ShiftPolicy{K, sigma, n}, n, count, work, st, nullptr, &X, &steps);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((slice_ritz_kernel<S>), dim3(count), dim3(kSignThreads), 0, st, K, work, X, x, lmin, flags,
                     nflag, n);
  return hipGetLastError();
}

}  // namespace

int sign_launches(int precision) {
  const double l0 = precision == VEMB_FP64 ? kNsResolved : kNsResolved32;
  const double stop = precision == VEMB_FP64 ? kNsStop : kNsStop32;
  return 2 * (int)ns_schedule(l0, stop).size() + 5;  // load, scale, the products, Pi, store, finish
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

hipError_t launch_lambda_min_slice(const double* K, double* x, double* sigma, double* lmin, int* flags, int* nflag,
                                   int n, int count, void* work, hipStream_t st, int precision) {
  if (count <= 0) return hipSuccess;
  if (n % 64 || n > kSignMax) return hipErrorInvalidValue;
  return precision == VEMB_FP64 ? slice_pass<double>(K, x, sigma, lmin, flags, nflag, n, count, work, st)
                                : slice_pass<float>(K, x, sigma, lmin, flags, nflag, n, count, work, st);
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
