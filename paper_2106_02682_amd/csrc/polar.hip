// PSD projection of one large symmetric matrix through the matrix sign function, on matrix cores.
//
// Pi(A) = (A + |A|) / 2 = (A + A sign(A)) / 2.  sign(A) is the limit of the scaled Newton-Schulz
// iteration X_0 = A / s (s = 1.01 ||A||_F > ||A||_2),
//     X_{k+1} = (a_k / 2) X_k (3 I - a_k^2 X_k^2),  a_k = sqrt(3 / (1 + l_k + l_k^2)),
//     l_{k+1} = (a_k l_k / 2) (3 - a_k^2 l_k^2),
// where l_k is a lower bound of |eigenvalue| / s still resolved: a_k balances the images of l_k and 1
// under y (3 - y^2) / 2, so the spectrum stays in [-1, -l] U [l, 1] and l grows by about
// 3 sqrt(3) / 2 per step while small, quadratically near 1 (Chen and Chow, SIAM J. Sci. Comput. 2014,
// derive the same scaling).  The schedule depends on l_0 only and is fixed on the host: eigenvalues
// with |lambda| < l_0 s are left partly unresolved, which moves Pi(A) by at most l_0 s per such
// eigenvalue.  Every step is two products of symmetric ld x ld matrices; a product is one launch
// over the upper-triangle 16 x 16 output tiles, one workgroup of four wavefronts per tile splitting
// the reduction, v_mfma_f64_16x16x4_f64 on operands read row-wise from L2 (symmetric operands:
// A(i, k) = A(k, i)), every result written exactly symmetric.
#include "polar.h"

#include <cmath>
#include <mutex>
#include <vector>

#include "mfma_tile.h"
#include "tile_map.h"

namespace vemb {
namespace {

constexpr int kNormBlocks = 64;

// partial[b] = sum of squares of the b-th slice of `in` (kNormBlocks workgroups of 256).
__global__ void __launch_bounds__(256) ns_norm_kernel(const double* in, long count, double* partial) {
  __shared__ double red[256];
  double acc = 0.0;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < count; e += (long)kNormBlocks * 256) acc += in[e] * in[e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// A = (in + in^T) / 2,  X = A / s with s = 1.01 ||in||_F: every |eigenvalue| of X is at most 0.99, so
// the largest ones map under the first scaled step (a_0 ~ sqrt 3) to at least 0.05 instead of to the
// root y = sqrt 3 of y (3 - y^2), where rounding could flip their sign (a rank-one input attains
// ||A||_2 = ||A||_F).
__global__ void __launch_bounds__(256) ns_init_kernel(const double* in, double* A, double* X, int ld,
                                                      const double* partial) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)ld * ld) return;
  const int i = (int)(e / ld), j = (int)(e % ld);
  double s2 = 0.0;
  for (int b = 0; b < kNormBlocks; ++b) s2 += partial[b];
  // a squared norm that overflows (entries beyond ~1e150: a diverged iterate) scales by NaN, so the
  // failure shows in every result instead of a silently wrong projection (a zero scale)
  const double inv = s2 > 0.0 ? (s2 < INFINITY ? 1.0 / (1.01 * sqrt(s2)) : NAN) : 1.0;
  const double a = 0.5 * (in[e] + in[(long)j * ld + i]);
  A[e] = a;
  X[e] = a * inv;
}

// out = c0 E + c1 P Q for symmetric P, Q, E whose product is symmetric (polynomials in one
// matrix), written exactly symmetric: one workgroup per upper-triangle tile (ti <= tj) stores the
// tile and its mirror, a diagonal tile stores its symmetric part.  Reading P(i, k) as P(k, i) is
// exact only for exactly symmetric P, and an asymmetric rounding residue would grow from step to
// step of the sign iteration, so every iterate is kept exactly symmetric.  E may be null.
// KW wavefronts split the reduction of a tile; each issues all its operand loads before its
// products (batches of 8), so a product waits on L2 latency about once.
template <int KW>
__global__ void __launch_bounds__(64 * KW) ns_gemm_kernel(const double* P, const double* Q, const double* E,
                                                          double* out, int ld, double c0, double c1) {
  int ti = 0, tj = 0;
  if (!upper_tile((int)blockIdx.x, ld / 16, &ti, &tj)) return;  // the grid holds the upper-triangle tiles only
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int r16 = l & 15, kk = l >> 4;
  const int chunk = ld / KW;  // reduction range of one wavefront (a multiple of 4)
  const double* pa = P + (long)(w * chunk + kk) * ld + ti * 16 + r16;  // P(i, k) read as P(k, i)
  const double* pb = Q + (long)(w * chunk + kk) * ld + tj * 16 + r16;  // Q(k, j)
  mf_d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < chunk; k0 += 32) {
    double av[8], bv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const bool in = k0 + 4 * u < chunk;
      av[u] = in ? pa[(long)(k0 + 4 * u) * ld] : 0.0;
      bv[u] = in ? pb[(long)(k0 + 4 * u) * ld] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = mfma_k4(av[u], bv[u], acc);
  }
  __shared__ double red[KW][256];
#pragma unroll
  for (int r = 0; r < 4; ++r) red[w][mfma_row<double>(l, r) * 16 + r16] = acc[r];
  __syncthreads();
  if (threadIdx.x >= 256) return;
  const int t = threadIdx.x, row = t >> 4, col = t & 15;
  double v = 0.0;
#pragma unroll
  for (int q = 0; q < KW; ++q) v += red[q][t];
  if (ti == tj) {
    const int tt = col * 16 + row;
    double vt = 0.0;
#pragma unroll
    for (int q = 0; q < KW; ++q) vt += red[q][tt];
    v = 0.5 * (v + vt);
  }
  const long o = (long)(ti * 16 + row) * ld + tj * 16 + col;
  const double val = E ? c0 * E[o] + c1 * v : c1 * v;
  out[o] = val;
  if (ti != tj) out[(long)(tj * 16 + col) * ld + ti * 16 + row] = val;
}

// One product with the widest split whose per-wavefront range is a multiple of 4.
void gemm(const double* P, const double* Q, const double* E, double* out, int ld, double c0, double c1, int blocks,
          hipStream_t st) {
  if (ld % 64 == 0)
    hipLaunchKernelGGL(ns_gemm_kernel<16>, dim3(blocks), dim3(1024), 0, st, P, Q, E, out, ld, c0, c1);
  else if (ld % 32 == 0)
    hipLaunchKernelGGL(ns_gemm_kernel<8>, dim3(blocks), dim3(512), 0, st, P, Q, E, out, ld, c0, c1);
  else
    hipLaunchKernelGGL(ns_gemm_kernel<4>, dim3(blocks), dim3(256), 0, st, P, Q, E, out, ld, c0, c1);
}

// Scratch of the allocation-free entry point: A, X, Y, T and the norm partials of one projection of
// at most kStaticSignMaxN x kStaticSignMaxN, one copy per GPU, alive until the process ends.  Host
// code never uses this name as an address (in host code it is a stand-in, not device memory): the
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) double scratch[kStaticSignWords];

}  // namespace

hipError_t static_sign_scratch(double** ptr) {
  static std::mutex mu;
  static double* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    double* p = nullptr;
    e = hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

const std::vector<double>& ns_schedule_resolved() {
  static const std::vector<double> sched = ns_schedule(kNsResolved);
  return sched;
}

std::vector<double> ns_schedule(double l0, double stop) {
  std::vector<double> a;
  double l = l0;
  while (1.0 - l > stop && a.size() < 64) {
    const double al = std::sqrt(3.0 / (1.0 + l + l * l));
    a.push_back(al);
    l = 0.5 * al * l * (3.0 - al * al * l * l);
  }
  return a;
}

hipError_t launch_psd_project_ns(const double* in, double* out, int ld, double* work, const std::vector<double>& sched,
                                 hipStream_t st) {
  if (ld <= 0 || ld % 16) return hipErrorInvalidValue;
  const long nn = (long)ld * ld;
  double* A = work;
  double* X = A + nn;
  double* Y = X + nn;
  double* T = Y + nn;
  double* partial = T + nn;
  const int eblocks = (int)((nn + 255) / 256);
  const int tiles = upper_tile_count(ld / 16);  // one workgroup per upper-triangle tile
  hipLaunchKernelGGL(ns_norm_kernel, dim3(kNormBlocks), dim3(256), 0, st, in, nn, partial);
  hipLaunchKernelGGL(ns_init_kernel, dim3(eblocks), dim3(256), 0, st, in, A, X, ld, partial);
  for (double a : sched) {
    gemm(X, X, nullptr, Y, ld, 0.0, 1.0, tiles, st);
    gemm(X, Y, X, T, ld, 1.5 * a, -0.5 * a * a * a, tiles, st);
    std::swap(X, T);
  }
  // Pi(A) = (A + A S) / 2 (A and S commute: the product is symmetric up to rounding, written
  // exactly symmetric)
  gemm(A, X, A, out, ld, 0.5, 0.5, tiles, st);
  return hipGetLastError();
}

}  // namespace vemb
