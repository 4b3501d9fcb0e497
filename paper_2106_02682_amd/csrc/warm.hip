// Fixed-size encoding of a ring's Algorithm 6 state, for the learned warm start.
//
// Offsets d = 1..M-1 of a ring of M clusters are read as direction '+' at distance
// r = d when 2d <= M, else direction '-' at r = M - d.  Distances 1..near have
// their own blocks, every larger distance shares a 'far' block.  Per (direction,
// slot): X_0d, Lambda_d, Lambda1_d, Lambda2_d, rho~_d.  Vector = [X_00, rho_0,
// ('+' slots 1..near, far), ('-' slots 1..near, far)], row-major FP32.  With
// near >= M/2 the encoding is exact.
//
// Encoding (M >= near + 1) copies the blocks at d = r and d = M - r, and averages
// the far distances near+1..M/2 (zeros when there are none).  Decoding writes
// every offset from its slot, symmetrises (X_0,M-d = X_0d^T, so X is symmetric),
// fixes Tr rho_0 = 1 and leaves X' in the X-step buffer; the caller then projects
// X onto the PSD cone through its momentum blocks, so the Lagrangian bound at the
// decoded point is valid.  With far_cold the offsets beyond `near` take Section 4's cold start instead
// (X_0d = 0, multipliers 0, rho~_d = rho_d = I/n), the far slot unused.
#include "kernels.h"

namespace vemb {
namespace {

__device__ inline void slot_of(int d, int M, int near, int& dir, int& slot) {
  int r;
  if (2 * d <= M) {
    dir = 0;
    r = d;
  } else {
    dir = 1;
    r = M - d;
  }
  slot = (r <= near ? r : near + 1) - 1;
}

__device__ inline long block_base(const WarmLayout& w, int dir, int slot) {
  return w.block0 + (long)(dir * (w.near + 1) + slot) * w.bsz;
}

// Value of block element e (0..bsz) of offset d in the state.
__device__ inline double state_elem(const StepArgs& A, const WarmLayout& w, int d, long e) {
  const long nop2 = (long)A.n_op * A.n_op, n2 = (long)A.n * A.n, m2 = (long)A.m * A.m;
  if (e < w.oL) return A.X[d * nop2 + e];
  if (e < w.oL1) return A.Lam[(d - 1) * n2 + (e - w.oL)];
  if (e < w.oL2) return A.Lam1[(d - 1) * m2 + (e - w.oL1)];
  if (e < w.oR) return A.Lam2[(d - 1) * m2 + (e - w.oL2)];
  return A.rho_t[(d - 1) * n2 + (e - w.oR)];
}

__global__ void __launch_bounds__(256) warm_encode_kernel(StepArgs A, WarmLayout w, float* vec) {
  const int b = blockIdx.x;
  const int M = A.M;
  if (b == 0) {
    const long nop2 = (long)A.n_op * A.n_op;
    for (long e = threadIdx.x; e < nop2; e += 256) vec[w.x00 + e] = (float)A.X[e];
    for (long e = threadIdx.x; e < (long)A.m * A.m; e += 256) vec[w.rho0 + e] = (float)A.rho0[e];
    return;
  }
  const int dir = (b - 1) / (w.near + 1), slot = (b - 1) % (w.near + 1);
  float* out = vec + block_base(w, dir, slot);
  if (slot < w.near) {
    const int r = slot + 1;
    const int d = dir == 0 ? r : M - r;
    for (long e = threadIdx.x; e < w.bsz; e += 256) out[e] = (float)state_elem(A, w, d, e);
  } else {
    const int r0 = w.near + 1, r1 = M / 2;
    for (long e = threadIdx.x; e < w.bsz; e += 256) {
      double acc = 0.0;
      for (int r = r0; r <= r1; ++r) acc += state_elem(A, w, dir == 0 ? r : M - r, e);
      out[e] = r1 >= r0 ? (float)(acc / (r1 - r0 + 1)) : 0.0f;
    }
  }
}

// One workgroup per offset d = 0..M-1.
__global__ void __launch_bounds__(256) warm_decode_kernel(StepArgs A, WarmLayout w, const float* vec) {
  __shared__ double red[256];
  const int d = blockIdx.x;
  const int M = A.M, nop = A.n_op, n = A.n, m = A.m;
  const long nop2 = (long)nop * nop, n2 = (long)n * n, m2 = (long)m * m;
  if (d == 0) {
    for (long e = threadIdx.x; e < nop2; e += 256) {
      const long a = e / nop, c = e - a * nop;
      A.Xp[e] = 0.5 * ((double)vec[w.x00 + a * nop + c] + (double)vec[w.x00 + c * nop + a]);
    }
    double tr = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) tr += vec[w.rho0 + (long)i * m + i];
    red[threadIdx.x] = tr;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    const double shift = (1.0 - red[0]) / m;
    for (long e = threadIdx.x; e < m2; e += 256) {
      const long i = e / m, j = e - i * m;
      A.rho0[e] = 0.5 * ((double)vec[w.rho0 + i * m + j] + (double)vec[w.rho0 + j * m + i]) + (i == j ? shift : 0.0);
    }
    return;
  }
  int dir, slot, dir2, slot2;
  slot_of(d, M, w.near, dir, slot);
  slot_of(M - d, M, w.near, dir2, slot2);
  if (w.far_cold && slot == w.near) {  // a far offset (d and M - d lie at the same distance)
    for (long e = threadIdx.x; e < nop2; e += 256) A.Xp[d * nop2 + e] = 0.0;
    for (long e = threadIdx.x; e < n2; e += 256) {
      const long i = e / n, j = e - i * n;
      const double rt = i == j ? 1.0 / n : 0.0;
      A.Lam[(d - 1) * n2 + e] = 0.0;
      A.rho_t[(d - 1) * n2 + e] = rt;
      A.rho[(d - 1) * n2 + e] = rt;
    }
    for (long e = threadIdx.x; e < m2; e += 256) {
      A.Lam1[(d - 1) * m2 + e] = 0.0;
      A.Lam2[(d - 1) * m2 + e] = 0.0;
    }
    return;
  }
  const float* P = vec + block_base(w, dir, slot);
  const float* Q = vec + block_base(w, dir2, slot2);
  for (long e = threadIdx.x; e < nop2; e += 256) {  // X_0d = (P_d + P_{M-d}^T) / 2
    const long a = e / nop, c = e - a * nop;
    A.Xp[d * nop2 + e] = 0.5 * ((double)P[w.oX + a * nop + c] + (double)Q[w.oX + c * nop + a]);
  }
  for (long e = threadIdx.x; e < n2; e += 256) {
    const long i = e / n, j = e - i * n;
    const double lam = 0.5 * ((double)P[w.oL + i * n + j] + (double)P[w.oL + j * n + i]);
    const double rt = 0.5 * ((double)P[w.oR + i * n + j] + (double)P[w.oR + j * n + i]);
    A.Lam[(d - 1) * n2 + e] = lam;
    A.rho_t[(d - 1) * n2 + e] = rt;
    A.rho[(d - 1) * n2 + e] = rt;
  }
  for (long e = threadIdx.x; e < m2; e += 256) {
    const long i = e / m, j = e - i * m;
    A.Lam1[(d - 1) * m2 + e] = 0.5 * ((double)P[w.oL1 + i * m + j] + (double)P[w.oL1 + j * m + i]);
    A.Lam2[(d - 1) * m2 + e] = 0.5 * ((double)P[w.oL2 + i * m + j] + (double)P[w.oL2 + j * m + i]);
  }
}

}  // namespace

WarmLayout warm_layout(const StepArgs& a, int near) {
  WarmLayout w{};
  w.near = near;
  const long nop2 = (long)a.n_op * a.n_op, n2 = (long)a.n * a.n, m2 = (long)a.m * a.m;
  w.x00 = 0;
  w.rho0 = nop2;
  w.block0 = nop2 + m2;
  w.oX = 0;
  w.oL = nop2;
  w.oL1 = nop2 + n2;
  w.oL2 = w.oL1 + m2;
  w.oR = w.oL2 + m2;
  w.bsz = nop2 + 2 * n2 + 2 * m2;
  w.total = w.block0 + 2L * (near + 1) * w.bsz;
  return w;
}

hipError_t launch_warm_encode(const StepArgs& a, int near, float* vec, hipStream_t st) {
  hipLaunchKernelGGL(warm_encode_kernel, dim3(1 + 2 * (near + 1)), dim3(256), 0, st, a, warm_layout(a, near), vec);
  return hipGetLastError();
}

hipError_t launch_warm_decode(const StepArgs& a, int near, const float* vec, hipStream_t st, int far_cold) {
  WarmLayout w = warm_layout(a, near);
  w.far_cold = far_cold ? 1 : 0;
  hipLaunchKernelGGL(warm_decode_kernel, dim3(a.M), dim3(256), 0, st, a, w, vec);
  return hipGetLastError();
}

}  // namespace vemb
