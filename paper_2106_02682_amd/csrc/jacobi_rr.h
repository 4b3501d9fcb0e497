// Register-resident one-sided Jacobi sweeps for n = 64.
//
// The 64 columns of W (and of V when eigenvectors are kept) form NB = 64 / BLK
// blocks of BLK columns (BLK = 8: 4 wavefronts; BLK = 4: 8 wavefronts).
// Wavefront w holds the blocks at positions w and NB-1-w in registers, one row per
// lane (lane = row), so a plane rotation of two columns it holds touches only its
// own registers.  A sweep visits every column pair once:
//   * intra-block: BLK-1 rounds of the round-robin (circle method) pairing of the
//     columns of each held block, BLK disjoint pairs per round;
//   * inter-block: NB-1 block rounds of the circle method over the NB blocks (the
//     block at position 0 stays, positions 1..NB-1 rotate), each pairing the two
//     held blocks in BLK sub-rounds of BLK disjoint pairs (x_i, y_(i+s) mod BLK);
//     between block rounds the blocks move through LDS.
// Each round reduces the partial sums of its BLK pairs (|a|^2, |b|^2, conj(a) b)
// over the 64 lanes at once: log2(BLK) halving exchanges over the top lane bits
// leave lane group p = lane / (64/BLK) with pair p's partial sums, the remaining
// exchanges finish them.  Each lane group computes its pair's rotation; the
// rotation is broadcast to the wavefront through scalar registers (readlane) and
// applied only when the pair rotates (uniform branch).  Blocks return to their
// home positions after a full sweep, so columns keep their places in LDS.
#pragma once

#include "jacobi_common.h"

namespace vemb {

// Circle-method pairing of N players (N even): game g (0..N/2-1) of round r (0..N-2).
__device__ constexpr int rrc_p(int r, int g, int N) { return g == 0 ? N - 1 : (r + g) % (N - 1); }
__device__ constexpr int rrc_q(int r, int g, int N) { return g == 0 ? r : (r - g + N - 1) % (N - 1); }
// Next position of a block under the block rotation (0 fixed, 1 -> 2 -> ... -> NB-1 -> 1).
__device__ constexpr int rrc_next(int pos, int NB) { return pos == 0 ? 0 : pos % (NB - 1) + 1; }

__device__ inline int lane_bcast(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }
__device__ inline float lane_bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ inline double lane_bcast(double v, int lane) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename T> __device__ inline cplx<T> lane_bcast(cplx<T> v, int lane) {
  return {lane_bcast(v.re, lane), lane_bcast(v.im, lane)};
}

template <typename S> __device__ inline typename scalar_traits<S>::real re_of(S v) { return v; }
template <typename T> __device__ inline T re_of(cplx<T> v) { return v.re; }
template <typename S> __device__ inline typename scalar_traits<S>::real im_of(S) { return 0; }
template <typename T> __device__ inline T im_of(cplx<T> v) { return v.im; }
template <typename S> __device__ inline S make_s(typename scalar_traits<S>::real re, typename scalar_traits<S>::real) {
  return re;
}
template <> __device__ inline cplx<double> make_s<cplx<double>>(double re, double im) { return {re, im}; }
template <> __device__ inline cplx<float> make_s<cplx<float>>(float re, float im) { return {re, im}; }

// One round: the BLK disjoint pairs (X[p], Y[p]) of register slots.  Returns 1 when
// any pair rotated.
template <typename S, bool TRACKV, int BLK>
__device__ inline int rr_round(S (&Wr)[2 * BLK], S (&Vr)[2 * BLK], const int (&X)[BLK], const int (&Y)[BLK],
                               typename scalar_traits<S>::real tol, typename scalar_traits<S>::real floor2, int l) {
  using R = typename scalar_traits<S>::real;
  constexpr int NV = scalar_traits<S>::is_complex ? 4 : 3;
  constexpr int LOGB = BLK == 8 ? 3 : (BLK == 4 ? 2 : 1);
  constexpr int GROUP = 64 / BLK;  // lanes per pair after the reduction
  R v[BLK][NV];
#pragma unroll
  for (int p = 0; p < BLK; ++p) {
    const S a = Wr[X[p]], b = Wr[Y[p]];
    const S g = conj_mul(a, b);
    v[p][0] = abs2(a);
    v[p][1] = abs2(b);
    v[p][2] = re_of(g);
    if constexpr (NV == 4) v[p][3] = im_of(g);
  }
  // halving exchanges over lane bits 5, 4, ...: keep the half of the pairs named by the bit
#pragma unroll
  for (int st = 0; st < LOGB; ++st) {
    const int mask = 32 >> st;
    const int half = BLK >> (st + 1);
    const bool hi = (l & mask) != 0;
#pragma unroll
    for (int k = 0; k < half; ++k)
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        const R lo_v = v[k][c], hi_v = v[k + half][c];
        const R send = hi ? lo_v : hi_v;
        v[k][c] = (hi ? hi_v : lo_v) + __shfl_xor(send, mask);
      }
  }
  // lanes of a group share the pair: finish the sums over the low lane bits
#pragma unroll
  for (int m = GROUP / 2; m > 0; m >>= 1)
#pragma unroll
    for (int c = 0; c < NV; ++c) v[0][c] += __shfl_xor(v[0][c], m);
  const R alpha = v[0][0], beta = v[0][1];
  const S gam = make_s<S>(v[0][2], NV == 4 ? v[0][NV - 1] : R(0));
  const R ag = modulus(gam);
  const R small = alpha < beta ? alpha : beta;
  int rot = 0;
  R c = R(1), s = R(0);
  S ph = one_of<S>();
  if (small > floor2 && ag > tol * dev_sqrt(alpha * beta) && ag > R(0)) {
    const R zeta = (beta - alpha) / (R(2) * ag);
    R t = R(1) / (dev_abs(zeta) + dev_sqrt(R(1) + zeta * zeta));
    if (zeta < R(0)) t = -t;
    c = R(1) / dev_sqrt(R(1) + t * t);
    s = c * t;
    ph = conj_phase(gam, ag);
    rot = 1;
  }
  int any = 0;
#pragma unroll
  for (int p = 0; p < BLK; ++p) {
    if (lane_bcast(rot, GROUP * p)) {
      const R cp = lane_bcast(c, GROUP * p), sp = lane_bcast(s, GROUP * p);
      const S pp = lane_bcast(ph, GROUP * p);
      {
        const S a = Wr[X[p]], b = mul_phase(pp, Wr[Y[p]]);
        Wr[X[p]] = scale_by(cp, a) - scale_by(sp, b);
        Wr[Y[p]] = scale_by(sp, a) + scale_by(cp, b);
      }
      if constexpr (TRACKV) {
        const S a = Vr[X[p]], b = mul_phase(pp, Vr[Y[p]]);
        Vr[X[p]] = scale_by(cp, a) - scale_by(sp, b);
        Vr[Y[p]] = scale_by(sp, a) + scale_by(cp, b);
      }
      any = 1;
    }
  }
  return any;
}

// Sweeps over W (and V) held column-major in LDS with leading dimension LD, n = 64,
// blockDim = 64 * (64 / BLK) / 2.  Returns the number of sweeps that rotated.
// flags: one int of LDS per wavefront.
template <typename S, bool TRACKV, int BLK>
__device__ int rr_sweeps(S* W, S* V, int LD, int max_sweeps, typename scalar_traits<S>::real tol,
                         typename scalar_traits<S>::real floor2, int* flags) {
  constexpr int NB = 64 / BLK, NW = NB / 2;
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
  const int pA = w, pB = NB - 1 - w;
  S Wr[2 * BLK], Vr[2 * BLK];
#pragma unroll
  for (int c = 0; c < BLK; ++c) {
    Wr[c] = W[(BLK * pA + c) * LD + l];
    Wr[BLK + c] = W[(BLK * pB + c) * LD + l];
    if constexpr (TRACKV) {
      Vr[c] = V[(BLK * pA + c) * LD + l];
      Vr[BLK + c] = V[(BLK * pB + c) * LD + l];
    } else {
      Vr[c] = Vr[BLK + c] = s_zero<S>();
    }
  }
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    int any = 0;
#pragma unroll
    for (int r = 0; r < BLK - 1; ++r) {
      int X[BLK], Y[BLK];
#pragma unroll
      for (int g = 0; g < BLK / 2; ++g) {
        X[g] = rrc_p(r, g, BLK);
        Y[g] = rrc_q(r, g, BLK);
        X[g + BLK / 2] = BLK + rrc_p(r, g, BLK);
        Y[g + BLK / 2] = BLK + rrc_q(r, g, BLK);
      }
      any |= rr_round<S, TRACKV, BLK>(Wr, Vr, X, Y, tol, floor2, l);
    }
    for (int br = 0; br < NB - 1; ++br) {
#pragma unroll
      for (int sr = 0; sr < BLK; ++sr) {
        int X[BLK], Y[BLK];
#pragma unroll
        for (int p = 0; p < BLK; ++p) {
          X[p] = p;
          Y[p] = BLK + (p + sr) % BLK;
        }
        any |= rr_round<S, TRACKV, BLK>(Wr, Vr, X, Y, tol, floor2, l);
      }
      // blocks move on: write to the next positions, read the blocks now at home
      __syncthreads();
      const int nA = rrc_next(pA, NB), nB = rrc_next(pB, NB);
#pragma unroll
      for (int c = 0; c < BLK; ++c) {
        W[(BLK * nA + c) * LD + l] = Wr[c];
        W[(BLK * nB + c) * LD + l] = Wr[BLK + c];
        if constexpr (TRACKV) {
          V[(BLK * nA + c) * LD + l] = Vr[c];
          V[(BLK * nB + c) * LD + l] = Vr[BLK + c];
        }
      }
      __syncthreads();
#pragma unroll
      for (int c = 0; c < BLK; ++c) {
        Wr[c] = W[(BLK * pA + c) * LD + l];
        Wr[BLK + c] = W[(BLK * pB + c) * LD + l];
        if constexpr (TRACKV) {
          Vr[c] = V[(BLK * pA + c) * LD + l];
          Vr[BLK + c] = V[(BLK * pB + c) * LD + l];
        }
      }
    }
    if (l == 0) flags[w] = any;
    __syncthreads();
    int all = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) all |= flags[k];
    if (!all) break;
  }
  // every block is home again in LDS (the last exchange of a sweep restores the
  // positions), matching the registers
  __syncthreads();
  return sweep;
}

}  // namespace vemb
