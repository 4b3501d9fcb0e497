// 16 x 16 matrix-core tiles over LDS operands (the eigensolver's dense products).
//
// v_mfma_f64_16x16x4_f64 / v_mfma_f32_16x16x4_f32: lane l supplies A(i, k) with
// i = l & 15, k = l >> 4 and B(k, j) with k = l >> 4, j = l & 15.  The result tile
// D(i, j) sits in lane j + 16 * (i % 4), register i / 4 for FP64, and in lane
// j + 16 * (i / 4), register i % 4 for FP32 (checked on gfx950).  Complex products
// take four real products per k-step.
#pragma once

#include "common.h"

namespace vemb {

typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));

template <typename R> struct MfmaAcc;
template <> struct MfmaAcc<double> { using T = mf_d4; };
template <> struct MfmaAcc<float> { using T = mf_f4; };

__device__ inline mf_d4 mfma_k4(double a, double b, mf_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline mf_f4 mfma_k4(float a, float b, mf_f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Row, within the tile, of result register r of lane l (the column is l & 15).
template <typename R> __device__ inline int mfma_row(int l, int r);
template <> __device__ inline int mfma_row<double>(int l, int r) { return (l >> 4) + 4 * r; }
template <> __device__ inline int mfma_row<float>(int l, int r) { return 4 * (l >> 4) + r; }

template <typename S> struct TileAcc {
  typename MfmaAcc<typename scalar_traits<S>::real>::T re, im;
};

// C = sum_{k < K} A(i0 + i, k) B(k, j0 + j) for the 16 x 16 tile at (i0, j0); K a
// multiple of 4; fa(i, k) and fb(k, j) read the operands (LDS).  One wavefront.
template <typename S, typename FA, typename FB>
__device__ inline TileAcc<S> tile_gemm(FA fa, FB fb, int K, int i0, int j0, int l) {
  using R = typename scalar_traits<S>::real;
  using A4 = typename MfmaAcc<R>::T;
  TileAcc<S> c;
  c.re = A4{R(0), R(0), R(0), R(0)};
  c.im = A4{R(0), R(0), R(0), R(0)};
  const int ia = i0 + (l & 15), kk = l >> 4, jb = j0 + (l & 15);
  for (int k0 = 0; k0 < K; k0 += 4) {
    const S a = fa(ia, k0 + kk);
    const S b = fb(k0 + kk, jb);
    if constexpr (scalar_traits<S>::is_complex) {
      c.re = mfma_k4(a.re, b.re, c.re);
      c.re = mfma_k4(-a.im, b.im, c.re);
      c.im = mfma_k4(a.re, b.im, c.im);
      c.im = mfma_k4(a.im, b.re, c.im);
    } else {
      c.re = mfma_k4(a, b, c.re);
    }
  }
  return c;
}

template <typename S> __device__ inline S tile_value(const TileAcc<S>& c, int r) {
  if constexpr (scalar_traits<S>::is_complex)
    return S{c.re[r], c.im[r]};
  else
    return c.re[r];
}

}  // namespace vemb
