// Internal helpers shared by the HIP translation units of libvemb.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/vemb.h"

namespace vemb {

// Threads-per-workgroup codes naming the register-resident n = 64 Jacobi kernels
// (jacobi_rr.h): 8-column blocks on 4 wavefronts, 4-column blocks on 8.
constexpr int kTpbRegister8 = 64;
constexpr int kTpbRegister4 = 128;

// Thread-local last-error message (set on every failing ABI call).
void set_error(const std::string& msg);

#define VEMB_HIP_CHECK(expr)                                                                  \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      ::vemb::set_error(std::string(#expr) + " failed: " + hipGetErrorString(e_));             \
      return VEMB_E_HIP;                                                                      \
    }                                                                                         \
  } while (0)

// ---------------------------------------------------------------------------
// Minimal complex type usable in device code and in templates over T.
// ---------------------------------------------------------------------------
template <typename T>
struct cplx {
  T re, im;
};

template <typename T>
struct scalar_traits {
  using real = T;
  static constexpr bool is_complex = false;
};
template <typename T>
struct scalar_traits<cplx<T>> {
  using real = T;
  static constexpr bool is_complex = true;
};

template <typename T> __host__ __device__ inline T s_zero() { return T(0); }
template <> __host__ __device__ inline cplx<double> s_zero<cplx<double>>() { return {0.0, 0.0}; }
template <> __host__ __device__ inline cplx<float> s_zero<cplx<float>>() { return {0.0f, 0.0f}; }

__host__ __device__ inline double abs2(double a) { return a * a; }
__host__ __device__ inline float abs2(float a) { return a * a; }
template <typename T> __host__ __device__ inline T abs2(cplx<T> a) { return a.re * a.re + a.im * a.im; }

__host__ __device__ inline double conj_mul(double a, double b) { return a * b; }  // conj(a) * b
__host__ __device__ inline float conj_mul(float a, float b) { return a * b; }
template <typename T> __host__ __device__ inline cplx<T> conj_mul(cplx<T> a, cplx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}

template <typename T> __host__ __device__ inline cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __host__ __device__ inline cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __host__ __device__ inline cplx<T> operator*(T s, cplx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> __host__ __device__ inline cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __host__ __device__ inline cplx<T> conjugate(cplx<T> a) { return {a.re, -a.im}; }
__host__ __device__ inline double conjugate(double a) { return a; }
__host__ __device__ inline float conjugate(float a) { return a; }

// Real part (identity for real scalars).
__host__ __device__ inline double re_part(double a) { return a; }
__host__ __device__ inline float re_part(float a) { return a; }
template <typename T> __host__ __device__ inline T re_part(cplx<T> a) { return a.re; }

// Conversions between precisions (FP64 storage <-> compute type).
template <typename D, typename S> struct convert;
template <typename D> struct convert<D, D> { __host__ __device__ static D go(D a) { return a; } };
template <> struct convert<float, double> { __host__ __device__ static float go(double a) { return (float)a; } };
template <> struct convert<double, float> { __host__ __device__ static double go(float a) { return (double)a; } };
template <> struct convert<cplx<float>, cplx<double>> {
  __host__ __device__ static cplx<float> go(cplx<double> a) { return {(float)a.re, (float)a.im}; }
};
template <> struct convert<cplx<double>, cplx<float>> {
  __host__ __device__ static cplx<double> go(cplx<float> a) { return {(double)a.re, (double)a.im}; }
};

// ---------------------------------------------------------------------------
// Operator-collection tables for PAULI1 (signed permutations, Section 2.2):
// O_alpha[u][v] = sign[alpha][u] / sqrt(m) when v = perm[alpha][u], else 0.
// ---------------------------------------------------------------------------
// Jordan-Wigner parity sign of fermionic pair blocks (complete collection): an odd matrix
// unit E_ce of the second cluster (popcount(c) + popcount(e) odd), taken to the pair's
// order, carries the first cluster's parity string, which multiplies the unit E_ba of the
// first cluster by (-1)^popcount(a).
__device__ inline double jw_sign(int a, int c, int e) {
  const int pc = __builtin_popcount((unsigned)c), pe = __builtin_popcount((unsigned)e);
  return (((pc + pe) & __builtin_popcount((unsigned)a)) & 1) ? -1.0 : 1.0;
}

constexpr int kMaxOps = 12;  // 3 L for L <= 4
constexpr int kMaxM = 16;

struct OpTables {
  int n_op;
  int8_t perm[kMaxOps][kMaxM];
  int8_t sign[kMaxOps][kMaxM];
};

}  // namespace vemb
