// Device helpers and load/store policies shared by the Jacobi eigensolver kernels
// (jacobi.hip: matrices held in LDS; jacobi_big.hip: matrices streamed through LDS).
#pragma once

#include <cfloat>

#include "kernels.h"

namespace vemb {
namespace {

constexpr int kThreads = 256;

template <typename R> struct eps_of;
template <> struct eps_of<double> { static constexpr double v = DBL_EPSILON; };
template <> struct eps_of<float> { static constexpr float v = FLT_EPSILON; };

__device__ inline double dev_sqrt(double x) { return sqrt(x); }
__device__ inline float dev_sqrt(float x) { return sqrtf(x); }
__device__ inline double dev_abs(double x) { return fabs(x); }
__device__ inline float dev_abs(float x) { return fabsf(x); }

template <typename T> __device__ inline T shfl_x(T v, int m) { return __shfl_xor(v, m); }
template <typename T> __device__ inline cplx<T> shfl_x(cplx<T> v, int m) {
  return {__shfl_xor(v.re, m), __shfl_xor(v.im, m)};
}

// Sum over aligned groups of G lanes (G a power of two up to 64), the same bits in every lane of a
// group.  Within a row of 16 lanes the DPP network adds operand pairs at register latency instead of
// the LDS crossbar's: rotations by 8, 4, 2, 1 for 16 lanes; for 8 lanes the half-row mirror
// (lane i with 7 - i) and the quad permutations swapping lanes 1 apart and 2 apart.  Every step
// adds two values that the partner lane adds in the other order, so a group agrees bit for bit.
// Offsets of 16 and 32 go through shuffles.
template <int CTRL> __device__ inline double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL> __device__ inline float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
constexpr int kDppQuadXor1 = 0xB1;     // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadXor2 = 0x4E;     // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;  // row_half_mirror
constexpr int kDppRowRor = 0x120;      // row_ror:N is kDppRowRor + N
template <int G, typename R> __device__ inline R group_sum(R v) {
  static_assert(G >= 1 && G <= 64 && (G & (G - 1)) == 0, "groups of a power of two lanes within a wavefront");
  if constexpr (G == 2 || G == 4) {
    v = v + dpp_mov<kDppQuadXor1>(v);
    if constexpr (G == 4) v = v + dpp_mov<kDppQuadXor2>(v);
  } else if constexpr (G == 8) {
    v = v + dpp_mov<kDppHalfMirror>(v);
    v = v + dpp_mov<kDppQuadXor1>(v);
    v = v + dpp_mov<kDppQuadXor2>(v);
  } else if constexpr (G >= 16) {
    v = v + dpp_mov<kDppRowRor + 8>(v);
    v = v + dpp_mov<kDppRowRor + 4>(v);
    v = v + dpp_mov<kDppRowRor + 2>(v);
    v = v + dpp_mov<kDppRowRor + 1>(v);
#pragma unroll
    for (int off = 16; off < G; off <<= 1) v = v + __shfl_xor(v, off);
  }
  return v;
}
template <int G, typename R> __device__ inline cplx<R> group_sum(cplx<R> v) {
  return {group_sum<G>(v.re), group_sum<G>(v.im)};
}

template <typename R> __device__ inline R scale_by(R s, R a) { return s * a; }
template <typename R> __device__ inline cplx<R> scale_by(R s, cplx<R> a) { return {s * a.re, s * a.im}; }

// Multiply by a unit phase (complex) or a sign (real).
template <typename R> __device__ inline R mul_phase(R ph, R a) { return ph * a; }
template <typename R> __device__ inline cplx<R> mul_phase(cplx<R> ph, cplx<R> a) { return ph * a; }

template <typename R> __device__ inline R modulus(R a) { return dev_abs(a); }
// |a| with scaling, so that tiny moduli do not underflow in the squares
template <typename R> __device__ inline R modulus(cplx<R> a) {
  const R x = dev_abs(a.re), y = dev_abs(a.im);
  const R big = x > y ? x : y;
  if (big == R(0)) return R(0);
  const R xs = x / big, ys = y / big;
  return big * dev_sqrt(xs * xs + ys * ys);
}

// 1/x and 1/sqrt(x) for the rotation parameters: the hardware estimates (v_rcp_f64, v_rsq_f64)
// refined by two Newton steps each (the error squares per step), instead of the correctly rounded
// division and square root sequences.  x > 0 and normal (the callers' arguments are at least 1 or a
// rotated |gamma| above the noise floor).  FP32 keeps the library operations.
__device__ inline double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  return fma(y, fma(-x, y, 1.0), y);
}
__device__ inline float rcp_nr(float x) { return 1.0f / x; }
__device__ inline double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}
__device__ inline float rsqrt_nr(float x) { return 1.0f / sqrtf(x); }

// |a| without the rescaling where the squares can neither overflow nor underflow.
template <typename R> struct square_safe;
template <> struct square_safe<double> { static constexpr double lo = 0x1p-500, hi = 0x1p500; };
template <> struct square_safe<float> { static constexpr float lo = 0x1p-60f, hi = 0x1p60f; };
template <typename R> __device__ inline R modulus_fast(R a) { return dev_abs(a); }
template <typename R> __device__ inline R modulus_fast(cplx<R> a) {
  const R x = dev_abs(a.re), y = dev_abs(a.im);
  const R big = x > y ? x : y;
  if (big > square_safe<R>::lo && big < square_safe<R>::hi) return dev_sqrt(a.re * a.re + a.im * a.im);
  return modulus(a);
}
// conj(gamma)/|gamma| from 1/|gamma| (complex); the exact sign of gamma (real).
template <typename R> __device__ inline R conj_phase_inv(R g, R) { return g < R(0) ? R(-1) : R(1); }
template <typename R> __device__ inline cplx<R> conj_phase_inv(cplx<R> g, R inv_absg) {
  return {g.re * inv_absg, -g.im * inv_absg};
}

// conj(gamma)/|gamma| for complex, sign(gamma) for real.
template <typename R> __device__ inline R conj_phase(R g, R absg) { return g / absg; }
template <typename R> __device__ inline cplx<R> conj_phase(cplx<R> g, R absg) { return {g.re / absg, -g.im / absg}; }

template <typename S> __device__ inline S hermitian_avg(S a, S b_transposed) {
  // (a + conj(b)) / 2
  using R = typename scalar_traits<S>::real;
  S cb = conjugate(b_transposed);
  return scale_by(R(0.5), a + cb);
}
template <> __device__ inline double hermitian_avg<double>(double a, double b) { return 0.5 * (a + b); }
template <> __device__ inline float hermitian_avg<float>(float a, float b) { return 0.5f * (a + b); }

template <typename S> __device__ inline S add_real(S a, typename scalar_traits<S>::real r) { return a + r; }
template <> __device__ inline cplx<double> add_real<cplx<double>>(cplx<double> a, double r) { return {a.re + r, a.im}; }
template <> __device__ inline cplx<float> add_real<cplx<float>>(cplx<float> a, float r) { return {a.re + r, a.im}; }

template <typename S> __device__ inline S drop_imag(S a) { return a; }
template <> __device__ inline cplx<double> drop_imag<cplx<double>>(cplx<double> a) { return {a.re, 0.0}; }
template <> __device__ inline cplx<float> drop_imag<cplx<float>>(cplx<float> a) { return {a.re, 0.0f}; }

template <typename S> struct wide { using type = double; };
template <> struct wide<float> { using type = double; };
template <> struct wide<cplx<double>> { using type = cplx<double>; };
template <> struct wide<cplx<float>> { using type = cplx<double>; };

template <typename S> __device__ inline S narrow(typename wide<S>::type v);
template <> __device__ inline double narrow<double>(double v) { return v; }
template <> __device__ inline float narrow<float>(double v) { return (float)v; }
template <> __device__ inline cplx<double> narrow<cplx<double>>(cplx<double> v) { return v; }
template <> __device__ inline cplx<float> narrow<cplx<float>>(cplx<double> v) { return {(float)v.re, (float)v.im}; }
__device__ inline double widen(double v) { return v; }
__device__ inline double widen(float v) { return (double)v; }
__device__ inline cplx<double> widen(cplx<double> v) { return v; }
__device__ inline cplx<double> widen(cplx<float> v) { return {(double)v.re, (double)v.im}; }

template <typename S> __device__ inline S one_of() { return S(1); }
template <> __device__ inline cplx<double> one_of<cplx<double>>() { return {1.0, 0.0}; }
template <> __device__ inline cplx<float> one_of<cplx<float>>() { return {1.0f, 0.0f}; }

// Block-wide reductions through LDS (blockDim.x threads, a power of two; red holds blockDim.x).
template <typename R>
__device__ R block_max(R v, R* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = (int)blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) red[t] = red[t] > red[t + s] ? red[t] : red[t + s];
    __syncthreads();
  }
  R r = red[0];
  __syncthreads();
  return r;
}

template <typename R>
__device__ R block_sum_r(R v, R* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = (int)blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  R r = red[0];
  __syncthreads();
  return r;
}

__device__ double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = (int)blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// Round-robin (circle method) pairing of np = n rounded up to even players.
__device__ inline void rr_pair(int round, int g, int np, int& p, int& q) {
  const int k = np - 1;
  if (g == 0) {
    p = k;
    q = round;
  } else {
    p = (round + g) % k;
    q = (round - g + k) % k;
  }
}

// kProject: Pi(C) through the policy's store; kEigvals: sorted eigenvalues;
// kVectors: only the eigenvectors (kept V), for a later refinement pass.
enum Mode { kProject = 0, kEigvals = 1, kVectors = 2 };

// ---------------------------------------------------------------------------
// Policies
// ---------------------------------------------------------------------------
template <typename S> __device__ inline S from_double(double v);
template <> __device__ inline double from_double<double>(double v) { return v; }
template <> __device__ inline float from_double<float>(double v) { return (float)v; }

__device__ inline double to_double(double v) { return v; }
__device__ inline double to_double(float v) { return (double)v; }

// Every policy also names where matrix `mat` keeps its eigenvectors (vslot).
struct PairPolicy {
  const double* rho;
  double* Lam;
  double* rho_t;
  double* feas;
  int* sweeps;
  int n;
  double mu;
  template <typename S> __device__ S load(int mat, int i, int j) const {
    const size_t o = (size_t)mat * n * n + (size_t)i * n + j;
    return from_double<S>(rho[o] - Lam[o] / mu);
  }
  template <typename S> __device__ double store(int mat, int i, int k, S v) const {
    const size_t o = (size_t)mat * n * n + (size_t)i * n + k;
    const double pv = to_double(v);
    const double r = rho[o];
    rho_t[o] = pv;
    Lam[o] = Lam[o] + mu * (pv - r);
    const double dlt = r - pv;
    return dlt * dlt;
  }
  __device__ void finish(int mat, double tot) const { feas[mat] = tot; }
  __device__ void record_sweeps(int mat, int s) const {
    if (sweeps) sweeps[mat] = s;
  }
  __device__ void store_eig(int, int, double) const {}
  template <typename D> __device__ D* vslot(void* base, int mat, size_t nn) const {
    return static_cast<D*>(base) + (size_t)mat * nn;
  }
};

struct MomentumPolicy {
  double* Xh;  // interleaved complex
  int* sweeps;
  int n;
  template <typename S> __device__ S load(int mat, int i, int j) const {
    const size_t o = 2 * ((size_t)mat * n * n + (size_t)i * n + j);
    using R = typename scalar_traits<S>::real;
    return S{(R)Xh[o], (R)Xh[o + 1]};
  }
  template <typename S> __device__ double store(int mat, int i, int k, S v) const {
    const size_t o = 2 * ((size_t)mat * n * n + (size_t)i * n + k);
    Xh[o] = (double)v.re;
    Xh[o + 1] = (double)v.im;
    return 0.0;
  }
  __device__ void finish(int, double) const {}
  __device__ void record_sweeps(int mat, int s) const {
    if (sweeps) sweeps[mat] = s;
  }
  __device__ void store_eig(int, int, double) const {}
  template <typename D> __device__ D* vslot(void* base, int mat, size_t nn) const {
    return static_cast<D*>(base) + (size_t)mat * nn;
  }
};

// Real or complex matrices in plain arrays (isolated entry points and the bound).
template <bool CPLX>
struct ArrayPolicy {
  const double* in;
  double* out;   // projection output (may alias in)
  double* w;     // eigenvalues (kEigvals)
  double* wmin;  // smallest eigenvalue only
  int* sweeps;
  int n;
  template <typename S> __device__ S load(int mat, int i, int j) const {
    if constexpr (CPLX) {
      const size_t o = 2 * ((size_t)mat * n * n + (size_t)i * n + j);
      using R = typename scalar_traits<S>::real;
      return S{(R)in[o], (R)in[o + 1]};
    } else {
      return from_double<S>(in[(size_t)mat * n * n + (size_t)i * n + j]);
    }
  }
  template <typename S> __device__ double store(int mat, int i, int k, S v) const {
    if constexpr (CPLX) {
      const size_t o = 2 * ((size_t)mat * n * n + (size_t)i * n + k);
      out[o] = (double)v.re;
      out[o + 1] = (double)v.im;
    } else {
      out[(size_t)mat * n * n + (size_t)i * n + k] = to_double(v);
    }
    return 0.0;
  }
  __device__ void finish(int, double) const {}
  __device__ void record_sweeps(int mat, int s) const {
    if (sweeps) sweeps[mat] = s;
  }
  __device__ void store_eig(int mat, int rank, double v) const {
    if (w) w[(size_t)mat * n + rank] = v;
    if (wmin && rank == 0) wmin[mat] = v;
  }
  template <typename D> __device__ D* vslot(void* base, int mat, size_t nn) const {
    return static_cast<D*>(base) + (size_t)mat * nn;
  }
};

// Batched policies: one launch covers the matrices of many problems of the same
// size; item[mat] = (instance, local index), per-instance pointers in `inst`.
struct BatchedPairPolicy {
  const int2* item;
  const PairPtrs* inst;
  int n;
  int record;  // write sweep counts
  template <typename S> __device__ S load(int mat, int i, int j) const {
    const int2 w = item[mat];
    const PairPtrs& P = inst[w.x];
    const size_t o = (size_t)w.y * n * n + (size_t)i * n + j;
    return from_double<S>(P.rho[o] - P.Lam[o] / P.mu);
  }
  template <typename S> __device__ double store(int mat, int i, int k, S v) const {
    const int2 w = item[mat];
    const PairPtrs& P = inst[w.x];
    const size_t o = (size_t)w.y * n * n + (size_t)i * n + k;
    const double pv = to_double(v);
    const double r = P.rho[o];
    P.rho_t[o] = pv;
    P.Lam[o] = P.Lam[o] + P.mu * (pv - r);
    const double dlt = r - pv;
    return dlt * dlt;
  }
  __device__ void finish(int mat, double tot) const {
    const int2 w = item[mat];
    inst[w.x].feas[w.y] = tot;
  }
  __device__ void record_sweeps(int mat, int s) const {
    const int2 w = item[mat];
    if (record && inst[w.x].sweeps) inst[w.x].sweeps[w.y] = s;
  }
  __device__ void store_eig(int, int, double) const {}
  template <typename D> __device__ D* vslot(void*, int mat, size_t nn) const {
    const int2 w = item[mat];
    return reinterpret_cast<D*>(inst[w.x].vstore) + (size_t)w.y * nn;
  }
};

// Whether a solve's matrix belongs to an instance that is being stepped: always for single problems; a
// batch skips the blocks of a masked instance (their workgroups return before any work).
template <typename Policy> __device__ inline bool policy_active(const Policy&, int) { return true; }
__device__ inline bool policy_active(const BatchedPairPolicy& p, int mat) { return p.inst[p.item[mat].x].active != 0; }

struct BatchedMomentumPolicy {
  const int2* item;
  const MomPtrs* inst;
  int n;
  int record;
  template <typename S> __device__ S load(int mat, int i, int j) const {
    const int2 w = item[mat];
    const size_t o = 2 * ((size_t)w.y * n * n + (size_t)i * n + j);
    using R = typename scalar_traits<S>::real;
    const double* X = inst[w.x].Xh;
    return S{(R)X[o], (R)X[o + 1]};
  }
  template <typename S> __device__ double store(int mat, int i, int k, S v) const {
    const int2 w = item[mat];
    const size_t o = 2 * ((size_t)w.y * n * n + (size_t)i * n + k);
    double* X = inst[w.x].Xh;
    X[o] = (double)v.re;
    X[o + 1] = (double)v.im;
    return 0.0;
  }
  __device__ void finish(int, double) const {}
  __device__ void record_sweeps(int mat, int s) const {
    const int2 w = item[mat];
    if (record && inst[w.x].sweeps) inst[w.x].sweeps[w.y] = s;
  }
  __device__ void store_eig(int, int, double) const {}
  template <typename D> __device__ D* vslot(void*, int mat, size_t nn) const {
    const int2 w = item[mat];
    return reinterpret_cast<D*>(inst[w.x].vstore) + (size_t)w.y * nn;
  }
};
__device__ inline bool policy_active(const BatchedMomentumPolicy& p, int mat) {
  return p.inst[p.item[mat].x].active != 0;
}


}  // namespace
}  // namespace vemb
