// PSD projection / eigenvalues for matrices too large to hold in LDS (n up to 256):
// the same one-sided Jacobi method as jacobi.hip (shift by the Gershgorin bound,
// orthogonalise the columns of W = B V, Pi(C) = sum (sigma - s)/sigma^2 w w^H),
// with W and V kept in global scratch and streamed through LDS in column blocks.
//
// Block Jacobi: the n columns form nb = n/BLK blocks.  A sweep rotates every pair
// of columns once: first all pairs inside each block (round-robin on BLK columns),
// then, for every block pair (I, J), the BLK x BLK cross pairs in BLK rounds of
// BLK disjoint pairs (I_i, J_{(i+r) mod BLK}).  Two blocks of W and V sit in LDS
// at a time (4 x BLK x (n+1) scalars, 132 KB at n = 256).  Warm start: W = (T + sI)
// V_prev by an LDS-tiled GEMM, where T is the Hermitian part of C.  One workgroup
// (256 threads) per matrix.
#include "jacobi_common.h"

namespace vemb {
namespace {

constexpr int kBigMax = 256;  // largest n

template <typename S> struct big_block { static constexpr int v = 16; };
template <> struct big_block<cplx<double>> { static constexpr int v = 8; };
template <> struct big_block<float> { static constexpr int v = 32; };
template <> struct big_block<cplx<float>> { static constexpr int v = 16; };

// Rotates the column pair (Wp, Wq) (and Vp, Vq) held in LDS, G lanes per pair,
// rows l, l+G, ... < n.  Returns |gamma| / sqrt(alpha beta) when this group rotated, else 0.
template <typename S, int G, bool TRACKV>
__device__ typename scalar_traits<S>::real rotate_pair(S* Wp, S* Wq, S* Vp, S* Vq, int n, int l, bool live,
                            typename scalar_traits<S>::real tol, typename scalar_traits<S>::real floor2) {
  using R = typename scalar_traits<S>::real;
  constexpr int RPL = (kBigMax + G - 1) / G;
  S a[RPL], b[RPL];
  R alpha = R(0), beta = R(0);
  S gam = s_zero<S>();
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int i = l + r * G;
    if (live && i < n) {
      a[r] = Wp[i];
      b[r] = Wq[i];
    } else {
      a[r] = s_zero<S>();
      b[r] = s_zero<S>();
    }
    alpha += abs2(a[r]);
    beta += abs2(b[r]);
    gam = gam + conj_mul(a[r], b[r]);
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) {
    alpha += shfl_x(alpha, off);
    beta += shfl_x(beta, off);
    gam = gam + shfl_x(gam, off);
  }
  const R ag = modulus(gam);
  const R small = alpha < beta ? alpha : beta;
  const R gab = dev_sqrt(alpha * beta);
  if (!(live && small > floor2 && ag > tol * gab && ag > R(0))) return R(0);
  const R zeta = (beta - alpha) / (R(2) * ag);
  R t = R(1) / (dev_abs(zeta) + dev_sqrt(R(1) + zeta * zeta));
  if (zeta < R(0)) t = -t;
  const R c = R(1) / dev_sqrt(R(1) + t * t);
  const R s = c * t;
  const S ph = conj_phase(gam, ag);
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int i = l + r * G;
    if (i < n) {
      const S bq = mul_phase(ph, b[r]);
      Wp[i] = scale_by(c, a[r]) - scale_by(s, bq);
      Wq[i] = scale_by(s, a[r]) + scale_by(c, bq);
      if constexpr (TRACKV) {
        const S va = Vp[i];
        const S vb = mul_phase(ph, Vq[i]);
        Vp[i] = scale_by(c, va) - scale_by(s, vb);
        Vq[i] = scale_by(s, va) + scale_by(c, vb);
      }
    }
  }
  return ag / gab;
}

// C (n x n, column-major) = A (n x K) * op(B) where A(i, k) = a(i, k) and the
// second operand is read through b(k, j); out(i, j, value) consumes each entry.
// 64 x 64 output tiles, K in chunks of 16, 4 x 4 register tile per thread.
template <typename S, typename FA, typename FB, typename FOut>
__device__ void tiled_gemm(int n, int K, S* lds, FA a, FB b, FOut out) {
  constexpr int TM = 64, KC = 16;
  S* As = lds;             // [KC][TM]
  S* Bs = lds + KC * TM;   // [KC][TM]
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;
  for (int i0 = 0; i0 < n; i0 += TM)
    for (int j0 = 0; j0 < n; j0 += TM) {
      S acc[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = s_zero<S>();
      for (int k0 = 0; k0 < K; k0 += KC) {
        for (int e = tid; e < KC * TM; e += kThreads) {
          const int kk = e / TM, ii = e % TM;
          const int i = i0 + ii, k = k0 + kk;
          As[kk * TM + ii] = (i < n && k < K) ? a(i, k) : s_zero<S>();
          const int j = j0 + ii;
          Bs[kk * TM + ii] = (j < n && k < K) ? b(k, j) : s_zero<S>();
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < KC; ++kk) {
          S av[4], bv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            av[u] = As[kk * TM + ty * 4 + u];
            bv[u] = Bs[kk * TM + tx * 4 + u];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = acc[u][v] + av[u] * bv[v];
        }
        __syncthreads();
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = i0 + ty * 4 + u, j = j0 + tx * 4 + v;
          if (i < n && j < n) out(i, j, acc[u][v]);
        }
    }
}

template <typename S, int MODE, bool TRACKV, typename Policy>
__global__ void __launch_bounds__(kThreads) jacobi_big_kernel(Policy pol, int n, int max_sweeps, void* vstore_raw,
                                                              S* wscr, S* tscr, int cold) {
  using R = typename scalar_traits<S>::real;
  using D = typename wide<S>::type;
  constexpr int BLK = big_block<S>::v;
  constexpr int LDC = kBigMax + 1;
  __shared__ S L[4 * BLK * LDC];
  __shared__ R red[kThreads];
  __shared__ double red_d[kThreads];
  __shared__ R colf[kBigMax];
  __shared__ int active[kBigMax];
  __shared__ int nact_s;
  __shared__ int rotated;

  const int mat = blockIdx.x, tid = threadIdx.x;
  const size_t nn = (size_t)n * n;
  S* W = wscr + mat * nn;  // column-major: W(i, j) = W[j*n + i]
  S* T = tscr + mat * nn;
  D* Vg = TRACKV ? pol.template vslot<D>(vstore_raw, mat, nn) : nullptr;

  // 0. cold == 2: orthonormalise the kept V (from a lower-precision solve) by one
  // Newton-Schulz step V <- V (3I - V^H V)/2, with G in T and the result via W.
  if constexpr (TRACKV) {
    if (cold == 2) {
      tiled_gemm<S>(
          n, n, L, [&](int i, int k) { return conjugate(narrow<S>(Vg[(size_t)i * n + k])); },
          [&](int k, int j) { return narrow<S>(Vg[(size_t)j * n + k]); },
          [&](int i, int j, S v) { T[(size_t)j * n + i] = v; });
      __syncthreads();
      tiled_gemm<S>(
          n, n, L, [&](int i, int k) { return narrow<S>(Vg[(size_t)k * n + i]); },
          [&](int k, int j) { return T[(size_t)j * n + k]; },
          [&](int i, int j, S v) {
            W[(size_t)j * n + i] = scale_by(R(1.5), narrow<S>(Vg[(size_t)j * n + i])) - scale_by(R(0.5), v);
          });
      __syncthreads();
      for (size_t idx = tid; idx < nn; idx += kThreads) Vg[idx] = widen(W[idx]);
      __syncthreads();
    }
  }

  // 1. T = Hermitian part of C
  for (size_t idx = tid; idx < nn; idx += kThreads) {
    const int j = (int)(idx / n), i = (int)(idx % n);
    S v;
    if (i == j)
      v = drop_imag(pol.template load<S>(mat, i, i));
    else
      v = hermitian_avg(pol.template load<S>(mat, i, j), pol.template load<S>(mat, j, i));
    T[idx] = v;
  }
  __syncthreads();

  // 2. Gershgorin shift
  R shift;
  {
    R v = R(0);
    for (int i = tid; i < n; i += kThreads) {
      R rad = R(0);
      for (int j = 0; j < n; ++j)
        if (j != i) rad += modulus(T[(size_t)j * n + i]);
      const R e = rad - re_part(T[(size_t)i * n + i]);
      v = e > v ? e : v;
    }
    // Pi needs only s >= -lambda_min(C)/2: every negative eigenvalue b of B then has
    // |b| <= s, so it and any column one-sided Jacobi mixes with it (same |b|) fall at or
    // below the cut sigma > s.  Half the Gershgorin bound satisfies this and halves the
    // shift's share of the rounding error.  Eigenvalue mode needs B >= 0: full bound.
    shift = block_max(v, red);
    if constexpr (MODE != kEigvals) shift *= R(0.5);
  }

  // 3. W = (T + s I) V_prev (warm) or T + s I (cold, V = I)
  if (TRACKV && cold != 1) {
    tiled_gemm<S>(
        n, n, L, [&](int i, int k) { return T[(size_t)k * n + i]; },
        [&](int k, int j) { return narrow<S>(Vg[(size_t)j * n + k]); },
        [&](int i, int j, S v) { W[(size_t)j * n + i] = v + scale_by(shift, narrow<S>(Vg[(size_t)j * n + i])); });
  } else {
    for (size_t idx = tid; idx < nn; idx += kThreads) {
      const int j = (int)(idx / n), i = (int)(idx % n);
      W[idx] = (i == j) ? add_real(T[idx], shift) : T[idx];
      if constexpr (TRACKV) Vg[idx] = widen(i == j ? one_of<S>() : s_zero<S>());
    }
  }
  __syncthreads();

  R floor2;
  {
    R v = R(0);
    for (size_t idx = tid; idx < nn; idx += kThreads) v += abs2(W[idx]);
    const R eta = R(n > 16 ? n : 16) * eps_of<R>::v;
    floor2 = eta * eta * block_sum_r(v, red);
  }
  const R tol = R(n > 16 ? n : 16) * eps_of<R>::v;
  const int nb = n / BLK;

  auto load_block = [&](int blk, int slot) {
    for (int e = tid; e < BLK * n; e += kThreads) {
      const int c = e / n, i = e % n;
      L[(slot * BLK + c) * LDC + i] = W[(size_t)(blk * BLK + c) * n + i];
      if constexpr (TRACKV) L[((slot + 2) * BLK + c) * LDC + i] = narrow<S>(Vg[(size_t)(blk * BLK + c) * n + i]);
    }
  };
  auto store_block = [&](int blk, int slot) {
    for (int e = tid; e < BLK * n; e += kThreads) {
      const int c = e / n, i = e % n;
      W[(size_t)(blk * BLK + c) * n + i] = L[(slot * BLK + c) * LDC + i];
      if constexpr (TRACKV) Vg[(size_t)(blk * BLK + c) * n + i] = widen(L[((slot + 2) * BLK + c) * LDC + i]);
    }
  };

  // 4. sweeps (ended early as in the LDS solver: once the largest rotation of a sweep is below
  // sqrt(tol) / 16, the next sweep would rotate nothing)
  const R early = dev_sqrt(tol) * R(0.0625);
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    R relmax = R(0);
    if (tid == 0) rotated = 0;
    __syncthreads();
    // 4a. pairs inside each block: round-robin on BLK columns, BLK/2 pairs per round
    {
      constexpr int NP = BLK / 2;
      constexpr int G0 = kThreads / NP;
      constexpr int G = G0 > 64 ? 64 : G0;
      const int g = tid / G, l = tid % G;
      for (int blk = 0; blk < nb; ++blk) {
        load_block(blk, 0);
        __syncthreads();
        for (int round = 0; round < BLK - 1; ++round) {
          int p = 0, q = 0;
          const bool live = g < NP;
          if (live) rr_pair(round, g, BLK, p, q);
          const R rel = rotate_pair<S, G, TRACKV>(&L[p * LDC], &L[q * LDC], &L[(2 * BLK + p) * LDC],
                                                  &L[(2 * BLK + q) * LDC], n, l, live, tol, floor2);
          relmax = rel > relmax ? rel : relmax;
          if (rel > R(0) && l == 0) rotated = 1;
          __syncthreads();
        }
        store_block(blk, 0);
        __syncthreads();
      }
    }
    // 4b. cross pairs of every block pair
    {
      constexpr int G0 = kThreads / BLK;
      constexpr int G = G0 > 64 ? 64 : G0;
      const int g = tid / G, l = tid % G;
      for (int bi = 0; bi < nb; ++bi)
        for (int bj = bi + 1; bj < nb; ++bj) {
          load_block(bi, 0);
          load_block(bj, 1);
          __syncthreads();
          for (int r = 0; r < BLK; ++r) {
            const bool live = g < BLK;
            const int p = g, q = BLK + (g + r) % BLK;
            const R rel = rotate_pair<S, G, TRACKV>(&L[p * LDC], &L[q * LDC], &L[(2 * BLK + p) * LDC],
                                                    &L[(2 * BLK + q) * LDC], n, l, live, tol, floor2);
            relmax = rel > relmax ? rel : relmax;
            if (rel > R(0) && l == 0) rotated = 1;
            __syncthreads();
          }
          store_block(bi, 0);
          store_block(bj, 1);
          __syncthreads();
        }
    }
    const int any = rotated;
    __syncthreads();
    if (!any) break;
    if (block_max(relmax, red) < early) {
      ++sweep;
      break;
    }
  }
  if (tid == 0) pol.record_sweeps(mat, sweep);
  if constexpr (MODE == kVectors) return;

  // 5. column norms
  for (int j = tid; j < n; j += kThreads) {
    R s2 = R(0);
    for (int i = 0; i < n; ++i) s2 += abs2(W[(size_t)j * n + i]);
    colf[j] = dev_sqrt(s2);
  }
  __syncthreads();

  if constexpr (MODE == kEigvals) {
    for (int j = tid; j < n; j += kThreads) {
      const R v = colf[j] - shift;
      int rank = 0;
      for (int k = 0; k < n; ++k) {
        const R u = colf[k] - shift;
        rank += (u < v) || (u == v && k < j);
      }
      pol.store_eig(mat, rank, (double)v);
    }
  } else {
    if (tid == 0) {
      int k = 0;
      for (int j = 0; j < n; ++j)
        if (colf[j] > shift) active[k++] = j;
      nact_s = k;
    }
    __syncthreads();
    const int nact = nact_s;
    // U_j = sqrt(sigma_j - s)/sigma_j w_j, packed into T's columns 0..nact-1
    for (size_t e = tid; e < (size_t)nact * n; e += kThreads) {
      const int jj = (int)(e / n), i = (int)(e % n);
      const int j = active[jj];
      const R f = dev_sqrt(colf[j] - shift) / colf[j];
      T[(size_t)jj * n + i] = scale_by(f, W[(size_t)j * n + i]);
    }
    __syncthreads();
    double part = 0.0;
    tiled_gemm<S>(
        n, nact, L, [&](int i, int k) { return T[(size_t)k * n + i]; },
        [&](int k, int j) { return conjugate(T[(size_t)k * n + j]); },
        [&](int i, int j, S v) { part += pol.store(mat, i, j, v); });
    const double tot = block_sum(part, red_d);
    if (tid == 0) pol.finish(mat, tot);
  }
}

}  // namespace

template <typename S, int MODE, typename Policy>
hipError_t big_dispatch(const Policy& pol, int n, int count, int max_sweeps, double* vstore, void* wscr, void* tscr,
                        int cold, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (n > kBigMax || n % big_block<S>::v) return hipErrorInvalidValue;
  if (vstore && MODE != kEigvals)
    hipLaunchKernelGGL((jacobi_big_kernel<S, MODE, true, Policy>), dim3(count), dim3(kThreads), 0, st, pol, n,
                       max_sweeps, (void*)vstore, (S*)wscr, (S*)tscr, cold);
  else
    hipLaunchKernelGGL((jacobi_big_kernel<S, MODE, false, Policy>), dim3(count), dim3(kThreads), 0, st, pol, n,
                       max_sweeps, nullptr, (S*)wscr, (S*)tscr, 1);
  return hipGetLastError();
}

// FP64, FP32, or MIXED (FP32 sweeps for the eigenvectors, then one warm FP64 sweep + FP64 rebuild).
template <typename S32, typename S64, typename Policy>
hipError_t big_by_precision(const Policy& pol, const Policy& quiet, int n, int count, int precision, int max_sweeps,
                            double* vstore, int cold, void* wscr, void* tscr, hipStream_t st) {
  if (precision == VEMB_FP32) return big_dispatch<S32, kProject>(pol, n, count, max_sweeps, vstore, wscr, tscr, cold, st);
  if (precision == VEMB_MIXED && vstore) {
    hipError_t e = big_dispatch<S32, kVectors>(pol, n, count, max_sweeps, vstore, wscr, tscr, cold, st);
    if (e != hipSuccess) return e;
    return big_dispatch<S64, kProject>(quiet, n, count, 3, vstore, wscr, tscr, 2, st);
  }
  return big_dispatch<S64, kProject>(pol, n, count, max_sweeps, vstore, wscr, tscr, cold, st);
}

hipError_t launch_pair_projection_big(const double* rho, double* Lam, double* rho_t, double* feas, int n, int P,
                                      double mu, int precision, int max_sweeps, int* sweeps, double* vstore, int cold,
                                      void* wscr, void* tscr, hipStream_t st) {
  PairPolicy pol{rho, Lam, rho_t, feas, sweeps, n, mu};
  PairPolicy quiet{rho, Lam, rho_t, feas, nullptr, n, mu};
  return big_by_precision<float, double>(pol, quiet, n, P, precision, max_sweeps, vstore, cold, wscr, tscr, st);
}

hipError_t launch_momentum_projection_big(double* Xh, int n_op, int K, int precision, int max_sweeps, int* sweeps,
                                          double* vstore, int cold, void* wscr, void* tscr, hipStream_t st) {
  MomentumPolicy pol{Xh, sweeps, n_op};
  MomentumPolicy quiet{Xh, nullptr, n_op};
  return big_by_precision<cplx<float>, cplx<double>>(pol, quiet, n_op, K, precision, max_sweeps, vstore, cold, wscr,
                                                     tscr, st);
}

hipError_t launch_psd_batched_big(const double* in, double* out, int n, int batch, bool is_complex, int precision,
                                  int max_sweeps, int* sweeps, double* vstore, void* wscr, void* tscr, hipStream_t st,
                                  int cold) {
  if (!vstore) cold = 1;
  if (is_complex) {
    ArrayPolicy<true> pol{in, out, nullptr, nullptr, sweeps, n};
    ArrayPolicy<true> quiet{in, out, nullptr, nullptr, nullptr, n};
    return big_by_precision<cplx<float>, cplx<double>>(pol, quiet, n, batch, precision, max_sweeps, vstore, cold,
                                                       wscr, tscr, st);
  }
  ArrayPolicy<false> pol{in, out, nullptr, nullptr, sweeps, n};
  ArrayPolicy<false> quiet{in, out, nullptr, nullptr, nullptr, n};
  return big_by_precision<float, double>(pol, quiet, n, batch, precision, max_sweeps, vstore, cold, wscr, tscr, st);
}

hipError_t launch_projection_group_lds(int kind, int n, int count, int precision, int max_sweeps, int cold, int tpb,
                                       const int2* item, const void* ptrs, void* vstore_any, hipStream_t st);

hipError_t launch_projection_group(int kind, int n, int count, int precision, int max_sweeps, int cold, int tpb,
                                   const int2* item, const void* ptrs, void* vstore_any, void* wscr, void* tscr,
                                   hipStream_t st) {
  const bool lds = n <= 64;
  if (lds) return launch_projection_group_lds(kind, n, count, precision, max_sweeps, cold, tpb, item, ptrs, vstore_any, st);
  double* vs = static_cast<double*>(vstore_any);
  if (kind == 0) {
    BatchedPairPolicy pol{item, static_cast<const PairPtrs*>(ptrs), n, 1};
    BatchedPairPolicy quiet{item, static_cast<const PairPtrs*>(ptrs), n, 0};
    return big_by_precision<float, double>(pol, quiet, n, count, precision, max_sweeps, vs, cold, wscr, tscr, st);
  }
  BatchedMomentumPolicy pol{item, static_cast<const MomPtrs*>(ptrs), n, 1};
  BatchedMomentumPolicy quiet{item, static_cast<const MomPtrs*>(ptrs), n, 0};
  return big_by_precision<cplx<float>, cplx<double>>(pol, quiet, n, count, precision, max_sweeps, vs, cold, wscr,
                                                     tscr, st);
}

hipError_t launch_eigvals_big(const double* in, double* w, double* wmin, int n, int count, bool is_complex,
                              int max_sweeps, int* sweeps, void* wscr, void* tscr, hipStream_t st) {
  if (is_complex) {
    ArrayPolicy<true> pol{in, nullptr, w, wmin, sweeps, n};
    return big_dispatch<cplx<double>, kEigvals>(pol, n, count, max_sweeps, nullptr, wscr, tscr, 1, st);
  }
  ArrayPolicy<false> pol{in, nullptr, w, wmin, sweeps, n};
  return big_dispatch<double, kEigvals>(pol, n, count, max_sweeps, nullptr, wscr, tscr, 1, st);
}

}  // namespace vemb
