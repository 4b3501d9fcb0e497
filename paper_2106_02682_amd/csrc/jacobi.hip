// Batched PSD projection Pi(C) = argmin_{S >= 0} ||S - C||_F (Section 3, definition of Pi)
// by a one-sided (Hestenes) Jacobi eigensolver held in LDS, one workgroup per matrix.
//
// Method.  Pi needs the eigenpairs of C with positive eigenvalues.  The kernel
// shifts C to B = C + s I with s from the Gershgorin bound g = max(0, max_i (r_i - c_ii))
// >= -lambda_min(C) (s = g for eigenvalues, g/2 for Pi, see below), then
// orthogonalises the columns of W = B by
// plane rotations W <- W J (round-robin parallel ordering: n/2 disjoint column
// pairs per round, every pair once per sweep).  At convergence W = B V with V
// orthogonal and W's columns mutually orthogonal, hence w_j = lambda_j(B) v_j
// and ||w_j|| = lambda_j(B) >= 0.  Then
//     Pi(C) = sum_{||w_j|| > s} (||w_j|| - s) / ||w_j||^2  w_j w_j^H,
// so V is not needed for Pi.  Eigenvalues of C are ||w_j|| - s when B is PSD.
// One-sided Jacobi sees only |b| of B's eigenvalues, so +-b pairs can mix; with
// s >= -lambda_min/2 every such pair lies at or below the cut and Pi is unaffected.  Hermitian blocks use the complex rotation
// [w_p, w_q] <- [w_p, conj(e) w_q] R(c, s) with e = gamma/|gamma|.
//
// Work split: 256 threads; each column pair of a round is owned by a group of G
// lanes of one wavefront (G = 256 / (n/2), at most 64), each lane holding n/G
// rows; the three dot products are reduced with wavefront shuffles.  One
// barrier per round.  Sweeps stop when no pair rotated, or after a sweep whose rotations were all
// small enough that the next one would rotate nothing (|gamma| <= tol
// sqrt(alpha beta), tol = max(n, 16) * machine epsilon of the compute type);
// columns of negligible norm (rounding noise left by an exactly singular B) are
// not rotated, see below.
#include <type_traits>

#include "jacobi_common.h"
#include "jacobi_rr.h"
#include "mfma_tile.h"

namespace vemb {
namespace {

// ---------------------------------------------------------------------------
// Core kernel.  S: compute scalar (double, float, cplx<double>, cplx<float>);
// NMAX: capacity (n <= NMAX, NMAX even); Policy: load / store of one matrix.
// ---------------------------------------------------------------------------
// LDS layout of one solve (byte offsets, 16-byte aligned): W and V (n x n, padded columns), the
// reduction buffers, the column norms, the active-column list and a few flags.
constexpr size_t lds_align(size_t b) { return (b + 15) & ~size_t(15); }
template <typename S, int NMAX, bool WARM, int NT>
struct JacobiLds {
  using R = typename scalar_traits<S>::real;
  static constexpr int LD = NMAX + 1;
  static constexpr size_t oV = lds_align(sizeof(S) * NMAX * LD);
  static constexpr size_t oRed = lds_align(oV + sizeof(S) * (WARM ? NMAX * LD : 1));
  static constexpr size_t oRedD = lds_align(oRed + sizeof(R) * NT);
  static constexpr size_t oColf = lds_align(oRedD + sizeof(double) * NT);
  static constexpr size_t oCn = lds_align(oColf + sizeof(R) * NMAX);
  static constexpr size_t oAct = lds_align(oCn + sizeof(R) * NMAX);
  static constexpr size_t oInts = lds_align(oAct + sizeof(int) * NMAX);  // nact, rotated, 8 wavefront flags
  static constexpr size_t bytes = lds_align(oInts + sizeof(int) * 10);
};

// One matrix (index mat of the policy) per workgroup, in the LDS area smem (JacobiLds bytes).
template <typename S, int NMAX, int MODE, bool WARM, int NT, typename Policy, bool REG = false, bool VG = false>
__device__ __attribute__((always_inline)) void jacobi_body(Policy pol, int n, int max_sweeps, void* vstore_raw,
                                                           int cold, const int mat, unsigned char* smem) {
  static_assert(!REG || (NMAX == 64 && (NT == 256 || NT == 512)), "register-resident sweeps: n = 64, 4 or 8 waves");
  // VG: a warm projection solve whose kept V is read from its slot by the warm-start product instead of
  // being staged in LDS (cold must not be 2), so the solve's LDS holds W alone
  static_assert(!VG || (WARM && MODE == kProject && !REG), "V from its slot: warm projection solves only");
  using R = typename scalar_traits<S>::real;
  using D = typename wide<S>::type;  // FP64 storage type of V
  constexpr int LD = NMAX + 1;  // padded column stride (wider padding measured no faster)
  constexpr int NPAIR = NMAX / 2;
  constexpr int G0 = NT / NPAIR;
  constexpr int G = G0 > 64 ? 64 : G0;  // lanes per pair, within one wavefront
  constexpr int RPL = (NMAX + G - 1) / G;  // rows per lane
  // Projection solves keep no rotated copy of V during the sweeps: at convergence W = B V has
  // mutually orthogonal columns (to the relative tolerance, checked on the stored W), so w_j / ||w_j||
  // is an orthonormal eigenbasis of B (sign(lambda_j) v_j) and is what the next warm start needs.
  // A block with a column at the noise floor (never rotated, so not orthogonal to the rest) keeps the
  // identity instead, which makes its next solve cold.  Half of every round's LDS traffic and
  // arithmetic (the V columns) goes away.
  constexpr bool VFW = WARM && MODE == kProject && !REG;
  using L = JacobiLds<S, NMAX, WARM && !VG, NT>;
  S* const W = reinterpret_cast<S*>(smem);
  S* const V = reinterpret_cast<S*>(smem + L::oV);
  R* const red = reinterpret_cast<R*>(smem + L::oRed);
  double* const red_d = reinterpret_cast<double*>(smem + L::oRedD);
  R* const colf = reinterpret_cast<R*>(smem + L::oColf);
  R* const cn = reinterpret_cast<R*>(smem + L::oCn);  // squared column norms carried through a sweep
  int* const active = reinterpret_cast<int*>(smem + L::oAct);
  int* const ints = reinterpret_cast<int*>(smem + L::oInts);
  int& nact_s = ints[0];
  int& rotated = ints[1];
  int* const rr_flags = ints + 2;

  const int tid = threadIdx.x;
  const int nn = n * n;
  constexpr int NOUT = (NMAX * NMAX + NT - 1) / NT;
  // dense products on matrix cores: 16 x 16 tiles, n a multiple of 16
  constexpr int NWAVE = NT / 64;
  constexpr int TMAX = NMAX >= 16 ? (NMAX / 16) * (NMAX / 16) : 0;
  constexpr int TPW = TMAX > 0 ? (TMAX + NWAVE - 1) / NWAVE : 0;
  const bool use_mfma = TMAX > 0 && n % 16 == 0;
  const int wv = tid >> 6, ln = tid & 63;

  // 0. cold == 2: the kept V comes from a lower-precision solve; restore its
  // orthonormality first with one Newton-Schulz step V <- V (3I - V^H V)/2
  // (defect E -> O(E^2)), using W as the buffer for G = V^H V.
  if constexpr (WARM && !VG) {
    if (cold == 2) {
      const D* vin = pol.template vslot<D>(vstore_raw, mat, (size_t)nn);
      for (int idx = tid; idx < nn; idx += NT) {
        const int j = idx / n, i = idx - (idx / n) * n;
        V[j * LD + i] = narrow<S>(vin[idx]);
      }
      __syncthreads();
      S outv[NOUT];
      #pragma unroll
      for (int c = 0; c < NOUT; ++c) {  // compile-time c keeps outv in registers
        const int idx = tid + c * NT;
        if (idx >= nn) break;
        const int j = idx / n, i = idx - (idx / n) * n;
        S acc = s_zero<S>();
        for (int k = 0; k < n; ++k) acc = acc + conj_mul(V[i * LD + k], V[j * LD + k]);
        outv[c] = acc;  // G(i, j)
      }
      #pragma unroll
      for (int c = 0; c < NOUT; ++c) {  // compile-time c keeps outv in registers
        const int idx = tid + c * NT;
        if (idx >= nn) break;
        const int j = idx / n, i = idx - (idx / n) * n;
        W[j * LD + i] = outv[c];
      }
      __syncthreads();
      #pragma unroll
      for (int c = 0; c < NOUT; ++c) {  // compile-time c keeps outv in registers
        const int idx = tid + c * NT;
        if (idx >= nn) break;
        const int j = idx / n, i = idx - (idx / n) * n;
        S acc = s_zero<S>();
        for (int k = 0; k < n; ++k) acc = acc + V[k * LD + i] * W[j * LD + k];
        outv[c] = scale_by(R(1.5), V[j * LD + i]) - scale_by(R(0.5), acc);
      }
      __syncthreads();
      #pragma unroll
      for (int c = 0; c < NOUT; ++c) {  // compile-time c keeps outv in registers
        const int idx = tid + c * NT;
        if (idx >= nn) break;
        const int j = idx / n, i = idx - (idx / n) * n;
        V[j * LD + i] = outv[c];
      }
      __syncthreads();
    }
  }

  // 1. load C (column j at W[j*LD]) and take its Hermitian part
  for (int idx = tid; idx < nn; idx += NT) {
    const int i = idx / n, j = idx - (idx / n) * n;
    W[j * LD + i] = pol.template load<S>(mat, i, j);
  }
  __syncthreads();
  for (int idx = tid; idx < nn; idx += NT) {
    const int i = idx / n, j = idx - (idx / n) * n;
    if (i < j) {
      const S h = hermitian_avg(W[j * LD + i], W[i * LD + j]);
      W[j * LD + i] = h;
      W[i * LD + j] = conjugate(h);
    } else if (i == j) {
      W[i * LD + i] = drop_imag(W[i * LD + i]);
    }
  }
  __syncthreads();

  // 2. Gershgorin shift s >= -lambda_min(C)
  R shift;
  {
    R v = R(0);
    for (int i = tid; i < n; i += NT) {
      R rad = R(0);
      for (int j = 0; j < n; ++j)
        if (j != i) rad += modulus_fast(W[j * LD + i]);
      R d = re_part(W[i * LD + i]);
      R e = rad - d;
      v = e > v ? e : v;
    }
    // Pi needs only s >= -lambda_min(C)/2: every negative eigenvalue b of B then has
    // |b| <= s, so it and any column one-sided Jacobi mixes with it (same |b|) fall at or
    // below the cut sigma > s.  Half the Gershgorin bound satisfies this and halves the
    // shift's share of the rounding error.  Eigenvalue mode needs B >= 0: full bound.
    shift = block_max(v, red);
    if constexpr (MODE != kEigvals) shift *= R(0.5);
  }
  for (int i = tid; i < n; i += NT) W[i * LD + i] = add_real(W[i * LD + i], shift);
  __syncthreads();
  // Warm start: W = B V_prev, where V_prev holds the eigenvectors of the previous
  // solve of this matrix slot.  B V_prev is nearly column-orthogonal when the
  // matrix moved little, so few sweeps remain.  V accumulates the rotations (eigenvalue and
  // eigenvector solves; projection solves rebuild V from W at the end instead).
  if constexpr (VG) {
    // W <- B V_prev with V_prev read from its slot (column-major); a cold start keeps W = B (= B I)
    const D* vin = pol.template vslot<D>(vstore_raw, mat, (size_t)nn);
    if (cold != 1) {
      if (use_mfma) {
        if constexpr (TPW > 0) {
          const int nt = n / 16, T = nt * nt;
          TileAcc<S> acc[TPW];
#pragma unroll
          for (int q = 0; q < TPW; ++q) {
            const int t = wv + q * NWAVE;
            if (t < T)
              acc[q] = tile_gemm<S>([&](int i, int k) { return W[k * LD + i]; },
                                    [&](int k, int j) { return narrow<S>(vin[(size_t)j * n + k]); }, n,
                                    (t / nt) * 16, (t % nt) * 16, ln);
          }
          __syncthreads();
#pragma unroll
          for (int q = 0; q < TPW; ++q) {
            const int t = wv + q * NWAVE;
            if (t < T)
#pragma unroll
              for (int r = 0; r < 4; ++r)
                W[((t % nt) * 16 + (ln & 15)) * LD + (t / nt) * 16 + mfma_row<R>(ln, r)] = tile_value(acc[q], r);
          }
        }
      } else {
        S outv[NOUT];
        #pragma unroll
        for (int c = 0; c < NOUT; ++c) {  // compile-time c keeps outv in registers
          const int idx = tid + c * NT;
          if (idx >= nn) break;
          const int j = idx / n, i = idx - (idx / n) * n;
          S acc = s_zero<S>();
          for (int k = 0; k < n; ++k) acc = acc + W[k * LD + i] * narrow<S>(vin[(size_t)j * n + k]);
          outv[c] = acc;
        }
        __syncthreads();
        #pragma unroll
        for (int c = 0; c < NOUT; ++c) {  // compile-time c keeps outv in registers
          const int idx = tid + c * NT;
          if (idx >= nn) break;
          const int j = idx / n, i = idx - (idx / n) * n;
          W[j * LD + i] = outv[c];
        }
      }
    }
    __syncthreads();
  } else if constexpr (WARM) {
    const D* vin = pol.template vslot<D>(vstore_raw, mat, (size_t)nn);  // column-major: V(i, j) at [j*n + i]
    if (cold == 1) {
      for (int idx = tid; idx < nn; idx += NT) {
        const int j = idx / n, i = idx - (idx / n) * n;
        V[j * LD + i] = (i == j) ? one_of<S>() : s_zero<S>();
      }
    } else {
      if (cold != 2) {  // (cold == 2 loaded and orthonormalised V above)
        for (int idx = tid; idx < nn; idx += NT) {
          const int j = idx / n, i = idx - (idx / n) * n;
          V[j * LD + i] = narrow<S>(vin[idx]);
        }
      }
      __syncthreads();
      if constexpr (TPW > 0) {
        if (use_mfma) {  // W <- B V on matrix cores
          const int nt = n / 16, T = nt * nt;
          TileAcc<S> acc[TPW];
#pragma unroll
          for (int q = 0; q < TPW; ++q) {
            const int t = wv + q * NWAVE;
            if (t < T)
              acc[q] = tile_gemm<S>([&](int i, int k) { return W[k * LD + i]; },
                                    [&](int k, int j) { return V[j * LD + k]; }, n, (t / nt) * 16, (t % nt) * 16,
                                    ln);
          }
          __syncthreads();
#pragma unroll
          for (int q = 0; q < TPW; ++q) {
            const int t = wv + q * NWAVE;
            if (t < T)
#pragma unroll
              for (int r = 0; r < 4; ++r)
                W[((t % nt) * 16 + (ln & 15)) * LD + (t / nt) * 16 + mfma_row<R>(ln, r)] = tile_value(acc[q], r);
          }
        }
      }
      if (!use_mfma) {
        S outv[NOUT];
        #pragma unroll
        for (int c = 0; c < NOUT; ++c) {  // compile-time c keeps outv in registers
          const int idx = tid + c * NT;
          if (idx >= nn) break;
          const int j = idx / n, i = idx - (idx / n) * n;
          S acc = s_zero<S>();
          for (int k = 0; k < n; ++k) acc = acc + W[k * LD + i] * V[j * LD + k];
          outv[c] = acc;
        }
        __syncthreads();
        #pragma unroll
        for (int c = 0; c < NOUT; ++c) {  // compile-time c keeps outv in registers
          const int idx = tid + c * NT;
          if (idx >= nn) break;
          const int j = idx / n, i = idx - (idx / n) * n;
          W[j * LD + i] = outv[c];
        }
      }
    }
    __syncthreads();
  }

  // Columns whose squared norm falls below (eta ||B||_F)^2, eta = max(n,16) eps, hold only
  // rounding noise: they are left unrotated.  Rotating them never converges (the noise
  // is re-created parallel to the partner column) and their weight in Pi is below
  // eta ||B||_F.
  R floor2;
  {
    R v = R(0);
    for (int idx = tid; idx < nn; idx += NT) {
      const int i = idx / n, j = idx - (idx / n) * n;
      v += abs2(W[j * LD + i]);
    }
    const R eta = R(n > 16 ? n : 16) * eps_of<R>::v;
    floor2 = eta * eta * block_sum_r(v, red);
  }

  // 3. sweeps
  const R tol = R(n > 16 ? n : 16) * eps_of<R>::v;
  int sweep = 0;
  bool converged = false;  // a sweep rotated nothing, or the early stop applied, before the cap
  if constexpr (REG) {
    sweep = rr_sweeps<S, WARM, (NT == 256 ? 8 : 4)>(W, V, LD, max_sweeps, tol, floor2, rr_flags);
    converged = sweep < max_sweeps;
  } else {
    const int np = (n + 1) & ~1;
    const int npair = np / 2;
    const int g = tid / G;   // pair slot
    const int l = tid % G;   // lane within the group
    // A sweep whose largest rotated |gamma| / sqrt(alpha beta) stays below sqrt(tol) / 16 ends the
    // solve: cyclic Jacobi converges quadratically, so the next sweep's inner products would be
    // about tol / 256 and rotate nothing (it would only confirm convergence).  Within clusters of
    // nearly equal eigenvalues the convergence is slower; what is left there mixes eigenvectors of
    // nearly equal eigenvalues, which moves Pi only for clusters at the cut (eigenvalues near 0).
    const R early = dev_sqrt(tol) * R(0.0625);
    for (; sweep < max_sweeps; ++sweep) {
      // squared column norms, recomputed exactly once per sweep and carried through the
      // rotations in between (|w_p'|^2 = |w_p|^2 - t|gamma|, |w_q'|^2 = |w_q|^2 + t|gamma|),
      // so a round reduces only the inner products
      // largest rotated |gamma| / sqrt(alpha beta) of the sweep, kept as a fraction (num / den) so a
      // round needs no division for it
      R rnum = R(0), rden = R(1);
      if (tid == 0) rotated = 0;
      for (int j = tid; j < n; j += NT) {
        R s2 = R(0);
        for (int i = 0; i < n; ++i) s2 += abs2(W[j * LD + i]);
        cn[j] = s2;
      }
      __syncthreads();
      // the slot's pair of round 0, advanced by one (mod np - 1) per round: the circle method
      int p = 0, q = 0;
      if (g < npair) rr_pair(0, g, np, p, q);
      const int kk = np - 1;
      for (int round = 0; round < kk; ++round) {
        if (round > 0 && g < npair) {
          if (g > 0) p = p + 1 == kk ? 0 : p + 1;
          q = q + 1 == kk ? 0 : q + 1;
        }
        const bool live = g < npair && p < n && q < n;
        S a[RPL], b[RPL];
        S gam = s_zero<S>();
  #pragma unroll
        for (int r = 0; r < RPL; ++r) {
          const int i = l + r * G;
          if (live && i < n) {
            a[r] = W[p * LD + i];
            b[r] = W[q * LD + i];
          } else {
            a[r] = s_zero<S>();
            b[r] = s_zero<S>();
          }
          gam = gam + conj_mul(a[r], b[r]);
        }
        gam = group_sum<G>(gam);
        const R alpha = live ? cn[p] : R(0), beta = live ? cn[q] : R(0);
        const R ag = modulus_fast(gam);
        const R small = alpha < beta ? alpha : beta;
        const R gab = dev_sqrt(alpha * beta);
        if (live && small > floor2 && ag > tol * gab && ag > R(0)) {
          if (ag * rden > rnum * gab) {
            rnum = ag;
            rden = gab;
          }
          const R inv_ag = rcp_nr(ag);
          const R zeta = (beta - alpha) * (R(0.5) * inv_ag);
          const R az = dev_abs(zeta);
          const R z2 = R(1) + zeta * zeta;
          R t = rcp_nr(az + z2 * rsqrt_nr(z2));
          if (zeta < R(0)) t = -t;
          const R c = rsqrt_nr(R(1) + t * t);
          const R s = c * t;
          const S ph = conj_phase_inv(gam, inv_ag);  // conj(e)
          if (l == 0) {
            const R da = t * ag;
            cn[p] = alpha - da > R(0) ? alpha - da : R(0);
            cn[q] = beta + da;
          }
  #pragma unroll
          for (int r = 0; r < RPL; ++r) {
            const int i = l + r * G;
            if (i < n) {
              const S bq = mul_phase(ph, b[r]);
              W[p * LD + i] = scale_by(c, a[r]) - scale_by(s, bq);
              W[q * LD + i] = scale_by(s, a[r]) + scale_by(c, bq);
              if constexpr (WARM && !VFW) {
                const S va = V[p * LD + i];
                const S vb = mul_phase(ph, V[q * LD + i]);
                V[p * LD + i] = scale_by(c, va) - scale_by(s, vb);
                V[q * LD + i] = scale_by(s, va) + scale_by(c, vb);
              }
            }
          }
          if (l == 0) rotated = 1;
        }
        __syncthreads();
      }
      const int any = rotated;
      __syncthreads();
      if (!any) {
        converged = true;
        break;
      }
      if (block_max(rnum / rden, red) < early) {
        ++sweep;
        converged = true;
        break;
      }
    }
  }
  // an unconverged solve (stopped by the cap) records cap + 1
  if (tid == 0) pol.record_sweeps(mat, converged ? sweep : max_sweeps + 1);
  if constexpr (WARM && !VFW) {
    D* vout = pol.template vslot<D>(vstore_raw, mat, (size_t)nn);
    for (int idx = tid; idx < nn; idx += NT) {
      const int j = idx / n, i = idx - (idx / n) * n;
      vout[idx] = widen(V[j * LD + i]);
    }
  }
  if constexpr (MODE == kVectors) return;

  // 4. column norms sigma_j = lambda_j(B)
  R noise = R(0);
  for (int j = tid; j < n; j += NT) {
    R s2 = R(0);
    for (int i = 0; i < n; ++i) s2 += abs2(W[j * LD + i]);
    colf[j] = dev_sqrt(s2);
    if (s2 <= floor2) noise = R(1);
  }
  __syncthreads();
  if constexpr (VFW) {
    // The normalised columns of W are an orthonormal eigenbasis of B only at convergence: a block with a
    // noise-floor column or an unconverged solve keeps the identity, so its next solve starts cold.  (The
    // short FP64 refinement of MIXED, cold == 2, is capped on purpose; its vectors are orthonormalised
    // again before every use.)
    const bool ident = block_max(noise, red) > R(0) || (!converged && cold != 2);
    D* vout = pol.template vslot<D>(vstore_raw, mat, (size_t)nn);
    for (int idx = tid; idx < nn; idx += NT) {
      const int j = idx / n, i = idx - (idx / n) * n;
      vout[idx] = ident ? widen(i == j ? one_of<S>() : s_zero<S>()) : widen(scale_by(R(1) / colf[j], W[j * LD + i]));
    }
  }

  if constexpr (MODE == kEigvals) {
    // eigenvalues of C: sigma_j - s, sorted ascending by rank
    for (int j = tid; j < n; j += NT) {
      const R v = colf[j] - shift;
      int rank = 0;
      for (int k = 0; k < n; ++k) {
        const R u = colf[k] - shift;
        rank += (u < v) || (u == v && k < j);
      }
      pol.store_eig(mat, rank, (double)v);
    }
    return;
  } else {
    // 5. rebuild Pi(C) = U U^H with U_j = sqrt((sigma_j - s)/sigma_j^2) w_j over active columns
    if (tid == 0) {
      int k = 0;
      for (int j = 0; j < n; ++j)
        if (colf[j] > shift) active[k++] = j;
      nact_s = k;
    }
    __syncthreads();
    double part = 0.0;
    bool done = false;
    if constexpr (TPW > 0) {
      if (use_mfma) {  // U U^H on matrix cores over all n columns, inactive ones zeroed
        for (int idx = tid; idx < nn; idx += NT) {
          const int j = idx / n, i = idx - (idx / n) * n;
          const R sg = colf[j];
          W[j * LD + i] = sg > shift ? scale_by(dev_sqrt(sg - shift) / sg, W[j * LD + i]) : s_zero<S>();
        }
        __syncthreads();
        const int nt = n / 16, T = nt * nt;
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
          const int t = wv + q * NWAVE;
          if (t < T) {
            const int i0 = (t / nt) * 16, k0 = (t % nt) * 16;
            const TileAcc<S> acc = tile_gemm<S>([&](int i, int j) { return W[j * LD + i]; },
                                                [&](int j, int k) { return conjugate(W[j * LD + k]); }, n, i0, k0,
                                                ln);
#pragma unroll
            for (int r = 0; r < 4; ++r) part += pol.store(mat, i0 + mfma_row<R>(ln, r), k0 + (ln & 15), tile_value(acc, r));
          }
        }
        done = true;
      }
    }
    if (!done) {
      const int nact = nact_s;
      for (int idx = tid; idx < nact * n; idx += NT) {
        const int jj = idx / n, i = idx - (idx / n) * n;
        const int j = active[jj];
        const R sg = colf[j];
        const R f = dev_sqrt((sg - shift)) / sg;
        W[j * LD + i] = scale_by(f, W[j * LD + i]);
      }
      __syncthreads();
      for (int idx = tid; idx < nn; idx += NT) {
        const int i = idx / n, k = idx - (idx / n) * n;
        S acc = s_zero<S>();
        for (int jj = 0; jj < nact; ++jj) {
          const int j = active[jj];
          acc = acc + conj_mul(W[j * LD + k], W[j * LD + i]);  // U(i,j) conj(U(k,j))
        }
        part += pol.store(mat, i, k, acc);
      }
    }
    const double tot = block_sum(part, red_d);
    if (tid == 0) pol.finish(mat, tot);

  }
}

template <typename S, int NMAX, int MODE, bool WARM, int NT, typename Policy, bool REG = false, bool VG = false>
__global__ void __launch_bounds__(NT) jacobi_kernel(Policy pol, int n, int max_sweeps, void* vstore_raw, int cold) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[JacobiLds<S, NMAX, WARM && !VG, NT>::bytes];
  if (!policy_active(pol, blockIdx.x)) return;  // a masked batch instance: the whole workgroup
  jacobi_body<S, NMAX, MODE, WARM, NT, Policy, REG, VG>(pol, n, max_sweeps, vstore_raw, cold, blockIdx.x, smem);
}

// The pair and momentum projections of one iteration in one launch: workgroups below P take the
// (real) pair blocks, the rest the (complex) momentum blocks, both warm-started solves of blocks of
// 33..64 with NT threads, in the real type R (FP64, or FP32 with the FP32 rebuild).  The two sets touch
// disjoint data, and one launch on one stream needs no fork and join between streams.
template <int NT, typename R>
__global__ void __launch_bounds__(NT) fused_projection_kernel(PairPolicy pp, int n, int P, MomentumPolicy mp, int n_op,
                                                              int max_sweeps, void* vpair, void* vmom, int cold) {
  constexpr size_t bp = JacobiLds<R, 64, true, NT>::bytes, bm = JacobiLds<cplx<R>, 64, true, NT>::bytes;
  __shared__ __attribute__((aligned(16))) unsigned char smem[bp > bm ? bp : bm];
  if ((int)blockIdx.x < P)
    jacobi_body<R, 64, kProject, true, NT, PairPolicy>(pp, n, max_sweeps, vpair, cold, blockIdx.x, smem);
  else
    jacobi_body<cplx<R>, 64, kProject, true, NT, MomentumPolicy>(mp, n_op, max_sweeps, vmom, cold,
                                                                  (int)blockIdx.x - P, smem);
}

// vstore == nullptr: cold solve without eigenvector storage.  Otherwise the
// eigenvectors of every matrix slot are read (unless cold) and written back.
// tpb: threads per workgroup (256, 512 or 1024; others fall back to 256).  More
// threads give each column pair more lanes (fewer rows per lane) and put up to
// four wavefronts on each SIMD to hide the latency of a round.
// Batched FP64 projections of 64-blocks read the kept V from its slot: without V in LDS two workgroups of
// the complex solver fit on a CU, which the batches' thousands of blocks use.
template <typename S, int MODE, int NM, bool REG, typename Policy>
constexpr bool v_from_slot() {
  return MODE == kProject && NM == 64 && !REG && std::is_same<typename scalar_traits<S>::real, double>::value &&
         (std::is_same<Policy, BatchedPairPolicy>::value || std::is_same<Policy, BatchedMomentumPolicy>::value);
}

template <typename S, int MODE, int NM, int NT, typename Policy, bool REG = false>
hipError_t launch_one(const Policy& pol, int n, int count, int max_sweeps, hipStream_t st, void* vstore, int cold) {
  if constexpr (v_from_slot<S, MODE, NM, REG, Policy>()) {
    if (vstore && cold != 2) {
      hipLaunchKernelGGL((jacobi_kernel<S, NM, MODE, true, NT, Policy, REG, true>), dim3(count), dim3(NT), 0, st, pol,
                         n, max_sweeps, vstore, cold);
      return hipGetLastError();
    }
  }
  if (vstore)
    hipLaunchKernelGGL((jacobi_kernel<S, NM, MODE, true, NT, Policy, REG>), dim3(count), dim3(NT), 0, st, pol, n,
                       max_sweeps, vstore, cold);
  else
    hipLaunchKernelGGL((jacobi_kernel<S, NM, MODE, false, NT, Policy, REG>), dim3(count), dim3(NT), 0, st, pol, n,
                       max_sweeps, nullptr, 1);
  return hipGetLastError();
}

template <typename S, int MODE, int NM, typename Policy>
hipError_t launch_tpb(const Policy& pol, int n, int count, int max_sweeps, hipStream_t st, void* vstore, int cold,
                      int tpb) {
  if constexpr (NM == 64) {  // register-resident kernels (n = 64 exactly)
    if (tpb == kTpbRegister8 && n == 64)
      return launch_one<S, MODE, 64, 256, Policy, true>(pol, n, count, max_sweeps, st, vstore, cold);
    if (tpb == kTpbRegister4 && n == 64)
      return launch_one<S, MODE, 64, 512, Policy, true>(pol, n, count, max_sweeps, st, vstore, cold);
  }
  if constexpr (NM >= 16 && NM <= 64) {
    if (tpb == 1024) return launch_one<S, MODE, NM, 1024>(pol, n, count, max_sweeps, st, vstore, cold);
    if (tpb == 512) return launch_one<S, MODE, NM, 512>(pol, n, count, max_sweeps, st, vstore, cold);
  }
  return launch_one<S, MODE, NM, 256>(pol, n, count, max_sweeps, st, vstore, cold);
}

template <typename S, int MODE, typename Policy>
hipError_t dispatch(const Policy& pol, int n, int count, int max_sweeps, hipStream_t st, void* vstore = nullptr,
                    int cold = 1, int tpb = 256) {
  if (count <= 0) return hipSuccess;
  const int np = (n + 1) & ~1;
  if (np <= 4) return launch_tpb<S, MODE, 4>(pol, n, count, max_sweeps, st, vstore, cold, tpb);
  if (np <= 8) return launch_tpb<S, MODE, 8>(pol, n, count, max_sweeps, st, vstore, cold, tpb);
  if (np <= 16) return launch_tpb<S, MODE, 16>(pol, n, count, max_sweeps, st, vstore, cold, tpb);
  if (np <= 32) return launch_tpb<S, MODE, 32>(pol, n, count, max_sweeps, st, vstore, cold, tpb);
  if (np <= 64) return launch_tpb<S, MODE, 64>(pol, n, count, max_sweeps, st, vstore, cold, tpb);
  if constexpr (!scalar_traits<S>::is_complex) {
    if (np <= 128 && !vstore) {
      hipLaunchKernelGGL((jacobi_kernel<S, 128, MODE, false, 256, Policy>), dim3(count), dim3(256), 0, st, pol, n,
                         max_sweeps, nullptr, 1);
      return hipGetLastError();
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace

// Precision modes: FP64 solves; FP32 solves; MIXED = FP32 sweeps for the eigenvectors,
// then one FP64 sweep warm-started from them and the FP64 rebuild.
template <typename S32, typename S64, typename Policy>
hipError_t by_precision(const Policy& pol, const Policy& pol_quiet, int n, int count, int precision, int max_sweeps,
                        double* vstore, int cold, int tpb, hipStream_t st) {
  if (precision == VEMB_FP32) return dispatch<S32, kProject>(pol, n, count, max_sweeps, st, vstore, cold, tpb);
  if (precision == VEMB_MIXED && vstore) {
    hipError_t e = dispatch<S32, kVectors>(pol, n, count, max_sweeps, st, vstore, cold, tpb);
    if (e != hipSuccess) return e;
    return dispatch<S64, kProject>(pol_quiet, n, count, 2, st, vstore, 2, tpb);
  }
  return dispatch<S64, kProject>(pol, n, count, max_sweeps, st, vstore, cold, tpb);
}

hipError_t launch_pair_projection(const double* rho, double* Lam, double* rho_t, double* feas, int n, int P,
                                  double mu, int precision, int max_sweeps, int* sweeps, double* vstore, int cold,
                                  int tpb, hipStream_t st) {
  PairPolicy pol{rho, Lam, rho_t, feas, sweeps, n, mu};
  PairPolicy quiet{rho, Lam, rho_t, feas, nullptr, n, mu};
  return by_precision<float, double>(pol, quiet, n, P, precision, max_sweeps, vstore, cold, tpb, st);
}

hipError_t launch_momentum_projection(double* Xh, int n_op, int K, int precision, int max_sweeps, int* sweeps,
                                      double* vstore, int cold, int tpb, hipStream_t st) {
  MomentumPolicy pol{Xh, sweeps, n_op};
  MomentumPolicy quiet{Xh, nullptr, n_op};
  return by_precision<cplx<float>, cplx<double>>(pol, quiet, n_op, K, precision, max_sweeps, vstore, cold, tpb, st);
}

hipError_t launch_projections_fused(const double* rho, double* Lam, double* rho_t, double* feas, int n, int P,
                                   double mu, double* Xh, int n_op, int K, int max_sweeps, int* sweeps, double* vpair,
                                   double* vmom, int cold, hipStream_t st, int precision) {
  if (!fused_projection_fits(n, n_op) || !vpair || !vmom || P <= 0 || K <= 0) return hipErrorInvalidValue;
  PairPolicy pp{rho, Lam, rho_t, feas, sweeps, n, mu};
  MomentumPolicy mp{Xh, sweeps + P, n_op};
  if (precision == VEMB_FP64)
    hipLaunchKernelGGL((fused_projection_kernel<kFusedThreads, double>), dim3(P + K), dim3(kFusedThreads), 0, st, pp, n,
                       P, mp, n_op, max_sweeps, vpair, vmom, cold);
  else
    hipLaunchKernelGGL((fused_projection_kernel<kFusedThreads, float>), dim3(P + K), dim3(kFusedThreads), 0, st, pp, n,
                       P, mp, n_op, max_sweeps, vpair, vmom, cold);
  return hipGetLastError();
}

hipError_t launch_psd_batched(const double* in, double* out, int n, int batch, bool is_complex, int precision,
                              int max_sweeps, int* sweeps, double* vstore, int tpb, hipStream_t st, int cold) {
  if (!vstore) cold = 1;
  if (is_complex) {
    ArrayPolicy<true> pol{in, out, nullptr, nullptr, sweeps, n};
    ArrayPolicy<true> quiet{in, out, nullptr, nullptr, nullptr, n};
    return by_precision<cplx<float>, cplx<double>>(pol, quiet, n, batch, precision, max_sweeps, vstore, cold, tpb,
                                                   st);
  }
  ArrayPolicy<false> pol{in, out, nullptr, nullptr, sweeps, n};
  ArrayPolicy<false> quiet{in, out, nullptr, nullptr, nullptr, n};
  return by_precision<float, double>(pol, quiet, n, batch, precision, max_sweeps, vstore, cold, tpb, st);
}

hipError_t launch_projection_group_lds(int kind, int n, int count, int precision, int max_sweeps, int cold, int tpb,
                                       const int2* item, const void* ptrs, void* vstore_any, hipStream_t st) {
  double* vs = static_cast<double*>(vstore_any);
  if (kind == 0) {
    BatchedPairPolicy pol{item, static_cast<const PairPtrs*>(ptrs), n, 1};
    BatchedPairPolicy quiet{item, static_cast<const PairPtrs*>(ptrs), n, 0};
    return by_precision<float, double>(pol, quiet, n, count, precision, max_sweeps, vs, cold, tpb, st);
  }
  BatchedMomentumPolicy pol{item, static_cast<const MomPtrs*>(ptrs), n, 1};
  BatchedMomentumPolicy quiet{item, static_cast<const MomPtrs*>(ptrs), n, 0};
  return by_precision<cplx<float>, cplx<double>>(pol, quiet, n, count, precision, max_sweeps, vs, cold, tpb, st);
}

hipError_t launch_eigvalsh_batched(const double* in, double* w, int n, int batch, bool is_complex, int max_sweeps,
                                   int* sweeps, hipStream_t st) {
  if (is_complex) {
    ArrayPolicy<true> pol{in, nullptr, w, nullptr, sweeps, n};
    return dispatch<cplx<double>, kEigvals>(pol, n, batch, max_sweeps, st);
  }
  ArrayPolicy<false> pol{in, nullptr, w, nullptr, sweeps, n};
  return dispatch<double, kEigvals>(pol, n, batch, max_sweeps, st);
}

hipError_t launch_lambda_min(const double* K, double* lmin, int n, int count, int max_sweeps, int* sweeps,
                             hipStream_t st, int tpb, double* vstore, int cold) {
  ArrayPolicy<false> pol{K, nullptr, nullptr, lmin, sweeps, n};
  return dispatch<double, kEigvals>(pol, n, count, max_sweeps, st, vstore, vstore ? cold : 1, tpb);
}

}  // namespace vemb
