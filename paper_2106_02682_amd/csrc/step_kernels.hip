// Per-iteration kernels of Algorithm 6 other than the eigensolves:
//   pair_update     steps 1-2 (+ the G_0d part of step 6) for every offset d
//   cluster_update  steps 4-5 (rho_0 and the consistency multipliers) + G_00 of step 6
//   dft_mfma<true>  step 7  (momentum blocks of X', a product with the twiddle matrix on matrix cores)
//   dft_mfma<false> step 9  (first block row of X from the projected blocks, likewise)
//   bound_build     matrices whose smallest eigenvalues give the Lagrangian bound
//
// Index conventions: a pair index is (x, y) -> x*m + y (cluster 0 first).
// Matrix units O_(a,b) = E_ab give, for the complete operator collection,
//   R(X)_(x,y),(x',y') = X_(x',x),(y,y')   (pair correction of eq. effHam)
//   G_0d(rho)_(a,b),(c,e) = rho_(a,e),(b,c) (realignment)
//   C_0(X)_(b,e) = sum_a X_(a,b),(a,e);  G_00(rho0)_(a,b),(c,e) = delta_ac rho0_(e,b).
// The single-site Pauli collection uses signed-permutation tables instead.  Fermionic problems
// (appendix on fermions) multiply the pair entries by the Jordan-Wigner parity sign jw_sign.
#include "kernels.h"
#include "mfma_tile.h"

namespace vemb {
namespace {

constexpr int kBlock = 256;
// lattice DFT: 16 x 16 output tiles per wavefront strip, and the rows a workgroup covers
constexpr int kDftRowTiles = 4, kDftRows = 16 * kDftRowTiles;

// sum over the generic (signed permutation) operators:
// R(X)_(x,y),(x',y') = (1/m) sum_ab X_ab [x = perm_a(x')] sgn_a(x') [y' = perm_b(y)] sgn_b(y)
__device__ double rx_generic(const double* X, const OpTables& T, int m, int x, int y, int xp, int yp) {
  double acc = 0.0;
  for (int a = 0; a < T.n_op; ++a) {
    if (T.perm[a][xp] != x) continue;
    const double sa = T.sign[a][xp];
    for (int b = 0; b < T.n_op; ++b) {
      if (T.perm[b][y] != yp) continue;
      acc += X[a * T.n_op + b] * sa * T.sign[b][y];
    }
  }
  return acc / m;
}

__device__ inline double rx_value(const StepArgs& A, const double* Xd, int x, int y, int xp, int yp) {
  const int m = A.m;
  if (A.opset == VEMB_OPSET_COMPLETE) {
    const double v = Xd[(size_t)(xp * m + x) * A.n_op + (y * m + yp)];
    return A.fermionic ? jw_sign(xp, y, yp) * v : v;
  }
  return rx_generic(Xd, *A.ops, m, x, y, xp, yp);
}

// R_d(i, j) of eq. rhoijUpdate's right-hand side:
// mu rho~ + (nu rho0 - L1) x I + I x (nu rho0 - L2) + Lam - H'_d,  H'_d = H_d - RX - RX^T.
__device__ double rhs_value(const StepArgs& A, int pd, int i, int j) {
  const int m = A.m, n = A.n;
  const int x = i / m, y = i % m, xp = j / m, yp = j % m;
  const size_t o = (size_t)pd * n * n + (size_t)i * n + j;
  const double* Xd = A.X + (size_t)(pd + 1) * A.n_op * A.n_op;
  double v = A.mu * A.rho_t[o] + A.Lam[o];
  const int h = A.hd_index[pd];
  if (h >= 0) v -= A.Hd[(size_t)h * n * n + (size_t)i * n + j];
  v += rx_value(A, Xd, x, y, xp, yp) + rx_value(A, Xd, xp, yp, x, y);
  const size_t mo = (size_t)pd * m * m;
  if (y == yp) v += A.nu * A.rho0[x * m + xp] - A.Lam1[mo + x * m + xp];
  if (x == xp) v += A.nu * A.rho0[y * m + yp] - A.Lam2[mo + y * m + yp];
  return v;
}

// ---------------------------------------------------------------------------
// Steps 1-2 and X'_0d.  One workgroup per offset d.
// ---------------------------------------------------------------------------
// R is formed block by block: block (x, x') is the m x m submatrix of rows x m + y and columns
// x' m + y' (y, y' < m).  Thread t owns the entry (y, y') = ((t mod m^2) / m, t mod m) of every block
// it visits (the thread count is a multiple of m^2), so
//   * the pair corrections of eq. effHam read rows x' m + x and x m + x' of X_0d whole within a
//     wavefront (entries y m + y' and y' m + y), and the blocks of rho~, Lambda, H_0d as row segments;
//   * Tr_1 R (the sum of the diagonal blocks) accumulates in the thread's registers, and Tr_2 R (the
//     traces of the blocks) from the diagonal entries, without strided gathers.
// Blocks up to kStageN keep R in LDS; larger ones store R in the rho buffer of the pair between the two
// passes (a coalesced write and read of n^2 words) and overwrite it with rho.
constexpr int kStageN = 64;
// Threads of a pair-update workgroup: four entries of a 64 x 64 block per thread keep enough loads
// in flight (the step is bound by memory latency, one workgroup per pair).
constexpr int kPairThreads = 1024;
static_assert(kPairThreads % (kMaxM * kMaxM) == 0, "a thread keeps one (y, y') entry of every block");

__device__ void pair_update_body(const StepArgs& A, int bx) {
  constexpr int NT = kPairThreads;
  const int pd = bx;  // offset d = pd + 1
  const int m = A.m, n = A.n, mm = m * m, nn = n * n;
  const int tid = threadIdx.x;
  __shared__ double T2[kMaxM * kMaxM];  // Tr_2 R
  __shared__ double T1[kMaxM * kMaxM];  // Tr_1 R
  __shared__ double Rs[kStageN * kStageN];  // R (staged blocks) or the blocks' diagonals (larger ones)
  __shared__ double red[NT];
  __shared__ double trR_s;
  const bool staged = n <= kStageN;
  double* rho = A.rho + (size_t)pd * nn;
  // pass 1: every entry of R, block by block; Tr_1 R in registers, the blocks' diagonals in LDS
  // (forming several entries per step with all their loads first measured slower: the extra registers
  // cost the second workgroup per CU)
  const int r = tid % mm, y = r / m, yp = r % m;
  double t1 = 0.0;
  for (int e = tid; e < nn; e += NT) {
    const int blk = e / mm, x = blk / m, xp = blk % m;
    const int i = x * m + y, j = xp * m + yp;
    const double v = rhs_value(A, pd, i, j);
    if (staged)
      Rs[i * n + j] = v;
    else
      rho[(size_t)i * n + j] = v;  // R, overwritten by rho in pass 2
    if (x == xp) t1 += v;
    if (y == yp && !staged) Rs[blk * m + y] = v;  // m^2 blocks x m diagonal entries <= kStageN^2 words
  }
  red[tid] = t1;
  __syncthreads();
  for (int e = tid; e < mm; e += NT) {
    double acc = 0.0;
    for (int q = e; q < NT; q += mm) acc += red[q];  // the threads that own entry e of the blocks
    T1[e] = acc;
  }
  for (int e = tid; e < mm; e += NT) {  // Tr_2 R (x, x') = the trace of block (x, x')
    const int x = e / m, xp = e % m;
    double acc = 0.0;
    for (int k = 0; k < m; ++k) acc += staged ? Rs[(x * m + k) * n + xp * m + k] : Rs[e * m + k];
    T2[e] = acc;
  }
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int u = 0; u < m; ++u) t += T2[u * m + u];
    trR_s = t;
  }
  __threadfence_block();  // R stored in rho (larger blocks) is read back by other threads below
  __syncthreads();
  const double trR = trR_s;
  const double a = A.a, bm = A.b / m, cm2 = A.c / ((double)m * m) * trR;

  // pass 2, row-major: rho = a R + (b/m)(Tr_2 R x I + I x Tr_1 R) + (c/m^2) Tr R I, and Tr(H_0d rho)
  // (H_0d is symmetric: the real case)
  const int h = A.hd_index[pd];
  double epart = 0.0;
  for (int idx = tid; idx < nn; idx += NT) {
    const int i = idx / n, j = idx % n;
    const int x = i / m, y2 = i % m, xp = j / m, yp2 = j % m;
    double v = a * (staged ? Rs[idx] : rho[idx]);
    double corr = 0.0;
    if (y2 == yp2) corr += T2[x * m + xp];
    if (x == xp) corr += T1[y2 * m + yp2];
    v += bm * corr;
    if (i == j) v += cm2;
    rho[idx] = v;
    if (h >= 0) epart += A.Hd[(size_t)h * nn + idx] * v;
  }
  // A_1 rho = (a + b) Tr_2 R + ((b + c)/m) Tr R I ;  A_2 rho likewise with Tr_1 R
  const double ab = A.a + A.b, bc = (A.b + A.c) / m * trR;
  for (int e = tid; e < mm; e += NT) {
    const int u = e / m, w = e % m;
    A.tr2[(size_t)pd * mm + e] = ab * T2[e] + (u == w ? bc : 0.0);
    A.tr1[(size_t)pd * mm + e] = ab * T1[e] + (u == w ? bc : 0.0);
  }
  __syncthreads();  // red is reused for the energy
  red[tid] = epart;
  __syncthreads();
  for (int s2 = NT / 2; s2 > 0; s2 >>= 1) {
    if (tid < s2) red[tid] += red[tid + s2];
    __syncthreads();
  }
  if (tid == 0) A.e_pair[pd] = red[0];
}

// X'_0d = X_0d + sign eps G_0d(rho_0d) for d = 1..M-1, one thread per entry.
__device__ void pair_xstep_body(const StepArgs& A, int bx, int by) {
  const int pd = by;
  const int k = A.n_op, m = A.m, n = A.n;
  const int e = bx * kBlock + threadIdx.x;
  if (e >= k * k) return;
  const size_t xo = (size_t)(pd + 1) * k * k + e;
  const double* rho = A.rho + (size_t)pd * n * n;
  double g;
  if (A.opset == VEMB_OPSET_COMPLETE) {
    const int al = e / k, be = e % k;
    const int aa = al / m, bb = al % m, cc = be / m, ee = be % m;
    g = rho[(size_t)(aa * m + ee) * n + (bb * m + cc)];
    if (A.fermionic) g *= jw_sign(aa, cc, ee);
  } else {
    // G_ab = (1/m) sum_{x', y} sgn_a(x') sgn_b(y) rho_(x', perm_b(y)),(perm_a(x'), y)
    const OpTables& T = *A.ops;
    const int al = e / k, be = e % k;
    double acc = 0.0;
    for (int xp = 0; xp < m; ++xp)
      for (int y = 0; y < m; ++y)
        acc += T.sign[al][xp] * T.sign[be][y] *
               rho[(size_t)(xp * m + T.perm[be][y]) * n + (T.perm[al][xp] * m + y)];
    g = acc / m;
  }
  A.Xp[xo] = A.X[xo] + A.sign * A.eps * g;
}

// ---------------------------------------------------------------------------
// Steps 4-5 and X'_00.  A single workgroup.
// ---------------------------------------------------------------------------
__device__ double c0_value(const StepArgs& A, int b, int e) {
  const int m = A.m, k = A.n_op;
  if (A.opset == VEMB_OPSET_COMPLETE) {
    double acc = 0.0;
    for (int a = 0; a < m; ++a) acc += A.X[(size_t)(a * m + b) * k + (a * m + e)];
    return acc;
  }
  // sum_ab X_ab O_a^T O_b:  (O_a^T O_b)(u, w) = (1/m) sum_v [u = perm_a(v)][w = perm_b(v)] sgn_a(v) sgn_b(v)
  const OpTables& T = *A.ops;
  double acc = 0.0;
  for (int v = 0; v < m; ++v)
    for (int al = 0; al < k; ++al) {
      if (T.perm[al][v] != b) continue;
      for (int be = 0; be < k; ++be) {
        if (T.perm[be][v] != e) continue;
        acc += A.X[al * k + be] * T.sign[al][v] * T.sign[be][v];
      }
    }
  return acc / m;
}

constexpr int kClusterBlock = 1024;

__device__ void cluster_update_body(const StepArgs& A) {
  const int m = A.m, mm = m * m, P = A.P, k = A.n_op;
  const int tid = threadIdx.x;
  __shared__ double r0[kMaxM * kMaxM];
  __shared__ double red[kClusterBlock];
  __shared__ double z_s;
  // rho'_0 = [sum_d (nu A_1 rho_d + Lambda1_d) - H'_0] / (nu (M-1)); the sum over d
  // is split over kSplit lanes of one wavefront per entry, then reduced by shuffles
  {
    constexpr int kSplit = 16;
    for (int base = 0; base < mm; base += kClusterBlock / kSplit) {
      const int e = base + tid / kSplit, part = tid % kSplit;
      double acc = 0.0;
      if (e < mm)
        for (int d = part; d < P; d += kSplit) acc += A.nu * A.tr2[(size_t)d * mm + e] + A.Lam1[(size_t)d * mm + e];
#pragma unroll
      for (int off = kSplit / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
      if (e < mm && part == 0) {
        const double h0p = A.H0[e] - c0_value(A, e / m, e % m);
        r0[e] = (acc - h0p) / (A.nu * (A.M - 1));
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int u = 0; u < m; ++u) t += r0[u * m + u];
    z_s = (1.0 - t) / m;
  }
  __syncthreads();
  for (int e = tid; e < mm; e += kClusterBlock) {
    if (e / m == e % m) r0[e] += z_s;
  }
  __syncthreads();
  double part = 0.0, epart = 0.0;
  for (int e = tid; e < mm; e += kClusterBlock) {
    A.rho0[e] = r0[e];
    epart += A.H0[(e % m) * m + e / m] * r0[e];
  }
  // multipliers with the new rho_0, and the consistency residuals of eq. feasErr
  for (int idx = tid; idx < P * mm; idx += kClusterBlock) {
    const int e = idx % mm;
    const double d1 = A.tr2[idx] - r0[e];
    const double d2 = A.tr1[idx] - r0[e];
    A.Lam1[idx] += A.nu * d1;
    A.Lam2[idx] += A.nu * d2;
    part += d1 * d1 + d2 * d2;
  }
  // X'_00 = X_00 + sign eps G_00(rho_0)
  for (int e = tid; e < k * k; e += kClusterBlock) {
    const int al = e / k, be = e % k;
    double g;
    if (A.opset == VEMB_OPSET_COMPLETE) {
      const int aa = al / m, bb = al % m, cc = be / m, ee = be % m;
      g = (aa == cc) ? r0[ee * m + bb] : 0.0;
    } else {
      // Tr(O_a^T O_b rho0) = (1/m) sum_v sgn_a(v) sgn_b(v) rho0(perm_b(v), perm_a(v))
      const OpTables& T = *A.ops;
      double acc = 0.0;
      for (int v = 0; v < m; ++v) acc += T.sign[al][v] * T.sign[be][v] * r0[T.perm[be][v] * m + T.perm[al][v]];
      g = acc / m;
    }
    A.Xp[e] = A.X[e] + A.sign * A.eps * g;
  }
  red[tid] = part;
  __syncthreads();
  for (int s = kClusterBlock / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double cons = red[0];
  __syncthreads();
  red[tid] = epart;
  __syncthreads();
  for (int s = kClusterBlock / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) {
    A.scal[0] = red[0];
    A.scal[1] = cons;
  }
}

// Steps 7 and 9 as real products on matrix cores.  Forward: C = T X' with rows r = 2k + p of T(r, d) = part p of tw[k][d]
// (p = 0 real, 1 imaginary), C(r, e) -> part p of Xh_k(e).  Inverse: X(d, e) = sum_r U(d, r) Y(r, e)
// with U(d, 2k + p) = w_k (part p of tw[k][d]) and Y(2k + p, e) = part p of Y_k(e), which is
// w_k Re(conj(tw[k][d]) Y_k(e)) summed over k.  One wavefront per 16 x 16 output tile (four per
// workgroup along e, all on the same 16 rows), v_mfma_f64_16x16x4_f64; the 16 x 32 twiddle slice of each
// 32-deep reduction chunk is staged once per workgroup in LDS, read along the table's contiguous axis
// (forward: (reduction index, part) of one momentum's row pair; inverse: (row, part) of one momentum),
// instead of being gathered by each wavefront; rows, columns and the reduction are padded with zeros;
// each wavefront issues eight reduction steps of X' (Y) loads before their products.
constexpr int kDftTilePitch = 36;  // staged row pitch: the four reduction lanes of a row land in distinct banks
template <bool FWD>
__device__ void dft_tile_body(const StepArgs& A, int bx, int by) {
  __shared__ double At[16 * kDftTilePitch];
  const int E = A.n_op * A.n_op;
  const int R = FWD ? 2 * A.Ku : A.M;   // output rows
  const int Kr = FWD ? A.M : 2 * A.Ku;  // reduction length
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int i16 = l & 15, kk = l >> 4;
  const int row0 = by * 16, col0 = (bx * 4 + w) * 16;
  const bool live = col0 < E;  // wavefronts past the last column still stage and wait
  const int e = col0 + i16;    // operand column supplied by this lane
  mf_d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < Kr; k0 += 32) {
    for (int x = tid; x < 16 * 32; x += kBlock) {
      int rr, qq;
      if constexpr (FWD) {
        rr = 2 * (x >> 6) + (x & 1);
        qq = (x & 63) >> 1;
      } else {
        qq = 2 * (x >> 5) + (x & 1);
        rr = (x & 31) >> 1;
      }
      const int r = row0 + rr, q = k0 + qq;
      double a = 0.0;
      if (r < R && q < Kr)
        a = FWD ? A.tw[2 * ((size_t)(r >> 1) * A.M + q) + (r & 1)]
                : A.wk[q >> 1] * A.tw[2 * ((size_t)(q >> 1) * A.M + r) + (q & 1)];
      At[rr * kDftTilePitch + qq] = a;
    }
    __syncthreads();
    if (live) {
      double bv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = k0 + 4 * u + kk;  // reduction index supplied by this lane
        double b = 0.0;
        if (q < Kr && e < E) b = FWD ? A.Xp[(size_t)q * E + e] : A.Xh[2 * ((size_t)(q >> 1) * E + e) + (q & 1)];
        bv[u] = b;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = mfma_k4(At[i16 * kDftTilePitch + 4 * u + kk], bv[u], acc);
    }
    __syncthreads();
  }
  if (!live) return;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int orow = row0 + mfma_row<double>(l, g), ocol = col0 + i16;
    if (orow < R && ocol < E) {
      if constexpr (FWD)
        A.Xh[2 * ((size_t)(orow >> 1) * E + ocol) + (orow & 1)] = acc[g];
      else
        A.X[(size_t)orow * E + ocol] = acc[g];
    }
  }
}

// The same products over row strips, for launches large enough to fill the chip with kDftRows-row
// workgroups (dft_strips): a workgroup covers kDftRows x 64 outputs: per 16-deep
// reduction chunk the kDftRows x 16 twiddle slice is staged once in LDS with contiguous reads (it is shared
// by the four wavefronts), and each wavefront takes a 16-column strip of kDftRowTiles 16 x 16 tiles, so
// every X' (Y) element it loads feeds kDftRows output rows; v_mfma_f64_16x16x4_f64; rows, columns and the
// reduction are padded with zeros.
template <bool FWD>
__device__ void dft_strip_body(const StepArgs& A, int bx, int by) {
  __shared__ double As[kDftRows][16 + 1];
  const int E = A.n_op * A.n_op;
  const int R = FWD ? 2 * A.Ku : A.M;   // output rows
  const int Kr = FWD ? A.M : 2 * A.Ku;  // reduction length
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int i16 = l & 15, kk = l >> 4;
  const int row0 = by * kDftRows, col0 = (bx * 4 + w) * 16;
  const bool live = col0 < E;  // wavefronts past the last column still stage and wait
  const int e = col0 + i16;    // operand column supplied by this lane
  const bool eok = e < E;
  mf_d4 acc[kDftRowTiles];
#pragma unroll
  for (int t = 0; t < kDftRowTiles; ++t) acc[t] = mf_d4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < Kr; k0 += 16) {
    // twiddle slice rows row0.., reduction indices k0..k0+15, read along the table's contiguous axis:
    // forward (q, part) of one momentum pair of rows, inverse (row, part) of one momentum
    for (int x = tid; x < kDftRows * 16; x += kBlock) {
      int rr, qq;
      if constexpr (FWD) {
        rr = 2 * (x >> 5) + (x & 1);
        qq = (x & 31) >> 1;
      } else {
        qq = 2 * (x >> 7) + (x & 1);
        rr = (x & 127) >> 1;
      }
      const int r = row0 + rr, q = k0 + qq;
      double a = 0.0;
      if (r < R && q < Kr)
        a = FWD ? A.tw[2 * ((size_t)(r >> 1) * A.M + q) + (r & 1)]
                : A.wk[q >> 1] * A.tw[2 * ((size_t)(q >> 1) * A.M + r) + (q & 1)];
      As[rr][qq] = a;
    }
    __syncthreads();
    if (live) {
      double bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = k0 + 4 * u + kk;  // reduction index supplied by this lane
        double b = 0.0;
        if (q < Kr && eok) b = FWD ? A.Xp[(size_t)q * E + e] : A.Xh[2 * ((size_t)(q >> 1) * E + e) + (q & 1)];
        bv[u] = b;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int t = 0; t < kDftRowTiles; ++t) acc[t] = mfma_k4(As[t * 16 + i16][4 * u + kk], bv[u], acc[t]);
    }
    __syncthreads();
  }
  if (!live) return;
#pragma unroll
  for (int t = 0; t < kDftRowTiles; ++t)
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int orow = row0 + t * 16 + mfma_row<double>(l, g), ocol = col0 + i16;
      if (orow < R && ocol < E) {
        if constexpr (FWD)
          A.Xh[2 * ((size_t)(orow >> 1) * E + ocol) + (orow & 1)] = acc[t][g];
        else
          A.X[(size_t)orow * E + ocol] = acc[t][g];
      }
    }
}

// The inverse takes the row strips where they still give every CU a workgroup (measured on the batched
// sweep: 1.20 -> 0.68 ms per launch); the forward stays on 16-row tiles, which its twiddle gathers favour.
__host__ __device__ inline bool dft_strips(bool fwd, int E, int M) {
  return !fwd && ((E + 63) / 64) * ((M + kDftRows - 1) / kDftRows) >= 256;
}

template <bool FWD>
__device__ void dft_mfma_body(const StepArgs& A, int bx, int by) {
  if constexpr (!FWD) {
    if (dft_strips(false, A.n_op * A.n_op, A.M)) {
      dft_strip_body<false>(A, bx, by);
      return;
    }
  }
  dft_tile_body<FWD>(A, bx, by);
}

template <bool FWD>
__global__ void __launch_bounds__(kBlock) dft_mfma_kernel(StepArgs A) {
  dft_mfma_body<FWD>(A, blockIdx.x, blockIdx.y);
}

// Single-instance kernels and batched kernels.  A batched launch covers every
// instance of a batch: work[blockIdx.x] names the instance and its local block.
__global__ void __launch_bounds__(kPairThreads) pair_update_kernel(StepArgs A) { pair_update_body(A, blockIdx.x); }
__global__ void __launch_bounds__(kBlock) pair_xstep_kernel(StepArgs A) { pair_xstep_body(A, blockIdx.x, blockIdx.y); }
__global__ void __launch_bounds__(kClusterBlock) cluster_update_kernel(StepArgs A) { cluster_update_body(A); }

// A masked instance (args[i].active == 0) keeps its state: its workgroups return at once.
__global__ void __launch_bounds__(kPairThreads) pair_update_batched(const StepArgs* args, const WorkItem* work) {
  const WorkItem w = work[blockIdx.x];
  if (!args[w.inst].active) return;
  pair_update_body(args[w.inst], w.bx);
}
__global__ void __launch_bounds__(kBlock) pair_xstep_batched(const StepArgs* args, const WorkItem* work) {
  const WorkItem w = work[blockIdx.x];
  if (!args[w.inst].active) return;
  pair_xstep_body(args[w.inst], w.bx, w.by);
}
__global__ void __launch_bounds__(kClusterBlock) cluster_update_batched(const StepArgs* args) {
  if (!args[blockIdx.x].active) return;
  cluster_update_body(args[blockIdx.x]);
}
__global__ void __launch_bounds__(kBlock) dft_forward_batched(const StepArgs* args, const WorkItem* work) {
  const WorkItem w = work[blockIdx.x];
  if (!args[w.inst].active) return;
  dft_mfma_body<true>(args[w.inst], w.bx, w.by);
}
__global__ void __launch_bounds__(kBlock) dft_inverse_batched(const StepArgs* args, const WorkItem* work) {
  const WorkItem w = work[blockIdx.x];
  if (!args[w.inst].active) return;
  dft_mfma_body<false>(args[w.inst], w.bx, w.by);
}

// ---------------------------------------------------------------------------
// Bound matrices: K_d = H'_d + sym(L1_d) x I + I x sym(L2_d) (P of them) and
// K_0 = H'_0 - 1/2 sum_d (sym(L1_d) + sym(L2_d)) stored after them.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) bound_pair_kernel(StepArgs A) {
  const int pd = blockIdx.y;
  const int m = A.m, n = A.n;
  const int idx = blockIdx.x * kBlock + threadIdx.x;
  if (idx >= n * n) return;
  const int i = idx / n, j = idx % n;
  const int x = i / m, y = i % m, xp = j / m, yp = j % m;
  const double* Xd = A.X + (size_t)(pd + 1) * A.n_op * A.n_op;
  double v = -(rx_value(A, Xd, x, y, xp, yp) + rx_value(A, Xd, xp, yp, x, y));
  const int h = A.hd_index[pd];
  if (h >= 0) v += A.Hd[(size_t)h * n * n + idx];
  const size_t mo = (size_t)pd * m * m;
  if (y == yp) v += 0.5 * (A.Lam1[mo + x * m + xp] + A.Lam1[mo + xp * m + x]);
  if (x == xp) v += 0.5 * (A.Lam2[mo + y * m + yp] + A.Lam2[mo + yp * m + y]);
  A.Kbuf[(size_t)pd * n * n + idx] = v;
}

__global__ void __launch_bounds__(kBlock) bound_cluster_kernel(StepArgs A) {
  const int m = A.m, mm = m * m;
  double* K0 = A.Kbuf + (size_t)A.P * A.n * A.n;
  for (int e = threadIdx.x; e < mm; e += kBlock) {
    const int u = e / m, w = e % m;
    double acc = 0.0;
    for (int d = 0; d < A.P; ++d) {
      const size_t o = (size_t)d * mm;
      acc += 0.5 * (A.Lam1[o + e] + A.Lam1[o + w * m + u]) + 0.5 * (A.Lam2[o + e] + A.Lam2[o + w * m + u]);
    }
    K0[e] = A.H0[e] - c0_value(A, u, w) - 0.5 * acc;
  }
}

}  // namespace

hipError_t launch_pair_update(const StepArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(pair_update_kernel, dim3(a.P), dim3(kPairThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_pair_xstep(const StepArgs& a, hipStream_t st) {
  const int E = a.n_op * a.n_op;
  hipLaunchKernelGGL(pair_xstep_kernel, dim3((E + kBlock - 1) / kBlock, a.P), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_cluster_update(const StepArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(cluster_update_kernel, dim3(1), dim3(kClusterBlock), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_dft_forward(const StepArgs& a, hipStream_t st) {
  const int E = a.n_op * a.n_op;
  hipLaunchKernelGGL(dft_mfma_kernel<true>, dim3((E + 63) / 64, (2 * a.Ku + 15) / 16), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_dft_inverse(const StepArgs& a, hipStream_t st) {
  const int E = a.n_op * a.n_op;
  const int rows = dft_strips(false, E, a.M) ? kDftRows : 16;
  hipLaunchKernelGGL(dft_mfma_kernel<false>, dim3((E + 63) / 64, (a.M + rows - 1) / rows), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

void local_grids(const StepArgs& a, int grid[5][2]) {
  const int E = a.n_op * a.n_op;
  const int ebx = (E + kBlock - 1) / kBlock;
  grid[0][0] = a.P;  // pair update
  grid[0][1] = 1;
  grid[1][0] = ebx;  // X step
  grid[1][1] = a.P;
  grid[2][0] = 1;  // cluster update
  grid[2][1] = 1;
  grid[3][0] = (E + 63) / 64;  // forward DFT: 16 x 64 output tiles of (2 K_u) x E
  grid[3][1] = (2 * a.Ku + 15) / 16;
  const int inv_rows = dft_strips(false, E, a.M) ? kDftRows : 16;
  grid[4][0] = (E + 63) / 64;  // inverse DFT: inv_rows x 64 output tiles of M x E
  grid[4][1] = (a.M + inv_rows - 1) / inv_rows;
}

hipError_t launch_step_batched(int which, const StepArgs* args, const WorkItem* work, int nwork, hipStream_t st) {
  if (nwork <= 0) return hipSuccess;
  switch (which) {
    case 0:
      hipLaunchKernelGGL(pair_update_batched, dim3(nwork), dim3(kPairThreads), 0, st, args, work);
      break;
    case 1:
      hipLaunchKernelGGL(pair_xstep_batched, dim3(nwork), dim3(kBlock), 0, st, args, work);
      break;
    case 2:
      hipLaunchKernelGGL(cluster_update_batched, dim3(nwork), dim3(kClusterBlock), 0, st, args);
      break;
    case 3:
      hipLaunchKernelGGL(dft_forward_batched, dim3(nwork), dim3(kBlock), 0, st, args, work);
      break;
    case 4:
      hipLaunchKernelGGL(dft_inverse_batched, dim3(nwork), dim3(kBlock), 0, st, args, work);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_bound_build(const StepArgs& a, hipStream_t st) {
  const int nn = a.n * a.n;
  hipLaunchKernelGGL(bound_pair_kernel, dim3((nn + kBlock - 1) / kBlock, a.P), dim3(kBlock), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(bound_cluster_kernel, dim3(1), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

}  // namespace vemb
