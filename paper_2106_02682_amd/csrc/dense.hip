// Algorithm 5 without translation invariance (Section 3.2): one marginal per
// cluster, one per unordered cluster pair i < j, and a dense (M n_op) x (M n_op)
// dual X.  The per-pair work is that of Algorithm 6 with the pair's own X block
// X_ij (row stride K = M n_op) and the two clusters' marginals; the cluster
// update gathers the pairs that contain the cluster; X' is built block by block
// (G_00(rho_i) on the diagonal, G_0d(rho_ij) and its transpose off it) and
// projected as one dense matrix.  Cluster Hamiltonians may differ (one-site
// fields), pair Hamiltonians come from the bond structure.
#include "dense.h"

namespace vemb {
namespace {

constexpr int kBlock = 256;

// R(X_ij)_(x,y),(x',y') for the pair block starting at Xd (row stride ld).
__device__ double rx_dense(const DenseArgs& A, const double* Xd, int x, int y, int xp, int yp) {
  const int m = A.m;
  const long ld = A.ld;
  if (A.opset == VEMB_OPSET_COMPLETE) {
    const double v = Xd[(long)(xp * m + x) * ld + (y * m + yp)];
    return A.fermionic ? jw_sign(xp, y, yp) * v : v;
  }
  // (1/m) sum_ab X_ab [x = perm_a(x')] sgn_a(x') [y' = perm_b(y)] sgn_b(y)
  const OpTables& T = *A.ops;
  double acc = 0.0;
  for (int a = 0; a < T.n_op; ++a) {
    if (T.perm[a][xp] != x) continue;
    const double sa = T.sign[a][xp];
    for (int b = 0; b < T.n_op; ++b) {
      if (T.perm[b][y] != yp) continue;
      acc += Xd[(long)a * ld + b] * sa * T.sign[b][y];
    }
  }
  return acc / m;
}

__device__ inline const double* pair_block(const DenseArgs& A, int i, int j) {
  return A.X + (long)i * A.k * A.ld + (long)j * A.k;
}

// Right-hand side of eq. rhoijUpdate for pair e = (i, j):
// mu rho~ + Lam - H'_ij + (nu rho_i - L1) x I + I x (nu rho_j - L2),  H'_ij = H_ij - R - R^T.
__device__ double rhs_dense(const DenseArgs& A, int e, int i0, int j0, int r, int c) {
  const int m = A.m, n = A.n;
  const int x = r / m, y = r % m, xp = c / m, yp = c % m;
  const long o = (long)e * n * n + (long)r * n + c;
  const double* Xd = pair_block(A, i0, j0);
  double v = A.mu * A.rho_t[o] + A.Lam[o];
  const int h = A.hp_index[e];
  if (h >= 0) v -= A.Hp[(long)h * n * n + (long)r * n + c];
  v += rx_dense(A, Xd, x, y, xp, yp) + rx_dense(A, Xd, xp, yp, x, y);
  const long mo = (long)e * m * m;
  if (y == yp) v += A.nu * A.rho0[(long)i0 * m * m + x * m + xp] - A.Lam1[mo + x * m + xp];
  if (x == xp) v += A.nu * A.rho0[(long)j0 * m * m + y * m + yp] - A.Lam2[mo + y * m + yp];
  return v;
}

// Steps 1-2 for every pair (one workgroup per pair): rho_ij, A_1 rho, A_2 rho, Tr H_ij rho_ij.
__global__ void __launch_bounds__(kBlock) dense_pair_update_kernel(DenseArgs A) {
  const int e = blockIdx.x;
  const int2 pr = A.pairs[e];
  const int m = A.m, n = A.n, mm = m * m;
  const int tid = threadIdx.x;
  __shared__ double T2[kMaxM * kMaxM];
  __shared__ double T1[kMaxM * kMaxM];
  __shared__ double red[kBlock];
  __shared__ double trR_s;
  for (int q = tid; q < 2 * mm; q += kBlock) {
    const int which = q / mm, u = (q % mm) / m, w = q % m;
    double acc = 0.0;
    for (int t = 0; t < m; ++t)
      acc += which == 0 ? rhs_dense(A, e, pr.x, pr.y, u * m + t, w * m + t)
                        : rhs_dense(A, e, pr.x, pr.y, t * m + u, t * m + w);
    (which == 0 ? T2 : T1)[u * m + w] = acc;
  }
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int u = 0; u < m; ++u) t += T2[u * m + u];
    trR_s = t;
  }
  __syncthreads();
  const double trR = trR_s;
  const double a = A.a, bm = A.b / m, cm2 = A.c / ((double)m * m) * trR;
  const int h = A.hp_index[e];
  double epart = 0.0;
  for (int idx = tid; idx < n * n; idx += kBlock) {
    const int r = idx / n, c = idx % n;
    const int x = r / m, y = r % m, xp = c / m, yp = c % m;
    double v = a * rhs_dense(A, e, pr.x, pr.y, r, c);
    double corr = 0.0;
    if (y == yp) corr += T2[x * m + xp];
    if (x == xp) corr += T1[y * m + yp];
    v += bm * corr;
    if (r == c) v += cm2;
    A.rho[(long)e * n * n + idx] = v;
    if (h >= 0) epart += A.Hp[(long)h * n * n + (long)c * n + r] * v;
  }
  const double ab = A.a + A.b, bc = (A.b + A.c) / m * trR;
  for (int q = tid; q < mm; q += kBlock) {
    const int u = q / m, w = q % m;
    A.tr2[(long)e * mm + q] = ab * T2[q] + (u == w ? bc : 0.0);
    A.tr1[(long)e * mm + q] = ab * T1[q] + (u == w ? bc : 0.0);
  }
  red[tid] = epart;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) A.e_pair[e] = red[0];
}

// C_0(X_ii)(b, w) = sum over the operator collection (as in eq. effHam).
__device__ double c0_dense(const DenseArgs& A, int i, int b, int w) {
  const int m = A.m, k = A.k;
  const long ld = A.ld;
  const double* Xi = A.X + (long)i * k * ld + (long)i * k;
  if (A.opset == VEMB_OPSET_COMPLETE) {
    double acc = 0.0;
    for (int a = 0; a < m; ++a) acc += Xi[(long)(a * m + b) * ld + (a * m + w)];
    return acc;
  }
  const OpTables& T = *A.ops;
  double acc = 0.0;
  for (int v = 0; v < m; ++v)
    for (int al = 0; al < k; ++al) {
      if (T.perm[al][v] != b) continue;
      for (int be = 0; be < k; ++be) {
        if (T.perm[be][v] != w) continue;
        acc += Xi[(long)al * ld + be] * T.sign[al][v] * T.sign[be][v];
      }
    }
  return acc / m;
}

// Steps 4 and the diagonal blocks of step 6 for every cluster (one workgroup each):
// rho_i = [sum over pairs containing i of (nu A rho + L) - H'_i] / (nu (M-1)), unit trace;
// X'_ii = X_ii + sign eps G_00(rho_i);  Tr H_i rho_i.
__global__ void __launch_bounds__(kBlock) dense_cluster_kernel(DenseArgs A) {
  const int i = blockIdx.x;
  const int m = A.m, mm = m * m, k = A.k;
  const long ld = A.ld;
  const int tid = threadIdx.x;
  __shared__ double r0[kMaxM * kMaxM];
  __shared__ double red[kBlock];
  __shared__ double z_s;
  for (int q = tid; q < mm; q += kBlock) {
    double acc = 0.0;
    for (int e = 0; e < A.Q; ++e) {
      const int2 pr = A.pairs[e];
      if (pr.x == i) acc += A.nu * A.tr2[(long)e * mm + q] + A.Lam1[(long)e * mm + q];
      else if (pr.y == i) acc += A.nu * A.tr1[(long)e * mm + q] + A.Lam2[(long)e * mm + q];
    }
    const double hp = A.Hc[(long)i * mm + q] - c0_dense(A, i, q / m, q % m);
    r0[q] = (acc - hp) / (A.nu * (A.M - 1));
  }
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int u = 0; u < m; ++u) t += r0[u * m + u];
    z_s = (1.0 - t) / m;
  }
  __syncthreads();
  double epart = 0.0;
  for (int q = tid; q < mm; q += kBlock) {
    const double v = r0[q] + ((q / m == q % m) ? z_s : 0.0);
    r0[q] = v;  // each entry is read back by its own thread only until the barrier below
    A.rho0[(long)i * mm + q] = v;
    epart += A.Hc[(long)i * mm + (q % m) * m + q / m] * v;
  }
  __syncthreads();
  for (int q = tid; q < k * k; q += kBlock) {
    const int al = q / k, be = q % k;
    double g;
    if (A.opset == VEMB_OPSET_COMPLETE) {
      const int aa = al / m, bb = al % m, cc = be / m, ee = be % m;
      g = (aa == cc) ? r0[ee * m + bb] : 0.0;
    } else {
      const OpTables& T = *A.ops;
      double acc = 0.0;
      for (int v = 0; v < m; ++v) acc += T.sign[al][v] * T.sign[be][v] * r0[T.perm[be][v] * m + T.perm[al][v]];
      g = acc / m;
    }
    const long o = ((long)i * k + al) * ld + (long)i * k + be;
    A.Xp[o] = A.X[o] + A.sign * A.eps * g;
  }
  red[tid] = epart;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) A.e_clu[i] = red[0];
}

// Step 5 for every pair: Lambda1 += nu (A_1 rho - rho_i), Lambda2 += nu (A_2 rho - rho_j), and
// the consistency residual of eq. feasErr.
__global__ void __launch_bounds__(kBlock) dense_mult_kernel(DenseArgs A) {
  const int e = blockIdx.x;
  const int2 pr = A.pairs[e];
  const int mm = A.m * A.m;
  __shared__ double red[kBlock];
  double part = 0.0;
  for (int q = threadIdx.x; q < mm; q += kBlock) {
    const long o = (long)e * mm + q;
    const double d1 = A.tr2[o] - A.rho0[(long)pr.x * mm + q];
    const double d2 = A.tr1[o] - A.rho0[(long)pr.y * mm + q];
    A.Lam1[o] += A.nu * d1;
    A.Lam2[o] += A.nu * d2;
    part += d1 * d1 + d2 * d2;
  }
  red[threadIdx.x] = part;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) A.cons[e] = red[0];
}

// Off-diagonal blocks of step 6: X'_ij = X_ij + sign eps G_0d(rho_ij), X'_ji = X_ji + sign eps G_0d(rho_ij)^T.
__global__ void __launch_bounds__(kBlock) dense_xstep_kernel(DenseArgs A) {
  const int e = blockIdx.y;
  const int k = A.k, m = A.m, n = A.n;
  const int q = blockIdx.x * kBlock + threadIdx.x;
  if (q >= k * k) return;
  const int2 pr = A.pairs[e];
  const double* rho = A.rho + (long)e * n * n;
  const int al = q / k, be = q % k;
  double g;
  if (A.opset == VEMB_OPSET_COMPLETE) {
    const int aa = al / m, bb = al % m, cc = be / m, ee = be % m;
    g = rho[(long)(aa * m + ee) * n + (bb * m + cc)];
    if (A.fermionic) g *= jw_sign(aa, cc, ee);
  } else {
    const OpTables& T = *A.ops;
    double acc = 0.0;
    for (int xp = 0; xp < m; ++xp)
      for (int y = 0; y < m; ++y)
        acc += T.sign[al][xp] * T.sign[be][y] * rho[(long)(xp * m + T.perm[be][y]) * n + (T.perm[al][xp] * m + y)];
    g = acc / m;
  }
  const long ld = A.ld;
  const long o = ((long)pr.x * k + al) * ld + (long)pr.y * k + be;
  const long ot = ((long)pr.y * k + be) * ld + (long)pr.x * k + al;
  const double step = A.sign * A.eps * g;
  A.Xp[o] = A.X[o] + step;
  A.Xp[ot] = A.X[ot] + step;
}

// Bound matrices: pair K_e = H_e - R - R^T + sym(L1) x I + I x sym(L2) (Q of them, n x n), then
// cluster A_i = H_i - C_0(X_ii) - sum_{(i,b)} sym(L1) - sum_{(a,i)} sym(L2) (M of them, m x m).
__global__ void __launch_bounds__(kBlock) dense_bound_pair_kernel(DenseArgs A) {
  const int e = blockIdx.y;
  const int m = A.m, n = A.n;
  const int idx = blockIdx.x * kBlock + threadIdx.x;
  if (idx >= n * n) return;
  const int2 pr = A.pairs[e];
  const int r = idx / n, c = idx % n;
  const int x = r / m, y = r % m, xp = c / m, yp = c % m;
  const double* Xd = pair_block(A, pr.x, pr.y);
  double v = -(rx_dense(A, Xd, x, y, xp, yp) + rx_dense(A, Xd, xp, yp, x, y));
  const int h = A.hp_index[e];
  if (h >= 0) v += A.Hp[(long)h * n * n + idx];
  const long mo = (long)e * m * m;
  if (y == yp) v += 0.5 * (A.Lam1[mo + x * m + xp] + A.Lam1[mo + xp * m + x]);
  if (x == xp) v += 0.5 * (A.Lam2[mo + y * m + yp] + A.Lam2[mo + yp * m + y]);
  A.Kbuf[(long)e * n * n + idx] = v;
}

__global__ void __launch_bounds__(kBlock) dense_bound_cluster_kernel(DenseArgs A) {
  const int i = blockIdx.x;
  const int m = A.m, mm = m * m;
  double* Ki = A.Kbuf + (long)A.Q * A.n * A.n + (long)i * mm;
  for (int q = threadIdx.x; q < mm; q += kBlock) {
    const int u = q / m, w = q % m;
    double v = A.Hc[(long)i * mm + q] - c0_dense(A, i, u, w);
    for (int e = 0; e < A.Q; ++e) {
      const int2 pr = A.pairs[e];
      const long mo = (long)e * mm;
      if (pr.x == i) v -= 0.5 * (A.Lam1[mo + u * m + w] + A.Lam1[mo + w * m + u]);
      else if (pr.y == i) v -= 0.5 * (A.Lam2[mo + u * m + w] + A.Lam2[mo + w * m + u]);
    }
    Ki[q] = v;
  }
}

}  // namespace

hipError_t launch_dense_pair_update(const DenseArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(dense_pair_update_kernel, dim3(a.Q), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_dense_cluster(const DenseArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(dense_cluster_kernel, dim3(a.M), dim3(kBlock), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dense_mult_kernel, dim3(a.Q), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_dense_xstep(const DenseArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(dense_xstep_kernel, dim3((a.k * a.k + kBlock - 1) / kBlock, a.Q), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_dense_bound_build(const DenseArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(dense_bound_pair_kernel, dim3((a.n * a.n + kBlock - 1) / kBlock, a.Q), dim3(kBlock), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dense_bound_cluster_kernel, dim3(a.M), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

}  // namespace vemb
