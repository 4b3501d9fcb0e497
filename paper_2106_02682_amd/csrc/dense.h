// Device side of dense Algorithm 5 (no translation invariance): arguments and launchers
// of the kernels in dense.hip.  Pairs e = (i, j), i < j, in lexicographic order.
#pragma once

#include "kernels.h"

namespace vemb {

struct DenseArgs {
  int M, Q, m, n, k, K;  // clusters, pairs, cluster / pair dimension, operators per cluster, K = M k
  int ld;                // row stride of X and X' (K, or K rounded up for the streamed eigensolver;
                         // rows and columns K..ld-1 stay zero, which the projection preserves)
  int opset;
  int fermionic;             // 1: Jordan-Wigner parity signs on the pair blocks (complete collection)
  double mu, nu, eps, sign;  // sign = -1 for X - eps G
  double a, b, c;            // closed-form inverse coefficients of the pair system
  const int2* pairs;         // Q cluster pairs (i, j), i < j
  const double* Hc;          // M x m x m cluster Hamiltonians (site fields included)
  const double* Hp;          // compact pair Hamiltonians, n x n each
  const int* hp_index;       // Q: index into Hp, or -1 for pairs without a bond
  const OpTables* ops;       // device copy (PAULI1)
  double* X;      // K x K dual (ld x ld storage)
  double* Xp;     // K x K: X - eps G, the input of the projection (ld x ld storage)
  double* rho0;   // M x m x m cluster marginals
  double* rho;    // Q x n x n pair marginals of the latest pair update
  double* rho_t;  // Q x n x n
  double* Lam;    // Q x n x n
  double* Lam1;   // Q x m x m
  double* Lam2;   // Q x m x m
  double* tr2;    // Q x m x m: A_1 rho_ij
  double* tr1;    // Q x m x m: A_2 rho_ij
  double* e_pair; // Q: Tr H_ij rho_ij
  double* e_clu;  // M: Tr H_i rho_i
  double* cons;   // Q: ||A_1 rho_ij - rho_i||^2 + ||A_2 rho_ij - rho_j||^2
  double* Kbuf;   // Q x n x n pair bound matrices, then M x m x m cluster ones
};

// Steps 1-2 for every pair (rho_ij, its partial traces, the pair energies).
hipError_t launch_dense_pair_update(const DenseArgs& a, hipStream_t st);
// Steps 4-5 and the diagonal blocks of X' (cluster marginals, consistency multipliers).
hipError_t launch_dense_cluster(const DenseArgs& a, hipStream_t st);
// Off-diagonal blocks of X' = X - eps G (both triangles).
hipError_t launch_dense_xstep(const DenseArgs& a, hipStream_t st);
// Matrices of the Lagrangian bound (their smallest eigenvalues are summed on the host).
hipError_t launch_dense_bound_build(const DenseArgs& a, hipStream_t st);

}  // namespace vemb
