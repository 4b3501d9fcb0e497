// Launchers of the device kernels, called by the host runtime (api.cpp).
#pragma once

#include "common.h"

namespace vemb {

// ----- Jacobi PSD projection / eigenvalues (jacobi.hip) -------------------
// Per-instance pointers for batched projections (one launch over many problems).
struct PairPtrs {
  const double* rho;
  double* Lam;
  double* rho_t;
  double* feas;
  int* sweeps;
  double* vstore;
  double mu;
  int active;  // 0: the instance is masked in its batch (its blocks are skipped)
};
struct MomPtrs {
  double* Xh;
  int* sweeps;
  double* vstore;
  int active;
};
// kind 0: pair projections (PairPtrs), kind 1: momentum projections (MomPtrs).
// item: device array count x int2 (instance, local index); ptrs: device array of
// PairPtrs / MomPtrs; vstore_any: any non-null pointer when eigenvectors are kept.
// Matrices above the LDS capacity use wscr / tscr (count x n x n, batch-owned).
hipError_t launch_projection_group(int kind, int n, int count, int precision, int max_sweeps, int cold, int tpb,
                                   const int2* item, const void* ptrs, void* vstore_any, void* wscr, void* tscr,
                                   hipStream_t st);
// All launchers enqueue on `st` and return hipSuccess or the launch error.

// Pair step 3 + Lambda update: C = rho - Lam/mu; rho_t = Pi(C); Lam += mu (rho_t - rho);
// feas[d] = ||rho_d - rho_t_d||_F^2.  P matrices of size n.
// vstore (P x n x n doubles, column-major per matrix) keeps each pair's eigenvectors for
// the warm start of the next iteration; cold = 1 ignores its content, cold = 0 starts
// from it, cold = 2 first restores its orthonormality (kept V from an FP32 solve).
hipError_t launch_pair_projection(const double* rho, double* Lam, double* rho_t, double* feas, int n, int P,
                                  double mu, int precision, int max_sweeps, int* sweeps, double* vstore, int cold,
                                  int tpb, hipStream_t st);

// Steps 8: Y_k = Pi((Xh_k + Xh_k^H)/2), in place on K complex n_op x n_op blocks
// (interleaved re/im doubles).
hipError_t launch_momentum_projection(double* Xh, int n_op, int K, int precision, int max_sweeps, int* sweeps,
                                      double* vstore, int cold, int tpb, hipStream_t st);

// Both of the above in one launch (warm-started, kFusedThreads threads per workgroup), for pair and
// momentum blocks of 33..64: workgroups [0, P) take the pair blocks, [P, P + K) the momentum blocks.
// vpair / vmom: the two eigenvector stores; sweeps[0, P) and sweeps[P, P + K).  precision: VEMB_FP64
// solves in FP64, VEMB_FP32 in FP32 (sweeps and matrix-core rebuild; state stays FP64).
constexpr int kFusedThreads = 512;
inline bool fused_projection_fits(int n, int n_op) { return n > 32 && n <= 64 && n_op > 32 && n_op <= 64; }
hipError_t launch_projections_fused(const double* rho, double* Lam, double* rho_t, double* feas, int n, int P,
                                   double mu, double* Xh, int n_op, int K, int max_sweeps, int* sweeps, double* vpair,
                                   double* vmom, int cold, hipStream_t st, int precision = VEMB_FP64);

// Isolated batched projection / eigenvalues (ABI entry points).
// vstore: eigenvector scratch (batch x n x n, complex doubles for Hermitian), needed by MIXED.
// tpb: LDS solver variant (256 / 512 / 1024 threads, 64 / 128 register-resident), see the
// autotuner in api.cpp.  cold = 0 starts from the eigenvectors in vstore (needs vstore).
hipError_t launch_psd_batched(const double* in, double* out, int n, int batch, bool is_complex, int precision,
                              int max_sweeps, int* sweeps, double* vstore, int tpb, hipStream_t st, int cold = 1);
hipError_t launch_eigvalsh_batched(const double* in, double* w, int n, int batch, bool is_complex,
                                   int max_sweeps, int* sweeps, hipStream_t st);

// Streaming variants for n > 64 (pairs) / n_op > 64 (momentum), n <= 256: W and T are
// per-matrix scratch of count x n x n compute scalars each (sized for FP64 / complex FP64).
hipError_t launch_pair_projection_big(const double* rho, double* Lam, double* rho_t, double* feas, int n, int P,
                                      double mu, int precision, int max_sweeps, int* sweeps, double* vstore, int cold,
                                      void* wscr, void* tscr, hipStream_t st);
hipError_t launch_momentum_projection_big(double* Xh, int n_op, int K, int precision, int max_sweeps, int* sweeps,
                                          double* vstore, int cold, void* wscr, void* tscr, hipStream_t st);
// cold = 0 starts from the eigenvectors in vstore (needs vstore).
hipError_t launch_psd_batched_big(const double* in, double* out, int n, int batch, bool is_complex, int precision,
                                  int max_sweeps, int* sweeps, double* vstore, void* wscr, void* tscr, hipStream_t st,
                                  int cold = 1);
hipError_t launch_eigvals_big(const double* in, double* w, double* wmin, int n, int count, bool is_complex,
                              int max_sweeps, int* sweeps, void* wscr, void* tscr, hipStream_t st);

// Smallest eigenvalue of `count` symmetric n x n matrices stored contiguously; with
// vstore (count x n x n) the eigenvectors are kept and, unless cold, reused as the start.
hipError_t launch_lambda_min(const double* K, double* lmin, int n, int count, int max_sweeps, int* sweeps,
                             hipStream_t st, int tpb = 256, double* vstore = nullptr, int cold = 1);

// ----- Iteration kernels (step_kernels.hip) ---------------------------------
struct StepArgs {
  // sizes
  int M, P, m, n, n_op, Ku;
  int opset;
  int fermionic;             // 1: Jordan-Wigner parity signs on the pair blocks (complete collection)
  double mu, nu, eps, sign;  // sign = -1 for X - eps G
  double a, b, c;            // closed-form inverse coefficients
  // fixed data
  const double* H0;      // m x m
  const double* Hd;      // nH x n x n (compact; only bonded offsets)
  const int* hd_index;   // P entries: index into Hd or -1
  const OpTables* ops;   // device copy (PAULI1)
  const double* tw;      // Ku x M complex (interleaved): M^{-1/2} exp(-2 pi i d.k / M)
  const double* wk;      // Ku weights (1 self-conjugate, 2 otherwise)
  // state
  double* X;     // M x n_op x n_op
  double* Xp;    // M x n_op x n_op  (X - eps G)
  double* Xh;    // Ku x n_op x n_op complex
  double* rho0;  // m x m
  double* rho;   // P x n x n
  double* rho_t; // P x n x n
  double* Lam;   // P x n x n
  double* Lam1;  // P x m x m
  double* Lam2;  // P x m x m
  double* tr2;   // P x m x m  (A_1 rho_d)
  double* tr1;   // P x m x m  (A_2 rho_d)
  // diagnostics
  double* e_pair;   // P: Tr(H_0d rho_d)
  double* feas;     // P: ||rho_d - rho~_d||^2
  double* scal;     // [0] Tr(H0 rho0), [1] sum_d ||A1 rho_d - rho0||^2 + ||A2 rho_d - rho0||^2
  double* Kbuf;     // P x n x n scratch for the bound, and m x m (K_0) after it
  double* lmin;     // P + 1
  int* sweeps;      // per-matrix sweep counters (P + Ku + P + 1)
  double* Vpair;    // P x n x n eigenvectors of the pair projections (warm start)
  double* Vmom;     // Ku x n_op x n_op complex eigenvectors of the momentum projections
  void* wscr_pair;  // streaming-solver scratch (n > 64): P x n x n doubles each
  void* tscr_pair;
  void* wscr_mom;   // (n_op > 64): Ku x n_op x n_op complex doubles each
  void* tscr_mom;
  int active;  // batches: 0 masks the instance (every batched kernel skips its blocks); 1 otherwise
};

// Batched step kernels: work[b] = {instance, local block x, local block y}.
struct WorkItem {
  int inst, bx, by, pad;
};
// Local grid (x, y) of the five step kernels of one instance, in the order
// 0 pair update, 1 X step, 2 cluster update, 3 forward DFT, 4 inverse DFT.
void local_grids(const StepArgs& a, int grid[5][2]);
// One launch of step kernel `which` (numbering above) over all work items;
// args is a device array of per-instance StepArgs.  which = 2 takes one block
// per instance (nwork = instance count, work unused).
hipError_t launch_step_batched(int which, const StepArgs* args, const WorkItem* work, int nwork, hipStream_t st);

hipError_t launch_pair_update(const StepArgs& a, hipStream_t st);
hipError_t launch_pair_xstep(const StepArgs& a, hipStream_t st);
hipError_t launch_cluster_update(const StepArgs& a, hipStream_t st);
hipError_t launch_dft_forward(const StepArgs& a, hipStream_t st);
hipError_t launch_dft_inverse(const StepArgs& a, hipStream_t st);
hipError_t launch_bound_build(const StepArgs& a, hipStream_t st);

// ----- Learned warm start: fixed-size state encoding of rings (warm.hip) -----
// `near` distances have blocks of their own, larger distances share a 'far' block.
struct WarmLayout {
  int near;
  int far_cold;  // decode: offsets beyond `near` take the cold start instead of the far slot
  long x00, rho0, block0, bsz, total;  // offsets / sizes in floats
  long oX, oL, oL1, oL2, oR;           // parts of a block
};
WarmLayout warm_layout(const StepArgs& a, int near);
// vec (device, warm_layout(a, near).total floats) <- state; needs M >= near + 1.
hipError_t launch_warm_encode(const StepArgs& a, int near, float* vec, hipStream_t st);
// State <- vec: X' (in Xp, to be projected), rho0, rho~ = rho, Lambda, Lambda1, Lambda2.
// far_cold: offsets at distances above `near` start cold (X_0d = 0, multipliers 0, rho~ = I/n).
hipError_t launch_warm_decode(const StepArgs& a, int near, const float* vec, hipStream_t st, int far_cold = 0);

}  // namespace vemb
