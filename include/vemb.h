/*
 * vemb.h -- C ABI of the MI355X library for the translation-invariant
 * two-marginal SDP relaxation of Khoo & Lindsey (arXiv 2106.02682).
 *
 * The library runs Algorithm 6 of the paper (translation-invariant ADMM /
 * projected dual gradient ascent, Section 3.3) on one GPU.  One iteration is
 *   1. effective Hamiltonians H'_0, H'_0d from the dual X      (eq. effHam)
 *   2. closed-form pair update rho_0d                          (eq. rhoijUpdate)
 *   3. PSD projection rho~_0d = Pi(rho_0d - Lambda_0d/mu)      (eq. rhoijTildeUpdate)
 *   4. cluster marginal rho_0 with trace fix                   (eq. rhoiUpdate)
 *   5. multiplier updates Lambda, Lambda1, Lambda2             (Algorithm 6)
 *   6. X' = X - eps G(rho)   (gradient of the partial dual is -G, eq. gradX)
 *   7. momentum blocks Xhat_k by a DFT over the cluster lattice (Section 3.3)
 *   8. Y_k = Pi(Hermitian part of Xhat_k)
 *   9. X_0d by the inverse DFT.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Status codes: 0 = VEMB_OK; negative values are errors (enum below).  No
 *   C++ exception crosses the ABI.  vemb_last_error() returns a thread-local
 *   message describing the last failure of the calling thread.
 * - All matrices are row-major, float64 unless stated.  A pair index is
 *   (x, y) -> x*m + y with cluster 0 the first (most significant) factor;
 *   inside a cluster, local site 0 is the most significant bit.
 * - Lattice: periodic Nx x Ny (Ny = 1 for a ring).  Site (x, y) belongs to
 *   cluster (x / Lx, y / Ly), flat cluster index cx*My + cy, local site index
 *   (x % Lx)*Ly + (y % Ly).  Offsets d = 1..M-1 use the flat cluster index.
 * - Device work is enqueued on the hipStream_t given at creation (NULL = the
 *   null stream).  The library owns all device memory of a problem; callers
 *   own every host buffer they pass.
 */
#ifndef VEMB_H
#define VEMB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum vemb_status {
  VEMB_OK = 0,
  VEMB_E_INVALID = -1,      /* NULL pointer, shape that does not tile, bad size or option */
  VEMB_E_UNSUPPORTED = -2,  /* M < 2, complex term, >2-site term, cluster too large, non-periodic */
  VEMB_E_NOMEM = -3,        /* device or host allocation failed */
  VEMB_E_HIP = -4,          /* a HIP runtime call failed (message names it) */
  VEMB_E_NUMERIC = -5,      /* non-finite value met by a diagnostic or by set_state */
  VEMB_E_DIVERGED = -6,     /* divergence watchdog fired (bound not finite or feasibility blowing up) */
  VEMB_E_NOCONV = -7        /* an eigensolver reached its sweep cap (result still written) */
};

/* VEMB_FHOP marks the two ends of a fermionic hopping (fermionic problems only). */
enum vemb_pauli { VEMB_I = 0, VEMB_X = 1, VEMB_Y = 2, VEMB_Z = 3, VEMB_FHOP = 4 };

/* One translation-invariant term: coeff * prod_s pauli[s] at site origin + offset[s].
 * nsites is 1 or 2 (pairwise Hamiltonians, Section 2.1).  The product must be
 * real (an even number of Y factors), as the paper treats the real case.
 * Fermionic problems (vemb_options.fermionic = 1; spinless fermions of the
 * appendix on fermions): a two-site term with pauli = {VEMB_FHOP, VEMB_FHOP} is
 * coeff (a_i^dag a_j + a_j^dag a_i) between its two sites, and VEMB_Z stands for
 * 1 - 2 n (so (n_i - 1/2)(n_j - 1/2) = Z_i Z_j / 4); X and Y are rejected.  Each
 * cluster uses the Jordan-Wigner order of its local sites, each cluster pair the
 * order (first cluster's sites, then the second's), cluster 0 first for the
 * offsets d; occupied = |1>. */
typedef struct {
  double coeff;
  int32_t nsites;
  int32_t pauli[2];
  int32_t offset[2][2]; /* (dx, dy) per factor */
} vemb_term;

typedef struct {
  int32_t nterms;
  const vemb_term* terms;
} vemb_hamiltonian;

typedef struct {
  int32_t ndim;        /* 1 or 2 */
  int32_t extent[2];   /* Nx, Ny (Ny = 1 when ndim = 1) */
  int32_t periodic[2]; /* must be 1: translation invariance needs a torus */
} vemb_lattice;

typedef struct {
  int32_t shape[2]; /* Lx, Ly; must divide the extents (Section 2.3, clusters as supersites) */
} vemb_clusters;

enum vemb_opset { VEMB_OPSET_COMPLETE = 0, VEMB_OPSET_PAULI1 = 1 };
/* Precision of a problem's iterations.  VEMB_FP64: every eigensolve in FP64.  VEMB_MIXED: the
 * eigensolves of vemb_step run in FP32 -- Jacobi rotations, the rebuild on FP32 matrix cores with FP32
 * accumulation, and for 256 x 256 blocks the sign-function products on FP32 matrix cores (eigenvalues
 * above 1e-6 of the block's norm resolved); the state stays FP64, and so do the diagnostics (bound,
 * energy, feasibility residuals) and vemb_refine, the closing FP64 iterations warm-started from the FP32
 * eigenvectors.  The bound of an FP32 iterate is evaluated in FP64 on an X that is PSD to FP32 rounding;
 * after vemb_refine it is certified.  VEMB_FP32: the same as VEMB_MIXED for problems.  For the isolated
 * vemb_psd_project_batched, VEMB_MIXED means FP32 sweeps followed by one FP64 refinement sweep and an
 * FP64 rebuild, VEMB_FP32 FP32 throughout. */
enum vemb_precision { VEMB_FP64 = 0, VEMB_MIXED = 1, VEMB_FP32 = 2 };

typedef struct {
  double mu, nu, eps;  /* penalty and step parameters (Section 4 uses 10, 10, 2) */
  int32_t opset;       /* vemb_opset: operator collection defining G (Section 2.2) */
  int32_t precision;   /* vemb_precision */
  int32_t max_sweeps;  /* Jacobi sweep cap per eigensolve (0 = default 40) */
  int32_t sign;        /* -1: X <- Pi(X - eps G) (default when 0); +1: the printed + sign */
  int32_t warm_refresh; /* eigensolves start from the previous iteration's eigenvectors; every
                           warm_refresh-th iteration (t % warm_refresh == 0) starts cold.
                           0 = default 64; negative = always cold. */
  int32_t tpb;          /* LDS eigensolver variant: 256, 512 or 1024 threads per workgroup
                           (columns round-trip through LDS every round); or, for 64 x 64
                           matrices, columns held in registers: 64 = 8-column blocks on 4
                           wavefronts, 128 = 4-column blocks on 8 wavefronts (blocks move
                           through LDS once per block round); other sizes then use 256.
                           0 = chosen by the autotuner (vemb_tuned_threads). */
  int32_t fermionic;    /* 1: spinless fermions (appendix on fermions): VEMB_FHOP terms, and the
                           off-diagonal G blocks and pair corrections of eq. effHam take the
                           Jordan-Wigner parity sign of the pair order (an odd operator of the
                           second cluster carries the first cluster's parity).  Needs
                           VEMB_OPSET_COMPLETE.  0 (default): spins. */
  int32_t lb_every;     /* > 0: vemb_step evaluates the FP64 diagnostics (bound, energy, feasibility) every
                           lb_every iterations, queued on the stream and read back one interval later, and
                           stops with the watchdog's status (vemb_divergence_check) when it fires:
                           VEMB_E_NUMERIC or VEMB_E_DIVERGED, naming the iteration.  While it is on, the
                           library owns the queued diagnostics (vemb_diagnostics_collect returns the latest
                           it queued).  0 (default): no diagnostics inside vemb_step. */
  int32_t adapt_every;  /* > 0: adaptive parameters (Section 4 notes that tuning mu, nu, eps to a problem could
                           smooth convergence).  (mu, nu, eps) = c (mu_0, nu_0, eps_0) from the values above;
                           every adapt_every iterations vemb_step evaluates the FP64 diagnostics after the
                           iteration (the equality residual of eq. feasErr and the relative primal-dual gap
                           |E_p - LB| / |LB|, a bound evaluation) and multiplies c by 1.25 when both fell since
                           the previous check by more than a relative 1e-6, by 0.5 when either rose by more (a
                           quantity whose two values lie below 1e-12 counts as neither), c within [1, 8]; the
                           first check only records them.  The multipliers are unscaled, so a change keeps every
                           fixed point.  Single translation-invariant problems only (vemb_batch_create and
                           vemb_dense_create refuse it).  0 (default): the fixed parameters of the paper's
                           runs. */
} vemb_options;

typedef struct vemb_problem vemb_problem;

/* Sizes of a created problem. */
typedef struct {
  int32_t M, P, L, m, n, n_op, Mx, My, K_unique;
  int64_t t; /* iterations done */
} vemb_info;

/* Device memory.  By default the library takes device memory with hipMalloc and returns it with
 * hipFree.  vemb_set_allocator routes every later device allocation of the library through the caller's
 * functions instead (e.g. torch's caching allocator): the state of problems, batches, dense problems
 * and networks, the autotuner's buffers and the scratch of the isolated entry points.  alloc(bytes, ctx)
 * returns device memory of at least `bytes` bytes, aligned to 256 bytes, on the current device, or NULL
 * (the library then fails with VEMB_E_NOMEM); free(ptr, ctx) takes back a pointer alloc returned, after
 * the library has synchronised the streams that used it.  Both NULL restores hipMalloc / hipFree.  Each
 * object keeps the allocator in effect when it was created and returns its memory through it.  Pinned
 * host buffers are not routed (hipHostMalloc).  The functions may be called from any thread that calls
 * the library.  Errors: VEMB_E_INVALID when only one of the two is NULL, or while any problem, batch,
 * dense problem or network is alive (switch allocators between objects' lifetimes). */
typedef void* (*vemb_alloc_fn)(size_t bytes, void* ctx);
typedef void (*vemb_free_fn)(void* ptr, void* ctx);
int vemb_set_allocator(vemb_alloc_fn alloc_fn, vemb_free_fn free_fn, void* ctx);

/* Fills *opts with the paper's parameters (mu = nu = 10, eps = 2), COMPLETE, FP64. */
void vemb_default_options(vemb_options* opts);

/* Builds H_0 and H_0d on the host from the translation-invariant terms,
 * allocates device state and initialises it as in Section 4 (multipliers 0,
 * marginals identity / trace, X_00 = I, X_0d = 0).  Inputs are copied.
 * Errors: VEMB_E_INVALID, VEMB_E_UNSUPPORTED, VEMB_E_NOMEM, VEMB_E_HIP. */
int vemb_create_problem(const vemb_hamiltonian* H, const vemb_lattice* lattice, const vemb_clusters* clusters,
                        const vemb_options* opts, void* hip_stream, vemb_problem** out);

int vemb_problem_info(const vemb_problem* p, vemb_info* info);

/* Enqueues `iters` iterations of Algorithm 6 on the problem's stream.
 * Asynchronous: returns once the work is enqueued. */
int vemb_step(vemb_problem* p, int iters);

/* Mixed precision's final refinement: enqueues `iters` iterations whose eigensolves run in FP64;
 * the first starts from the eigenvectors the FP32 solves kept, orthonormalised by one Newton-Schulz
 * step (256 x 256 blocks: the FP64 sign function).  Same as vemb_step for an FP64 problem.
 * Asynchronous. */
int vemb_refine(vemb_problem* p, int iters);

/* FP64 Lagrangian lower bound per site (valid for any PSD X and any symmetric
 * Lambda1, Lambda2; derived from the partial dual, Section 2.4):
 *   (1/L)[lmin(H'_0 - 1/2 sum_d(L1_d + L2_d)) + 1/2 sum_d lmin(H'_0d + L1_d x I + I x L2_d)].
 * Synchronises the stream.  VEMB_E_NUMERIC on non-finite results. */
int vemb_dual_bound(vemb_problem* p, double* lb_per_site);

/* vemb_dual_bound and vemb_primal_energy in one call with one synchronisation
 * (lb required; e_per_site / feas_err may be NULL). */
int vemb_diagnostics(vemb_problem* p, double* lb_per_site, double* e_per_site, double* feas_err);
/* The same diagnostics without stopping the stream: _enqueue queues the bound
 * kernels and copies of the current state's diagnostics into pinned host memory
 * (later iterations queued after it do not change what it reports); _collect
 * waits for the last enqueued set and returns it (VEMB_E_INVALID if none). */
int vemb_diagnostics_enqueue(vemb_problem* p);
int vemb_diagnostics_collect(vemb_problem* p, double* lb_per_site, double* e_per_site, double* feas_err);

/* Primal energy per site [Tr H_0 rho_0 + 1/2 sum_d Tr H_0d rho_0d]/L of the
 * latest pair update and the feasibility error of eq. feasErr.  Synchronises. */
int vemb_primal_energy(vemb_problem* p, double* e_per_site, double* feas_err);

enum vemb_which { VEMB_RHO = 0, VEMB_RHO_TILDE = 1 };

/* Copies rho_0 (m*m doubles) and the pair marginals (P*n*n doubles; rho_0d of
 * the latest pair update, or rho~_0d) into caller-owned host buffers.
 * Either pointer may be NULL to skip it.  Synchronises. */
int vemb_marginals(vemb_problem* p, int which, double* rho0, double* rho_pairs);

/* Full iteration state, host buffers owned by the caller, sizes from vemb_info:
 * X: M*n_op*n_op (first block row X_0d, d = 0..M-1), rho0: m*m, rho: P*n*n,
 * rho_t: P*n*n, Lam: P*n*n, Lam1: P*m*m, Lam2: P*m*m.  It is the checkpoint
 * format and the warm-start input.  Optional (may be NULL): the eigenvectors
 * the eigensolves keep between iterations, Vpair: P*n*n and Vmom:
 * K_unique*n_op*n_op*2 (complex, interleaved), column-major per matrix.
 * Restoring them makes a resumed FP64 run bit-identical to an uninterrupted
 * one; without them the next iteration solves cold (same result up to rounding). */
typedef struct {
  int64_t t;
  double* X;
  double* rho0;
  double* rho;
  double* rho_t;
  double* Lam;
  double* Lam1;
  double* Lam2;
  double* Vpair;
  double* Vmom;
} vemb_state;

int vemb_get_state(vemb_problem* p, vemb_state* s);
/* Validates finiteness (VEMB_E_NUMERIC) and copies the state to the device. */
int vemb_set_state(vemb_problem* p, const vemb_state* s);

/* Largest Jacobi sweep count over the pair projections and over the momentum
 * projections of the last iteration (synchronises).  An eigensolve of the LDS solver
 * (blocks up to 64 x 64 complex / 128 x 128 real) that stopped at the sweep cap unconverged
 * records cap + 1; its kept eigenvectors are then reset to the identity, so its next solve
 * starts cold.  Returns VEMB_E_NOCONV (with both counts written) when a count exceeds the cap. */
int vemb_last_sweeps(vemb_problem* p, int* pair_max, int* momentum_max);

/* Parameters in force (adaptive mode, vemb_options.adapt_every): *mu, *nu, *eps, the joint scale *scale
 * (1 without adaptation), and *last_feas, *last_gap, feasErr (eq. feasErr) and the relative primal-dual gap
 * at the last check (-1 before the first).  Any output pointer may be NULL.  Errors: VEMB_E_INVALID for a
 * NULL problem. */
int vemb_penalties(const vemb_problem* p, double* mu, double* nu, double* eps, double* scale, double* last_feas,
                   double* last_gap);
/* Resume an adaptive run: sets the joint scale (within [1, 8]) and the values of the last check (either
 * negative: none, the next check only records); the parameters become scale times the created ones.
 * Errors: VEMB_E_INVALID (NULL problem, scale outside [1, 8] or not finite). */
int vemb_set_penalty_scale(vemb_problem* p, double scale, double last_feas, double last_gap);

/* The divergence watchdog's rule, on the host (no device work): feas[0..count) are the feasibility
 * errors (eq. feasErr) of successive diagnostics, oldest first; lb and energy the latest bound and
 * energy per site.  Returns VEMB_E_NUMERIC if the latest values are not finite; VEMB_E_DIVERGED if the
 * latest feasibility error exceeds 1e3 (marginals have unit trace, so a bounded iteration keeps it O(1)),
 * or if it rose at each of the last 5 checks and is at least 100 times the smallest seen; else VEMB_OK.
 * The printed "+ eps G" step (vemb_options.sign = +1) is the natural diverging case.  Errors:
 * VEMB_E_INVALID for count < 1 or NULL feas. */
int vemb_divergence_check(const double* feas, int count, double lb, double energy);

/* Kernel-level timing.  With profiling on, every kernel the problem launches is
 * bracketed by HIP events recorded on the problem's stream; vemb_get_profile
 * synchronises and returns the accumulated device milliseconds and launch counts
 * per kernel since profiling was (re)enabled. */
enum vemb_kernel_id {
  VEMB_K_PAIR_UPDATE = 0,  /* steps 1-2 */
  VEMB_K_PAIR_XSTEP = 1,   /* step 6, d != 0 */
  VEMB_K_PAIR_PROJ = 2,    /* step 3 + Lambda update */
  VEMB_K_CLUSTER = 3,      /* steps 4-5 + step 6, d = 0 */
  VEMB_K_DFT_FWD = 4,      /* step 7 */
  VEMB_K_MOM_PROJ = 5,     /* step 8 */
  VEMB_K_DFT_INV = 6,      /* step 9 */
  VEMB_K_BOUND_BUILD = 7,  /* bound matrices */
  VEMB_K_LMIN = 8,         /* bound eigenvalues */
  VEMB_K_PROJ = 9,         /* steps 3 and 8 in one launch (FP64 blocks of 33..64 with matching solver variants) */
  VEMB_K_COUNT = 10
};
typedef struct {
  double ms[VEMB_K_COUNT];
  int64_t launches[VEMB_K_COUNT];
} vemb_profile;

int vemb_set_profiling(vemb_problem* p, int enable);
/* As vemb_set_profiling with a bit mask of the kernels to time (bit vemb_kernel_id);
 * 0 turns timing off.  Fewer events per iteration disturb the timed run less. */
int vemb_set_profiling_mask(vemb_problem* p, uint32_t kernels);
/* Times only the iterations whose index t (iterations done so far on the problem) is a multiple of
 * `every` (>= 1; default 1, every iteration): each timed launch adds two event packets to the
 * stream, and sampling keeps their cost out of most iterations.  Errors: VEMB_E_INVALID for a NULL
 * problem or every < 1. */
int vemb_set_profiling_every(vemb_problem* p, int every);
int vemb_get_profile(vemb_problem* p, vemb_profile* out);

/* Autotuner of the LDS eigensolver variant (256 / 512 / 1024 threads, and the
 * register-resident 64 / 128 for n = 64) for
 * batches of `batch` n x n matrices: times the candidates with HIP events on
 * hip_stream on warm-started solves (a cold solve of seeded synthetic matrices,
 * then the timed solve of the same matrices moved by 1e-3, started from the kept
 * eigenvectors, as in the iteration) and returns the fastest (>0), or a
 * negative status.  Results are cached per (device, n, real/complex, precision,
 * batch rounded up to a power of two) in memory and in the text file
 * $VEMB_TUNE_CACHE (default $HOME/.cache/vemb_tune.txt; "none" = memory only).
 * Synchronises the stream.  vemb_create_problem calls it unless opts->tpb is set. */
int vemb_tuned_threads(int n, int is_complex, int precision, int batch, void* hip_stream);
/* Threads per workgroup the problem's pair and momentum eigensolves use. */
int vemb_problem_threads(const vemb_problem* p, int* pair_tpb, int* momentum_tpb);

void vemb_destroy(vemb_problem* p);
const char* vemb_last_error(void);

/* Isolated batched PSD projection (eq. rhoijTildeUpdate's Pi applied to a
 * batch): out[b] = argmin_{S >= 0} ||S - in[b]||_F for `batch` symmetric
 * (is_complex = 0; n*n doubles each) or Hermitian (is_complex = 1; n*n
 * interleaved re/im double pairs each) matrices.  `in` and `out` are DEVICE
 * pointers (they may alias).  precision: VEMB_FP64 or VEMB_MIXED.
 * Asynchronous on hip_stream for n <= 128 real / n <= 64 complex (matrix held in
 * LDS); larger n (<= 256, multiple of 16) use the streamed solver with scratch
 * allocated for the call, and the call synchronises the stream. */
int vemb_psd_project_batched(const double* in, double* out, int n, int batch, int is_complex, int precision,
                             void* hip_stream);

/* As vemb_psd_project_batched, with an explicit sweep cap (0 = default 40), an
 * optional DEVICE array sweeps[batch] receiving the sweeps each matrix used, and
 * the LDS solver variant tpb (as vemb_options.tpb; 0 = autotuned). */
int vemb_psd_project_batched_ex(const double* in, double* out, int n, int batch, int is_complex, int precision,
                                int max_sweeps, int* sweeps, int tpb, void* hip_stream);

/* Eigenvalues of a batch of symmetric / Hermitian matrices (device pointers;
 * w receives batch*n doubles in ascending order), by the same Jacobi solver. */
/* Pi(sym(in)) of ONE n x n matrix (n a positive multiple of 16, at most 4096; DEVICE row-major
 * FP64, in may alias out) by the matrix-sign route of the dense solver: (A + A sign(A)) / 2 with
 * sign(A) from 38 scaled Newton-Schulz steps on matrix cores, every eigenvalue above
 * 1e-14 ||A||_F resolved.  Allocates 4 n^2 + 64 doubles of scratch for the call and synchronises
 * hip_stream.  Errors: VEMB_E_INVALID, VEMB_E_NOMEM, VEMB_E_HIP. */
int vemb_psd_project_sign(const double* in, double* out, int n, void* hip_stream);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): vemb_psd_project_sign without any allocation.  Same arguments,
 * result and kernels; n a positive multiple of 16, at most 512 (VEMB_E_INVALID beyond, with a
 * message).  The scratch (4 n^2 + 64 doubles) lives in a static device array of 4 * 512^2 + 64
 * doubles (8 MiB) that each GPU the call runs on holds until the process ends; its device address
 * is looked up once per device on the first call.  Nothing in it needs to start at zero: each call
 * writes every scratch word it reads.  Asynchronous on hip_stream (it does not synchronise).  Every
 * call on one GPU shares that GPU's array, so calls that overlap on one GPU (different streams or
 * host threads without ordering) race and give wrong results: order them, e.g. on one stream.
 * Errors: VEMB_E_INVALID, VEMB_E_HIP. */
int vemb_psd_project_sign_noalloc(const double* in, double* out, int n, void* hip_stream);
int vemb_eigvalsh_batched(const double* in, double* w, int n, int batch, int is_complex, void* hip_stream);

/* Workgroup -> output tile map of the symmetric-product kernels, computed on the host by the same
 * functions the kernels and their launchers use, so that callers and tests can check a launch covers
 * every tile once and no workgroup reaches past the last one.  kind 0: the single-matrix product of the
 * sign projection (vemb_psd_project_sign, the dense X projection), n a multiple of 16 up to 4096, 16 x 16
 * tiles; kind 1: the batched products of the 4-site-cluster blocks, n a multiple of 64 up to 256, 64 x 64
 * tiles, `count` blocks, a 2-D grid (upper-triangle tiles, count) listed as bx + tiles_upper * by.
 * *grid receives the launch's workgroup count; map (host, 4 * grid ints, may be NULL to query the grid)
 * receives per workgroup {live, block, tile row, tile column} (live 0: the workgroup returns at once;
 * its other fields are -1).  Only the upper triangle (row <= column) is mapped.
 * Errors: VEMB_E_INVALID. */
int vemb_tile_map(int kind, int n, int count, int* grid, int* map);

/* ---- Batches: many independent problems stepped together --------------------
 * Parameter sweeps (Section 4's tables: one solve per field value or coupling)
 * and uneven mixes of cluster sizes.  A batch refers to existing problems (it
 * does not own them; destroy the batch first).  One iteration of a batch issues
 * one launch per step kernel for all instances and one eigensolver launch per
 * (kind, size, precision) class, with threads per workgroup from the autotuner,
 * and is captured in HIP graphs (an all-warm and a cold-refresh iteration) that
 * vemb_batch_step replays.  Every instance goes through the same arithmetic
 * as vemb_step alone (separately compiled kernels: results agree to rounding),
 * except that an iteration starts all eigensolves
 * cold when any instance needs a cold start (t % warm_refresh == 0, or no kept
 * eigenvectors).  All problems must be on the same device and share max_sweeps
 * and warm_refresh.  Errors: VEMB_E_INVALID, VEMB_E_NOMEM, VEMB_E_HIP. */
typedef struct vemb_batch vemb_batch;

/* use_graph = 0 launches the kernels directly each iteration (same results). */
int vemb_batch_create(vemb_problem* const* problems, int count, int use_graph, vemb_batch** out);
/* Enqueues `iters` iterations on the batch's own stream, ordered after work
 * already queued on each problem's stream; later work on a problem's stream
 * is ordered after them.  Asynchronous. */
int vemb_batch_step(vemb_batch* b, int iters);
/* Host arrays of length count: per-problem vemb_dual_bound results and status
 * codes (status may be NULL).  Synchronises; returns the last failing status.  An instance whose
 * bound is not finite (VEMB_E_NUMERIC) is masked (vemb_batch_set_active): later steps skip it. */
int vemb_batch_dual_bounds(vemb_batch* b, double* lb_per_site, int* status);
/* Host arrays of length count (either may be NULL): vemb_primal_energy per problem.  An instance whose
 * energy or feasibility error is not finite is masked, as above. */
int vemb_batch_primal_energies(vemb_batch* b, double* e_per_site, double* feas_err);
/* Failure masking.  A masked instance (active = 0) is skipped by every launch of later steps -- its
 * workgroups return at once, inside graph replays too -- so its state and iteration count stay as they
 * were (for inspection, or vemb_set_state and unmasking) and a diverged instance no longer costs its
 * eigensolves' sweep cap in every class launch; the other instances step exactly as before.  index in
 * [0, count); synchronises the batch stream.  Errors: VEMB_E_INVALID. */
int vemb_batch_set_active(vemb_batch* b, int index, int active);
/* Host array of length count: 1 for stepped instances, 0 for masked ones. */
int vemb_batch_get_active(const vemb_batch* b, int* active);
/* Number of eigensolver size classes and kernel launches per iteration. */
int vemb_batch_info(const vemb_batch* b, int* classes, int* launches_per_iteration);
/* Sampled kernel timing of a batch.  every >= 1: the iterations whose batch iteration index (counted
 * from the batch's creation) is a multiple of `every` are enqueued directly instead of replaying the
 * graph, with HIP events around each step kernel launch, each Jacobi class launch and each product
 * launch of the sign-function projections, recorded on the stream the launch runs on; every = 0 turns
 * timing off.  Resets the accumulated times.  vemb_batch_get_profile synchronises and returns the
 * accumulated device milliseconds and launch counts per kernel id since the last reset.
 * Errors: VEMB_E_INVALID (NULL batch, every < 0). */
enum vemb_batch_kernel_id {
  VEMB_BK_PAIR_UPDATE = 0,     /* steps 1-2, all instances in one launch */
  VEMB_BK_PAIR_XSTEP = 1,      /* step 6, d != 0 */
  VEMB_BK_CLUSTER = 2,         /* steps 4-5 + step 6, d = 0 */
  VEMB_BK_DFT_FWD = 3,         /* step 7 */
  VEMB_BK_DFT_INV = 4,         /* step 9 */
  VEMB_BK_PAIR_JACOBI = 5,     /* a Jacobi pair-projection launch (one per size class) */
  VEMB_BK_MOM_JACOBI = 6,      /* a Jacobi momentum-projection launch (one per size class) */
  VEMB_BK_SIGN_GEMM_REAL = 7,  /* one product launch of the pair sign projections (all blocks of the class) */
  VEMB_BK_SIGN_GEMM_CPLX = 8,  /* one product launch of the momentum sign projections */
  VEMB_BK_COUNT = 9
};
typedef struct {
  double ms[VEMB_BK_COUNT];
  int64_t launches[VEMB_BK_COUNT];
} vemb_batch_profile;
int vemb_batch_set_profiling(vemb_batch* b, int every);
int vemb_batch_get_profile(vemb_batch* b, vemb_batch_profile* out);
int vemb_batch_sync(vemb_batch* b);
void vemb_batch_destroy(vemb_batch* b);

/* ---- Dense Algorithm 5: no translation invariance (Section 3.2) --------------
 * One marginal rho_i per cluster and rho_ij, rho~_ij, Lambda_ij, Lambda1_ij,
 * Lambda2_ij per unordered cluster pair i < j (Q = M(M-1)/2 pairs, ordered
 * (0,1), (0,2), ..., (1,2), ...), and one dense dual X of size K = M n_op
 * (block (i, j) couples the operators of clusters i and j).  One iteration:
 *   1. pair update of every rho_ij with H'_ij = H_ij - R(X_ij) - R(X_ij)^T   (eq. rhoijUpdate)
 *   2. rho~_ij = Pi(rho_ij - Lambda_ij / mu), Lambda_ij update            (eq. rhoijTildeUpdate)
 *   3. rho_i from the pairs that contain i: A_1 terms of pairs (i, j > i),
 *      A_2 terms of pairs (j < i, i), divided by nu (M-1), unit trace      (eq. rhoiUpdate)
 *   4. Lambda1_ij, Lambda2_ij updates with the new rho_i, rho_j
 *   5. X <- Pi(X - eps G) for the dense G of Section 2.2 (diagonal blocks
 *      G_00(rho_i), off-diagonal blocks G_0d(rho_ij) and their transposes),
 *      one eigensolve of the whole K x K matrix.
 * The bonds are those of the translation-invariant term list on the torus
 * (H_ij = H_0d with d the offset from i to j); one-site fields may differ from
 * site to site (disorder), which translation invariance cannot represent.
 * Limits: K <= 1024, pair matrices n <= 256.  K <= 64: the X projection is a
 * one-sided Jacobi eigensolve (warm starts as vemb_problem; precision modes as the isolated
 * vemb_psd_project_batched: MIXED = FP32 sweeps, one FP64 refinement sweep and an FP64 rebuild).
 * K > 64: Pi(A) = (A + A sign(A)) / 2 with sign(A) from a fixed schedule of 38
 * scaled Newton-Schulz steps on matrix cores (FP64 in every precision mode; X
 * stored padded with zeros to a multiple of 32), resolving every eigenvalue
 * above 1e-14 ||A||_F.  Same option struct as vemb_problem. */
typedef struct vemb_dense vemb_dense;

/* One-site term coeff * pauli at lattice site (x, y) (wrapped onto the torus),
 * added to the Hamiltonian of the cluster holding the site.  pauli: VEMB_X or
 * VEMB_Z (real operators). */
typedef struct {
  int32_t x, y;
  int32_t pauli;
  double coeff;
} vemb_site_field;

typedef struct {
  int32_t M, Q, L, m, n, n_op, K;
  int64_t t; /* iterations done */
} vemb_dense_info;

/* Host buffers (each may be NULL): X (K x K), rho0 (M x m x m), rho, rho_t, Lam
 * (Q x n x n), Lam1, Lam2 (Q x m x m); rho is the latest pair update. */
typedef struct {
  int64_t t;
  double* X;
  double* rho0;
  double* rho;
  double* rho_t;
  double* Lam;
  double* Lam1;
  double* Lam2;
} vemb_dense_state;

/* Builds the cluster Hamiltonians (translation-invariant terms plus `nfields`
 * site fields, copied), allocates device state and initialises it as in
 * Section 4 (multipliers 0, marginals identity / trace, X = I).
 * Errors: VEMB_E_INVALID, VEMB_E_UNSUPPORTED (K or n above 256, a field other
 * than X or Z), VEMB_E_NOMEM, VEMB_E_HIP. */
int vemb_dense_create(const vemb_hamiltonian* H, const vemb_lattice* lattice, const vemb_clusters* clusters,
                      const vemb_site_field* fields, int nfields, const vemb_options* opts, void* hip_stream,
                      vemb_dense** out);
int vemb_dense_get_info(const vemb_dense* d, vemb_dense_info* info);
/* Enqueues `iters` iterations.  Asynchronous. */
int vemb_dense_step(vemb_dense* d, int iters);
/* Lagrangian lower bound per site at the current X, Lambda1, Lambda2 (Section 2.4
 * pair by pair): [sum_i lmin(H'_i - sum_{(i,b)} sym Lambda1 - sum_{(a,i)} sym Lambda2)
 * + sum_{i<j} lmin(H'_ij + sym Lambda1_ij x I + I x sym Lambda2_ij)] / N, with
 * H'_i = H_i - C_0(X_ii).  Synchronises.  VEMB_E_NUMERIC if not finite. */
int vemb_dense_dual_bound(vemb_dense* d, double* lb_per_site);
/* Energy per site of the latest pair update, [sum_i Tr H_i rho_i + sum_{i<j}
 * Tr H_ij rho_ij] / N, and the feasibility error sqrt(sum over pairs of the
 * consistency and rho = rho~ residuals / M) (eq. feasErr).  Either may be NULL.
 * Synchronises. */
int vemb_dense_primal_energy(vemb_dense* d, double* e_per_site, double* feas_err);
/* Copies the state to the host buffers of *st (NULL members skipped).  Synchronises. */
int vemb_dense_get_state(vemb_dense* d, vemb_dense_state* st);
/* Replaces the members of the state that are not NULL (X should be symmetric: the
 * projection reads its symmetric part); the next eigensolves start cold.
 * VEMB_E_NUMERIC for a non-finite value (nothing is changed then). */
int vemb_dense_set_state(vemb_dense* d, const vemb_dense_state* st);
/* Sweeps of the last pair projections (maximum) and of the last X projection
 * (for K > 64: the number of Newton-Schulz steps). */
int vemb_dense_last_sweeps(vemb_dense* d, int* pair_max, int* x_sweeps);
void vemb_dense_destroy(vemb_dense* d);

/* ---- Learned warm start ------------------------------------------------------
 * A multilayer perceptron maps Hamiltonian parameters to a fixed-size encoding
 * of a converged state, and the encoding becomes the starting point of a new
 * solve.  Any decoded point is valid: X is projected onto the PSD cone, so the
 * Lagrangian bound (Section 2.4) at it is a lower bound, and the plain cold
 * start stays the reference the network is judged against.
 *
 * Encoding of a ring of M clusters (vemb_warm_size floats, FP32, row-major
 * matrices): [X_00, rho_0, then for direction '+' and '-' the slots of distance
 * 1..near and 'far' (> near), each X_0d, Lambda_d, Lambda1_d, Lambda2_d, rho~_d].
 * Offset d is direction '+' at distance d when 2d <= M, else '-' at M - d.  With
 * near >= M/2 the encoding is exact; a smaller near gives a size independent of
 * M, the far slot averaging distances near+1..M/2. */
int vemb_warm_size(const vemb_problem* p, int near, int64_t* count);
/* vec (DEVICE, vemb_warm_size floats) <- the problem's current state.  Needs
 * M >= near + 1.  Asynchronous.  VEMB_E_UNSUPPORTED for 2-D lattices. */
int vemb_warm_encode(vemb_problem* p, int near, float* vec);
/* The problem's state <- decode(vec) (DEVICE): every offset takes its slot's
 * blocks, X_0,M-d = X_0d^T and X_00, rho_0, rho~, Lambdas symmetrised, Tr rho_0
 * = 1, rho = rho~, then X projected onto the PSD cone through its momentum
 * blocks (FP64).  Resets the iteration count (eigensolves restart cold).
 * Asynchronous. */
int vemb_warm_start(vemb_problem* p, int near, const float* vec);
/* As vemb_warm_start; far_cold = 1 starts the offsets at distances above `near` cold instead of from the
 * far slot (X_0d = 0, multipliers 0, rho~_d = rho_d = I/n: Section 4's start), the far slot unused. */
int vemb_warm_start_ex(vemb_problem* p, int near, const float* vec, int far_cold);

/* Network: dims[0] inputs, dims[1..n_dims-2] silu hidden layers, dims[n_dims-1]
 * outputs.  Parameters flat FP32 in the order W_0 (dims[1] x dims[0], row-major),
 * b_0, W_1, b_1, ...; the passes read the weights rounded to bfloat16 (nearest
 * even) and multiply on the BF16 matrix cores with FP32 accumulation, FP32
 * activations and gradients entering as exact sums of three bfloat16 terms (the
 * accuracy of an FP32 product).  Targets are learned normalised per output,
 * t_hat = (t - mean) / std; the loss is the mean of (y - t_hat)^2 over batch and
 * outputs; Adam (b1 0.9, b2 0.999, eps 1e-8) updates the FP32 parameters.
 * All x / y / target / row arrays below are DEVICE pointers, row-major. */
typedef struct vemb_mlp vemb_mlp;
/* params: host array of vemb_mlp_num_params floats, or NULL for zeros.  Work
 * buffers are sized for up to max_batch rows.  Synchronises hip_stream. */
int vemb_mlp_create(const int32_t* dims, int n_dims, const float* params, int max_batch, void* hip_stream,
                    vemb_mlp** out);
int vemb_mlp_num_params(const vemb_mlp* n, int64_t* count);
int vemb_mlp_set_params(vemb_mlp* n, const float* params_host);
int vemb_mlp_get_params(vemb_mlp* n, float* params_host);
/* mean / std per output over `count` target rows (FP64 sums); std floored at
 * max(1e-6, rel_floor * largest std) so that near-constant outputs are not
 * magnified into noise. */
int vemb_mlp_fit_normalization(vemb_mlp* n, const float* targets, int count, float rel_floor);
int vemb_mlp_get_normalization(vemb_mlp* n, float* mean_host, float* std_host);
int vemb_mlp_set_normalization(vemb_mlp* n, const float* mean_host, const float* std_host);
/* y (batch x outputs) = denormalised network output for x (batch x inputs). */
int vemb_mlp_forward(vemb_mlp* n, const float* x, float* y, int batch);
/* Loss and gradient for one batch; grad (DEVICE, num_params floats) may be NULL;
 * loss (host) may be NULL, else the call synchronises. */
int vemb_mlp_gradients(vemb_mlp* n, const float* x, const float* targets, int batch, double* loss, float* grad);
/* One Adam step with the gradient of the last vemb_mlp_gradients / train step. */
int vemb_mlp_adam_step(vemb_mlp* n, float lr);
/* Gradient + Adam on the rows `rows[0..batch)` (DEVICE int32, indices into the
 * count rows of X and T; NULL = the first batch rows).  Rows outside 0..count-1
 * read as zeros.  loss (host) may be NULL, else the call synchronises. */
int vemb_mlp_train_step(vemb_mlp* n, const float* X, const float* T, int count, const int32_t* rows, int batch,
                        float lr, double* loss);
void vemb_mlp_destroy(vemb_mlp* n);

#ifdef __cplusplus
}
#endif
#endif /* VEMB_H */
