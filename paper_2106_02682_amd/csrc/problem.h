// Internal definition of a problem (shared by the C ABI in api.cpp and the batch in batch.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "alloc.h"
#include "host_model.h"
#include "kernels.h"

struct vemb_problem {
  vemb::Geometry g;
  int P = 0, n_op = 0, Ku = 0;
  vemb_options opt{};
  hipStream_t stream = nullptr;
  // The pair projection feeds only the next iteration (rho_t, Lambda), so it runs on
  // a side stream concurrently with the cluster update, the DFTs and the momentum
  // projections: fork after the X step, join at the end of the iteration.
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  int64_t t = 0;
  vemb::HostModel host;
  vemb::OpTables ops_host{};
  vemb::StepArgs a{};
  vemb::DeviceMemory mem;  // every device allocation of the problem
  // device fixed data
  double *H0 = nullptr, *Hd = nullptr, *tw = nullptr, *wk = nullptr;
  int* hd_index = nullptr;
  vemb::OpTables* ops = nullptr;
  // kernel timing (vemb_set_profiling)
  bool profiling = false;
  uint32_t prof_mask = 0;  // kernels timed (bit per vemb_kernel_id)
  int prof_every = 1;      // timed iterations: those with t a multiple of prof_every
  // asynchronous diagnostics: pinned host copies [lmin (P+1) | e_pair (P) | feas (P) | scal (4)]
  double* diag_host = nullptr;
  hipEvent_t diag_ev = nullptr;
  bool diag_pending = false;
  double adapt_scale = 1.0;   // joint scale of (mu, nu, eps) (vemb_options.adapt_every)
  double adapt_last = -1.0;   // feasErr at the last adaptation check, < 0 before the first
  double adapt_last_gap = -1.0;  // relative primal-dual gap at the last check
  std::vector<double> feas_hist;  // feasibility errors of the watchdog's checks (vemb_options.lb_every)
  struct Mark { int id; hipEvent_t start, stop; };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> free_events;
  double prof_ms[VEMB_K_COUNT] = {};
  bool v_valid = false;  // Vpair / Vmom hold eigenvectors of the previous iteration
  bool v_fp32 = false;   // ... found by FP32 solves (an FP64 solve orthonormalises them first)
  double* Kv = nullptr;   // eigenvectors of the bound matrices (pair blocks up to 128), kept between bounds
  bool k_valid = false;
  int64_t k_uses = 0;  // bound evaluations; every 16th restarts them cold (orthogonality drift)
  int tpb_pair = 256, tpb_mom = 256;  // threads per workgroup of the LDS solver (autotuned)
  // FP64 blocks above 64 (4-site clusters): scratch of the sign-function projections (else null)
  void* sign_pair = nullptr;
  void* sign_mom = nullptr;
  // Bound matrices above 128 (spectral slicing): last Ritz vectors (P x n, zero before the first
  // evaluation), shifts, per-block flags and their count
  double* slice_x = nullptr;
  double* slice_sigma = nullptr;
  int* slice_flags = nullptr;
  int* slice_nflag = nullptr;
  bool slice_started = false;
  int64_t prof_n[VEMB_K_COUNT] = {};
};

namespace vemb {
// The arithmetic of a mode's per-iteration eigensolves: FP64 for VEMB_FP64, FP32 for MIXED and FP32
// (state, diagnostics and vemb_refine stay FP64).
inline int solve_precision(int precision) { return precision == VEMB_FP64 ? VEMB_FP64 : VEMB_FP32; }
int fail(int code, const std::string& msg);
int hip_rc(hipError_t e, const char* what);
int tuned_tpb(int n, bool cplx, int precision, int count, hipStream_t st);
}  // namespace vemb

#define VEMB_TRY(expr)              \
  do {                              \
    int rc_ = (expr);               \
    if (rc_ != VEMB_OK) return rc_; \
  } while (0)
