// PSD projection of one large symmetric matrix by the scaled Newton-Schulz sign iteration on
// matrix cores (polar.hip).
#pragma once

#include <vector>

#include "common.h"

namespace vemb {

// Scaling factors a_k of the iteration for a resolved fraction l0 of ||A||_F (host), until the
// resolved bound l_k is within `stop` of 1.
std::vector<double> ns_schedule(double l0, double stop = 1e-15);

// out = Pi((in + in^T) / 2) for one ld x ld matrix, ld a multiple of 16 (row-major, FP64).
// work: 4 ld^2 + 64 doubles of device scratch.  `in` may alias `out`.  Enqueued on st.
hipError_t launch_psd_project_ns(const double* in, double* out, int ld, double* work, const std::vector<double>& sched,
                                 hipStream_t st);

// Resolved fraction used by the library: eigenvalues below 1e-14 ||A||_F may stay partly unresolved.
constexpr double kNsResolved = 1e-14;
constexpr double kNsStop = 1e-15;
// FP32 iterations: eigenvalues below 1e-6 ||A||_F, and the last 1e-7 of the convergence to 1 (FP32
// rounding), are left.
constexpr double kNsResolved32 = 1e-6;
constexpr double kNsStop32 = 1e-7;

// The schedule for kNsResolved, computed once on the host.
const std::vector<double>& ns_schedule_resolved();

// Allocation-free projections: the largest matrix and the scratch words (4 n^2 + 64) they need.
constexpr int kStaticSignMaxN = 512;
constexpr size_t kStaticSignWords = 4 * (size_t)kStaticSignMaxN * kStaticSignMaxN + 64;
constexpr int kMaxDevices = 64;

// Device address of the current device's static scratch array (kStaticSignWords doubles), looked up
// with hipGetSymbolAddress on the first call for each device and kept.
hipError_t static_sign_scratch(double** ptr);

}  // namespace vemb
