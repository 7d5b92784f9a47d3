// Internal interface between the C-ABI layer (mss_api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "mss_device.h"

namespace mss {

// Scan tiling: one wave owns kScanTile consecutive matrices, each lane a
// run of kScanPerLane of them.
constexpr int kScanPerLane = 4;
constexpr int kScanTile = 64 * kScanPerLane;

struct IntegrateArgs {
  FieldProgram fp;
  IntervalGrid g;
};

// host helpers shared by the C-ABI translation units (mss_api.hip)
mss_status api_fail(mss_status s, const char* fmt, ...);
mss_status api_fail_text(mss_status s, const std::string& msg);
mss_status api_ok();
mss_status api_hip_fail(hipError_t e, const char* what);
std::string api_last_error_copy();
mss_status api_validate_problem(const mss_problem* p);
// a spin-1 problem with a term on U_1, U_2, V_1 or V_2 (the full su(3) basis)
bool api_full_basis(const mss_problem* p);
// the term checks of api_validate_problem for a term list on its own
mss_status api_validate_terms(int spin_twice, const mss_term* terms, int n_terms, int n_params);
// a problem run with a sampler: its parameter vector covers what the
// sampler reads, and its spin suits the sampler's components
mss_status api_sampler_check_problem(mss_sampler s, const mss_problem* p);
int api_device_cu_count();
int api_plan_slices(int64_t K, int32_t L, int cu);
int api_ilog2(int x);
// launch shape (lane-slices per interval, block size) of one simulation;
// given: whether the caller fixed the slices
mss_status api_resolve_launch(const mss_problem* p, const mss_launch* in, int* slices, int* block,
                              bool* given);
// lane segments of a grid launch with S0 slices (IntervalGrid), given the
// number of waves that run at once (slots; 0: unknown, one segment)
void api_plan_lane_segments(IntervalGrid& g, int S0, bool given, int64_t slots);
// waves of a planned grid launch
int64_t api_grid_waves(const IntervalGrid& g);
// waves of integrate_kernel<N> in blocks of `block` threads that run at once
// on the current device (0 if unknown)
int64_t integrate_slots(int N, int block);

// work-queue integrator of a user sampler's module on the current device
// (loads the module there on first use)
mss_status api_sampler_work_function(mss_sampler s, hipFunction_t* fn);

hipError_t launch_integrate(int N, const IntegrateArgs& a, int block, hipStream_t st);
hipError_t launch_scan_reduce(int N, const double* M, int64_t n, double* agg, hipStream_t st);
hipError_t launch_scan_apply(int N, const double* M, int64_t n, const double* start, double* before,
                             double* after_last, hipStream_t st, double* spin = nullptr);

// levels 1 and 2 of a two-level single-sequence scan in one workgroup
// (n1 level-1 elements in at most 16 tiles)
hipError_t launch_scan_top(int N, const double* M1, int64_t n1, const double* start,
                           double* before1, hipStream_t st);

hipError_t launch_spin_projection(int N, const double* psi, int64_t K, double* out,
                                  hipStream_t st);

}  // namespace mss
