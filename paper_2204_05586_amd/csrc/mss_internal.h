// Internal interface between the C-ABI layer (mss_api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "mss_device.h"

namespace mss {

// Scan tiling: one wave owns kScanTile consecutive matrices, each lane a
// run of kScanPerLane of them.
constexpr int kScanPerLane = 4;
constexpr int kScanTile = 64 * kScanPerLane;

struct IntegrateArgs {
  FieldProgram fp;
  const double* params;
  double* U;
  double* time;
  double t_start;
  double dt_out;  // Dt
  double dt;      // Dt / L
  int64_t K;
  int32_t L;
  int32_t tau;
  int32_t frame;
  int32_t slices_log2;
};

hipError_t launch_integrate(int N, const IntegrateArgs& a, int block, hipStream_t st);
hipError_t launch_scan_reduce(int N, const double* M, int64_t n, double* agg, hipStream_t st);
hipError_t launch_scan_apply(int N, const double* M, int64_t n, const double* start, double* before,
                             double* after_last, hipStream_t st);

}  // namespace mss
