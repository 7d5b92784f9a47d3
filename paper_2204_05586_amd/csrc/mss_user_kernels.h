// Integrator kernels around a user-supplied field function.  This header is
// compiled at run time (hiprtc) by the sampler entry points, after the
// user's source, which defines
//
//   __device__ void mss_user_field(double t, const double* params, double* field);
//
// field arrives zeroed and receives f_x, f_y, f_z, f_q in Hz at time t (s);
// params is the simulation's parameter vector.  This is the counterpart of
// the paper's field function compiled into its integrator (Sec.
// "Compilation of integrator"): the user's code is inlined into the same
// interval operator as the field-program interpreter.
#pragma once

#include "mss_device.h"
#include "mss_work_device.h"

__device__ void mss_user_field(double t, const double* params, double* field);

struct MssUserField {};

// Found by argument-dependent lookup from the interval operator's templates.
__device__ __forceinline__ void field_eval(const MssUserField&, const double* __restrict__ params,
                                           double t, double f[4]) {
  f[0] = 0.0;
  f[1] = 0.0;
  f[2] = 0.0;
  f[3] = 0.0;
  mss_user_field(t, params, f);
}

extern "C" __global__ void __launch_bounds__(256) mss_user_integrate_2(const mss::IntervalGrid g) {
  mss::integrate_lanes<2>(MssUserField{}, g);
}

extern "C" __global__ void __launch_bounds__(256) mss_user_integrate_3(const mss::IntervalGrid g) {
  mss::integrate_lanes<3>(MssUserField{}, g);
}

// Every descriptor of a batch takes its field from the user function.
struct MssUserSource {
  __device__ __forceinline__ MssUserField operator()(const mss::IntegrateWorkArgs&,
                                                     const mss::SimDesc&) const {
    return MssUserField{};
  }
};

extern "C" __global__ void __launch_bounds__(256) mss_user_work_integrate(
    const mss::IntegrateWorkArgs A) {
  mss::work_integrate_loop(A, MssUserSource{});
}

extern "C" __global__ void __launch_bounds__(256, 2) mss_user_work_chained(
    const mss::IntegrateWorkArgs A) {
  mss::chained_integrate_loop(A, MssUserSource{});
}
