// Device side of work sets (mss_work.h): the descriptor of one sequence and
// the persistent work-queue integrator, generic over the field source so
// that the field-program kernel and a user sampler's kernel (compiled at
// run time) share it.
#pragma once

#include "mss_device.h"

namespace mss {

struct SimDesc {
  double t_start, dt_out, dt;
  int64_t k_first;   // first interval integrated by this descriptor
  int64_t k_count;   // intervals integrated (0: none)
  int64_t K_total;   // length of the whole sequence (for the scan)
  int64_t item_off;  // first integrator work item
  const double* params;
  const double* psi0;  // [N]
  double* psi;         // [K_total][N]
  double* psi_final;   // [N] or null
  double* U;           // [K_total][N][N]
  double* scan_ws;     // scan levels 1..top: per level [n_l][N][N] then [n_l][N]
  int32_t spin_twice, n_terms, term_off, n_fine;
  int32_t tau, frame, slices_log2, top;  // top: scan levels above 0; -1: no scan
  int32_t method, full;  // full: spin-1 in the full su(3) basis
};

struct IntegrateWorkArgs {
  const SimDesc* sims;
  const mss_term* terms;
  unsigned long long* counter;
  int64_t n_items;
  int32_t n_sims;
};

__device__ __forceinline__ int64_t wave_broadcast(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffff));
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return ((int64_t)hi << 32) | (uint32_t)lo;
}

// One work item: 64 / S consecutive intervals of descriptor s, S lane-slices
// each.  source(A, s) gives the field source of the descriptor.
template <int N, class Source>
__device__ __forceinline__ void work_item(const IntegrateWorkArgs& A, const SimDesc& s,
                                          int64_t local, int lane, const Source& source) {
  const int sl = s.slices_log2;
  const int64_t j = local * (64 >> sl) + (lane >> sl);  // interval within the range
  const int slice = lane & ((1 << sl) - 1);
  const bool active = j < s.k_count;
  const int64_t k = s.k_first + j;
  Mat<N> U;
  double tk;
  using Terms = decltype(source(A, s));
  bool done = false;
  if constexpr (N == 3 && has_full_basis<Terms>::value) {
    if (s.full) {
      interval_operator<3, true>(source(A, s), s.params, s.t_start, s.dt_out, s.dt, s.n_fine,
                                 s.tau, s.frame, s.method, k, slice, sl, active, U, &tk);
      done = true;
    }
  }
  if (!done)
    interval_operator<N>(source(A, s), s.params, s.t_start, s.dt_out, s.dt, s.n_fine, s.tau,
                         s.frame, s.method, k, slice, sl, active, U, &tk);
  if (active && slice == 0) store_mat<N>(s.U + (size_t)k * 2 * N * N, U);
}

// Persistent loop: each wave takes items from the counter until it passes
// the item count, so every wave exits once the queue is drained and no wave
// waits for another.
template <class Source>
__device__ __forceinline__ void work_integrate_loop(const IntegrateWorkArgs& A,
                                                    const Source& source) {
  const int lane = threadIdx.x & 63;
  for (;;) {
    int64_t item = 0;
    if (lane == 0) item = (int64_t)atomicAdd(A.counter, 1ull);
    item = wave_broadcast(item);
    if (item >= A.n_items) break;
    int lo = 0, hi = A.n_sims - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (A.sims[mid].item_off <= item) lo = mid;
      else hi = mid - 1;
    }
    const SimDesc& s = A.sims[lo];
    const int64_t local = item - s.item_off;
    if (s.spin_twice == 2) work_item<3>(A, s, local, lane, source);
    else work_item<2>(A, s, local, lane, source);
  }
}

}  // namespace mss
