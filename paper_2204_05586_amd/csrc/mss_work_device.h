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
  int32_t method, pad;
};

struct IntegrateWorkArgs {
  const SimDesc* sims;
  const mss_term* terms;
  unsigned long long* counter;
  int64_t n_items;
  int32_t n_sims;
  int32_t store_u;  // fused form: also write U_k (0: states only)
  // fused form (integrator and ordered product in one launch): per work
  // item a flag, 0 until the state leaving the item is in tile_out
  unsigned long long* flags;  // [n_items]
  double* tile_out;           // [n_items][6]
};

// Spin limit of the wait for the preceding item (each trip sleeps 2 x 64
// clocks: about 0.5 s in all, far above the longest legitimate wait, one
// item's integration).  Reaching it means the preceding item never
// published: the item's states are then written as NaN, and the wave never
// waits again (its later items are NaN too), so a launch ends within one
// limit of its normal time whatever happens.
constexpr uint32_t kChainSpinLimit = 1u << 23;

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
  interval_operator<N>(source(A, s), s.params, s.t_start, s.dt_out, s.dt, s.n_fine, s.tau,
                       s.frame, s.method, k, slice, sl, active, U, &tk);
  if (active && slice == 0) store_mat<N>(s.U + (size_t)k * 2 * N * N, U);
}

// Fused form of one work item (every descriptor integrates its whole
// sequence, k_first = 0): after its operators, the wave forms their ordered
// inclusive products with wave shuffles, takes the state entering the item
// (psi0 for the first item of a sequence, else the state the preceding item
// published: a chained single-pass scan), writes the states of its
// intervals and publishes the state leaving the item.  The preceding item
// was taken from the counter earlier, by a wave that is running and waits
// only on items before it, so the wait ends; a spin limit bounds it anyway.
template <int N, class Source>
__device__ __forceinline__ void work_item_scan(const IntegrateWorkArgs& A, const SimDesc& s,
                                               int64_t item, int64_t local, int lane,
                                               const Source& source, bool& degraded) {
  const int sl = s.slices_log2;
  const int per = 64 >> sl;                // intervals per item
  const int jl = lane >> sl;               // interval within the item
  const int slice = lane & ((1 << sl) - 1);
  const int64_t j = local * per + jl;      // interval within the sequence
  const bool active = j < s.k_count;
  Mat<N> P;
  double tk;
  interval_operator<N>(source(A, s), s.params, s.t_start, s.dt_out, s.dt, s.n_fine, s.tau,
                       s.frame, s.method, j, slice, sl, active, P, &tk);
  if (!active) set_identity<N>(P);
  if (A.store_u && active && slice == 0) store_mat<N>(s.U + (size_t)j * 2 * N * N, P);
  // inclusive products over the item's intervals, later on the left (the
  // slice-0 lanes hold the operators, 2^sl lanes apart)
  for (int d = 1; d < per; d <<= 1) {
    const Mat<N> o = shfl_up_mat<N>(P, d << sl);
    if (jl >= d) {
      Mat<N> t;
      matmul<N>(P, o, t);
      P = t;
    }
  }
  Mat<N> X = shfl_up_mat<N>(P, 1 << sl);
  if (jl == 0) set_identity<N>(X);
  // state entering the item
  const double* src = s.psi0;
  bool ok = true;
  if (local > 0) {
    ok = !degraded;
    uint32_t spins = 0;
    while (ok) {
      const unsigned long long f =
          __hip_atomic_load(A.flags + item - 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
      if (f != 0ull) break;
      if (++spins > kChainSpinLimit) ok = false;
      else __builtin_amdgcn_s_sleep(2);
    }
    // one wave-wide verdict (lanes read the same flag; this keeps them together)
    ok = __builtin_amdgcn_readfirstlane((int)ok) != 0;
    if (!ok) degraded = true;
    src = A.tile_out + (size_t)(item - 1) * 6;
  }
  double vr[N], vi[N];
#pragma unroll
  for (int a = 0; a < N; ++a) {
    vr[a] = ok ? src[2 * a] : __builtin_nan("");
    vi[a] = ok ? src[2 * a + 1] : __builtin_nan("");
  }
  // psi_j = X v (the state entering interval j)
  if (active && slice == 0) {
    double* o = s.psi + (size_t)j * 2 * N;
#pragma unroll
    for (int a = 0; a < N; ++a) {
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int b = 0; b < N; ++b) {
        re = fma(X.r[a][b], vr[b], re);
        re = fma(-X.i[a][b], vi[b], re);
        im = fma(X.r[a][b], vi[b], im);
        im = fma(X.i[a][b], vr[b], im);
      }
      o[2 * a] = re;
      o[2 * a + 1] = im;
    }
  }
  // the state leaving the item, from the lane of its last interval
  const int64_t left = s.k_count - local * per;
  const int jlast = (int)(left < per ? left : per) - 1;
  if (slice == 0 && jl == jlast) {
    double* out = A.tile_out + (size_t)item * 6;
    const bool last_item = left <= per;
#pragma unroll
    for (int a = 0; a < N; ++a) {
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int b = 0; b < N; ++b) {
        re = fma(P.r[a][b], vr[b], re);
        re = fma(-P.i[a][b], vi[b], re);
        im = fma(P.r[a][b], vi[b], im);
        im = fma(P.i[a][b], vr[b], im);
      }
      out[2 * a] = re;
      out[2 * a + 1] = im;
      if (last_item && s.psi_final) {
        s.psi_final[2 * a] = re;
        s.psi_final[2 * a + 1] = im;
      }
    }
    __hip_atomic_store(A.flags + item, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Persistent loop: each wave takes items from the counter until it passes
// the item count, so every wave exits once the queue is drained.  In the
// plain form no wave waits for another; in the fused form (Fused = true) a
// wave waits only for the item before its own (work_item_scan).
template <bool Fused = false, class Source>
__device__ __forceinline__ void work_integrate_loop(const IntegrateWorkArgs& A,
                                                    const Source& source) {
  const int lane = threadIdx.x & 63;
  bool degraded = false;  // fused form: set once a wait of this wave timed out
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
    if (Fused) {
      if (s.spin_twice == 2) work_item_scan<3>(A, s, item, local, lane, source, degraded);
      else work_item_scan<2>(A, s, item, local, lane, source, degraded);
    } else {
      if (s.spin_twice == 2) work_item<3>(A, s, local, lane, source);
      else work_item<2>(A, s, local, lane, source);
    }
  }
}

}  // namespace mss
