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

// Chained runs: the states are formed inside the integrator's launch.  Each
// simulation has one slot through which its work items pass the state on:
// item r of the simulation writes the state leaving its last interval and
// then its tag, chain_tag(call, r); item r + 1 waits for that tag.
struct ChainSlot {
  unsigned long long tag;
  unsigned long long pad;
  double psi[6];  // N complex
};
static_assert(sizeof(ChainSlot) == 64, "one chain slot is 64 bytes");

// Head of a chained run's workspace: the item counter, the number of the
// last call (incremented by the reset kernel before each run) and the tag of
// a call whose bounded wait ran out (0 if none ever did).
struct ChainSync {
  unsigned long long counter;
  unsigned long long epoch;
  unsigned long long failed;
  unsigned long long pad[29];
};
static_assert(sizeof(ChainSync) == 256, "the chain head is one 256-byte block");

struct IntegrateWorkArgs {
  const SimDesc* sims;
  const mss_term* terms;
  unsigned long long* counter;
  int64_t n_items;
  int32_t n_sims;
  // chained runs only: the interleaved item order and the chain slots.
  // Items go round by round (item r of every simulation that has one, then
  // item r + 1, ...), simulations within a round by decreasing item count,
  // so a round's simulations are a prefix of `order`.  Rounds with the same
  // simulation count form a group: group g starts at item group_item0[g]
  // and round group_round0[g] and holds group_count[g] simulations per round.
  int32_t n_groups;
  const int64_t* group_item0;   // [n_groups]
  const int64_t* group_round0;  // [n_groups]
  const int32_t* group_count;   // [n_groups]
  const int32_t* order;         // [n_sims]
  ChainSlot* slots;             // [n_sims]
  ChainSync* sync;
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

// ---------------------------------------------------------------------------
// chained runs
// ---------------------------------------------------------------------------
// The finalizer of SplitMix64 (Steele, Lea and Flood, 2014): a bijection of
// 64-bit words.  The tag of item r in call c is the image of c 2^40 + r, so
// no two (call, item) pairs share a tag (r < 2^40, calls counted modulo
// 2^24) and whatever a slot held before matches only by a 2^-64 chance.
__device__ __forceinline__ unsigned long long chain_tag(unsigned long long call, int64_t r) {
  unsigned long long c = (call << 40) | ((unsigned long long)r & ((1ull << 40) - 1));
  c ^= c >> 30;
  c *= 0xbf58476d1ce4e5b9ull;
  c ^= c >> 27;
  c *= 0x94d049bb133111ebull;
  c ^= c >> 31;
  return c;
}

// Upper bound of one wait, in ticks of the 100 MHz real-time counter (10 s,
// far beyond any real wait: an item waits at most for the items dequeued
// before it).
constexpr unsigned long long kChainWaitTicks = 1000000000ull;

// Every lane polls until *p == want; false when the bound ran out.
__device__ __forceinline__ bool chain_wait(const unsigned long long* p, unsigned long long want) {
  const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
  for (;;) {
    const unsigned long long v = __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    if (__all(v == want)) return true;
    if (__builtin_amdgcn_s_memrealtime() - t0 > kChainWaitTicks) return false;
    __builtin_amdgcn_s_sleep(2);
  }
}

// One chained item: the operators of 64 / S consecutive intervals (written
// to U when the descriptor has one), their ordered products within the
// wave, the entering state from the item before (or psi0), and every
// interval's entering state; the state leaving the last interval goes to
// the slot (and to psi_final after the last interval of the simulation).
template <int N, class Source>
__device__ __forceinline__ void chained_item(const IntegrateWorkArgs& A, const SimDesc& s,
                                             ChainSlot* slot, int64_t local, int lane,
                                             unsigned long long call, const Source& source) {
  const int sl = s.slices_log2;
  const int per = 64 >> sl;
  const int jl = lane >> sl;  // interval within the item
  const int slice = lane & ((1 << sl) - 1);
  const int64_t k = local * per + jl;
  const bool active = k < s.K_total;
  Mat<N> P;
  double tk;
  using Terms = decltype(source(A, s));
  bool done = false;
  if constexpr (N == 3 && has_full_basis<Terms>::value) {
    if (s.full) {
      interval_operator<3, true>(source(A, s), s.params, s.t_start, s.dt_out, s.dt, s.n_fine,
                                 s.tau, s.frame, s.method, k, slice, sl, active, P, &tk);
      done = true;
    }
  }
  if (!done)
    interval_operator<N>(source(A, s), s.params, s.t_start, s.dt_out, s.dt, s.n_fine, s.tau,
                         s.frame, s.method, k, slice, sl, active, P, &tk);
  if (active && slice == 0 && s.U) store_mat<N>(s.U + (size_t)k * 2 * N * N, P);
  if (!active) set_identity<N>(P);
  // P_j = U_j ... U_0 over the item's intervals (lanes with slice 0; the
  // other lanes compute values nobody reads)
  for (int d = 1; d < per; d <<= 1) {
    const Mat<N> o = shfl_up_mat<N>(P, d << sl);
    if (jl >= d) {
      Mat<N> t;
      matmul<N>(P, o, t);
      P = t;
    }
  }
  // entering state of the item
  double xr[N], xi[N];
  const double* src = s.psi0;
  if (local > 0) {
    if (!chain_wait(&slot->tag, chain_tag(call, local - 1)) && lane == 0)
      __hip_atomic_store(&A.sync->failed, chain_tag(call, local - 1), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    src = slot->psi;
  }
#pragma unroll
  for (int a = 0; a < N; ++a) {
    xr[a] = src[2 * a];
    xi[a] = src[2 * a + 1];
  }
  // y = P_j x: the state leaving interval j; the one entering it is the
  // previous interval's leaving state (x for the first)
  double yr[N], yi[N];
#pragma unroll
  for (int a = 0; a < N; ++a) {
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int b = 0; b < N; ++b) {
      re = fma(P.r[a][b], xr[b], re);
      re = fma(-P.i[a][b], xi[b], re);
      im = fma(P.r[a][b], xi[b], im);
      im = fma(P.i[a][b], xr[b], im);
    }
    yr[a] = re;
    yi[a] = im;
  }
  double er[N], ei[N];
#pragma unroll
  for (int a = 0; a < N; ++a) {
    er[a] = __shfl_up(yr[a], 1 << sl, 64);
    ei[a] = __shfl_up(yi[a], 1 << sl, 64);
    if (jl == 0) {
      er[a] = xr[a];
      ei[a] = xi[a];
    }
  }
  if (active && slice == 0) {
    double* o = s.psi + (size_t)k * 2 * N;
#pragma unroll
    for (int a = 0; a < N; ++a) {
      o[2 * a] = er[a];
      o[2 * a + 1] = ei[a];
    }
    const int64_t last = (local + 1) * per < s.K_total ? (local + 1) * per - 1 : s.K_total - 1;
    if (k == last) {
      if (k == s.K_total - 1) {
        if (s.psi_final) {
#pragma unroll
          for (int a = 0; a < N; ++a) {
            s.psi_final[2 * a] = yr[a];
            s.psi_final[2 * a + 1] = yi[a];
          }
        }
      } else {
#pragma unroll
        for (int a = 0; a < N; ++a) {
          slot->psi[2 * a] = yr[a];
          slot->psi[2 * a + 1] = yi[a];
        }
        __hip_atomic_store(&slot->tag, chain_tag(call, local), __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

// Persistent loop of a chained run.  An item waits only for the item of
// its simulation one round earlier, which was taken from the counter
// before it by a wave that is running, so every wait ends; every wave exits
// once the queue is drained.
template <class Source>
__device__ __forceinline__ void chained_integrate_loop(const IntegrateWorkArgs& A,
                                                       const Source& source) {
  const int lane = threadIdx.x & 63;
  const unsigned long long call =
      __hip_atomic_load(&A.sync->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (;;) {
    int64_t item = 0;
    if (lane == 0) item = (int64_t)atomicAdd(A.counter, 1ull);
    item = wave_broadcast(item);
    if (item >= A.n_items) break;
    int lo = 0, hi = A.n_groups - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (A.group_item0[mid] <= item) lo = mid;
      else hi = mid - 1;
    }
    const int64_t off = item - A.group_item0[lo];
    const int64_t cnt = A.group_count[lo];
    const int64_t round = A.group_round0[lo] + off / cnt;
    const int sim = A.order[off % cnt];
    const SimDesc& s = A.sims[sim];
    if (s.spin_twice == 2) chained_item<3>(A, s, A.slots + sim, round, lane, call, source);
    else chained_item<2>(A, s, A.slots + sim, round, lane, call, source);
  }
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
