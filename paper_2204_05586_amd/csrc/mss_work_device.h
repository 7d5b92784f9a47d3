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
// simulation has one slot through which its work units pass the state on.
// The state (N complex = 4N 32-bit halves) travels in 4N 64-bit words, each
// holding one half in its low 32 bits and the tag r + 1 of the unit r that
// wrote it in its high 32 bits.  Words are written (exchange) and read
// (compare-and-swap, chain_read) only by atomic read-modify-write
// operations at agent scope, which take effect at the device's coherence
// point whichever XCD issues them, so a reader sees each word either old or
// new and needs no cache maintenance or fence (a plain or relaxed load, by
// contrast, can keep returning a line its XCD's L2 holds): once all
// 4N words carry the tag it waits for, they hold that unit's state.  A
// reset kernel zeroes every slot before each run, so a word can only hold
// 0 or the tag of an earlier unit of the same run.
struct ChainSlot {
  unsigned long long w[16];  // 4N words used
};
static_assert(sizeof(ChainSlot) == 128, "one chain slot is 128 bytes");

// Head of a chained run's workspace: the unit counter and the tag of a
// wait that ran out in this run (0 if none did), both cleared by the reset
// kernel.
struct ChainSync {
  unsigned long long counter;
  unsigned long long failed;
  unsigned long long pad[30];
};
static_assert(sizeof(ChainSync) == 256, "the chain head is one 256-byte block");

struct IntegrateWorkArgs {
  const SimDesc* sims;
  const mss_term* terms;
  unsigned long long* counter;
  int64_t n_items;
  int32_t n_sims;
  // chained runs only (n_items then counts units of kChainPerLane 64 / S
  // intervals): the interleaved unit order, the chain slots and the bound
  // of one wait (ticks of the 100 MHz real-time counter).  Units go round by round
  // (unit r of every simulation that has one, then unit r + 1, ...),
  // simulations within a round by decreasing unit count, so a round's
  // simulations are a prefix of `order`.  Rounds with the same simulation
  // count form a group: group g starts at unit group_item0[g] and round
  // group_round0[g] and holds group_count[g] simulations per round.
  int32_t n_groups;
  const int64_t* group_item0;   // [n_groups]
  const int64_t* group_round0;  // [n_groups]
  const int32_t* group_count;   // [n_groups]
  const int32_t* order;         // [n_sims]
  ChainSlot* slots;             // [n_sims]
  ChainSync* sync;
  unsigned long long wait_ticks;
};

__device__ __forceinline__ int64_t wave_broadcast(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffff));
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return ((int64_t)hi << 32) | (uint32_t)lo;
}

// Largest i in [0, n) with key(i) <= x, for a non-decreasing key with
// key(0) <= x, found by the whole wave: each step splits what is left into
// 64 buckets, lane l tests the first key of bucket l, and the highest lane
// whose key is <= x picks the bucket.  Two dependent vector loads for 4096
// keys instead of twelve dependent scalar loads of a binary search.
template <class Key>
__device__ __forceinline__ int wave_search(const Key& key, int n, int64_t x, int lane) {
  int base = 0, span = n;
  while (span > 1) {
    const int stride = (span + 63) >> 6;
    const bool ok = lane * stride < span && key(base + lane * stride) <= x;
    const unsigned long long m = __ballot(ok);
    const int last = 63 - __builtin_clzll(m);  // m != 0: key(base) <= x
    base += last * stride;
    span = min(stride, span - last * stride);
  }
  return base;
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
// Default bound of one wait, in ticks of the 100 MHz real-time counter
// (10 s, far beyond any real wait: a unit waits at most for the units
// dequeued before it).
constexpr unsigned long long kChainWaitTicks = 1000000000ull;

// The current value of a word, read by an atomic compare-and-swap of 0
// with 0 (it writes only a 0 that is already there): a real read-modify-
// write, which the compiler cannot turn into a plain load (as it does with
// an idempotent fetch-add or fetch-or) and which takes effect at the
// device's coherence point like the work counter's increments.
__device__ __forceinline__ unsigned long long chain_read(unsigned long long* p) {
  unsigned long long v = 0ull;
  __hip_atomic_compare_exchange_strong(p, &v, 0ull, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return v;
}

// A wave-uniform truth value as a scalar, so that branches on it are
// scalar branches and never split the wave's execution mask.
__device__ __forceinline__ bool wave_uniform(bool b) {
  return __builtin_amdgcn_readfirstlane((int)b) != 0;
}

// The state the unit with tag `tag` left in the slot (every lane receives
// it): lanes 0 .. 4N - 1 hold one word each, v (read earlier), and read it
// again until all carry the tag.  The loop's exits are wave-uniform.
// Returns false when the wait ran past wait_ticks (it then writes its tag
// into the failure word), or when a wait of this run already had (the
// kernel then only drains its queue; the states are undefined).
template <int N>
__device__ __forceinline__ bool chain_receive(ChainSlot* slot, unsigned tag, ChainSync* sync,
                                              unsigned long long wait_ticks, int lane,
                                              unsigned long long v, double* xr, double* xi) {
  const bool mine = lane < 4 * N;
  bool ok = true;
  const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
  for (;;) {
    if (wave_uniform(__all(!mine || (unsigned)(v >> 32) == tag))) break;
    // not there yet: give up at once if a wait of this run already ran out
    unsigned long long f = 0ull;
    if (lane == 0) f = chain_read(&sync->failed);
    if (wave_uniform(f != 0ull)) {
      ok = false;
      break;
    }
    if (__builtin_amdgcn_s_memrealtime() - t0 > wait_ticks) {
      ok = false;
      if (lane == 0)
        (void)__hip_atomic_exchange(&sync->failed, (unsigned long long)tag, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    __builtin_amdgcn_s_sleep(2);
    if (mine) v = chain_read(&slot->w[lane]);
  }
  const unsigned lo32 = (unsigned)v;
#pragma unroll
  for (int a = 0; a < N; ++a) {
    const unsigned long long rl = (unsigned)__shfl((int)lo32, 4 * a, 64);
    const unsigned long long rh = (unsigned)__shfl((int)lo32, 4 * a + 1, 64);
    const unsigned long long il = (unsigned)__shfl((int)lo32, 4 * a + 2, 64);
    const unsigned long long ih = (unsigned)__shfl((int)lo32, 4 * a + 3, 64);
    xr[a] = __longlong_as_double((long long)(rl | (rh << 32)));
    xi[a] = __longlong_as_double((long long)(il | (ih << 32)));
  }
  return ok;
}

// Lanes 0 .. 4N - 1 write the state (the same in every lane) into the slot
// with tag `tag`.
template <int N>
__device__ __forceinline__ void chain_send(ChainSlot* slot, unsigned tag, int lane,
                                           const double* xr, const double* xi) {
  const int a = lane >> 2;
  double d = 0.0;
#pragma unroll
  for (int b = 0; b < N; ++b)
    if (a == b) d = (lane & 2) ? xi[b] : xr[b];
  const unsigned long long bits = (unsigned long long)__double_as_longlong(d);
  const unsigned long long half = (lane & 1) ? (bits >> 32) : (bits & 0xffffffffull);
  if (lane < 4 * N)
    (void)__hip_atomic_exchange(&slot->w[lane], ((unsigned long long)tag << 32) | half,
                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Intervals per lane group in a chained unit: a unit is 64 / S groups of
// kChainPerLane consecutive intervals.  More than one cuts the unit's scan
// and hand-off per interval; a group's earlier operators wait in LDS while
// the last is integrated, so the integration needs no more registers.
constexpr int kChainPerLane = 3;
// doubles of LDS per wave for the parked operators (spin-1 size)
constexpr int kChainParkDoubles = (kChainPerLane - 1) * 2 * 3 * 3 * 64;

// A parked operator in LDS: 2 N^2 doubles per lane, element e of lane l at
// [e * 64 + l] (64 consecutive doubles per element, no bank conflicts).
template <int N>
__device__ __forceinline__ void park_mat(double* __restrict__ lds, int lane, const Mat<N>& m) {
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int b = 0; b < N; ++b) {
      lds[(2 * (a * N + b)) * 64 + lane] = m.r[a][b];
      lds[(2 * (a * N + b) + 1) * 64 + lane] = m.i[a][b];
    }
}

template <int N>
__device__ __forceinline__ void unpark_mat(const double* __restrict__ lds, int lane, Mat<N>& m) {
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int b = 0; b < N; ++b) {
      m.r[a][b] = lds[(2 * (a * N + b)) * 64 + lane];
      m.i[a][b] = lds[(2 * (a * N + b) + 1) * 64 + lane];
    }
}

// One chained unit: 64 / S groups of E = kChainPerLane consecutive
// intervals of one simulation, from interval E unit 64 / S on; lanes
// jS .. jS + S - 1 form group j.  The operators (written to U when the
// descriptor has one), the group products Q_j = U_{Ej+E-1} ... U_{Ej}, their
// ordered products within the wave, the entering state (psi0 for the
// simulation's first unit, otherwise the state the unit before left in the
// slot) and every interval's entering state; the state leaving the unit
// goes to the slot, or to psi_final after the simulation's last interval.
// Every branch on the unit's shape is wave-uniform.  lds: this wave's
// kChainParkDoubles doubles.
template <int N, class Source>
__device__ __forceinline__ void chained_unit(const IntegrateWorkArgs& A, const SimDesc& s,
                                             ChainSlot* slot, int64_t unit, int lane,
                                             double* __restrict__ lds, const Source& source) {
  constexpr int E = kChainPerLane;
  constexpr int kPark = 2 * N * N * 64;  // doubles per parked operator
  const int sl = s.slices_log2;
  const int per = 64 >> sl;   // groups in the unit
  const int jl = lane >> sl;  // this lane's group
  const int slice = lane & ((1 << sl) - 1);
  const int64_t span = (int64_t)per * E;
  const int64_t kb = unit * span;
  const int64_t k0 = kb + (int64_t)jl * E;  // the group's first interval
  using Terms = decltype(source(A, s));
  // the state the unit before left is read now: with a round's units spread
  // over the queue it is usually there already, and the read's round trip
  // then overlaps this unit's integration
  const bool first = wave_uniform(unit == 0);
  unsigned long long early = 0ull;
  if (!first && lane < 4 * N) early = chain_read(&slot->w[lane]);
  // Q_j = U_{k0+E-1} ... U_{k0}: each operator but the last is parked while
  // the next is integrated (one copy of the integration code: the loop is
  // not unrolled), so that nothing but parked operators outlives an
  // integration
  Mat<N> U;
#pragma unroll 1
  for (int e = 0;; ++e) {
    const int64_t k = k0 + e;
    const bool active = k < s.K_total;
    double tk;
    bool done = false;
    if constexpr (N == 3 && has_full_basis<Terms>::value) {
      if (s.full) {
        interval_operator<3, true, true>(source(A, s), s.params, s.t_start, s.dt_out, s.dt,
                                         s.n_fine, s.tau, s.frame, s.method, k, slice, sl,
                                         active, U, &tk);
        done = true;
      }
    }
    if (!done)
      interval_operator<N, false, true>(source(A, s), s.params, s.t_start, s.dt_out, s.dt,
                                        s.n_fine, s.tau, s.frame, s.method, k, slice, sl,
                                        active, U, &tk);
    if (active && slice == 0 && s.U) store_mat<N>(s.U + (size_t)k * 2 * N * N, U);
    if (!active) set_identity<N>(U);
    if (e + 1 == E) break;
    park_mat<N>(lds + e * kPark, lane, U);
  }
  Mat<N> P = U;
#pragma unroll
  for (int e = E - 2; e >= 0; --e) {
    Mat<N> Ue, t;
    unpark_mat<N>(lds + e * kPark, lane, Ue);
    matmul<N>(P, Ue, t);
    P = t;
  }
  // P_j = Q_j ... Q_0 over the unit's groups (lanes with slice 0; the other
  // lanes compute values nobody reads)
  for (int d = 1; d < per; d <<= 1) {
    const Mat<N> o = shfl_up_mat<N>(P, d << sl);
    if (jl >= d) {
      Mat<N> t;
      matmul<N>(P, o, t);
      P = t;
    }
  }
  // the entering state: psi0, or what the unit before left
  double xr[N], xi[N];
  if (first) {
#pragma unroll
    for (int a = 0; a < N; ++a) {
      xr[a] = s.psi0[2 * a];
      xi[a] = s.psi0[2 * a + 1];
    }
  } else {
    (void)chain_receive<N>(slot, (unsigned)unit, A.sync, A.wait_ticks, lane, early, xr, xi);
  }
  // y = P_j x: the state leaving group j; the one entering it is the group
  // before's leaving state (x for the first), and the parked operators
  // carry it through the group's earlier intervals
  double yr[N], yi[N];
  matvec<N>(P, xr, xi, yr, yi);
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
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (slice == 0 && k0 + e < s.K_total) {
      double* o = s.psi + (size_t)(k0 + e) * 2 * N;
#pragma unroll
      for (int a = 0; a < N; ++a) {
        o[2 * a] = er[a];
        o[2 * a + 1] = ei[a];
      }
    }
    if (e + 1 < E) {
      Mat<N> Ue;
      unpark_mat<N>(lds + e * kPark, lane, Ue);
      double fr[N], fi[N];
      matvec<N>(Ue, er, ei, fr, fi);
#pragma unroll
      for (int a = 0; a < N; ++a) {
        er[a] = fr[a];
        ei[a] = fi[a];
      }
    }
  }
  // the state leaving the unit: that of the group holding its last interval
  const int64_t n_here = s.K_total - kb < span ? s.K_total - kb : span;
  const int last = ((int)(n_here - 1) / E) << sl;
#pragma unroll
  for (int a = 0; a < N; ++a) {
    xr[a] = __shfl(yr[a], last, 64);
    xi[a] = __shfl(yi[a], last, 64);
  }
  // Both outputs are written by lane-indexed selects under wave-uniform
  // conditions: an if / else-if with a one-lane branch here made the
  // compiler build the persistent loop as a divergent loop, in which a
  // wave could reach the next dequeue without lane 0 and run a unit twice.
  const bool more = wave_uniform(kb + span < s.K_total);
  if (more) chain_send<N>(slot, (unsigned)(unit + 1), lane, xr, xi);
  double f = 0.0;
#pragma unroll
  for (int a = 0; a < N; ++a) {
    if (lane == 2 * a) f = xr[a];
    if (lane == 2 * a + 1) f = xi[a];
  }
  if (!more && s.psi_final && lane < 2 * N) s.psi_final[lane] = f;
}

// Persistent loop of a chained run.  A unit waits only for the unit of its
// simulation one round earlier, which was taken from the counter before it
// by a wave that is running, so every wait ends; every wave exits once the
// queue is drained.
template <class Source>
__device__ __forceinline__ void chained_integrate_loop(const IntegrateWorkArgs& A,
                                                       const Source& source) {
  const int lane = threadIdx.x & 63;
  // each wave's parking space for its lanes' parked operators; the launches use
  // 256-lane blocks, and a wider one fails the run instead of overrunning it
  __shared__ double park[4 * kChainParkDoubles];
  if (blockDim.x > 256) {
    if (threadIdx.x == 0)
      (void)__hip_atomic_exchange(&A.sync->failed, ~0ull, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  double* lds = park + (threadIdx.x >> 6) * kChainParkDoubles;
  int64_t item = 0;
  if (lane == 0) item = (int64_t)atomicAdd(A.counter, 1ull);
  item = wave_broadcast(item);
  while (item < A.n_items) {
    // every lane must be here: a wave without lane 0 would take no unit from
    // the counter and broadcast another lane's 0 instead; it stops and
    // marks the run failed (never seen with the loop compiled uniform)
    if (__builtin_amdgcn_read_exec() != ~0ull) {
      if (lane == __builtin_amdgcn_readfirstlane(lane))
        (void)__hip_atomic_exchange(&A.sync->failed, ~0ull, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    // while a whole grid's worth of units remains, the next unit is taken
    // now, so the counter's round trip overlaps this unit's work (a held unit
    // is younger than the one its wave works on, so the oldest unfinished
    // unit always runs and every wait still ends); near the end it is taken
    // afterwards, so that the last units go to idle waves
    const bool ahead = item + (int64_t)gridDim.x * (blockDim.x >> 6) < A.n_items;
    int64_t next = 0;
    if (ahead && lane == 0) next = (int64_t)atomicAdd(A.counter, 1ull);
    const int lo = wave_search([&](int i) { return A.group_item0[i]; }, A.n_groups, item, lane);
    // the unit's round and simulation, made explicitly wave-uniform so that
    // every branch on the descriptor is a scalar branch
    const int64_t off = item - A.group_item0[lo];
    const int64_t cnt = A.group_count[lo];
    const int64_t round = wave_broadcast(A.group_round0[lo] + off / cnt);
    const int sim = __builtin_amdgcn_readfirstlane(A.order[off % cnt]);
    const SimDesc& s = A.sims[sim];
    if (s.spin_twice == 2) chained_unit<3>(A, s, A.slots + sim, round, lane, lds, source);
    else chained_unit<2>(A, s, A.slots + sim, round, lane, lds, source);
    if (!ahead && lane == 0) next = (int64_t)atomicAdd(A.counter, 1ull);
    item = wave_broadcast(next);
  }
}

// Persistent loop: each wave takes items from the counter until it passes
// the item count, so every wave exits once the queue is drained and no wave
// waits for another.  While a whole grid's worth of items remains, the next
// item is taken before the current one is worked on, so the counter's round
// trip overlaps that work; near the end it is taken afterwards, so that the
// last items go to idle waves.
template <class Source>
__device__ __forceinline__ void work_integrate_loop(const IntegrateWorkArgs& A,
                                                    const Source& source) {
  const int lane = threadIdx.x & 63;
  int64_t item = 0;
  if (lane == 0) item = (int64_t)atomicAdd(A.counter, 1ull);
  item = wave_broadcast(item);
  while (item < A.n_items) {
    const bool ahead = item + (int64_t)gridDim.x * (blockDim.x >> 6) < A.n_items;
    int64_t next = 0;
    if (ahead && lane == 0) next = (int64_t)atomicAdd(A.counter, 1ull);
    const int lo = wave_search([&](int i) { return A.sims[i].item_off; }, A.n_sims, item, lane);
    const SimDesc& s = A.sims[lo];
    const int64_t local = item - s.item_off;
    if (s.spin_twice == 2) work_item<3>(A, s, local, lane, source);
    else work_item<2>(A, s, local, lane, source);
    if (!ahead && lane == 0) next = (int64_t)atomicAdd(A.counter, 1ull);
    item = wave_broadcast(next);
  }
}

}  // namespace mss
