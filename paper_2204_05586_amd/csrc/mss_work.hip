// Kernels and host builder of work sets (see mss_work.h).
//
// Integrator: persistent waves take work items (64 / S consecutive
// intervals of one range, S lane-slices per interval) from an atomic
// counter until it passes the item count, so every wave exits once the
// queue is drained; no wave ever waits for another.
// Scan: level by level; a wave locates its sequence by binary search over
// the level's tile prefix and handles one tile of it.
#include <string.h>

#include <algorithm>

#include "mss_scan.h"
#include "mss_work.h"

namespace mss {

int scan_top(int64_t K, int tile) {
  int top = 0;
  int64_t n = K;
  while (n > tile) {
    n = (n + tile - 1) / tile;
    ++top;
  }
  return top;
}

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t scan_scratch_bytes(int N, int64_t K, int tile) {
  size_t b = 0;
  int64_t n = K;
  while (n > tile) {
    n = (n + tile - 1) / tile;
    b += (size_t)n * (N * N + N) * 16;
  }
  return a256(b);
}

// ---------------------------------------------------------------------------
// device
// ---------------------------------------------------------------------------
// largest i in [0, n) with prefix[i] <= x (non-decreasing prefix, prefix[0] = 0)
__device__ __forceinline__ int find_segment(const int64_t* __restrict__ prefix, int n, int64_t x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

struct ScanWorkArgs {
  const SimDesc* sims;
  const int64_t* tiles;  // prefix over sequences at this level
  int64_t n_tiles;
  int32_t n_sims;
  int32_t level;
};

__global__ void work_reset_kernel(unsigned long long* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0ull;
}

// Field-program source of a descriptor: its slice of the term table.
struct TableSource {
  __device__ __forceinline__ TableTerms operator()(const IntegrateWorkArgs& A,
                                                   const SimDesc& s) const {
    return TableTerms{A.terms + s.term_off, s.n_terms};
  }
};

__global__ void __launch_bounds__(256) work_integrate_kernel(const IntegrateWorkArgs A) {
  work_integrate_loop(A, TableSource{});
}

__global__ void __launch_bounds__(256, 2) work_chained_kernel(const IntegrateWorkArgs A) {
  chained_integrate_loop(A, TableSource{});
}

// Before a chained run: unit counter and failure word to 0, every slot
// word to 0 (tag 0, which no unit writes).  Atomic stores, like every
// other access to these words; a kernel rather than a memset, so a captured
// graph replays it as such.
__global__ void chain_reset_kernel(ChainSync* s, unsigned long long* words, int64_t n_words) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    __hip_atomic_store(&s->counter, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&s->failed, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (i < n_words) __hip_atomic_store(words + i, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Element count of a sequence at a scan level and the start of that level's
// arrays in the sequence's scratch (levels >= 1).
template <int N, int E>
__device__ __forceinline__ int64_t level_geometry(const SimDesc& s, int level, size_t* mats_off) {
  int64_t n = s.K_total;
  size_t off = 0;
  for (int l = 1; l <= level; ++l) {
    if (l > 1) off += (size_t)n * (N * N + N) * 2;
    n = (n + 64 * E - 1) / (64 * E);
  }
  *mats_off = off;  // in doubles
  return n;
}

template <int N, int E>
__device__ __forceinline__ void work_reduce_tile(const SimDesc& s, int level, int64_t local,
                                                 int lane) {
  size_t off = 0;
  const int64_t n = level_geometry<N, E>(s, level, &off);
  const double* M = level == 0 ? s.U : s.scan_ws + off;
  size_t up_off = 0;
  const int64_t n_up = level_geometry<N, E>(s, level + 1, &up_off);
  (void)n_up;
  double* out = s.scan_ws + up_off + (size_t)local * 2 * N * N;
  tile_reduce<N, E>(M, n, local, lane, out);
}

template <int N, int E>
__device__ __forceinline__ void work_apply_tile(const SimDesc& s, int level, int64_t local,
                                                int lane) {
  size_t off = 0;
  const int64_t n = level_geometry<N, E>(s, level, &off);
  const double* M = level == 0 ? s.U : s.scan_ws + off;
  double* before = level == 0 ? s.psi : s.scan_ws + off + (size_t)n * 2 * N * N;
  const double* start;
  if (level == s.top) {
    start = s.psi0;
  } else {
    size_t up_off = 0;
    const int64_t n_up = level_geometry<N, E>(s, level + 1, &up_off);
    start = s.scan_ws + up_off + (size_t)n_up * 2 * N * N + (size_t)local * 2 * N;
  }
  tile_apply<N, E, (E * 2 * N * N <= 36)>(M, n, local, lane, true, start, before,
                                           level == 0 ? s.psi_final : nullptr);
}

template <int E>
__global__ void __launch_bounds__(256) work_reduce_kernel(const ScanWorkArgs A) {
  const int lane = threadIdx.x & 63;
  const int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (tile >= A.n_tiles) return;  // the whole wave leaves together
  const int i = find_segment(A.tiles, A.n_sims, tile);
  const int64_t local = tile - A.tiles[i];
  const SimDesc& s = A.sims[i];
  if (s.spin_twice == 2) work_reduce_tile<3, E>(s, A.level, local, lane);
  else work_reduce_tile<2, E>(s, A.level, local, lane);
}

template <int E>
__global__ void __launch_bounds__(256) work_apply_kernel(const ScanWorkArgs A) {
  const int lane = threadIdx.x & 63;
  const int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (tile >= A.n_tiles) return;  // the whole wave leaves together
  const int i = find_segment(A.tiles, A.n_sims, tile);
  const int64_t local = tile - A.tiles[i];
  const SimDesc& s = A.sims[i];
  if (s.spin_twice == 2) work_apply_tile<3, E>(s, A.level, local, lane);
  else work_apply_tile<2, E>(s, A.level, local, lane);
}

// ---------------------------------------------------------------------------
// host
// ---------------------------------------------------------------------------
void WorkSet::add(const mss_problem& p, int slices_log2, int64_t k_first, int64_t k_count,
                  bool scan) {
  SimDesc d;
  memset(&d, 0, sizeof d);
  d.t_start = p.t_start;
  d.dt_out = p.dt_out;
  d.dt = p.dt_out / (double)p.n_fine;
  d.k_first = k_first;
  d.k_count = k_count;
  d.K_total = p.n_samples;
  d.spin_twice = p.spin_twice;
  d.n_terms = p.n_terms;
  d.n_fine = p.n_fine;
  d.tau = p.spin_twice == 2 ? p.n_squares : 0;
  d.frame = p.rotating_frame;
  d.method = p.method;
  d.full = api_full_basis(&p) ? 1 : 0;
  d.slices_log2 = slices_log2;
  d.top = scan ? scan_top(p.n_samples, 64 * scan_e) : -1;
  if (last_terms_ && last_n_terms_ == p.n_terms &&
      (p.n_terms == 0 || memcmp(last_terms_, p.terms, sizeof(mss_term) * p.n_terms) == 0)) {
    d.term_off = last_term_off_;
  } else {
    d.term_off = (int32_t)terms.size();
    for (int t = 0; t < p.n_terms; ++t) terms.push_back(p.terms[t]);
    last_terms_ = p.terms;
    last_n_terms_ = p.n_terms;
    last_term_off_ = d.term_off;
  }
  sims.push_back(d);
}

void WorkSet::finalize() {
  const int n = (int)sims.size();
  int64_t item = 0;
  n_levels = 0;
  for (SimDesc& d : sims) {
    d.item_off = item;
    const int64_t per = 64 >> d.slices_log2;
    item += (d.k_count + per - 1) / per;
    n_levels = std::max(n_levels, d.top);
  }
  n_items = item;
  if (chained) {
    // unit counts per sequence (kChainPerLane 64 / S intervals each),
    // sequences by decreasing count; walking from the shortest up, each new
    // count starts a group of rounds in which exactly the sequences before
    // it (in `order`) and itself take part
    std::vector<int64_t> cnt(n);
    n_units = 0;
    for (int i = 0; i < n; ++i) {
      const int64_t per = (int64_t)kChainPerLane * (64 >> sims[i].slices_log2);
      cnt[i] = (sims[i].k_count + per - 1) / per;
      n_units += cnt[i];
    }
    order.resize(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return cnt[a] > cnt[b]; });
    group_item0.clear();
    group_round0.clear();
    group_count.clear();
    int64_t round = 0, at = 0;
    for (int j = n - 1; j >= 0; --j) {
      const int64_t m = cnt[order[j]];
      if (m <= round) continue;
      group_item0.push_back(at);
      group_round0.push_back(round);
      group_count.push_back(j + 1);
      at += (m - round) * (j + 1);
      round = m;
    }
  }
  reduce_tiles.assign(n_levels, std::vector<int64_t>(n + 1, 0));
  apply_tiles.assign(n_levels + 1, std::vector<int64_t>(n + 1, 0));
  const int tile = 64 * scan_e;
  for (int i = 0; i < n; ++i) {
    const SimDesc& d = sims[i];
    int64_t cnt = d.K_total;
    for (int l = 0; l <= n_levels; ++l) {
      const int64_t tiles = (cnt + tile - 1) / tile;
      const bool scans = d.top >= 0;
      if (l < n_levels) reduce_tiles[l][i + 1] = reduce_tiles[l][i] + (scans && l < d.top ? tiles : 0);
      apply_tiles[l][i + 1] = apply_tiles[l][i] + (scans && l <= d.top ? tiles : 0);
      cnt = tiles;
    }
  }
}

// chained tables: group_item0, group_round0, group_count, order
static size_t chain_table_bytes(size_t groups, size_t sims) {
  return 2 * a256(std::max<size_t>(1, groups) * sizeof(int64_t)) +
         a256(std::max<size_t>(1, groups) * sizeof(int32_t)) +
         a256(std::max<size_t>(1, sims) * sizeof(int32_t));
}

size_t WorkSet::packed_bytes() const {
  size_t b = a256(sims.size() * sizeof(SimDesc)) + a256(std::max<size_t>(1, terms.size()) * sizeof(mss_term));
  b += (reduce_tiles.size() + apply_tiles.size()) * a256((sims.size() + 1) * sizeof(int64_t));
  if (chained) b += chain_table_bytes(group_item0.size(), sims.size());
  return b;
}

void WorkSet::pack(char* dst, size_t* o_sims, size_t* o_terms, std::vector<size_t>* o_reduce,
                   std::vector<size_t>* o_apply, size_t* o_chain) const {
  size_t off = 0;
  *o_sims = off;
  memcpy(dst + off, sims.data(), sims.size() * sizeof(SimDesc));
  off += a256(sims.size() * sizeof(SimDesc));
  *o_terms = off;
  if (!terms.empty()) memcpy(dst + off, terms.data(), terms.size() * sizeof(mss_term));
  off += a256(std::max<size_t>(1, terms.size()) * sizeof(mss_term));
  const size_t tb = a256((sims.size() + 1) * sizeof(int64_t));
  o_reduce->clear();
  for (const auto& t : reduce_tiles) {
    o_reduce->push_back(off);
    memcpy(dst + off, t.data(), t.size() * sizeof(int64_t));
    off += tb;
  }
  o_apply->clear();
  for (const auto& t : apply_tiles) {
    o_apply->push_back(off);
    memcpy(dst + off, t.data(), t.size() * sizeof(int64_t));
    off += tb;
  }
  if (o_chain) *o_chain = off;
  if (chained) {
    const size_t g = group_item0.size();
    memcpy(dst + off, group_item0.data(), g * sizeof(int64_t));
    off += a256(std::max<size_t>(1, g) * sizeof(int64_t));
    memcpy(dst + off, group_round0.data(), g * sizeof(int64_t));
    off += a256(std::max<size_t>(1, g) * sizeof(int64_t));
    memcpy(dst + off, group_count.data(), g * sizeof(int32_t));
    off += a256(std::max<size_t>(1, g) * sizeof(int32_t));
    memcpy(dst + off, order.data(), order.size() * sizeof(int32_t));
  }
}

DevWork device_view(const WorkSet& w, const char* dev_base, size_t o_sims, size_t o_terms,
                    const std::vector<size_t>& o_reduce, const std::vector<size_t>& o_apply,
                    size_t o_chain) {
  DevWork d;
  if (w.chained) {
    const size_t g = w.group_item0.size();
    d.n_groups = (int32_t)g;
    size_t off = o_chain;
    d.group_item0 = (const int64_t*)(dev_base + off);
    off += a256(std::max<size_t>(1, g) * sizeof(int64_t));
    d.group_round0 = (const int64_t*)(dev_base + off);
    off += a256(std::max<size_t>(1, g) * sizeof(int64_t));
    d.group_count = (const int32_t*)(dev_base + off);
    off += a256(std::max<size_t>(1, g) * sizeof(int32_t));
    d.order = (const int32_t*)(dev_base + off);
  }
  d.sims = (const SimDesc*)(dev_base + o_sims);
  d.terms = (const mss_term*)(dev_base + o_terms);
  d.n_sims = (int32_t)w.sims.size();
  d.n_items = w.n_items;
  d.n_levels = w.n_levels;
  d.scan_e = w.scan_e;
  d.n_units = w.n_units;
  for (size_t l = 0; l < o_reduce.size(); ++l) {
    d.reduce_tiles.push_back((const int64_t*)(dev_base + o_reduce[l]));
    d.reduce_total.push_back(w.reduce_tiles[l].back());
  }
  for (size_t l = 0; l < o_apply.size(); ++l) {
    d.apply_tiles.push_back((const int64_t*)(dev_base + o_apply[l]));
    d.apply_total.push_back(w.apply_tiles[l].back());
  }
  return d;
}

hipError_t launch_work_integrate(const DevWork& w, unsigned long long* counter, int grid_blocks,
                                 hipStream_t st, hipFunction_t user_fn, bool counter_zeroed) {
  if (w.n_items == 0) return hipSuccess;
  if (!counter_zeroed) hipLaunchKernelGGL(work_reset_kernel, dim3(1), dim3(64), 0, st, counter);
  IntegrateWorkArgs a{w.sims, w.terms, counter, w.n_items, w.n_sims};
  if (user_fn) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    void* args[] = {&a};
    return hipModuleLaunchKernel(user_fn, (unsigned)grid_blocks, 1, 1, 256, 1, 1, 0, st, args,
                                 nullptr);
  }
  hipLaunchKernelGGL(work_integrate_kernel, dim3(grid_blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

size_t chain_workspace_bytes(int32_t n_sims) {
  return sizeof(ChainSync) + a256((size_t)std::max(1, n_sims) * sizeof(ChainSlot));
}

hipError_t launch_work_chained(const DevWork& w, void* ws, int grid_blocks, hipStream_t st,
                               hipFunction_t user_fn, unsigned long long wait_ticks) {
  if (w.n_units == 0) return hipSuccess;
  ChainSync* sync = (ChainSync*)ws;
  const int64_t n_words = (int64_t)w.n_sims * (sizeof(ChainSlot) / sizeof(unsigned long long));
  ChainSlot* slots = (ChainSlot*)((char*)ws + sizeof(ChainSync));
  hipLaunchKernelGGL(chain_reset_kernel, dim3((unsigned)((n_words + 255) / 256)), dim3(256), 0, st,
                     sync, (unsigned long long*)slots, n_words);
  IntegrateWorkArgs a{w.sims, w.terms, &sync->counter, w.n_units, w.n_sims};
  a.n_groups = w.n_groups;
  a.group_item0 = w.group_item0;
  a.group_round0 = w.group_round0;
  a.group_count = w.group_count;
  a.order = w.order;
  a.slots = slots;
  a.sync = sync;
  a.wait_ticks = wait_ticks;
  if (user_fn) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    void* args[] = {&a};
    return hipModuleLaunchKernel(user_fn, (unsigned)grid_blocks, 1, 1, 256, 1, 1, 0, st, args,
                                 nullptr);
  }
  hipLaunchKernelGGL(work_chained_kernel, dim3(grid_blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int E>
static void scan_levels(const DevWork& w, hipStream_t st) {
  for (int l = 0; l < w.n_levels; ++l) {
    const int64_t tiles = w.reduce_total[l];
    if (!tiles) continue;
    ScanWorkArgs a{w.sims, w.reduce_tiles[l], tiles, w.n_sims, l};
    hipLaunchKernelGGL(work_reduce_kernel<E>, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, st,
                       a);
  }
  for (int l = w.n_levels; l >= 0; --l) {
    const int64_t tiles = w.apply_total[l];
    if (!tiles) continue;
    ScanWorkArgs a{w.sims, w.apply_tiles[l], tiles, w.n_sims, l};
    hipLaunchKernelGGL(work_apply_kernel<E>, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, st,
                       a);
  }
}

hipError_t launch_work_scan(const DevWork& w, hipStream_t st) {
  if (w.scan_e == 2) scan_levels<2>(w, st);
  else if (w.scan_e == 8) scan_levels<8>(w, st);
  else scan_levels<4>(w, st);
  return hipGetLastError();
}

}  // namespace mss
