// Batched execution: many independent simulations of uneven length (and
// possibly mixed spin) in one persistent integrator launch plus one
// segmented scan, optionally captured as a single HIP graph.
//
// Work decomposition: simulation i is cut into work items of 64 / S_i
// consecutive intervals (one wave's worth; S_i lane-slices per interval).
// Waves of the persistent integrator take items from an atomic counter
// until the counter passes the item count, so every wave exits once the
// queue is drained.  The scan runs level by level over per-simulation tile
// tables: a wave finds its simulation by binary search over the tile prefix
// of the level and scans that simulation's tile only.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "mss_internal.h"
#include "mss_scan.h"

namespace mss {

struct BatchSim {
  double t_start, dt_out, dt;
  int64_t K;
  int64_t param_off;  // doubles into params
  int64_t psi0_off;   // complex index into psi0 / psi_final
  int64_t state_off;  // complex index into psi
  int64_t op_off;     // complex index into the operator array
  int64_t item_off;   // first work item
  int32_t spin_twice, n_terms, term_off, n_fine, tau, frame, slices_log2, pad;
};

// Per-level tables (device pointers into the descriptor buffer) and the
// level's matrix / state arrays (device pointers supplied at run time).
struct LevelView {
  const int64_t* n;          // [n_sims] elements of each simulation
  const int64_t* elem_off;   // [n_sims] complex offset of its first matrix
  const int64_t* state_off;  // [n_sims] complex offset of its first entering state
  const int64_t* tile_off;   // [n_sims + 1] prefix of ceil(n / kScanTile)
  double* mats;
  double* states;
};

struct IntegrateBatchArgs {
  const BatchSim* sims;
  const mss_term* terms;
  const double* params;
  double* U;
  unsigned long long* counter;
  int64_t n_items;
  int32_t n_sims;
};

struct ScanBatchArgs {
  const BatchSim* sims;
  int32_t n_sims;
  int32_t is_top;
  LevelView lv;     // this level
  LevelView up;     // level above (reduce target / apply source)
  const double* psi0;
  double* psi_final;
};

__device__ __forceinline__ int find_segment(const int64_t* __restrict__ prefix, int n, int64_t x) {
  // largest i in [0, n) with prefix[i] <= x (prefix is non-decreasing, prefix[0] = 0)
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int64_t wave_broadcast(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffff));
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return ((int64_t)hi << 32) | (uint32_t)lo;
}

__global__ void batch_reset_kernel(unsigned long long* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0ull;
}

template <int N>
__device__ __forceinline__ void batch_item(const IntegrateBatchArgs& A, const BatchSim& s,
                                           int64_t local, int lane) {
  const int sl = s.slices_log2;
  const int64_t k = local * (64 >> sl) + (lane >> sl);
  const int slice = lane & ((1 << sl) - 1);
  const bool active = k < s.K;
  Mat<N> U;
  double tk;
  interval_operator<N>(TableTerms{A.terms + s.term_off, s.n_terms}, A.params + s.param_off,
                       s.t_start, s.dt_out, s.dt, s.n_fine, s.tau, s.frame, k, slice, sl, active,
                       U, &tk);
  if (active && slice == 0) store_mat<N>(A.U + 2 * ((size_t)s.op_off + (size_t)k * N * N), U);
}

__global__ void __launch_bounds__(256) batch_integrate_kernel(const IntegrateBatchArgs A) {
  const int lane = threadIdx.x & 63;
  for (;;) {
    int64_t item = 0;
    if (lane == 0) item = (int64_t)atomicAdd(A.counter, 1ull);
    item = wave_broadcast(item);
    if (item >= A.n_items) break;
    // simulation owning the item: item_off is the first field run of sims
    int lo = 0, hi = A.n_sims - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (A.sims[mid].item_off <= item) lo = mid;
      else hi = mid - 1;
    }
    const BatchSim& s = A.sims[lo];
    const int64_t local = item - s.item_off;
    if (s.spin_twice == 2) batch_item<3>(A, s, local, lane);
    else batch_item<2>(A, s, local, lane);
  }
}

template <int N>
__device__ __forceinline__ void batch_reduce_tile(const ScanBatchArgs& A, int i, int64_t local,
                                                  int lane) {
  const LevelView& v = A.lv;
  const int64_t n = v.n[i];
  const double* M = v.mats + 2 * v.elem_off[i];
  double* out = A.up.mats + 2 * (A.up.elem_off[i] + local * N * N);
  tile_reduce<N>(M, n, local, lane, out);
}

__global__ void __launch_bounds__(256) batch_scan_reduce_kernel(const ScanBatchArgs A,
                                                                int64_t n_tiles) {
  const int lane = threadIdx.x & 63;
  const int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (tile >= n_tiles) return;  // whole wave leaves together
  const int i = find_segment(A.lv.tile_off, A.n_sims, tile);
  const int64_t local = tile - A.lv.tile_off[i];
  if (A.sims[i].spin_twice == 2) batch_reduce_tile<3>(A, i, local, lane);
  else batch_reduce_tile<2>(A, i, local, lane);
}

template <int N>
__device__ __forceinline__ void batch_apply_tile(const ScanBatchArgs& A, int i, int64_t local,
                                                 int lane) {
  const LevelView& v = A.lv;
  const int64_t n = v.n[i];
  const double* M = v.mats + 2 * v.elem_off[i];
  const double* start = A.is_top ? A.psi0 + 2 * A.sims[i].psi0_off
                                 : A.up.states + 2 * (A.up.state_off[i] + local * N);
  double* before = v.states + 2 * v.state_off[i];
  double* after = A.psi_final ? A.psi_final + 2 * A.sims[i].psi0_off : nullptr;
  tile_apply<N>(M, n, local, lane, true, start, before, after);
}

__global__ void __launch_bounds__(256) batch_scan_apply_kernel(const ScanBatchArgs A,
                                                               int64_t n_tiles) {
  const int lane = threadIdx.x & 63;
  const int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (tile >= n_tiles) return;  // whole wave leaves together
  const int i = find_segment(A.lv.tile_off, A.n_sims, tile);
  const int64_t local = tile - A.lv.tile_off[i];
  if (A.sims[i].spin_twice == 2) batch_apply_tile<3>(A, i, local, lane);
  else batch_apply_tile<2>(A, i, local, lane);
}

}  // namespace mss

using namespace mss;

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct mss_batch_plan {
  int32_t n = 0;
  int64_t n_items = 0;
  int64_t psi0_total = 0, state_total = 0, op_total = 0;
  std::vector<int64_t> psi0_off, state_off, op_off;  // host copies, n + 1 entries
  std::vector<int32_t> dims;
  int n_levels = 0;                                   // levels above 0
  std::vector<int64_t> level_tiles;                   // [n_levels + 1]
  std::vector<size_t> level_mats_ws, level_states_ws; // ws offsets for levels >= 1
  size_t ws_counter = 0, ws_ops = 0, ws_bytes_levels = 0;
  void* desc = nullptr;                               // device descriptor buffer
  const BatchSim* d_sims = nullptr;
  const mss_term* d_terms = nullptr;
  std::vector<LevelView> views;                       // table pointers, buffers unset
  int grid_blocks = 0;
  mss_batch_options opt{};
  // graph cache
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* key[7] = {};
  int device = 0;
};

namespace {

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

template <class T>
size_t put(std::vector<char>& buf, const T* data, size_t count) {
  const size_t off = a256(buf.size());
  buf.resize(off + sizeof(T) * count);
  if (count) memcpy(buf.data() + off, data, sizeof(T) * count);
  return off;
}

void release(mss_batch_plan* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
  if (p->desc) (void)hipFree(p->desc);
  delete p;
}

// Workspace: counter (256 B) | operators, when the caller keeps no U |
// level arrays starting at lv_base.
std::vector<LevelView> level_views(const mss_batch_plan* P, double* ops, double* psi, char* ws,
                                   size_t lv_base) {
  std::vector<LevelView> lv = P->views;
  lv[0].mats = ops;
  lv[0].states = psi;
  for (int l = 1; l <= P->n_levels; ++l) {
    lv[l].mats = (double*)(ws + lv_base + P->level_mats_ws[l]);
    lv[l].states = (double*)(ws + lv_base + P->level_states_ws[l]);
  }
  return lv;
}

void enqueue_integrate(const mss_batch_plan* P, const double* params, double* ops, char* ws,
                       hipStream_t st) {
  unsigned long long* counter = (unsigned long long*)(ws + P->ws_counter);
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, st, counter);
  IntegrateBatchArgs ia{P->d_sims, P->d_terms, params, ops, counter, P->n_items, P->n};
  hipLaunchKernelGGL(batch_integrate_kernel, dim3(P->grid_blocks), dim3(256), 0, st, ia);
}

void enqueue_propagate(const mss_batch_plan* P, const double* psi0, double* psi, double* psi_final,
                       double* ops, char* ws, size_t lv_base, hipStream_t st) {
  const std::vector<LevelView> lv = level_views(P, ops, psi, ws, lv_base);
  for (int l = 0; l < P->n_levels; ++l) {
    ScanBatchArgs sa{P->d_sims, P->n, 0, lv[l], lv[l + 1], psi0, nullptr};
    const int64_t tiles = P->level_tiles[l];
    hipLaunchKernelGGL(batch_scan_reduce_kernel, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0,
                       st, sa, tiles);
  }
  for (int l = P->n_levels; l >= 0; --l) {
    ScanBatchArgs sa{P->d_sims, P->n, l == P->n_levels ? 1 : 0, lv[l],
                     l < P->n_levels ? lv[l + 1] : lv[l], psi0, l == 0 ? psi_final : nullptr};
    const int64_t tiles = P->level_tiles[l];
    hipLaunchKernelGGL(batch_scan_apply_kernel, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0,
                       st, sa, tiles);
  }
}

mss_status enqueue(mss_batch_plan* P, const double* params, const double* psi0, double* psi,
                   double* psi_final, double* U, char* ws, size_t lv_base, hipStream_t st) {
  double* ops = U ? U : (double*)(ws + P->ws_ops);
  enqueue_integrate(P, params, ops, ws, st);
  enqueue_propagate(P, psi0, psi, psi_final, ops, ws, lv_base, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return mss::api_hip_fail(e, "batch launch");
  return MSS_OK;
}

mss_status check_ws(const mss_batch_plan* P, bool store_u, const void* ws, size_t ws_bytes) {
  size_t need = 256 + P->ws_bytes_levels + (store_u ? 0 : a256((size_t)P->op_total * 16));
  if (!ws || ws_bytes < need)
    return api_fail(MSS_E_NOMEM, "workspace too small: need %zu bytes, got %zu", need,
                    ws ? ws_bytes : (size_t)0);
  return MSS_OK;
}

}  // namespace

extern "C" {

mss_status mss_batch_plan_create(int32_t n, const mss_problem* problems, const int64_t* param_off,
                                 const mss_batch_options* options, mss_batch_plan** out) {
  if (!out) return api_fail(MSS_E_INVALID, "out is NULL");
  *out = nullptr;
  if (n < 1) return api_fail(MSS_E_INVALID, "a batch needs at least one simulation");
  if (!problems) return api_fail(MSS_E_INVALID, "problems is NULL");
  mss_batch_options opt{};
  if (options) opt = *options;
  if (opt.slices_spin_half < 0 || opt.slices_spin_half > 64 ||
      (opt.slices_spin_half & (opt.slices_spin_half - 1)) != 0 || opt.slices_spin_one < 0 ||
      opt.slices_spin_one > 64 || (opt.slices_spin_one & (opt.slices_spin_one - 1)) != 0)
    return api_fail(MSS_E_INVALID, "slices must be 0 (choose) or a power of two <= 64");
  if (opt.waves_per_simd < 0 || opt.waves_per_simd > 8)
    return api_fail(MSS_E_INVALID, "waves_per_simd must be in [0, 8]");
  for (int i = 0; i < n; ++i) {
    mss_status s = api_validate_problem(&problems[i]);
    if (s != MSS_OK) {
      std::string m = api_last_error_copy();
      return api_fail(s, "simulation %d: %s", i, m.c_str());
    }
    if (problems[i].n_params > 0) {
      if (!param_off) return api_fail(MSS_E_INVALID, "param_off is NULL but simulation %d has parameters", i);
      if (param_off[i] < 0) return api_fail(MSS_E_INVALID, "simulation %d: negative param_off", i);
    }
  }
  const int cu = api_device_cu_count();
  // slice choice per spin class, from the class's total interval count
  int64_t k_class[2] = {0, 0};
  int32_t l_class[2] = {1 << 30, 1 << 30};
  for (int i = 0; i < n; ++i) {
    const int c = problems[i].spin_twice - 1;
    k_class[c] += problems[i].n_samples;
    l_class[c] = std::min(l_class[c], problems[i].n_fine);
  }
  int S_class[2];
  for (int c = 0; c < 2; ++c) {
    const int given = c == 0 ? opt.slices_spin_half : opt.slices_spin_one;
    S_class[c] = given ? given : (k_class[c] ? api_plan_slices(k_class[c], l_class[c], cu) : 1);
  }

  mss_batch_plan* P = new (std::nothrow) mss_batch_plan();
  if (!P) return api_fail(MSS_E_NOMEM, "host allocation failed");
  P->n = n;
  P->opt = opt;
  (void)hipGetDevice(&P->device);
  std::vector<BatchSim> sims(n);
  std::vector<mss_term> terms;
  P->psi0_off.assign(n + 1, 0);
  P->state_off.assign(n + 1, 0);
  P->op_off.assign(n + 1, 0);
  P->dims.resize(n);
  int64_t item = 0;
  int last_term_off = -1, last_n_terms = -1;
  const mss_term* last_terms = nullptr;
  for (int i = 0; i < n; ++i) {
    const mss_problem& q = problems[i];
    const int N = q.spin_twice + 1;
    P->dims[i] = N;
    BatchSim& s = sims[i];
    memset(&s, 0, sizeof s);
    s.t_start = q.t_start;
    s.dt_out = q.dt_out;
    s.dt = q.dt_out / (double)q.n_fine;
    s.K = q.n_samples;
    s.param_off = q.n_params > 0 ? param_off[i] : 0;
    s.psi0_off = P->psi0_off[i];
    s.state_off = P->state_off[i];
    s.op_off = P->op_off[i];
    P->psi0_off[i + 1] = P->psi0_off[i] + N;
    P->state_off[i + 1] = P->state_off[i] + q.n_samples * N;
    P->op_off[i + 1] = P->op_off[i] + q.n_samples * N * N;
    int S = S_class[q.spin_twice - 1];
    while (S > q.n_fine) S >>= 1;
    s.slices_log2 = api_ilog2(S);
    s.item_off = item;
    item += (q.n_samples + (64 / S) - 1) / (64 / S);
    s.spin_twice = q.spin_twice;
    s.n_terms = q.n_terms;
    s.n_fine = q.n_fine;
    s.tau = q.spin_twice == 2 ? q.n_squares : 0;
    s.frame = q.rotating_frame;
    // identical term lists (same content as the previous simulation's) are stored once
    if (last_terms && last_n_terms == q.n_terms &&
        (q.n_terms == 0 || memcmp(last_terms, q.terms, sizeof(mss_term) * q.n_terms) == 0)) {
      s.term_off = last_term_off;
    } else {
      s.term_off = (int32_t)terms.size();
      for (int t = 0; t < q.n_terms; ++t) terms.push_back(q.terms[t]);
      last_term_off = s.term_off;
      last_n_terms = q.n_terms;
      last_terms = q.terms;
    }
  }
  P->n_items = item;
  P->psi0_total = P->psi0_off[n];
  P->state_total = P->state_off[n];
  P->op_total = P->op_off[n];

  // scan levels: level 0 = the operators themselves
  std::vector<std::vector<int64_t>> ln, leo, lso, lto;
  std::vector<int64_t> cur(n);
  for (int i = 0; i < n; ++i) cur[i] = problems[i].n_samples;
  for (;;) {
    const int l = (int)ln.size();
    std::vector<int64_t> eo(n), so(n), to(n + 1, 0);
    int64_t e_acc = 0, s_acc = 0;
    for (int i = 0; i < n; ++i) {
      const int N = P->dims[i];
      if (l == 0) {
        eo[i] = P->op_off[i];
        so[i] = P->state_off[i];
      } else {
        eo[i] = e_acc;
        so[i] = s_acc;
        e_acc += cur[i] * N * N;
        s_acc += cur[i] * N;
      }
      to[i + 1] = to[i] + (cur[i] + kScanTile - 1) / kScanTile;
    }
    ln.push_back(cur);
    leo.push_back(eo);
    lso.push_back(so);
    lto.push_back(to);
    P->level_tiles.push_back(to[n]);
    if (l >= 1) {
      P->level_mats_ws.resize(l + 1, 0);
      P->level_states_ws.resize(l + 1, 0);
      P->level_mats_ws[l] = (size_t)e_acc * 16;   // sizes for now, offsets below
      P->level_states_ws[l] = (size_t)s_acc * 16;
    }
    int64_t mx = 0;
    for (int i = 0; i < n; ++i) mx = std::max(mx, cur[i]);
    if (mx <= kScanTile) break;
    for (int i = 0; i < n; ++i) cur[i] = (cur[i] + kScanTile - 1) / kScanTile;
    if (ln.size() > 8) break;
  }
  P->n_levels = (int)ln.size() - 1;
  // workspace layout: counter | operators (when not stored by the caller) | levels
  size_t off = 0;
  P->ws_counter = off;
  off += 256;
  P->ws_ops = off;
  size_t lv_off = 0;
  std::vector<size_t> mats_off(P->n_levels + 1, 0), states_off(P->n_levels + 1, 0);
  for (int l = 1; l <= P->n_levels; ++l) {
    mats_off[l] = lv_off;
    lv_off += a256(P->level_mats_ws[l]);
    states_off[l] = lv_off;
    lv_off += a256(P->level_states_ws[l]);
  }
  P->ws_bytes_levels = lv_off;
  // level offsets are relative to lv_base (after the optional operator block)
  for (int l = 1; l <= P->n_levels; ++l) {
    P->level_mats_ws[l] = mats_off[l];
    P->level_states_ws[l] = states_off[l];
  }

  // descriptor buffer
  std::vector<char> buf;
  const size_t o_sims = put(buf, sims.data(), sims.size());
  const size_t o_terms = put(buf, terms.data(), terms.size());
  std::vector<size_t> o_n(ln.size()), o_eo(ln.size()), o_so(ln.size()), o_to(ln.size());
  for (size_t l = 0; l < ln.size(); ++l) {
    o_n[l] = put(buf, ln[l].data(), ln[l].size());
    o_eo[l] = put(buf, leo[l].data(), leo[l].size());
    o_so[l] = put(buf, lso[l].data(), lso[l].size());
    o_to[l] = put(buf, lto[l].data(), lto[l].size());
  }
  hipError_t e = hipMalloc(&P->desc, a256(buf.size()));
  if (e != hipSuccess) {
    release(P);
    if (e == hipErrorOutOfMemory) return api_fail(MSS_E_NOMEM, "descriptor allocation failed");
    return api_hip_fail(e, "descriptor allocation");
  }
  e = hipMemcpy(P->desc, buf.data(), buf.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    release(P);
    return api_hip_fail(e, "descriptor upload");
  }
  char* d = (char*)P->desc;
  P->d_sims = (const BatchSim*)(d + o_sims);
  P->d_terms = (const mss_term*)(d + o_terms);
  P->views.resize(ln.size());
  for (size_t l = 0; l < ln.size(); ++l) {
    LevelView& v = P->views[l];
    v.n = (const int64_t*)(d + o_n[l]);
    v.elem_off = (const int64_t*)(d + o_eo[l]);
    v.state_off = (const int64_t*)(d + o_so[l]);
    v.tile_off = (const int64_t*)(d + o_to[l]);
    v.mats = nullptr;
    v.states = nullptr;
  }
  const int wps = opt.waves_per_simd ? opt.waves_per_simd : 2;
  int64_t blocks = (int64_t)cu * wps;  // 256-thread blocks = one wave per SIMD each
  const int64_t max_useful = (P->n_items + 3) / 4;
  P->grid_blocks = (int)std::max<int64_t>(1, std::min(blocks, max_useful));
  *out = P;
  return api_ok();
}

mss_status mss_batch_layout(const mss_batch_plan* P, int64_t* psi0_off, int64_t* state_off,
                            int64_t* op_off) {
  if (!P) return api_fail(MSS_E_INVALID, "plan is NULL");
  for (int i = 0; i <= P->n; ++i) {
    if (psi0_off) psi0_off[i] = P->psi0_off[i];
    if (state_off) state_off[i] = P->state_off[i];
    if (op_off) op_off[i] = P->op_off[i];
  }
  return api_ok();
}

mss_status mss_batch_workspace_size(const mss_batch_plan* P, int32_t store_u, size_t* bytes) {
  if (!P || !bytes) return api_fail(MSS_E_INVALID, "plan and bytes are required");
  size_t b = 256 + P->ws_bytes_levels;
  if (!store_u) b += a256((size_t)P->op_total * 16);
  *bytes = b;
  return api_ok();
}

mss_status mss_batch_run(mss_batch_plan* P, const double* params, const double* psi0, double* psi,
                         double* psi_final, double* U, void* ws, size_t ws_bytes, void* stream) {
  if (!P) return api_fail(MSS_E_INVALID, "plan is NULL");
  if (!psi0 || !psi) return api_fail(MSS_E_INVALID, "psi0 and psi are required");
  mss_status cs = check_ws(P, U != nullptr, ws, ws_bytes);
  if (cs != MSS_OK) return cs;
  // level arrays follow the counter (and the operator block when U is not stored)
  char* base = (char*)ws;
  const size_t lv_base = 256 + (U ? 0 : a256((size_t)P->op_total * 16));
  mss_batch_plan& Q = *P;
  hipStream_t st = (hipStream_t)stream;
  mss_status s;
  if (!Q.opt.use_graph) {
    s = enqueue(P, params, psi0, psi, psi_final, U, base, lv_base, st);
  } else {
    const void* key[7] = {params, psi0, psi, psi_final, U, ws, (const void*)lv_base};
    bool same = Q.exec != nullptr;
    for (int i = 0; i < 7 && same; ++i) same = Q.key[i] == key[i];
    s = MSS_OK;
    if (!same) {
      if (Q.exec) {
        (void)hipGraphExecDestroy(Q.exec);
        Q.exec = nullptr;
      }
      hipError_t e = hipSuccess;
      if (!Q.capture_stream) e = hipStreamCreateWithFlags(&Q.capture_stream, hipStreamNonBlocking);
      hipGraph_t g = nullptr;
      if (e == hipSuccess) e = hipStreamBeginCapture(Q.capture_stream, hipStreamCaptureModeRelaxed);
      if (e == hipSuccess) {
        s = enqueue(P, params, psi0, psi, psi_final, U, base, lv_base, Q.capture_stream);
        hipError_t e2 = hipStreamEndCapture(Q.capture_stream, &g);
        if (s == MSS_OK && e2 != hipSuccess) e = e2;
      }
      if (e == hipSuccess && s == MSS_OK) e = hipGraphInstantiate(&Q.exec, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      if (e != hipSuccess && s == MSS_OK) s = api_hip_fail(e, "batch graph capture");
      if (s == MSS_OK)
        for (int i = 0; i < 7; ++i) Q.key[i] = key[i];
    }
    if (s == MSS_OK) {
      hipError_t e = hipGraphLaunch(Q.exec, st);
      if (e != hipSuccess) s = api_hip_fail(e, "batch graph launch");
    }
  }
  return s == MSS_OK ? api_ok() : s;
}

mss_status mss_batch_info(const mss_batch_plan* P, mss_batch_info_t* info) {
  if (!P || !info) return api_fail(MSS_E_INVALID, "plan and info are required");
  info->n_sims = P->n;
  info->n_items = P->n_items;
  info->grid_blocks = P->grid_blocks;
  info->scan_levels = P->n_levels + 1;
  info->total_samples = 0;
  for (int i = 0; i < P->n; ++i)
    info->total_samples += (P->state_off[i + 1] - P->state_off[i]) / P->dims[i];
  return api_ok();
}

mss_status mss_batch_integrate(mss_batch_plan* P, const double* params, double* U, void* ws,
                               size_t ws_bytes, void* stream) {
  if (!P) return api_fail(MSS_E_INVALID, "plan is NULL");
  mss_status cs = check_ws(P, U != nullptr, ws, ws_bytes);
  if (cs != MSS_OK) return cs;
  char* base = (char*)ws;
  double* ops = U ? U : (double*)(base + P->ws_ops);
  enqueue_integrate(P, params, ops, base, (hipStream_t)stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return api_hip_fail(e, "batch integrate launch");
  return api_ok();
}

mss_status mss_batch_propagate(mss_batch_plan* P, const double* psi0, double* psi,
                               double* psi_final, const double* U, void* ws, size_t ws_bytes,
                               void* stream) {
  if (!P) return api_fail(MSS_E_INVALID, "plan is NULL");
  if (!psi0 || !psi) return api_fail(MSS_E_INVALID, "psi0 and psi are required");
  mss_status cs = check_ws(P, U != nullptr, ws, ws_bytes);
  if (cs != MSS_OK) return cs;
  char* base = (char*)ws;
  double* ops = U ? (double*)U : (double*)(base + P->ws_ops);
  const size_t lv_base = 256 + (U ? 0 : a256((size_t)P->op_total * 16));
  enqueue_propagate(P, psi0, psi, psi_final, ops, base, lv_base, (hipStream_t)stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return api_hip_fail(e, "batch propagate launch");
  return api_ok();
}

void mss_batch_plan_destroy(mss_batch_plan* P) { release(P); }

}  // extern "C"
