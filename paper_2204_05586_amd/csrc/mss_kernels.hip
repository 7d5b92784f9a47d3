// Kernels of the solver path:
//   integrate_kernel<N>  interval operators U_k (CF4 fine steps in the
//                        per-interval rotating frame, frame exit)
//   scan_reduce_kernel<N>, scan_apply_kernel<N>
//                        ordered prefix product psi_{k+1} = U_k psi_k as a
//                        two-level associative scan (wave shuffles)
#include "mss_internal.h"
#include "mss_scan.h"

namespace mss {

// One lane per (interval k, slice s); slice s integrates fine steps
// [s L / S, (s + 1) L / S) and the partial products are combined in order
// (later slices on the left) with wave shuffles.
template <int N>
__global__ void __launch_bounds__(256) integrate_kernel(const IntegrateArgs A) {
  integrate_lanes<N>(ArgTerms{A.fp}, A.g);
}

template <int N>
__global__ void __launch_bounds__(256) scan_reduce_kernel(const double* __restrict__ M, int64_t n,
                                                          double* __restrict__ agg) {
  const int lane = threadIdx.x & 63;
  const int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  tile_reduce<N, kScanPerLane>(M, n, tile, lane, tile < ntiles ? agg + (size_t)tile * 2 * N * N : nullptr);
}

template <int N>
__global__ void __launch_bounds__(256) scan_apply_kernel(const double* __restrict__ M, int64_t n,
                                                         const double* __restrict__ start,
                                                         double* __restrict__ before,
                                                         double* __restrict__ after_last,
                                                         double* __restrict__ spin) {
  const int lane = threadIdx.x & 63;
  const int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  const bool valid = tile < ntiles;
  tile_apply<N, kScanPerLane>(M, n, tile, lane, valid, valid ? start + (size_t)tile * 2 * N : nullptr, before,
                after_last, spin);
}

// Levels 1 and 2 of a two-level scan in one workgroup (n1 <= 16 tiles):
// wave w reduces level-1 tile w into LDS, wave 0 scans those aggregates
// from start, then wave w applies its tile from the state entering it.  The
// same tile routines on the same data as the separate launches, so the
// result is bitwise the same; the LDS holds the level-2 aggregates and
// entering states between the phases.
constexpr int kTopWaves = 16;

template <int N>
__global__ void __launch_bounds__(64 * kTopWaves) scan_top_kernel(const double* __restrict__ M1,
                                                                  int64_t n1,
                                                                  const double* __restrict__ start,
                                                                  double* __restrict__ before1) {
  __shared__ double agg2[kTopWaves * 2 * N * N];
  __shared__ double before2[kTopWaves * 2 * N];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t n2 = (n1 + kScanTile - 1) / kScanTile;
  tile_reduce<N, kScanPerLane>(M1, n1, wave, lane, agg2 + (size_t)wave * 2 * N * N);
  __syncthreads();
  if (wave == 0) tile_apply<N, kScanPerLane>(agg2, n2, 0, lane, true, start, before2, nullptr);
  __syncthreads();
  tile_apply<N, kScanPerLane>(M1, n1, wave, lane, true, before2 + (size_t)wave * 2 * N, before1,
                              nullptr);
}

// ---------------------------------------------------------------------------
// The whole scan of one sequence in one launch, for two or three levels
// (level 0 = the operators, at most 16 level-1 tiles).  One wave per
// level-0 tile, every workgroup resident at once, three phases:
//   1. every wave reduces its tile into the level-1 aggregates and
//      publishes it by writing the call's tag into the tile's tag word;
//   2. workgroup 0 waits for every tag, then does the upper levels exactly
//      as scan_apply_kernel (one level) or scan_top_kernel (two levels)
//      would, and publishes the entering states of the level-0 tiles;
//   3. every wave waits for that and applies its tile.
// The tile routines and their data are those of the separate launches, so
// the results are bitwise theirs.  The call number comes from the
// workspace itself (epoch + 1, written back by workgroup 0 once every tag
// is in), so a captured graph replays it correctly.  Tags and the ready
// word hold the call number passed through a 64-bit bijective mix
// (call_tag), so neither tags of earlier calls nor whatever the workspace
// held before (operators, states, other tags) match the current call
// except by a 2^-64 coincidence.
// Only workgroup 0 waits for later workgroups.  The host launches this
// kernel only when its grid needs at most a quarter of the workgroups the
// device holds at once, so the grid is resident even beside three more
// such scans on other streams; kernels that do not wait (the integrators)
// leave in time.  Every wait is bounded by kScanWaitTicks of the 100 MHz
// real-time counter (10 s, far beyond any real wait): one that runs out
// writes the call's tag into `failed` in the workspace and the kernel
// finishes without blocking (its results are then undefined).
// ---------------------------------------------------------------------------
struct ScanSync {
  unsigned long long epoch;  // number of the last completed call
  unsigned long long ready;  // call_tag(call) once the level-0 entering states are written
  unsigned long long failed; // call_tag(call) of a call whose bounded wait ran out
  unsigned long long pad[29];
};
static_assert(sizeof(ScanSync) == 256, "ScanSync is one 256-byte block");

constexpr unsigned long long kScanWaitTicks = 1000000000ull;  // 10 s at 100 MHz

// The finalizer of SplitMix64 (Steele, Lea and Flood, 2014), a bijection of
// 64-bit words that spreads small call numbers over all bits.
__device__ __forceinline__ unsigned long long call_tag(unsigned long long c) {
  c ^= c >> 30;
  c *= 0xbf58476d1ce4e5b9ull;
  c ^= c >> 27;
  c *= 0x94d049bb133111ebull;
  c ^= c >> 31;
  return c;
}

__device__ __forceinline__ void store_release(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// The current value of a word, read by an atomic compare-and-swap of 0
// with 0 (it writes only a 0 that is already there): a real read-modify-
// write at agent scope, which takes effect at the device's coherence point,
// whereas a plain or relaxed load (and an idempotent fetch-add, which the
// compiler turns into one) can keep returning a line the reading XCD's L2
// holds.
__device__ __forceinline__ unsigned long long coherent_read(unsigned long long* p) {
  unsigned long long v = 0ull;
  __hip_atomic_compare_exchange_strong(p, &v, 0ull, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return v;
}

// Every lane of the wave polls (coherent_read) until *p == want, then one
// acquire fence makes what was written before the tag visible; false when
// the bound ran out.
__device__ __forceinline__ bool wait_equal(unsigned long long* p, unsigned long long want) {
  const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
  bool ok = true;
  for (;;) {
    if (__all(coherent_read(p) == want)) break;
    if (__builtin_amdgcn_s_memrealtime() - t0 > kScanWaitTicks) {
      ok = false;
      break;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return ok;
}

struct OnePassArgs {
  const double* M0;     // operators [n0][N][N]
  int64_t n0;
  double* M1;           // level-1 aggregates [n1][N][N]
  double* st1;          // level-1 entering states [n1][N]
  int64_t n1;
  const double* psi0;
  double* psi;          // [n0][N]
  double* psi_final;    // [N] or null
  double* spin;         // [n0][3] or null
  ScanSync* sync;
  unsigned long long* tags;  // [n1]
  int32_t levels;       // 1 or 2 above the operators
};

template <int N>
__global__ void __launch_bounds__(256) scan_one_pass_kernel(const OnePassArgs A) {
  __shared__ double agg2[kTopWaves * 2 * N * N];
  __shared__ double before2[kTopWaves * 2 * N];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t tile = (int64_t)blockIdx.x * 4 + wave;
  const bool has_tile = tile < A.n1;
  const unsigned long long call =
      __hip_atomic_load(&A.sync->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1ull;
  const unsigned long long tag = call_tag(call);
  // 1. reduce the tile, publish its aggregate
  if (has_tile) {
    tile_reduce<N, kScanPerLane>(A.M0, A.n0, tile, lane, A.M1 + (size_t)tile * 2 * N * N);
    if (lane == 0) store_release(A.tags + tile, tag);
  }
  // 2. workgroup 0: the upper levels
  if (blockIdx.x == 0) {
    bool ok = true;
    for (int64_t base = (int64_t)wave * 64; base < A.n1; base += 256) {
      const int64_t idx = base + lane;
      unsigned long long* t = A.tags + (idx < A.n1 ? idx : A.n1 - 1);
      ok = ok && wait_equal(t, tag);
    }
    if (!ok && lane == 0) A.sync->failed = tag;
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // every aggregate read below is in
    if (A.levels == 1) {
      if (wave == 0) tile_apply<N, kScanPerLane>(A.M1, A.n1, 0, lane, true, A.psi0, A.st1, nullptr);
    } else {
      const int64_t n2 = (A.n1 + kScanTile - 1) / kScanTile;  // <= kTopWaves
      for (int64_t j = wave; j < n2; j += 4)
        tile_reduce<N, kScanPerLane>(A.M1, A.n1, j, lane, agg2 + (size_t)j * 2 * N * N);
      __syncthreads();
      if (wave == 0) tile_apply<N, kScanPerLane>(agg2, n2, 0, lane, true, A.psi0, before2, nullptr);
      __syncthreads();
      for (int64_t j = wave; j < n2; j += 4)
        tile_apply<N, kScanPerLane>(A.M1, A.n1, j, lane, true, before2 + (size_t)j * 2 * N, A.st1,
                                    nullptr);
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
      store_release(&A.sync->ready, tag);
      store_release(&A.sync->epoch, call);
    }
  }
  // 3. apply the tile from its entering state
  if (!has_tile) return;
  if (!wait_equal(&A.sync->ready, tag) && lane == 0) A.sync->failed = tag;
  tile_apply<N, kScanPerLane>(A.M0, A.n0, tile, lane, true, A.st1 + (size_t)tile * 2 * N, A.psi,
                              A.psi_final, A.spin);
}

// <J_a> = psi^H J_a psi for one state per lane (a = x, y, z), written as
// [K][3] doubles.  Spin-1/2: J = sigma/2; spin-1: J_x, J_y with 1/sqrt 2
// couplings between neighbouring levels, J_z = diag(1, 0, -1).
template <int N>
__global__ void __launch_bounds__(256) spin_projection_kernel(const double* __restrict__ psi,
                                                              int64_t K, double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const double* v = psi + (size_t)k * 2 * N;
  double vr[N], vi[N];
#pragma unroll
  for (int a = 0; a < N; ++a) {
    vr[a] = v[2 * a];
    vi[a] = v[2 * a + 1];
  }
  project_spin<N>(vr, vi, out + 3 * k);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int64_t integrate_slots(int N, int block) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  int cu = 0;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  int blocks = 0;
  const hipError_t e =
      N == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, integrate_kernel<2>, block, 0)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, integrate_kernel<3>, block, 0);
  if (e != hipSuccess) return 0;
  return (int64_t)blocks * (block / 64) * cu;
}

hipError_t launch_integrate(int N, const IntegrateArgs& a, int block, hipStream_t st) {
  const int64_t grid = (api_grid_waves(a.g) * 64 + block - 1) / block;
  if (N == 2)
    hipLaunchKernelGGL(integrate_kernel<2>, dim3((unsigned)grid), dim3(block), 0, st, a);
  else
    hipLaunchKernelGGL(integrate_kernel<3>, dim3((unsigned)grid), dim3(block), 0, st, a);
  return hipGetLastError();
}

static int64_t scan_grid(int64_t n) {
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  return (ntiles + 3) / 4;  // 4 waves per 256-thread block
}

hipError_t launch_scan_reduce(int N, const double* M, int64_t n, double* agg, hipStream_t st) {
  const dim3 grid((unsigned)scan_grid(n)), block(256);
  if (N == 2) hipLaunchKernelGGL(scan_reduce_kernel<2>, grid, block, 0, st, M, n, agg);
  else hipLaunchKernelGGL(scan_reduce_kernel<3>, grid, block, 0, st, M, n, agg);
  return hipGetLastError();
}

hipError_t launch_scan_apply(int N, const double* M, int64_t n, const double* start, double* before,
                             double* after_last, hipStream_t st, double* spin) {
  const dim3 grid((unsigned)scan_grid(n)), block(256);
  if (N == 2)
    hipLaunchKernelGGL(scan_apply_kernel<2>, grid, block, 0, st, M, n, start, before, after_last,
                       spin);
  else
    hipLaunchKernelGGL(scan_apply_kernel<3>, grid, block, 0, st, M, n, start, before, after_last,
                       spin);
  return hipGetLastError();
}

hipError_t launch_scan_top(int N, const double* M1, int64_t n1, const double* start,
                           double* before1, hipStream_t st) {
  const int64_t tiles = (n1 + kScanTile - 1) / kScanTile;
  if (tiles < 1 || tiles > kTopWaves) return hipErrorInvalidValue;
  const dim3 grid(1), block((unsigned)(64 * tiles));
  if (N == 2) hipLaunchKernelGGL(scan_top_kernel<2>, grid, block, 0, st, M1, n1, start, before1);
  else hipLaunchKernelGGL(scan_top_kernel<3>, grid, block, 0, st, M1, n1, start, before1);
  return hipGetLastError();
}

// Workgroups of scan_one_pass_kernel<N> that can be resident at once on the
// current device (0 if unknown); cached per device and N.
static int64_t one_pass_capacity(int N) {
  static int64_t cache[64][2] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  int64_t& c = cache[dev][N - 2];
  if (c) return c;
  int cu = 0, blocks = 0;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  const hipError_t e =
      N == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, scan_one_pass_kernel<2>, 256, 0)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, scan_one_pass_kernel<3>, 256, 0);
  if (e != hipSuccess) return 0;
  c = (int64_t)blocks * cu;
  return c;
}

bool scan_one_pass_fits(int N, int64_t n1) {
  const int64_t blocks = (n1 + 3) / 4;
  return 4 * blocks <= one_pass_capacity(N);
}

hipError_t launch_scan_one_pass(int N, const double* U, int64_t n0, double* M1, double* st1,
                                int64_t n1, int levels, const double* psi0, double* psi,
                                double* psi_final, double* spin, void* sync_tags,
                                hipStream_t st) {
  OnePassArgs a;
  a.M0 = U;
  a.n0 = n0;
  a.M1 = M1;
  a.st1 = st1;
  a.n1 = n1;
  a.psi0 = psi0;
  a.psi = psi;
  a.psi_final = psi_final;
  a.spin = spin;
  a.sync = (ScanSync*)sync_tags;
  a.tags = (unsigned long long*)((char*)sync_tags + sizeof(ScanSync));
  a.levels = levels;
  const dim3 grid((unsigned)((n1 + 3) / 4)), block(256);
  if (N == 2) hipLaunchKernelGGL(scan_one_pass_kernel<2>, grid, block, 0, st, a);
  else hipLaunchKernelGGL(scan_one_pass_kernel<3>, grid, block, 0, st, a);
  return hipGetLastError();
}

hipError_t launch_spin_projection(int N, const double* psi, int64_t K, double* out,
                                  hipStream_t st) {
  const dim3 grid((unsigned)((K + 255) / 256)), block(256);
  if (N == 2) hipLaunchKernelGGL(spin_projection_kernel<2>, grid, block, 0, st, psi, K, out);
  else hipLaunchKernelGGL(spin_projection_kernel<3>, grid, block, 0, st, psi, K, out);
  return hipGetLastError();
}

}  // namespace mss
