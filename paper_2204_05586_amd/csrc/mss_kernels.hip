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
  tile_apply<N, kScanPerLane, true>(M, n, tile, lane, valid,
                                    valid ? start + (size_t)tile * 2 * N : nullptr, before,
                                    after_last, spin);
}

// Level 0 of a one-level scan (n1 <= kScanTile tile aggregates A1) with the
// top level folded in: each wave scans its tile (its operators kept in
// registers), forms the state entering its tile from start as the level-1
// apply would (single_tile_state, the same operations), then walks its tile.
// Bitwise the result of the two launches.  The tile's loads are issued
// first, so their latency overlaps the level-1 work.
template <int N>
__global__ void __launch_bounds__(256) scan_apply_fold_kernel(const double* __restrict__ M,
                                                              int64_t n,
                                                              const double* __restrict__ A1,
                                                              int64_t n1,
                                                              const double* __restrict__ start,
                                                              double* __restrict__ before,
                                                              double* __restrict__ after_last,
                                                              double* __restrict__ spin) {
  constexpr int E = kScanPerLane;
  const int lane = threadIdx.x & 63;
  const int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const bool valid = tile < n1;
  const int64_t base = tile * kScanTile + (int64_t)lane * E;
  Mat<N> P;
  Mat<N> kept[E];
  lane_product_keep<N, E>(M, n, base, P, kept);
  wave_scan<N>(lane, lanes_with_data<E>(n, tile), P);
  double sr[N], si[N];
  single_tile_state<N, E>(A1, n1, valid ? tile : 0, lane, start, sr, si);
  tile_walk<N, E, true>(P, kept, M, n, base, lane, valid, sr, si, before, after_last, spin);
}

// Levels 1 and 2 of a two-level scan in one workgroup (n1 <= kTopWaves tiles of
// kScanTile level-1 elements), with one scan pass per wave: wave w forms
// the inclusive products P_j of its tile (lane_scan, as tile_reduce and
// tile_apply do) and leaves the tile total in LDS; wave 0 applies the
// level-2 tile of totals from start (tile_apply); every wave then applies
// its own tile from the state entering it with the P_j it still holds.
// The arithmetic is that of the separate reduce and apply launches, so the
// states are bitwise the same.

template <int N>
__global__ void __launch_bounds__(64 * kTopWaves) scan_top_kernel(const double* __restrict__ M1,
                                                                  int64_t n1,
                                                                  const double* __restrict__ start,
                                                                  double* __restrict__ before1) {
  constexpr int E = kScanPerLane;
  __shared__ double total[kTopWaves * 2 * N * N];
  __shared__ double enter[kTopWaves * 2 * N];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t n2 = blockDim.x >> 6;
  const int64_t base = (int64_t)wave * kScanTile + (int64_t)lane * E;
  const int L = lanes_with_data<E>(n1, wave);
  Mat<N> P;
  lane_scan<N, E>(M1, n1, base, lane, L, P);
  if (lane == L - 1) store_mat<N>(total + (size_t)wave * 2 * N * N, P);
  __syncthreads();
  if (wave == 0) tile_apply<N, E>(total, n2, 0, lane, true, start, enter, nullptr);
  __syncthreads();
  // the state entering this lane's first element: P_{lane-1} x (I x for lane 0)
  double xr[N], xi[N];
#pragma unroll
  for (int a = 0; a < N; ++a) {
    xr[a] = enter[wave * 2 * N + 2 * a];
    xi[a] = enter[wave * 2 * N + 2 * a + 1];
  }
  Mat<N> X = shfl_up_mat<N>(P, 1);
  if (lane == 0) set_identity<N>(X);
  double vr[N], vi[N];
  matvec<N>(X, xr, xi, vr, vi);
  // the lane's elements but its last, all loaded before the first product
  Mat<N> Y[E - 1];
#pragma unroll
  for (int e = 0; e < E - 1; ++e)
    if (base + e < n1) load_mat<N>(M1 + (size_t)(base + e) * 2 * N * N, Y[e]);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int64_t idx = base + e;
    if (idx < n1) {
      double* o = before1 + (size_t)idx * 2 * N;
#pragma unroll
      for (int a = 0; a < N; ++a) {
        o[2 * a] = vr[a];
        o[2 * a + 1] = vi[a];
      }
      if (e + 1 < E) {
        double wr_[N], wi_[N];
        matvec<N>(Y[e < E - 1 ? e : 0], vr, vi, wr_, wi_);
#pragma unroll
        for (int a = 0; a < N; ++a) {
          vr[a] = wr_[a];
          vi[a] = wi_[a];
        }
      }
    }
  }
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

// Launch shape of a scan pass over n elements, one wave per tile: four
// waves per workgroup, or one when the pass has fewer tiles than the
// device has CUs, so that each tile's wave has a CU's load path to itself
// (spin-1/2 1e4-operator scan: reduce 5.2 -> 4.5 us, fold 7.5 -> 6.1 us;
// at 782 tiles one wave per workgroup made the reduce slower).
static void scan_shape(int64_t n, dim3* grid, dim3* block) {
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  const int per = ntiles < api_device_cu_count() ? 1 : 4;
  *grid = dim3((unsigned)((ntiles + per - 1) / per));
  *block = dim3(64 * per);
}

hipError_t launch_scan_reduce(int N, const double* M, int64_t n, double* agg, hipStream_t st) {
  dim3 grid, block;
  scan_shape(n, &grid, &block);
  if (N == 2) hipLaunchKernelGGL(scan_reduce_kernel<2>, grid, block, 0, st, M, n, agg);
  else hipLaunchKernelGGL(scan_reduce_kernel<3>, grid, block, 0, st, M, n, agg);
  return hipGetLastError();
}

hipError_t launch_scan_apply(int N, const double* M, int64_t n, const double* start, double* before,
                             double* after_last, hipStream_t st, double* spin) {
  dim3 grid, block;
  scan_shape(n, &grid, &block);
  if (N == 2)
    hipLaunchKernelGGL(scan_apply_kernel<2>, grid, block, 0, st, M, n, start, before, after_last,
                       spin);
  else
    hipLaunchKernelGGL(scan_apply_kernel<3>, grid, block, 0, st, M, n, start, before, after_last,
                       spin);
  return hipGetLastError();
}

hipError_t launch_scan_apply_fold(int N, const double* M, int64_t n, const double* A1, int64_t n1,
                                  const double* start, double* before, double* after_last,
                                  hipStream_t st, double* spin) {
  if (n1 != (n + kScanTile - 1) / kScanTile || n1 > kScanTile) return hipErrorInvalidValue;
  dim3 grid, block;
  scan_shape(n, &grid, &block);
  if (N == 2)
    hipLaunchKernelGGL(scan_apply_fold_kernel<2>, grid, block, 0, st, M, n, A1, n1, start, before,
                       after_last, spin);
  else
    hipLaunchKernelGGL(scan_apply_fold_kernel<3>, grid, block, 0, st, M, n, A1, n1, start, before,
                       after_last, spin);
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

hipError_t launch_spin_projection(int N, const double* psi, int64_t K, double* out,
                                  hipStream_t st) {
  const dim3 grid((unsigned)((K + 255) / 256)), block(256);
  if (N == 2) hipLaunchKernelGGL(spin_projection_kernel<2>, grid, block, 0, st, psi, K, out);
  else hipLaunchKernelGGL(spin_projection_kernel<3>, grid, block, 0, st, psi, K, out);
  return hipGetLastError();
}

}  // namespace mss
