// Kernels of the solver path:
//   integrate_kernel<N>  interval operators U_k (CF4 fine steps in the
//                        per-interval rotating frame, frame exit)
//   scan_reduce_kernel<N>, scan_apply_kernel<N>
//                        ordered prefix product psi_{k+1} = U_k psi_k as a
//                        two-level associative scan (wave shuffles)
#include "mss_internal.h"

namespace mss {

// One lane per (interval k, slice s).  The S = 2^slices_log2 slices of an
// interval sit in consecutive lanes of one wave; slice s integrates fine
// steps [s L / S, (s + 1) L / S) and the partial products are combined in
// order (later slices on the left) with wave shuffles.
template <int N>
__global__ void __launch_bounds__(256) integrate_kernel(const IntegrateArgs A) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int sl = A.slices_log2;
  const int64_t k = gid >> sl;
  const int s = (int)(gid & ((1 << sl) - 1));
  const bool active = k < A.K;

  Mat<N> U;
  set_identity<N>(U);
  double tk = 0.0, wr = 0.0;
  if (active) {
    interval_setup(A.fp, A.params, A.t_start, A.dt_out, k, A.frame, &tk, &wr);
    const int l0 = (int)(((int64_t)s * A.L) >> sl);
    const int l1 = (int)(((int64_t)(s + 1) * A.L) >> sl);
    for (int l = l0; l < l1; ++l) {
      double th1[4], th2[4];
      cf4_angles(A.fp, A.params, tk, l, A.dt, wr, th1, th2);
      Mat<N> E;
      Exponentiator<N>::apply(th1, A.tau, E);
      premultiply<N>(E, U);
      Exponentiator<N>::apply(th2, A.tau, E);
      premultiply<N>(E, U);
    }
  }
  for (int d = 1; d < (1 << sl); d <<= 1) {
    const Mat<N> o = shfl_down_mat<N>(U, d);
    if ((s & (2 * d - 1)) == 0) premultiply<N>(o, U);
  }
  if (active && s == 0) {
    exit_frame<N>(wr, A.dt_out, U);
    store_mat<N>(A.U + (size_t)k * 2 * N * N, U);
    if (A.time) A.time[k] = tk;
  }
}

// Product of the lane's (up to) kScanPerLane consecutive matrices, later on the left.
template <int N>
__device__ __forceinline__ void lane_product(const double* __restrict__ M, int64_t n, int64_t base,
                                             Mat<N>& Q) {
  set_identity<N>(Q);
#pragma unroll
  for (int e = 0; e < kScanPerLane; ++e) {
    const int64_t idx = base + e;
    if (idx < n) {
      Mat<N> X;
      load_mat<N>(M + (size_t)idx * 2 * N * N, X);
      premultiply<N>(X, Q);
    }
  }
}

// agg[t] = M[t T + T - 1] ... M[t T], T = kScanTile, one wave per tile.
template <int N>
__global__ void __launch_bounds__(256) scan_reduce_kernel(const double* __restrict__ M, int64_t n,
                                                          double* __restrict__ agg) {
  const int lane = threadIdx.x & 63;
  const int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t base = tile * kScanTile + (int64_t)lane * kScanPerLane;
  Mat<N> Q;
  lane_product<N>(M, n, base, Q);
  for (int d = 1; d < 64; d <<= 1) {
    const Mat<N> o = shfl_down_mat<N>(Q, d);
    if ((lane & (2 * d - 1)) == 0) premultiply<N>(o, Q);
  }
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  if (lane == 0 && tile < ntiles) store_mat<N>(agg + (size_t)tile * 2 * N * N, Q);
}

// before[i] = M[i-1] ... M[t T] start[t] for i in tile t (the state entering
// element i); after_last (optional) = M[n-1] ... M[0] applied likewise.
template <int N>
__global__ void __launch_bounds__(256) scan_apply_kernel(const double* __restrict__ M, int64_t n,
                                                         const double* __restrict__ start,
                                                         double* __restrict__ before,
                                                         double* __restrict__ after_last) {
  const int lane = threadIdx.x & 63;
  const int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t base = tile * kScanTile + (int64_t)lane * kScanPerLane;
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  Mat<N> P;
  lane_product<N>(M, n, base, P);
  // inclusive scan over lanes: P_lane = Q_lane ... Q_0
  for (int d = 1; d < 64; d <<= 1) {
    const Mat<N> o = shfl_up_mat<N>(P, d);
    if (lane >= d) {
      Mat<N> t;
      matmul<N>(P, o, t);
      P = t;
    }
  }
  Mat<N> X = shfl_up_mat<N>(P, 1);
  if (lane == 0) set_identity<N>(X);
  if (tile >= ntiles) return;
  // v = X start[tile]
  double vr[N], vi[N];
  {
    const double* st = start + (size_t)tile * 2 * N;
    double sr[N], si[N];
#pragma unroll
    for (int a = 0; a < N; ++a) {
      sr[a] = st[2 * a];
      si[a] = st[2 * a + 1];
    }
#pragma unroll
    for (int a = 0; a < N; ++a) {
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int b = 0; b < N; ++b) {
        re = fma(X.r[a][b], sr[b], re);
        re = fma(-X.i[a][b], si[b], re);
        im = fma(X.r[a][b], si[b], im);
        im = fma(X.i[a][b], sr[b], im);
      }
      vr[a] = re;
      vi[a] = im;
    }
  }
#pragma unroll
  for (int e = 0; e < kScanPerLane; ++e) {
    const int64_t idx = base + e;
    if (idx < n) {
      double* o = before + (size_t)idx * 2 * N;
#pragma unroll
      for (int a = 0; a < N; ++a) {
        o[2 * a] = vr[a];
        o[2 * a + 1] = vi[a];
      }
      Mat<N> Y;
      load_mat<N>(M + (size_t)idx * 2 * N * N, Y);
      double wr_[N], wi_[N];
#pragma unroll
      for (int a = 0; a < N; ++a) {
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int b = 0; b < N; ++b) {
          re = fma(Y.r[a][b], vr[b], re);
          re = fma(-Y.i[a][b], vi[b], re);
          im = fma(Y.r[a][b], vi[b], im);
          im = fma(Y.i[a][b], vr[b], im);
        }
        wr_[a] = re;
        wi_[a] = im;
      }
#pragma unroll
      for (int a = 0; a < N; ++a) {
        vr[a] = wr_[a];
        vi[a] = wi_[a];
      }
      if (idx == n - 1 && after_last) {
#pragma unroll
        for (int a = 0; a < N; ++a) {
          after_last[2 * a] = vr[a];
          after_last[2 * a + 1] = vi[a];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_integrate(int N, const IntegrateArgs& a, int block, hipStream_t st) {
  const int64_t lanes = a.K << a.slices_log2;
  const int64_t grid = (lanes + block - 1) / block;
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
                             double* after_last, hipStream_t st) {
  const dim3 grid((unsigned)scan_grid(n)), block(256);
  if (N == 2)
    hipLaunchKernelGGL(scan_apply_kernel<2>, grid, block, 0, st, M, n, start, before, after_last);
  else
    hipLaunchKernelGGL(scan_apply_kernel<3>, grid, block, 0, st, M, n, start, before, after_last);
  return hipGetLastError();
}

}  // namespace mss
