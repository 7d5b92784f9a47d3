// Tile routines of the ordered prefix product psi_{k+1} = U_k psi_k
// (eq. integration_compilation): one wave owns a tile of 64 E consecutive
// N x N operators, each lane a run of E of them.
#pragma once

#include "mss_internal.h"

namespace mss {

// <J_a> = psi^H J_a psi of one state (a = x, y, z): spin-1/2 J = sigma/2;
// spin-1 J_x, J_y with 1/sqrt 2 couplings between neighbouring levels,
// J_z = diag(1, 0, -1).
template <int N>
__device__ __forceinline__ void project_spin(const double* vr, const double* vi, double* j3) {
  double jx, jy, jz;
  if (N == 2) {
    const double ar = vr[0], ai = vi[0], br = vr[1], bi = vi[1];
    // <J_x> = Re(conj(a) b), <J_y> = Im(conj(a) b), <J_z> = (|a|^2 - |b|^2) / 2
    jx = fma(ar, br, ai * bi);
    jy = fma(ar, bi, -ai * br);
    jz = 0.5 * (fma(ar, ar, ai * ai) - fma(br, br, bi * bi));
  } else {
    const double ar = vr[0], ai = vi[0], br = vr[1], bi = vi[1], cr = vr[N - 1], ci = vi[N - 1];
    // conj(a) b + conj(b) c, scaled by sqrt 2 (twice the 1/sqrt 2 couplings)
    const double sr = fma(ar, br, ai * bi) + fma(br, cr, bi * ci);
    const double si = fma(ar, bi, -ai * br) + fma(br, ci, -bi * cr);
    jx = 2.0 * kRsqrt2 * sr;
    jy = 2.0 * kRsqrt2 * si;
    jz = fma(ar, ar, ai * ai) - fma(cr, cr, ci * ci);
  }
  j3[0] = jx;
  j3[1] = jy;
  j3[2] = jz;
}

// Product of the lane's (up to) E consecutive matrices, later on the left
// (the identity for a lane past the end).  The first matrix is loaded as
// the start value: multiplying it into the identity would give the same
// entries.
template <int N, int E>
__device__ __forceinline__ void lane_product(const double* __restrict__ M, int64_t n, int64_t base,
                                             Mat<N>& Q) {
  if (base < n) load_mat<N>(M + (size_t)base * 2 * N * N, Q);
  else set_identity<N>(Q);
#pragma unroll
  for (int e = 1; e < E; ++e) {
    const int64_t idx = base + e;
    if (idx < n) {
      Mat<N> X;
      load_mat<N>(M + (size_t)idx * 2 * N * N, X);
      premultiply<N>(X, Q);
    }
  }
}

// The lane's (up to) E consecutive matrices kept in X, and their product as
// lane_product forms it (the same operations in the same order).
template <int N, int E>
__device__ __forceinline__ void lane_product_keep(const double* __restrict__ M, int64_t n,
                                                  int64_t base, Mat<N>& Q, Mat<N> (&X)[E]) {
#pragma unroll
  for (int e = 0; e < E; ++e)
    if (base + e < n) load_mat<N>(M + (size_t)(base + e) * 2 * N * N, X[e]);
  if (base < n) Q = X[0];
  else set_identity<N>(Q);
#pragma unroll
  for (int e = 1; e < E; ++e)
    if (base + e < n) premultiply<N>(X[e], Q);
}

// Lanes of tile t that hold elements (n elements in all): wave-uniform, at
// most 64, 0 or less past the last tile.
template <int E>
__device__ __forceinline__ int lanes_with_data(int64_t n, int64_t tile) {
  const int64_t left = n - tile * (64 * E);
  return left >= 64 * E ? 64 : (int)((left + E - 1) / E);
}

// Inclusive products over the wave's first L lanes: lane j's P (its Q_j on
// entry) becomes P_j = Q_j ... Q_0 for j < L, by shuffle levels of stride
// 1, 2, 4, ... below L (a level of stride L or more changes no lane below
// L, so stopping there gives those lanes the values the full six levels
// give).  L is wave-uniform.
template <int N>
__device__ __forceinline__ void wave_scan(int lane, int L, Mat<N>& P) {
  for (int d = 1; d < L; d <<= 1) {
    const Mat<N> o = shfl_up_mat<N>(P, d);
    if (lane >= d) {
      Mat<N> t;
      matmul<N>(P, o, t);
      P = t;
    }
  }
}

// Inclusive products over a tile: lane j < L ends with P_j = Q_j ... Q_0,
// Q_j the product of its E elements.  Every lane must call this.
template <int N, int E>
__device__ __forceinline__ void lane_scan(const double* __restrict__ M, int64_t n, int64_t base,
                                          int lane, int L, Mat<N>& P) {
  lane_product<N, E>(M, n, base, P);
  wave_scan<N>(lane, L, P);
}

// Tile reduce: agg = M[tT + T - 1] ... M[tT] of tile t (T = 64 E), one
// wave per tile: the inclusive product of the last lane holding elements,
// so that a tile's aggregate is bit for bit the total that tile_apply's
// scan forms.  M points at element 0 of the sequence, n its length.
template <int N, int E>
__device__ __forceinline__ void tile_reduce(const double* __restrict__ M, int64_t n, int64_t tile,
                                            int lane, double* __restrict__ agg_out) {
  const int64_t base = tile * (64 * E) + (int64_t)lane * E;
  const int L = lanes_with_data<E>(n, tile);
  Mat<N> P;
  lane_scan<N, E>(M, n, base, lane, L, P);
  if (lane == L - 1 && agg_out) store_mat<N>(agg_out, P);
}

// The walk of tile_apply: from the lane's inclusive product P (its Q_j on
// the scan's entry; kept[] its matrices when KEEP), the state entering the
// lane's first element is P_{lane-1} start (start for lane 0), carried
// through its elements; writes before[idx] (and spin, after_last) for the
// lane's elements base .. base + E - 1 below n.  Every lane must call this.
template <int N, int E, bool KEEP>
__device__ __forceinline__ void tile_walk(const Mat<N>& P, const Mat<N> (&kept)[KEEP ? E : 1],
                                          const double* __restrict__ M, int64_t n, int64_t base,
                                          int lane, bool valid, const double* sr,
                                          const double* si, double* __restrict__ before,
                                          double* __restrict__ after_last,
                                          double* __restrict__ spin) {
  Mat<N> X = shfl_up_mat<N>(P, 1);
  if (lane == 0) set_identity<N>(X);
  if (!valid) return;
  double vr[N], vi[N];
  matvec<N>(X, sr, si, vr, vi);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int64_t idx = base + e;
    if (idx < n) {
      double* o = before + (size_t)idx * 2 * N;
#pragma unroll
      for (int a = 0; a < N; ++a) {
        o[2 * a] = vr[a];
        o[2 * a + 1] = vi[a];
      }
      if (spin) project_spin<N>(vr, vi, spin + 3 * idx);
      Mat<N> Y;
      if constexpr (KEEP) Y = kept[e];
      else load_mat<N>(M + (size_t)idx * 2 * N * N, Y);
      double wr_[N], wi_[N];
      matvec<N>(Y, vr, vi, wr_, wi_);
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

// Tile apply: before[i] = M[i-1] ... M[tT] start for i in tile t (the state
// entering element i); after_last (optional) receives M[n-1] ... applied
// when the tile holds the last element; spin (optional, [n][3]) receives
// <J_x>, <J_y>, <J_z> of every state written.  Every lane must call this.
// KEEP: the lane's matrices stay in registers from the scan to the walk
// (one read of M instead of two); the values and operations are the same.
template <int N, int E, bool KEEP = false>
__device__ __forceinline__ void tile_apply(const double* __restrict__ M, int64_t n, int64_t tile,
                                           int lane, bool valid, const double* __restrict__ start,
                                           double* __restrict__ before,
                                           double* __restrict__ after_last,
                                           double* __restrict__ spin = nullptr) {
  const int64_t base = tile * (64 * E) + (int64_t)lane * E;
  // the entering state is read first, so its latency overlaps the scan's
  double sr[N], si[N];
#pragma unroll
  for (int a = 0; a < N; ++a) {
    sr[a] = valid ? start[2 * a] : 0.0;
    si[a] = valid ? start[2 * a + 1] : 0.0;
  }
  Mat<N> P;
  Mat<N> kept[KEEP ? E : 1];
  if constexpr (KEEP) lane_product_keep<N, E>(M, n, base, P, kept);
  else lane_product<N, E>(M, n, base, P);
  wave_scan<N>(lane, lanes_with_data<E>(n, tile), P);
  tile_walk<N, E, KEEP>(P, kept, M, n, base, lane, valid, sr, si, before, after_last, spin);
}

// The state entering element w of a sequence of n <= 64 E elements that
// starts from `start` (every lane gets it): what tile_apply writes for
// element w of tile 0, by the same operations (scan, the lane's prefix
// applied to start, its walk up to w).  The lane's elements stay in
// registers from the scan to the walk.  Every lane must call this.
template <int N, int E>
__device__ __forceinline__ void single_tile_state(const double* __restrict__ M, int64_t n,
                                                  int64_t w, int lane,
                                                  const double* __restrict__ start, double* vr,
                                                  double* vi) {
  const int64_t base = (int64_t)lane * E;
  Mat<N> P;
  Mat<N> kept[E];
  lane_product_keep<N, E>(M, n, base, P, kept);
  wave_scan<N>(lane, lanes_with_data<E>(n, 0), P);
  Mat<N> X = shfl_up_mat<N>(P, 1);
  if (lane == 0) set_identity<N>(X);
  double sr[N], si[N];
#pragma unroll
  for (int a = 0; a < N; ++a) {
    sr[a] = start[2 * a];
    si[a] = start[2 * a + 1];
  }
  double ur[N], ui[N];
  matvec<N>(X, sr, si, ur, ui);
  const int owner = (int)(w / E);
  const int steps = (int)(w % E);
#pragma unroll
  for (int e = 0; e < E - 1; ++e) {
    if (e < steps) {  // wave-uniform
      Mat<N> Y;
      if (base + e < n) Y = kept[e];
      else set_identity<N>(Y);
      double wr_[N], wi_[N];
      matvec<N>(Y, ur, ui, wr_, wi_);
#pragma unroll
      for (int a = 0; a < N; ++a) {
        ur[a] = wr_[a];
        ui[a] = wi_[a];
      }
    }
  }
#pragma unroll
  for (int a = 0; a < N; ++a) {
    vr[a] = __shfl(ur[a], owner, 64);
    vi[a] = __shfl(ui[a], owner, 64);
  }
}

}  // namespace mss
