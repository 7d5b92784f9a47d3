// Device-side building blocks of the solver: small complex matrices held in
// registers, the two exponentiators, the field-program interpreter and one
// CF4 fine step.  gfx950 only: FP64 on the vector ALUs (a 3x3 complex
// product is 108 FP64 FMAs and not a dense contraction worth MFMA).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mss.h"

namespace mss {

// ---------------------------------------------------------------------------
// constants (IEEE double values of the printed closed forms)
// ---------------------------------------------------------------------------
// Gauss-Legendre nodes (1 -/+ 1/sqrt 3) / 2 and CF4 weights (3 +/- 2 sqrt 3) / 12
// (Sec. "Unitary time evolution and the Magnus expansion", eqs. cf4_sample_1/2).
constexpr double kNode1 = 0x1.b0cb174df99c6p-3;
constexpr double kNode2 = 0x1.93cd3a2c8198ep-1;
constexpr double kWPlus = 0x1.13cd3a2c8198ep-1;
constexpr double kWMinus = -0x1.3cd3a2c8198e0p-5;
constexpr double kTwoPi = 0x1.921fb54442d18p+2;
constexpr double kRsqrt2 = 0x1.6a09e667f3bccp-1;

// Field program as a kernel argument (scalar-loaded, uniform across a wave).
struct FieldProgram {
  int32_t n_terms;
  int32_t pad;
  mss_term t[MSS_MAX_TERMS];
};

// Does a field source provide the full su(3) basis (the field-program
// interpreter does; a user field function gives four components)?
template <class T, class = void>
struct has_full_basis {
  static constexpr bool value = false;
};
template <class T>
struct has_full_basis<T, decltype((void)T::kFullBasis)> {
  static constexpr bool value = T::kFullBasis;
};

// Term sources for the interpreter: the kernel-argument program of a single
// simulation, or a slice of a term table in device memory (batches).
struct ArgTerms {
  static constexpr bool kFullBasis = true;  // field programs may use all eight components
  const FieldProgram& fp;
  __device__ __forceinline__ int size() const { return fp.n_terms; }
  __device__ __forceinline__ const mss_term& operator[](int i) const { return fp.t[i]; }
};
struct TableTerms {
  static constexpr bool kFullBasis = true;
  const mss_term* __restrict__ t;
  int n;
  __device__ __forceinline__ int size() const { return n; }
  __device__ __forceinline__ const mss_term& operator[](int i) const { return t[i]; }
};

template <int N>
struct Mat {
  double r[N][N];
  double i[N][N];
};

template <int N>
__device__ __forceinline__ void set_identity(Mat<N>& m) {
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int b = 0; b < N; ++b) {
      m.r[a][b] = (a == b) ? 1.0 : 0.0;
      m.i[a][b] = 0.0;
    }
}

// C = A * B (complex, N x N), 4 real FMAs per complex multiply-add.
template <int N>
__device__ __forceinline__ void matmul(const Mat<N>& A, const Mat<N>& B, Mat<N>& C) {
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int b = 0; b < N; ++b) {
      double re = A.r[a][0] * B.r[0][b];
      double im = A.r[a][0] * B.i[0][b];
      re = fma(-A.i[a][0], B.i[0][b], re);
      im = fma(A.i[a][0], B.r[0][b], im);
#pragma unroll
      for (int k = 1; k < N; ++k) {
        re = fma(A.r[a][k], B.r[k][b], re);
        re = fma(-A.i[a][k], B.i[k][b], re);
        im = fma(A.r[a][k], B.i[k][b], im);
        im = fma(A.i[a][k], B.r[k][b], im);
      }
      C.r[a][b] = re;
      C.i[a][b] = im;
    }
}

// M <- A * M
template <int N>
__device__ __forceinline__ void premultiply(const Mat<N>& A, Mat<N>& M) {
  Mat<N> t;
  matmul<N>(A, M, t);
  M = t;
}

// y = M x for a complex N x N matrix and an N-vector (re / im parts apart).
template <int N>
__device__ __forceinline__ void matvec(const Mat<N>& M, const double* xr, const double* xi,
                                       double* yr, double* yi) {
#pragma unroll
  for (int a = 0; a < N; ++a) {
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int b = 0; b < N; ++b) {
      re = fma(M.r[a][b], xr[b], re);
      re = fma(-M.i[a][b], xi[b], re);
      im = fma(M.r[a][b], xi[b], im);
      im = fma(M.i[a][b], xr[b], im);
    }
    yr[a] = re;
    yi[a] = im;
  }
}

template <int N>
__device__ __forceinline__ Mat<N> shfl_down_mat(const Mat<N>& m, int d) {
  Mat<N> o;
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int b = 0; b < N; ++b) {
      o.r[a][b] = __shfl_down(m.r[a][b], d, 64);
      o.i[a][b] = __shfl_down(m.i[a][b], d, 64);
    }
  return o;
}

template <int N>
__device__ __forceinline__ Mat<N> shfl_up_mat(const Mat<N>& m, int d) {
  Mat<N> o;
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int b = 0; b < N; ++b) {
      o.r[a][b] = __shfl_up(m.r[a][b], d, 64);
      o.i[a][b] = __shfl_up(m.i[a][b], d, 64);
    }
  return o;
}

template <int N>
__device__ __forceinline__ void load_mat(const double* __restrict__ p, Mat<N>& m) {
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int b = 0; b < N; ++b) {
      m.r[a][b] = p[2 * (a * N + b)];
      m.i[a][b] = p[2 * (a * N + b) + 1];
    }
}

template <int N>
__device__ __forceinline__ void store_mat(double* __restrict__ p, const Mat<N>& m) {
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int b = 0; b < N; ++b) {
      p[2 * (a * N + b)] = m.r[a][b];
      p[2 * (a * N + b) + 1] = m.i[a][b];
    }
}

// ---------------------------------------------------------------------------
// sine and cosine
// ---------------------------------------------------------------------------
// sincos_cw: Cody-Waite reduction x = k pi/2 + r with pi/2 split into three
// doubles (P1, P2 with 32 significant bits so k P1 and k P2 are exact for
// |k| < 2^20; P3 the rest), then the Taylor series of sin r to r^17 and of
// cos r to r^16 on |r| <= pi/4 (truncation < 1e-17), rotated by the
// quadrant k mod 4.  Beyond |x| = 1.5 * 2^20 the reduction is no longer
// exact and ocml's sincos is used.
constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;
constexpr double kPio2_1 = 0x1.921fb54400000p+0;
constexpr double kPio2_2 = 0x1.0b4611a600000p-34;
constexpr double kPio2_3 = 0x1.3198a2e037073p-69;

__device__ __forceinline__ void sincos_cw(double x, double* s, double* c) {
  if (!(fabs(x) < 0x1.8p+20)) {
    sincos(x, s, c);
    return;
  }
  const double k = rint(x * kTwoOverPi);
  double r = fma(-k, kPio2_1, x);
  r = fma(-k, kPio2_2, r);
  r = fma(-k, kPio2_3, r);
  const double r2 = r * r;
  double ps = 0x1.952c77030ad4ap-49;          //  1/17!
  ps = fma(ps, r2, -0x1.ae7f3e733b81fp-41);   // -1/15!
  ps = fma(ps, r2, 0x1.6124613a86d09p-33);    //  1/13!
  ps = fma(ps, r2, -0x1.ae64567f544e4p-26);   // -1/11!
  ps = fma(ps, r2, 0x1.71de3a556c734p-19);    //  1/9!
  ps = fma(ps, r2, -0x1.a01a01a01a01ap-13);   // -1/7!
  ps = fma(ps, r2, 0x1.1111111111111p-7);     //  1/5!
  ps = fma(ps, r2, -0x1.5555555555555p-3);    // -1/3!
  const double sn = fma(r * r2, ps, r);
  double pc = 0x1.ae7f3e733b81fp-45;          //  1/16!
  pc = fma(pc, r2, -0x1.93974a8c07c9dp-37);   // -1/14!
  pc = fma(pc, r2, 0x1.1eed8eff8d898p-29);    //  1/12!
  pc = fma(pc, r2, -0x1.27e4fb7789f5cp-22);   // -1/10!
  pc = fma(pc, r2, 0x1.a01a01a01a01ap-16);    //  1/8!
  pc = fma(pc, r2, -0x1.6c16c16c16c17p-10);   // -1/6!
  pc = fma(pc, r2, 0x1.5555555555555p-5);     //  1/4!
  pc = fma(pc, r2, -0.5);                     // -1/2!
  const double cn = fma(r2, pc, 1.0);
  const int q = ((int)k) & 3;
  const double s1 = (q & 1) ? cn : sn;
  const double c1 = (q & 1) ? sn : cn;
  *s = (q & 2) ? -s1 : s1;
  *c = ((q + 1) & 2) ? -c1 : c1;
}

// Tiny angles inside the exponentiators: below 2^-10 the Taylor series to
// x^5 (sin) and x^6 (cos) is exact to far below one ulp (next terms
// < 2e-22 relative); above it, sincos_cw.
__device__ __forceinline__ void sincos_small(double x, double* s, double* c) {
  if (fabs(x) < 0x1p-10) {
    const double x2 = x * x;
    *s = fma(x * x2, fma(x2, 1.0 / 120.0, -1.0 / 6.0), x);
    *c = fma(x2, fma(x2, fma(x2, -1.0 / 720.0, 1.0 / 24.0), -0.5), 1.0);
  } else {
    sincos_cw(x, s, c);
  }
}

// ---------------------------------------------------------------------------
// spin-1/2 exponential: exp(-i theta . sigma / 2)
// = cos(|theta|/2) I - i sin(|theta|/2) (theta/|theta|) . sigma
// ---------------------------------------------------------------------------
__device__ __forceinline__ void exp_half(const double th[4], int /*tau*/, Mat<2>& E) {
  const double t2 = fma(th[0], th[0], fma(th[1], th[1], th[2] * th[2]));
  const double big = sqrt(t2);
  const double x = 0.5 * big;
  double c, S;  // S = sin(|theta|/2) / |theta|
  if (x < 0x1p-10) {
    const double x2 = x * x;
    c = fma(x2, fma(x2, fma(x2, -1.0 / 720.0, 1.0 / 24.0), -0.5), 1.0);
    S = 0.5 * fma(x2, fma(x2, 1.0 / 120.0, -1.0 / 6.0), 1.0);
  } else {
    double s;
    sincos_cw(x, &s, &c);
    S = s / big;
  }
  E.r[0][0] = c;           E.i[0][0] = -S * th[2];
  E.r[0][1] = -S * th[1];  E.i[0][1] = -S * th[0];
  E.r[1][0] = S * th[1];   E.i[1][0] = -S * th[0];
  E.r[1][1] = c;           E.i[1][1] = S * th[2];
}

// ---------------------------------------------------------------------------
// spin-1 Lie-Trotter exponential (Sec. "Lie-Trotter based exponentiator")
// ---------------------------------------------------------------------------
// T = exp(-iD/2) exp(-i Phi J_phi) exp(-iD/2) with z = theta_z / n,
// q = theta_q / n, Phi = |theta_xy| / n, n = 2^tau (the symmetric split of
// the spin-1 Lie-Trotter step).  With P = diag(e^{-i phi}, 1, e^{i phi}),
// exp(-i Phi J_phi) = P exp(-i Phi J_x) P^H and P commutes with D, so
// T = P T' P^H where T' is the same split at phi = 0.  T' is complex
// symmetric (J_x real symmetric, D diagonal), and so is every residual
// squaring of it (a polynomial in the residual); T^(2^tau) = P T'^(2^tau) P^H.
// The squarings therefore run on the six entries on and above the diagonal
// and the phases e^{-i phi (m_j - m_k)}, m = (1, 0, -1), are put back once.
//
// Complex symmetric 3x3 residual: entries 0..2 the diagonal, 3 = (0,1),
// 4 = (0,2), 5 = (1,2).
struct Sym3 {
  double r[6], i[6];
};

// Residual a' = T' - I, written entry by entry (element-wise form of the
// paper at phi = 0, the T_13 and T_22 misprints corrected); diagonals as
// (e^{i b} - 1) - k S^2 e^{i b} with e^{i b} - 1 = -2 sin^2(b/2) + i sin b,
// so nothing cancels.  Returns e^{i phi} = (theta_x + i theta_y) / rho.
__device__ __forceinline__ void lie_trotter_residual(const double th[4], int tau, Sym3& a,
                                                     double* ep_r, double* ep_i) {
  const double ninv = ldexp(1.0, -tau);
  const double z = th[2] * ninv;
  const double q = th[3] * ninv;
  const double rho = sqrt(fma(th[0], th[0], th[1] * th[1]));  // angles are far from overflow
  const double Phi = rho * ninv;
  double epr = 1.0, epi = 0.0;
  if (rho > 0.0) {
    const double inv = 1.0 / rho;
    epr = th[0] * inv;
    epi = th[1] * inv;
  }
  *ep_r = epr;
  *ep_i = epi;
  double S, C;
  sincos_small(0.5 * Phi, &S, &C);
  const double S2 = S * S;
  const double rs = kRsqrt2 * (2.0 * S * C);  // sin(Phi) / sqrt 2
  double sz, cz, sq, cq;
  sincos_small(0.5 * z, &sz, &cz);           // e^{i z/2}
  sincos_small(q * (1.0 / 6.0), &sq, &cq);   // e^{i q/6}
  // g = e^{iq/6} e^{-iz/2}, h = e^{iq/6} e^{iz/2}
  const double gr = fma(cq, cz, sq * sz), gi = fma(sq, cz, -cq * sz);
  const double hr = fma(cq, cz, -sq * sz), hi = fma(sq, cz, cq * sz);
  // T'_12 = -i rs g, T'_23 = -i rs h; (-i rs) (x + i y) = rs y - i rs x
  a.r[3] = rs * gi;  a.i[3] = -rs * gr;
  a.r[5] = rs * hi;  a.i[5] = -rs * hr;
  // T'_13 = -S^2 e^{-iq/3}
  const double e3r = fma(cq, cq, -sq * sq), e3i = -2.0 * sq * cq;
  a.r[4] = -S2 * e3r;
  a.i[4] = -S2 * e3i;
  // diagonals, b1 = -z - q/3, b2 = 2q/3, b3 = z - q/3: the half-angle
  // exponentials e^{i b_j / 2} are conj(h), conj(e^{-iq/3}) and conj(g)
  const double shv[3] = {-hi, -e3i, -gi};  // sin(b_j / 2)
  const double chv[3] = {hr, e3r, gr};     // cos(b_j / 2)
  const double k[3] = {S2, 2.0 * S2, S2};
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const double sh = shv[j], ch = chv[j];
    const double mr = -2.0 * sh * sh;  // Re(e^{ib} - 1)
    const double mi = 2.0 * sh * ch;   // Im = sin b
    a.r[j] = fma(-k[j], 1.0 + mr, mr);
    a.i[j] = fma(-k[j], mi, mi);
  }
}

// One residual squaring y = (x + 2I) x of a complex symmetric x:
//   y_jj = (x_jj + 2) x_jj + x_jk^2 + x_jl^2
//   y_jk = x_jk (x_jj + 2 + x_kk) + x_jl x_kl        ({j, k, l} = {0, 1, 2})
// 63 instructions where the general 3x3 product takes 111.
__device__ __forceinline__ void residual_square(const Sym3& x, Sym3& y) {
  const double b0 = x.r[0] + 2.0, b1 = x.r[1] + 2.0, b2 = x.r[2] + 2.0;
  // squares of the off-diagonal entries
  double sr[3], si[3];
#pragma unroll
  for (int o = 0; o < 3; ++o) {
    const double xr = x.r[3 + o], xi = x.i[3 + o];
    const double t = xr * xi;
    sr[o] = fma(xr, xr, -xi * xi);
    si[o] = t + t;
  }
  // diagonal j adds the squares of the two off-diagonal entries in its row:
  // row 0: (0,1), (0,2); row 1: (0,1), (1,2); row 2: (0,2), (1,2)
  {
    const double ar = sr[0] + sr[1], ai = si[0] + si[1];
    y.r[0] = fma(b0, x.r[0], fma(-x.i[0], x.i[0], ar));
    y.i[0] = fma(b0, x.i[0], fma(x.i[0], x.r[0], ai));
  }
  {
    const double ar = sr[0] + sr[2], ai = si[0] + si[2];
    y.r[1] = fma(b1, x.r[1], fma(-x.i[1], x.i[1], ar));
    y.i[1] = fma(b1, x.i[1], fma(x.i[1], x.r[1], ai));
  }
  {
    const double ar = sr[1] + sr[2], ai = si[1] + si[2];
    y.r[2] = fma(b2, x.r[2], fma(-x.i[2], x.i[2], ar));
    y.i[2] = fma(b2, x.i[2], fma(x.i[2], x.r[2], ai));
  }
  // (0,1) = x01 (x00 + 2 + x11) + x02 x12
  {
    const double cr = b0 + x.r[1], ci = x.i[0] + x.i[1];
    y.r[3] = fma(x.r[3], cr, fma(-x.i[3], ci, fma(x.r[4], x.r[5], -x.i[4] * x.i[5])));
    y.i[3] = fma(x.r[3], ci, fma(x.i[3], cr, fma(x.r[4], x.i[5], x.i[4] * x.r[5])));
  }
  // (0,2) = x02 (x00 + 2 + x22) + x01 x12
  {
    const double cr = b0 + x.r[2], ci = x.i[0] + x.i[2];
    y.r[4] = fma(x.r[4], cr, fma(-x.i[4], ci, fma(x.r[3], x.r[5], -x.i[3] * x.i[5])));
    y.i[4] = fma(x.r[4], ci, fma(x.i[4], cr, fma(x.r[3], x.i[5], x.i[3] * x.r[5])));
  }
  // (1,2) = x12 (x11 + 2 + x22) + x01 x02
  {
    const double cr = b1 + x.r[2], ci = x.i[1] + x.i[2];
    y.r[5] = fma(x.r[5], cr, fma(-x.i[5], ci, fma(x.r[3], x.r[4], -x.i[3] * x.i[4])));
    y.i[5] = fma(x.r[5], ci, fma(x.i[5], cr, fma(x.r[3], x.i[4], x.i[3] * x.r[4])));
  }
}

// M = P (s + d I) P^H for a complex symmetric s: the off-diagonal entries
// take the phases e^{-i phi (m_j - m_k)}, m = (1, 0, -1), of
// e^{i phi} = (epr, epi); d is added to the real diagonal.
__device__ __forceinline__ void sym_to_full(const Sym3& s, double d, double epr, double epi,
                                            Mat<3>& M) {
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    M.r[j][j] = s.r[j] + d;
    M.i[j][j] = s.i[j];
  }
  // (0,1), (1,2) carry e^{-i phi}, (1,0), (2,1) carry e^{i phi}
  M.r[0][1] = fma(s.r[3], epr, s.i[3] * epi);
  M.i[0][1] = fma(s.i[3], epr, -s.r[3] * epi);
  M.r[1][0] = fma(s.r[3], epr, -s.i[3] * epi);
  M.i[1][0] = fma(s.i[3], epr, s.r[3] * epi);
  M.r[1][2] = fma(s.r[5], epr, s.i[5] * epi);
  M.i[1][2] = fma(s.i[5], epr, -s.r[5] * epi);
  M.r[2][1] = fma(s.r[5], epr, -s.i[5] * epi);
  M.i[2][1] = fma(s.i[5], epr, s.r[5] * epi);
  // (0,2) carries e^{-2i phi}, (2,0) carries e^{2i phi}
  const double e2r = fma(epr, epr, -epi * epi), e2i = 2.0 * epr * epi;
  M.r[0][2] = fma(s.r[4], e2r, s.i[4] * e2i);
  M.i[0][2] = fma(s.i[4], e2r, -s.r[4] * e2i);
  M.r[2][0] = fma(s.r[4], e2r, -s.i[4] * e2i);
  M.i[2][0] = fma(s.i[4], e2r, s.r[4] * e2i);
}

// tau residual squarings a' <- (a' + 2I) a' (two per trip, alternating
// between two register sets, so nothing is copied), then
// E = P (I + a') P^H.
__device__ __forceinline__ void exp_one(const double th[4], int tau, Mat<3>& E) {
  Sym3 a, b;
  double epr, epi;
  lie_trotter_residual(th, tau, a, &epr, &epi);
  for (int s = 0; s + 2 <= tau; s += 2) {
    residual_square(a, b);
    residual_square(b, a);
  }
  if (tau & 1) {
    residual_square(a, b);
    a = b;
  }
  sym_to_full(a, 1.0, epr, epi, E);
}

template <int N> struct Exponentiator;
template <> struct Exponentiator<2> {
  static __device__ __forceinline__ void apply(const double th[4], int tau, Mat<2>& E) {
    exp_half(th, tau, E);
  }
};
template <> struct Exponentiator<3> {
  static __device__ __forceinline__ void apply(const double th[4], int tau, Mat<3>& E) {
    exp_one(th, tau, E);
  }
};

// ---------------------------------------------------------------------------
// field program interpreter and node arithmetic.  Multiply-adds are kept
// unfused here, so node times and phase arguments (up to ~1e6 rad) round
// exactly as the plain definition t_k = t_start + k Dt,
// tau_i = (l + c_i) dt, phase = 2 pi (f t) + phi prescribes.
// ---------------------------------------------------------------------------
template <class Terms>
__device__ __forceinline__ void field_eval(const Terms& fp, const double* __restrict__ params,
                                           double t, double f[4]) {
#pragma clang fp contract(off)
  double fx = 0.0, fy = 0.0, fz = 0.0, fq = 0.0;
  const int nt = fp.size();
  for (int n = 0; n < nt; ++n) {
    const mss_term& tm = fp[n];
    if (!(tm.t_on < t && t < tm.t_off)) continue;
    double amp = tm.a_slot >= 0 ? params[tm.a_slot] : tm.a;
    const double fr = tm.f_slot >= 0 ? params[tm.f_slot] : tm.f;
    double ph = tm.phi_slot >= 0 ? params[tm.phi_slot] : tm.phi;
    const int kind = tm.kind;
    if (kind >= MSS_TERM_PWC) {
      const double x = (t - tm.seg_t0) / tm.seg_len;
      const double fl = floor(x);
      int s = fl < 0.0 ? 0 : (fl > (double)(tm.n_seg - 1) ? tm.n_seg - 1 : (int)fl);
      if (tm.seg_a_slot >= 0) amp = params[tm.seg_a_slot + s];
      if (tm.seg_phi_slot >= 0) ph = params[tm.seg_phi_slot + s];
    }
    double v;
    if (kind == MSS_TERM_CONST || kind == MSS_TERM_PWC) {
      v = amp;
    } else {
      const double ft = fr * t;
      const double x = kTwoPi * ft;
      const double arg = x + ph;
      double sn, cs;
      sincos_cw(arg, &sn, &cs);
      v = amp * ((kind == MSS_TERM_COS || kind == MSS_TERM_PWC_COS) ? cs : sn);
    }
    switch (tm.comp) {
      case 0: fx = fx + v; break;
      case 1: fy = fy + v; break;
      case 2: fz = fz + v; break;
      default: fq = fq + v; break;
    }
  }
  f[0] = fx; f[1] = fy; f[2] = fz; f[3] = fq;
}

// Frame rotations of the two CF4 nodes of a run of fine steps: cos and sin
// of wr tau_i at tau_i = (l + c_i) dt, taken directly at the run's first
// step and advanced by the rotation over one fine step (angle addition),
// so a step costs two complex products instead of two sines and cosines.
struct NodeRotations {
  double c[2], s[2];  // cos, sin of wr tau_i for the current step
  double cd, sd;      // cos, sin of wr dt
  __device__ __forceinline__ void start(double wr, int l, double dt) {
#pragma clang fp contract(off)
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const double tau_i = ((double)l + (i == 0 ? kNode1 : kNode2)) * dt;
      sincos_cw(wr * tau_i, &s[i], &c[i]);
    }
    sincos_cw(wr * dt, &sd, &cd);
  }
  // the node rotations of step l alone, taken directly (no step rotation)
  __device__ __forceinline__ void at(double wr, int l, double dt) {
#pragma clang fp contract(off)
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const double tau_i = ((double)l + (i == 0 ? kNode1 : kNode2)) * dt;
      sincos_cw(wr * tau_i, &s[i], &c[i]);
    }
  }
  __device__ __forceinline__ void advance() {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const double cn = fma(c[i], cd, -s[i] * sd);
      const double sn = fma(s[i], cd, c[i] * sd);
      c[i] = cn;
      s[i] = sn;
    }
  }
};

// Angles theta_{1,2} = omega_bar_{1,2} dt of one CF4 fine step starting at
// t_k + l dt, in the frame rotating at wr about z (wr = 0: lab frame; then
// rot is not read).
template <class Terms>
__device__ __forceinline__ void cf4_angles(const Terms& fp, const double* __restrict__ params,
                                           double tk, int l, double dt, double wr,
                                           const NodeRotations& rot, double th1[4],
                                           double th2[4]) {
#pragma clang fp contract(off)
  double w[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double tau_i = ((double)l + (i == 0 ? kNode1 : kNode2)) * dt;
    double f[4];
    field_eval(fp, params, tk + tau_i, f);
#pragma unroll
    for (int j = 0; j < 4; ++j) w[i][j] = kTwoPi * f[j];
    if (wr != 0.0) {
      // (w_x + i w_y) e^{-i wr tau_i}
      const double c = rot.c[i], s = rot.s[i];
      const double xr = w[i][0] * c + w[i][1] * s;
      const double xi = w[i][1] * c - w[i][0] * s;
      w[i][0] = xr;
      w[i][1] = xi;
      w[i][2] = w[i][2] - wr;
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    th1[j] = (kWPlus * w[0][j] + kWMinus * w[1][j]) * dt;
    th2[j] = (kWMinus * w[0][j] + kWPlus * w[1][j]) * dt;
  }
}

// Angles of one Euler-family step (one exponential): H sampled at the
// midpoint (method 1) or averaged over both ends of the step (method 2).
template <class Terms>
__device__ __forceinline__ void euler_angles(const Terms& fp, const double* __restrict__ params,
                                             double tk, int l, double dt, double wr, int method,
                                             double th[4]) {
#pragma clang fp contract(off)
  const int nn = method == 1 ? 1 : 2;
  double w[2][4];
  for (int i = 0; i < nn; ++i) {
    const double c = method == 1 ? 0.5 : (i == 0 ? 0.0 : 1.0);
    const double tau_i = ((double)l + c) * dt;
    double f[4];
    field_eval(fp, params, tk + tau_i, f);
#pragma unroll
    for (int j = 0; j < 4; ++j) w[i][j] = kTwoPi * f[j];
    if (wr != 0.0) {
      double s, cs;
      sincos_cw(wr * tau_i, &s, &cs);
      const double xr = w[i][0] * cs + w[i][1] * s;
      const double xi = w[i][1] * cs - w[i][0] * s;
      w[i][0] = xr;
      w[i][1] = xi;
      w[i][2] = w[i][2] - wr;
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) th[j] = (method == 1 ? w[0][j] : (w[0][j] + w[1][j]) / 2.0) * dt;
}

// Start time of interval k and the frame rate omega_r = 2 pi f_z(t_k + Dt/2).
template <class Terms>
__device__ __forceinline__ void interval_setup(const Terms& fp, const double* __restrict__ params,
                                               double t_start, double Dt, int64_t k, int frame,
                                               double* tk_out, double* wr_out) {
#pragma clang fp contract(off)
  const double tk = t_start + (double)k * Dt;
  double wr = 0.0;
  if (frame) {
    double f[4];
    field_eval(fp, params, tk + Dt / 2.0, f);
    wr = kTwoPi * f[2];
  }
  *tk_out = tk;
  *wr_out = wr;
}

// U <- diag(exp(-i m wr Dt)) U, m = +s ... -s  (eq. exit_rotating_frame)
template <int N>
__device__ __forceinline__ void exit_frame(double wr, double Dt, Mat<N>& U) {
  if (wr == 0.0) return;
  const double beta = wr * Dt;
#pragma unroll
  for (int a = 0; a < N; ++a) {
    const double m = (N == 2) ? (a == 0 ? 0.5 : -0.5) : (double)(1 - a);
    if (m == 0.0) continue;
    double s, c;
    sincos_cw(-(m * beta), &s, &c);
#pragma unroll
    for (int b = 0; b < N; ++b) {
      const double xr = U.r[a][b], xi = U.i[a][b];
      U.r[a][b] = fma(c, xr, -s * xi);
      U.i[a][b] = fma(c, xi, s * xr);
    }
  }
}

// ---------------------------------------------------------------------------
// spin-1 in the full su(3) basis: components x, y, z, q, u1, u2, v1, v2 of
// H = 2 pi (f_x J_x + f_y J_y + f_z J_z + f_q Q + f_u1 U_1 + f_u2 U_2 + f_v1 V_1
// + f_v2 V_2), with U_1 = J_x^2 - J_y^2, U_2 = J_x J_y + J_y J_x (Delta m = 2)
// and V_1 = J_z J_x + J_x J_z, V_2 = J_y J_z + J_z J_y (Delta m = 1).  A
// spin-1 problem takes this path when a term is on u1, u2, v1 or v2.
// ---------------------------------------------------------------------------
constexpr int kFullComps = 8;

// The field at time t over the eight components, terms summed in list order
// (the interpreter's arithmetic of field_eval).
template <class Terms>
__device__ __forceinline__ void field_eval_full(const Terms& fp, const double* __restrict__ params,
                                                double t, double f[kFullComps]) {
#pragma clang fp contract(off)
#pragma unroll
  for (int j = 0; j < kFullComps; ++j) f[j] = 0.0;
  const int nt = fp.size();
  for (int n = 0; n < nt; ++n) {
    const mss_term& tm = fp[n];
    if (!(tm.t_on < t && t < tm.t_off)) continue;
    double amp = tm.a_slot >= 0 ? params[tm.a_slot] : tm.a;
    const double fr = tm.f_slot >= 0 ? params[tm.f_slot] : tm.f;
    double ph = tm.phi_slot >= 0 ? params[tm.phi_slot] : tm.phi;
    const int kind = tm.kind;
    if (kind >= MSS_TERM_PWC) {
      const double x = (t - tm.seg_t0) / tm.seg_len;
      const double fl = floor(x);
      int s = fl < 0.0 ? 0 : (fl > (double)(tm.n_seg - 1) ? tm.n_seg - 1 : (int)fl);
      if (tm.seg_a_slot >= 0) amp = params[tm.seg_a_slot + s];
      if (tm.seg_phi_slot >= 0) ph = params[tm.seg_phi_slot + s];
    }
    double v;
    if (kind == MSS_TERM_CONST || kind == MSS_TERM_PWC) {
      v = amp;
    } else {
      const double ft = fr * t;
      const double x = kTwoPi * ft;
      const double arg = x + ph;
      double sn, cs;
      sincos_cw(arg, &sn, &cs);
      v = amp * ((kind == MSS_TERM_COS || kind == MSS_TERM_PWC_COS) ? cs : sn);
    }
    switch (tm.comp) {
      case 0: f[0] = f[0] + v; break;
      case 1: f[1] = f[1] + v; break;
      case 2: f[2] = f[2] + v; break;
      case 3: f[3] = f[3] + v; break;
      case 4: f[4] = f[4] + v; break;
      case 5: f[5] = f[5] + v; break;
      case 6: f[6] = f[6] + v; break;
      default: f[7] = f[7] + v; break;
    }
  }
}

// Node field in the rotating frame: (x + i y) and (v1 + i v2) times
// e^{-i wr tau}, (u1 + i u2) times e^{-2i wr tau} (Delta m = 1 and 2 under
// rotations about z), z - wr; (c, s) = (cos, sin)(wr tau).
__device__ __forceinline__ void frame_full(double w[kFullComps], double c, double s, double wr) {
#pragma clang fp contract(off)
  const double c2 = c * c - s * s, s2 = 2.0 * (c * s);
  const double xr = w[0] * c + w[1] * s, xi = w[1] * c - w[0] * s;
  const double ur = w[4] * c2 + w[5] * s2, ui = w[5] * c2 - w[4] * s2;
  const double vr = w[6] * c + w[7] * s, vi = w[7] * c - w[6] * s;
  w[0] = xr;
  w[1] = xi;
  w[2] = w[2] - wr;
  w[4] = ur;
  w[5] = ui;
  w[6] = vr;
  w[7] = vi;
}

template <class Terms>
__device__ __forceinline__ void cf4_angles_full(const Terms& fp, const double* __restrict__ params,
                                                double tk, int l, double dt, double wr,
                                                const NodeRotations& rot,
                                                double th1[kFullComps], double th2[kFullComps]) {
#pragma clang fp contract(off)
  double w[2][kFullComps];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double tau_i = ((double)l + (i == 0 ? kNode1 : kNode2)) * dt;
    double f[kFullComps];
    field_eval_full(fp, params, tk + tau_i, f);
#pragma unroll
    for (int j = 0; j < kFullComps; ++j) w[i][j] = kTwoPi * f[j];
    if (wr != 0.0) frame_full(w[i], rot.c[i], rot.s[i], wr);
  }
#pragma unroll
  for (int j = 0; j < kFullComps; ++j) {
    th1[j] = (kWPlus * w[0][j] + kWMinus * w[1][j]) * dt;
    th2[j] = (kWMinus * w[0][j] + kWPlus * w[1][j]) * dt;
  }
}

template <class Terms>
__device__ __forceinline__ void euler_angles_full(const Terms& fp,
                                                  const double* __restrict__ params, double tk,
                                                  int l, double dt, double wr, int method,
                                                  double th[kFullComps]) {
#pragma clang fp contract(off)
  const int nn = method == 1 ? 1 : 2;
  double w[2][kFullComps] = {};
#pragma unroll
  for (int i = 0; i < 2; ++i) {  // a fixed trip count keeps w in registers
    if (i >= nn) break;
    const double c = method == 1 ? 0.5 : (i == 0 ? 0.0 : 1.0);
    const double tau_i = ((double)l + c) * dt;
    double f[kFullComps];
    field_eval_full(fp, params, tk + tau_i, f);
#pragma unroll
    for (int j = 0; j < kFullComps; ++j) w[i][j] = kTwoPi * f[j];
    if (wr != 0.0) {
      double s, cs;
      sincos_cw(wr * tau_i, &s, &cs);
      frame_full(w[i], cs, s, wr);
    }
  }
#pragma unroll
  for (int j = 0; j < kFullComps; ++j)
    th[j] = (method == 1 ? w[0][j] : (w[0][j] + w[1][j]) / 2.0) * dt;
}

// One general residual squaring y = (x + 2I) x.
__device__ __forceinline__ void residual_square_full(const Mat<3>& x, Mat<3>& y) {
  Mat<3> b = x;
  b.r[0][0] += 2.0;
  b.r[1][1] += 2.0;
  b.r[2][2] += 2.0;
  matmul<3>(b, x, y);
}

// exp(-i G), G = sum_j theta_j A_j over the full basis, by scaling and
// squaring: X = -i G / n with n = 2^tau, the residual of exp(X) from its
// degree-4 Taylor polynomial in Horner form, X (I + X/2 (I + X/3 (I + X/4)))
// (no identity term, nothing cancels), then tau residual squarings, I + a.
__device__ __forceinline__ void exp_full(const double th[kFullComps], int tau, Mat<3>& E) {
  const double ninv = ldexp(1.0, -tau);
  // G entry by entry: J_x, J_y, V_1, V_2 couple neighbouring levels (1/sqrt 2),
  // U_1, U_2 the outer pair; J_z and Q on the diagonal.
  const double g00 = th[2] + th[3] * (1.0 / 3.0);
  const double g11 = th[3] * (-2.0 / 3.0);
  const double g22 = -th[2] + th[3] * (1.0 / 3.0);
  const double g01r = kRsqrt2 * (th[0] + th[6]), g01i = -kRsqrt2 * (th[1] + th[7]);
  const double g12r = kRsqrt2 * (th[0] - th[6]), g12i = -kRsqrt2 * (th[1] - th[7]);
  const double g02r = th[4], g02i = -th[5];
  // X = -i G / n: -i (gr + i gi) = gi - i gr; the lower triangle holds conj(G)
  Mat<3> X;
  X.r[0][0] = 0.0;  X.i[0][0] = -g00 * ninv;
  X.r[1][1] = 0.0;  X.i[1][1] = -g11 * ninv;
  X.r[2][2] = 0.0;  X.i[2][2] = -g22 * ninv;
  X.r[0][1] = g01i * ninv;   X.i[0][1] = -g01r * ninv;
  X.r[1][0] = -g01i * ninv;  X.i[1][0] = -g01r * ninv;
  X.r[1][2] = g12i * ninv;   X.i[1][2] = -g12r * ninv;
  X.r[2][1] = -g12i * ninv;  X.i[2][1] = -g12r * ninv;
  X.r[0][2] = g02i * ninv;   X.i[0][2] = -g02r * ninv;
  X.r[2][0] = -g02i * ninv;  X.i[2][0] = -g02r * ninv;
  Mat<3> a, t;
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      a.r[p][q] = X.r[p][q] * 0.25 + (p == q ? 1.0 : 0.0);
      a.i[p][q] = X.i[p][q] * 0.25;
    }
  const double inv_k[2] = {1.0 / 3.0, 0.5};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    matmul<3>(X, a, t);
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        a.r[p][q] = t.r[p][q] * inv_k[h] + (p == q ? 1.0 : 0.0);
        a.i[p][q] = t.i[p][q] * inv_k[h];
      }
  }
  matmul<3>(X, a, t);
  for (int s = 0; s + 2 <= tau; s += 2) {
    residual_square_full(t, a);
    residual_square_full(a, t);
  }
  if (tau & 1) {
    residual_square_full(t, a);
    t = a;
  }
  E = t;
  E.r[0][0] += 1.0;
  E.r[1][1] += 1.0;
  E.r[2][2] += 1.0;
}

// The wave's issue priority, rotated with the fine step: the hardware slot
// number offsets the rotation, so waves sharing a SIMD take turns at the
// highest of the four levels and advance at the same rate.  (Among waves
// of equal priority the arbiter prefers the older one, which in a
// persistent launch with two blocks per CU runs the first block's waves
// about 2.4 times as fast as the second's for the whole launch.)  Lanes
// may disagree on the step (several slices per interval): the first active
// lane's sets the level.
__device__ __forceinline__ void rotate_priority(int step, int slot) {
  switch (__builtin_amdgcn_readfirstlane(step + slot) & 3) {
    case 0: __builtin_amdgcn_s_setprio(0); break;
    case 1: __builtin_amdgcn_s_setprio(1); break;
    case 2: __builtin_amdgcn_s_setprio(2); break;
    default: __builtin_amdgcn_s_setprio(3); break;
  }
}

// The wave's slot on its SIMD (HW_ID bits 3:0).
__device__ __forceinline__ int wave_slot() {
  return (int)(__builtin_amdgcn_s_getreg(4 | (3 << 11)) & 15u);
}

// Operator of one interval (rows a1-a9) computed by S = 2^sl cooperating
// lanes: slice s integrates fine steps [s L / S, (s + 1) L / S) and the
// partial products are combined in order with wave shuffles; the full
// U_k (frame exit applied) ends up in the lane with s == 0.  Every lane of
// the wave must call this (the shuffles need the whole wave).  SHARE: the
// wave rotates its issue priority every fine step (rotate_priority), for
// launches whose waves wait on one another's results.
template <int N, bool FULL = false, bool SHARE = false, class Terms>
__device__ __forceinline__ void interval_operator(const Terms& terms, const double* __restrict__ params,
                                                  double t_start, double Dt, double dt, int L,
                                                  int tau, int frame, int method, int64_t k, int s,
                                                  int sl, bool active, Mat<N>& U, double* tk_out) {
  static_assert(!FULL || N == 3, "the full basis is spin-1 only");
  set_identity<N>(U);
  double tk = 0.0, wr = 0.0;
  if (active) {
    interval_setup(terms, params, t_start, Dt, k, frame, &tk, &wr);
    const int l0 = (int)(((int64_t)s * L) >> sl);
    const int l1 = (int)(((int64_t)(s + 1) * L) >> sl);
    const int slot = SHARE ? wave_slot() : 0;
    if constexpr (FULL) {
      if (method == 0) {
        NodeRotations rot;
        if (wr != 0.0) rot.start(wr, l0, dt);
        for (int l = l0; l < l1; ++l) {
          if constexpr (SHARE) rotate_priority(l, slot);
          double th1[kFullComps], th2[kFullComps];
          cf4_angles_full(terms, params, tk, l, dt, wr, rot, th1, th2);
          if (wr != 0.0) rot.advance();
          Mat<3> E;
          exp_full(th1, tau, E);
          premultiply<3>(E, U);
          exp_full(th2, tau, E);
          premultiply<3>(E, U);
        }
      } else {
        for (int l = l0; l < l1; ++l) {
          if constexpr (SHARE) rotate_priority(l, slot);
          double th[kFullComps];
          euler_angles_full(terms, params, tk, l, dt, wr, method, th);
          Mat<3> E;
          exp_full(th, tau, E);
          premultiply<3>(E, U);
        }
      }
    } else if (method == 0) {
      NodeRotations rot;
      if (wr != 0.0) rot.start(wr, l0, dt);
      for (int l = l0; l < l1; ++l) {
        if constexpr (SHARE) rotate_priority(l, slot);
        double th1[4], th2[4];
        cf4_angles(terms, params, tk, l, dt, wr, rot, th1, th2);
        if (wr != 0.0) rot.advance();
        Mat<N> E;
        Exponentiator<N>::apply(th1, tau, E);
        premultiply<N>(E, U);
        Exponentiator<N>::apply(th2, tau, E);
        premultiply<N>(E, U);
      }
    } else {
      for (int l = l0; l < l1; ++l) {
        if constexpr (SHARE) rotate_priority(l, slot);
        double th[4];
        euler_angles(terms, params, tk, l, dt, wr, method, th);
        Mat<N> E;
        Exponentiator<N>::apply(th, tau, E);
        premultiply<N>(E, U);
      }
    }
  }
  for (int d = 1; d < (1 << sl); d <<= 1) {
    const Mat<N> o = shfl_down_mat<N>(U, d);
    if ((s & (2 * d - 1)) == 0) premultiply<N>(o, U);
  }
  if (active && s == 0) exit_frame<N>(wr, Dt, U);
  *tk_out = tk;
}

// Time grid, outputs and options of one simulation's integrator launch
// (everything but the field source).  The intervals form up to two
// segments with their own lane-slice counts: segment j holds intervals
// [seg_k0[j], next segment's first or K) on waves from seg_w0[j] on, 64 /
// 2^seg_sl[j] intervals per wave.  A second segment re-slices the intervals
// left over after the last full round of waves more finely, so the final
// round is short.
struct IntervalGrid {
  const double* params;  // the simulation's parameter vector (may be null)
  double* U;             // [K][N][N] complex
  double* time;          // [K] interval start times, or null
  double t_start;
  double dt_out;         // Dt
  double dt;             // Dt / L
  int64_t K;
  int32_t L;
  int32_t tau;
  int32_t frame;
  int32_t method;
  int32_t n_seg;         // 1 or 2
  int32_t seg_sl[2];     // log2 of the lane-slices per interval
  int32_t full;          // spin-1 in the full su(3) basis
  int64_t seg_k0[2];     // first interval of each segment
  int64_t seg_w0[2];     // first wave of each segment
};

// Lane body of the single-simulation integrator: one lane per (interval k,
// slice s), the S = 2^sl slices of an interval in consecutive lanes of one
// wave; the whole wave must call it.  `terms` is any field source
// field_eval accepts.
template <int N, class Terms>
__device__ __forceinline__ void integrate_lanes(const Terms& terms, const IntervalGrid& g) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t wave = gid >> 6;
  const int lane = (int)(gid & 63);
  const int j = (g.n_seg > 1 && wave >= g.seg_w0[1]) ? 1 : 0;  // uniform across the wave
  const int sl = g.seg_sl[j];
  const int64_t k = g.seg_k0[j] + ((wave - g.seg_w0[j]) << (6 - sl)) + (lane >> sl);
  const int s = lane & ((1 << sl) - 1);
  const bool active = k < (j + 1 < g.n_seg ? g.seg_k0[j + 1] : g.K);
  Mat<N> U;
  double tk;
  bool done = false;
  if constexpr (N == 3 && has_full_basis<Terms>::value) {
    if (g.full) {
      interval_operator<3, true>(terms, g.params, g.t_start, g.dt_out, g.dt, g.L, g.tau, g.frame,
                                 g.method, k, s, sl, active, U, &tk);
      done = true;
    }
  }
  if (!done)
    interval_operator<N>(terms, g.params, g.t_start, g.dt_out, g.dt, g.L, g.tau, g.frame,
                         g.method, k, s, sl, active, U, &tk);
  if (active && s == 0) {
    store_mat<N>(g.U + (size_t)k * 2 * N * N, U);
    if (g.time) g.time[k] = tk;
  }
}

}  // namespace mss
