// CPU oracle for the spin-1/2 / spin-1 time-dependent Schroedinger solver of
// arXiv:2204.05586 ("Spinsim").
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, scalar reference
// that the GPU path is checked against.  Only the tests, the smoke check and
// the benchmark's CPU-baseline leg may load it.  It shares no code, header,
// constant or helper with the GPU library: it parses the same field-program
// data format with its own structures.
//
// Every step follows the paper in its own order and notation:
//   * CF4 step (Sec. "Unitary time evolution and the Magnus expansion",
//     eqs. cf4_sample_1, cf4_sample_2, cf4_implementation):
//     Gauss nodes t_{1,2} = t + (1 -/+ 1/sqrt 3) dt / 2, weights
//     w_{+/-} = (3 +/- 2 sqrt 3) / 12, u = exp(-i Hbar_2 dt) exp(-i Hbar_1 dt).
//   * Spin-1/2 exponential: analytic SU(2) form (Sec. "Lie-Trotter based
//     exponentiator"; the formula itself is not printed, the textbook
//     exp(-i theta.sigma/2) = cos(|theta|/2) I - i sin(|theta|/2) n.sigma is used).
//   * Spin-1 exponential: Lie-Trotter with the symmetric (leapfrog) split
//     T = exp(-i D/2) exp(-i Phi J_phi) exp(-i D/2), n = 2^tau, written
//     element-wise (eq. lie_trotter_4, with its two misprints corrected:
//     T_13 carries exp(-i q/6) inside the square and T_22 = cos(Phi) exp(2iq/3)),
//     built as the residual a = T - I with expm1-style diagonals, then tau
//     residual squarings a <- (a + 2I) a, then I + a.
//   * Spin-1 with the full su(3) basis (Sec. "Spin-one" extension to
//     H = ... + w_u1 U_1 + w_u2 U_2 + w_v1 V_1 + w_v2 V_2): the paper takes
//     U_1, U_2, V_1, V_2 from a reference it does not print, and includes a
//     general exponentiator without describing it.  Readings here:
//     U_1 = J_x^2 - J_y^2, U_2 = J_x J_y + J_y J_x (the Delta m = +-2
//     quadrupoles) and V_1 = J_z J_x + J_x J_z, V_2 = J_y J_z + J_z J_y (the
//     Delta m = +-1 quadrupoles); exp(-i G) by scaling and squaring: the
//     residual of exp(-i G / n), n = 2^tau, as its Taylor polynomial of degree
//     4, then the same tau residual squarings.  A spin-1 problem uses it when
//     any of its terms is on U_1, U_2, V_1 or V_2.
//   * Dynamic rotating frame (Sec. "Dynamically rotating frame"):
//     omega_r = omega_z(t_k + Dt/2); within an interval the transverse field
//     is rotated by exp(-i omega_r (t - t_k)) and omega_z -> omega_z - omega_r;
//     the full-basis pairs (w_u1 + i w_u2) and (w_v1 + i w_v2) by
//     exp(-2i omega_r (t - t_k)) and exp(-i omega_r (t - t_k)) (they carry
//     Delta m = 2 and 1 under rotations about z);
//     on exit U_k = R(-Dt) U_k^r = diag(exp(-i m omega_r Dt)) U_k^r
//     (eq. exit_rotating_frame).
//   * Discretisation (Sec. "Discretization and parallelization"): t_k =
//     t_start + k Dt, L fine steps of dt = Dt / L per interval, each U_k the
//     ordered product of its fine steps, and the state series
//     psi_{k+1} = U_k psi_k (eq. integration_compilation) computed
//     sequentially, as the paper's CPU state compiler does.
//
// Floating point: compiled with -ffp-contract=off on a baseline x86-64
// target, so no multiply-add is ever fused.  Node times and phase arguments
// are formed as t_k = t_start + (k * Dt), tau_i = (l + c_i) * dt,
// t_i = t_k + tau_i and phase = 2 pi * (f * t) + phi.
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

#include <omp.h>

namespace {

// ---- problem description (own copy of the field-program data format) ------
struct OTerm {
  int32_t kind, comp;
  int32_t a_slot, f_slot, phi_slot;
  int32_t n_seg, seg_a_slot, seg_phi_slot;
  double a, f, phi;
  double t_on, t_off;
  double seg_t0, seg_len;
};

// A field function supplied by the caller instead of terms, with the
// paper's calling convention for the user's field function (Sec.
// "Compilation of integrator"): time, sweep parameters, and the field
// sample f_x, f_y, f_z, f_q (Hz) to fill.  Double precision only.
typedef void (*OFieldFn)(double t, const double* params, double* field);

struct OProblem {
  int32_t spin_twice;  // 1: spin-1/2, 2: spin-1
  int32_t n_terms;
  int32_t n_fine;      // L
  int32_t n_squares;   // tau
  int32_t rotating_frame;
  int32_t n_params;
  int32_t method;      // 0: CF4, 1: midpoint (modified Euler), 2: Heun (improved Euler)
  int64_t n_samples;   // K
  double t_start;
  double dt_out;       // Dt
  const OTerm* terms;
  OFieldFn field_fn;   // non-null: the field comes from this function, terms unused
};

enum { K_CONST = 0, K_COS = 1, K_SIN = 2, K_PWC = 3, K_PWC_COS = 4, K_PWC_SIN = 5 };

// field components: x, y, z, q, then the full-basis quadrupoles u1, u2, v1, v2
constexpr int kComps = 8;

// Does the problem need the full su(3) basis (a term on u1, u2, v1 or v2)?
inline bool full_basis(const OProblem& p) {
  if (p.spin_twice != 2 || p.field_fn) return false;
  for (int i = 0; i < p.n_terms; ++i)
    if (p.terms[i].comp >= 4) return true;
  return false;
}

template <class R> using cx = std::complex<R>;

using std::acos;
using std::atan2;
using std::cos;
using std::floor;
using std::hypot;
using std::ldexp;
using std::sin;
using std::sqrt;

template <class R> R two_pi() { return R(2) * acos(R(-1)); }

template <class R> cx<R> expi(R x) { return cx<R>(cos(x), sin(x)); }

// ---- field program ---------------------------------------------------------
template <class R>
R param_or(const R* params, int32_t slot, double literal) {
  return slot >= 0 ? params[slot] : R(literal);
}

template <class R>
R phase(R f, R t, R phi) {
  R ft = f * t;
  R x = two_pi<R>() * ft;
  return x + phi;
}

template <class R>
int64_t segment(const OTerm& tm, R t) {
  R x = (t - R(tm.seg_t0)) / R(tm.seg_len);
  R fl = floor(x);
  int64_t s;
  if (fl < R(0)) s = 0;
  else if (fl > R(tm.n_seg - 1)) s = tm.n_seg - 1;
  else s = (int64_t)fl;
  return s;
}

// The caller's field function (double only: the entry points refuse a field
// function for other number types).
inline void call_field_fn(const OProblem& p, const double* params, double t, double out[4]) {
  p.field_fn(t, params, out);
}
template <class R>
void call_field_fn(const OProblem&, const R*, R, R*) {}

// Field functions f_j(t) in Hz, j = x, y, z, q, u1, u2, v1, v2.  Terms are
// summed in list order.  A field function fills the first four.
template <class R>
void field(const OProblem& p, const R* params, R t, R out[kComps]) {
  for (int j = 0; j < kComps; ++j) out[j] = R(0);
  if (p.field_fn) {
    call_field_fn(p, params, t, out);
    return;
  }
  for (int i = 0; i < p.n_terms; ++i) {
    const OTerm& tm = p.terms[i];
    if (!(R(tm.t_on) < t && t < R(tm.t_off))) continue;
    R v = R(0);
    R amp = param_or(params, tm.a_slot, tm.a);
    R fr = param_or(params, tm.f_slot, tm.f);
    R ph = param_or(params, tm.phi_slot, tm.phi);
    if (tm.kind == K_PWC || tm.kind == K_PWC_COS || tm.kind == K_PWC_SIN) {
      int64_t s = segment(tm, t);
      if (tm.seg_a_slot >= 0) amp = params[tm.seg_a_slot + s];
      if (tm.seg_phi_slot >= 0) ph = params[tm.seg_phi_slot + s];
    }
    switch (tm.kind) {
      case K_CONST: case K_PWC: v = amp; break;
      case K_COS: case K_PWC_COS: v = amp * cos(phase(fr, t, ph)); break;
      case K_SIN: case K_PWC_SIN: v = amp * sin(phase(fr, t, ph)); break;
      default: v = R(0); break;
    }
    out[tm.comp] = out[tm.comp] + v;
  }
}

// ---- forward-mode dual numbers --------------------------------------------
// v + dx e_x + dy e_y with e_x e_x = e_x e_y = e_y e_y = 0: carried through the
// exponentiators they give E together with dE/dtheta_x and dE/dtheta_y.
template <class R>
struct Dual {
  R v, dx, dy;
  Dual() : v(0), dx(0), dy(0) {}
  Dual(R a) : v(a), dx(0), dy(0) {}
  Dual(R a, R b, R c) : v(a), dx(b), dy(c) {}
};
template <class R> Dual<R> operator+(const Dual<R>& a, const Dual<R>& b) { return {a.v + b.v, a.dx + b.dx, a.dy + b.dy}; }
template <class R> Dual<R> operator-(const Dual<R>& a, const Dual<R>& b) { return {a.v - b.v, a.dx - b.dx, a.dy - b.dy}; }
template <class R> Dual<R> operator-(const Dual<R>& a) { return {-a.v, -a.dx, -a.dy}; }
template <class R> Dual<R> operator*(const Dual<R>& a, const Dual<R>& b) {
  return {a.v * b.v, a.dx * b.v + a.v * b.dx, a.dy * b.v + a.v * b.dy};
}
template <class R> Dual<R> operator/(const Dual<R>& a, const Dual<R>& b) {
  const R q = a.v / b.v;
  return {q, (a.dx - q * b.dx) / b.v, (a.dy - q * b.dy) / b.v};
}
template <class R> Dual<R>& operator+=(Dual<R>& a, const Dual<R>& b) { return a = a + b; }
template <class R> Dual<R>& operator-=(Dual<R>& a, const Dual<R>& b) { return a = a - b; }
template <class R> Dual<R>& operator*=(Dual<R>& a, const Dual<R>& b) { return a = a * b; }
template <class R> Dual<R>& operator/=(Dual<R>& a, const Dual<R>& b) { return a = a / b; }
template <class R> bool operator==(const Dual<R>& a, const Dual<R>& b) { return a.v == b.v; }
template <class R> bool operator!=(const Dual<R>& a, const Dual<R>& b) { return a.v != b.v; }
template <class R> Dual<R> cos(const Dual<R>& a) {
  const R s = std::sin(a.v);
  return {std::cos(a.v), -s * a.dx, -s * a.dy};
}
template <class R> Dual<R> sin(const Dual<R>& a) {
  const R c = std::cos(a.v);
  return {std::sin(a.v), c * a.dx, c * a.dy};
}
template <class R> Dual<R> sqrt(const Dual<R>& a) {
  const R r = std::sqrt(a.v);
  return {r, a.dx / (R(2) * r), a.dy / (R(2) * r)};
}
// hypot and atan2 are not differentiable at x = y = 0; the spin-1 factor
// that uses them is, and lie_trotter_residual takes that point apart.
template <class R> Dual<R> hypot(const Dual<R>& x, const Dual<R>& y) {
  const R h = std::hypot(x.v, y.v);
  const R cx_ = x.v / h, sy = y.v / h;
  return {h, cx_ * x.dx + sy * y.dx, cx_ * x.dy + sy * y.dy};
}
template <class R> Dual<R> atan2(const Dual<R>& y, const Dual<R>& x) {
  const R h = std::hypot(x.v, y.v);
  const R cx_ = x.v / h, sy = y.v / h;
  return {std::atan2(y.v, x.v), (cx_ * y.dx - sy * x.dx) / h, (cx_ * y.dy - sy * x.dy) / h};
}
template <class R> Dual<R> ldexp(const Dual<R>& a, int e) {
  return {std::ldexp(a.v, e), std::ldexp(a.dx, e), std::ldexp(a.dy, e)};
}

// ---- small dense complex matrices -----------------------------------------
template <class R, int N>
struct Mat {
  cx<R> m[N][N];
  static Mat identity() {
    Mat r;
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) r.m[i][j] = cx<R>(i == j ? R(1) : R(0), R(0));
    return r;
  }
};

template <class R, int N>
Mat<R, N> matmul(const Mat<R, N>& A, const Mat<R, N>& B) {
  Mat<R, N> C;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      cx<R> s(0, 0);
      for (int k = 0; k < N; ++k) s += A.m[i][k] * B.m[k][j];
      C.m[i][j] = s;
    }
  return C;
}

// ---- exponentiators ---------------------------------------------------------
// Spin-1/2: exp(-i (theta_x J_x + theta_y J_y + theta_z J_z)), J = sigma / 2.
// At theta = 0 the formula is taken at its limit, cos -> 1 and
// sin(|theta|/2)/|theta| -> 1/2: E = I, and with dual numbers the tangent
// -i sigma_a / 2 along theta_a (the map is analytic there; the square root
// of |theta|^2 is not).
template <class R>
Mat<R, 2> exp_half(const R th[3]) {
  const R big2 = th[0] * th[0] + th[1] * th[1] + th[2] * th[2];
  R c = R(1), s = R(1) / R(2);
  if (big2 != R(0)) {
    const R big = sqrt(big2);
    c = cos(big / R(2));
    s = sin(big / R(2)) / big;
  }
  Mat<R, 2> e;
  e.m[0][0] = cx<R>(c, -s * th[2]);
  e.m[0][1] = cx<R>(-s * th[1], -s * th[0]);
  e.m[1][0] = cx<R>(s * th[1], -s * th[0]);
  e.m[1][1] = cx<R>(c, s * th[2]);
  return e;
}

// e^{i beta} - 1 without cancellation.
template <class R>
cx<R> expim1(R beta) {
  R h = sin(beta / R(2));
  return cx<R>(R(-2) * h * h, sin(beta));
}

// Residual a = T - I of the symmetric Lie-Trotter factor (eq. lie_trotter_4,
// corrected) from z = theta_z / n, q = theta_q / n, Phi and e^{i phi}.
template <class R>
Mat<R, 3> lie_trotter_residual_polar(R z, R q, R Phi, cx<R> eiphi) {
  const cx<R> emphi = std::conj(eiphi);  // e^{-i phi}
  const R C = cos(Phi / R(2));
  const R S = sin(Phi / R(2));
  const R sPhi = sin(Phi);
  const R r = R(1) / sqrt(R(2));
  (void)C;
  const cx<R> mi(R(0), R(-1));
  const cx<R> off = mi * cx<R>(r * sPhi, R(0));  // (-i / sqrt 2) sin(Phi)
  Mat<R, 3> a;
  // off-diagonal entries of T (eq. lie_trotter_4, corrected)
  a.m[0][1] = off * expi(q / R(6)) * expi(-z / R(2)) * emphi;
  a.m[1][0] = off * expi(q / R(6)) * expi(-z / R(2)) * eiphi;
  a.m[1][2] = off * expi(q / R(6)) * expi(z / R(2)) * emphi;
  a.m[2][1] = off * expi(q / R(6)) * expi(z / R(2)) * eiphi;
  {
    cx<R> w = cx<R>(S, R(0)) * expi(-q / R(6)) * emphi;
    a.m[0][2] = -(w * w);
    cx<R> v = cx<R>(S, R(0)) * expi(-q / R(6)) * eiphi;
    a.m[2][0] = -(v * v);
  }
  // diagonal entries of T - I: T_11 = C^2 e^{i b1}, T_22 = cos(Phi) e^{i b2},
  // T_33 = C^2 e^{i b3}; T_jj - 1 = (e^{i b} - 1) - k S^2 e^{i b}, k = 1, 2, 1.
  const R b1 = -z - q / R(3);
  const R b2 = R(2) * q / R(3);
  const R b3 = z - q / R(3);
  const R S2 = S * S;
  a.m[0][0] = expim1(b1) - cx<R>(S2, R(0)) * expi(b1);
  a.m[1][1] = expim1(b2) - cx<R>(R(2) * S2, R(0)) * expi(b2);
  a.m[2][2] = expim1(b3) - cx<R>(S2, R(0)) * expi(b3);
  return a;
}

// The same for the step angles theta = (theta_x, theta_y, theta_z, theta_q)
// and n = 2^tau: Phi = rho / n with rho = |theta_x + i theta_y| and
// phi = atan2(theta_y, theta_x) (Sec. "Lie-Trotter based exponentiator";
// phi = atan2(0, 0) = 0 at rho = 0).
template <class R>
Mat<R, 3> lie_trotter_residual(const R th[4], int tau) {
  const R n = ldexp(R(1), tau);
  const R phi = atan2(th[1], th[0]);
  return lie_trotter_residual_polar(th[2] / n, th[3] / n, hypot(th[0], th[1]) / n, expi(phi));
}

// Dual numbers at rho = 0, where Phi and phi have no derivative but T has:
// on the line theta_y = 0 the form at phi = 0 with the signed Phi = theta_x / n
// is T itself (a negative Phi at phi = 0 gives the entries of |Phi| at
// phi = pi), so its tangent is the theta_x part of dT; on theta_x = 0 the
// form at phi = pi/2 (e^{i phi} = i) with Phi = theta_y / n gives the theta_y
// part.  Both evaluate T at Phi = 0, where it does not depend on phi, and the
// chain rule adds the two tangents.
template <class R>
Mat<Dual<R>, 3> lie_trotter_residual(const Dual<R> th[4], int tau) {
  if (std::hypot(th[0].v, th[1].v) != R(0)) {
    const Dual<R> n = ldexp(Dual<R>(R(1)), tau);
    const Dual<R> phi = atan2(th[1], th[0]);
    return lie_trotter_residual_polar(th[2] / n, th[3] / n, hypot(th[0], th[1]) / n, expi(phi));
  }
  using D = Dual<R>;
  const R n = std::ldexp(R(1), tau);
  const cx<D> one(D(R(1)), D(R(0))), i_(D(R(0)), D(R(1)));
  const Mat<D, 3> ax = lie_trotter_residual_polar(th[2] / D(n), th[3] / D(n), th[0] / D(n), one);
  const Mat<D, 3> ay = lie_trotter_residual_polar(D(th[2].v / n), D(th[3].v / n), th[1] / D(n), i_);
  Mat<D, 3> a;
  for (int j = 0; j < 3; ++j)
    for (int k = 0; k < 3; ++k) {
      const cx<D>& x = ax.m[j][k];
      const cx<D>& y = ay.m[j][k];
      a.m[j][k] = cx<D>(D(x.real().v, x.real().dx + y.real().dx, x.real().dy + y.real().dy),
                        D(x.imag().v, x.imag().dx + y.imag().dx, x.imag().dy + y.imag().dy));
    }
  return a;
}

// Spin-1: exp(-i (theta_x J_x + theta_y J_y + theta_z J_z + theta_q Q)) by
// T^(2^tau), squared through the residual a = T - I.
template <class R>
Mat<R, 3> exp_one(const R th[4], int tau) {
  Mat<R, 3> a = lie_trotter_residual(th, tau);
  for (int s = 0; s < tau; ++s) {
    Mat<R, 3> b = a;
    for (int i = 0; i < 3; ++i) b.m[i][i] += cx<R>(R(2), R(0));
    a = matmul(b, a);
  }
  for (int i = 0; i < 3; ++i) a.m[i][i] += cx<R>(R(1), R(0));
  return a;
}

// The eight spin-1 basis operators A_j, j = x, y, z, q, u1, u2, v1, v2, in
// the basis |+1>, |0>, |-1>: J_x, J_y with 1/sqrt 2 couplings between
// neighbouring levels, J_z = diag(1, 0, -1), Q = diag(1, -2, 1) / 3,
// U_1 = J_x^2 - J_y^2, U_2 = J_x J_y + J_y J_x, V_1 = J_z J_x + J_x J_z,
// V_2 = J_y J_z + J_z J_y (products formed here, not written out).
template <class R>
Mat<R, 3> basis_operator(int j) {
  const R r = R(1) / sqrt(R(2));
  Mat<R, 3> Jx, Jy, Jz;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Jx.m[a][b] = Jy.m[a][b] = Jz.m[a][b] = cx<R>(0, 0);
  Jx.m[0][1] = Jx.m[1][0] = Jx.m[1][2] = Jx.m[2][1] = cx<R>(r, 0);
  Jy.m[0][1] = Jy.m[1][2] = cx<R>(0, -r);
  Jy.m[1][0] = Jy.m[2][1] = cx<R>(0, r);
  Jz.m[0][0] = cx<R>(1, 0);
  Jz.m[2][2] = cx<R>(-1, 0);
  auto add = [](const Mat<R, 3>& A, const Mat<R, 3>& B, R sb) {
    Mat<R, 3> C;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) C.m[a][b] = A.m[a][b] + sb * B.m[a][b];
    return C;
  };
  switch (j) {
    case 0: return Jx;
    case 1: return Jy;
    case 2: return Jz;
    case 3: {
      Mat<R, 3> Q = Mat<R, 3>::identity();
      Q.m[0][0] = cx<R>(R(1) / R(3), 0);
      Q.m[1][1] = cx<R>(R(-2) / R(3), 0);
      Q.m[2][2] = cx<R>(R(1) / R(3), 0);
      return Q;
    }
    case 4: return add(matmul(Jx, Jx), matmul(Jy, Jy), R(-1));
    case 5: return add(matmul(Jx, Jy), matmul(Jy, Jx), R(1));
    case 6: return add(matmul(Jz, Jx), matmul(Jx, Jz), R(1));
    default: return add(matmul(Jy, Jz), matmul(Jz, Jy), R(1));
  }
}

// Spin-1, full basis: exp(-i G), G = sum_j theta_j A_j, by scaling and
// squaring.  X = -i G / n with n = 2^tau; the residual of exp(X) from its
// degree-4 Taylor polynomial, a = X + X^2/2 + X^3/6 + X^4/24 (no identity
// term, so nothing cancels), then tau residual squarings and I + a.
template <class R>
Mat<R, 3> exp_full(const R th[kComps], int tau) {
  const R n = ldexp(R(1), tau);
  Mat<R, 3> X;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) X.m[a][b] = cx<R>(0, 0);
  for (int j = 0; j < kComps; ++j) {
    const Mat<R, 3> A = basis_operator<R>(j);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) X.m[a][b] += cx<R>(th[j], 0) * A.m[a][b];
  }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) X.m[a][b] = cx<R>(0, -1) * X.m[a][b] / n;
  Mat<R, 3> a = Mat<R, 3>::identity();  // Horner: I + X/4, I + X/3 (...), I + X/2 (...)
  for (int k = 4; k >= 2; --k) {
    Mat<R, 3> t = matmul(X, a);
    a = Mat<R, 3>::identity();
    for (int i = 0; i < 3; ++i)
      for (int jj = 0; jj < 3; ++jj) a.m[i][jj] += t.m[i][jj] / R(k);
  }
  a = matmul(X, a);
  for (int s = 0; s < tau; ++s) {
    Mat<R, 3> b = a;
    for (int i = 0; i < 3; ++i) b.m[i][i] += cx<R>(R(2), R(0));
    a = matmul(b, a);
  }
  for (int i = 0; i < 3; ++i) a.m[i][i] += cx<R>(R(1), R(0));
  return a;
}

// the exponential of one step's angles (full: the su(3) exponentiator)
template <class R, int N> struct Exp;
template <class R> struct Exp<R, 2> {
  static Mat<R, 2> apply(const R th[kComps], int, bool) { return exp_half(th); }
};
template <class R> struct Exp<R, 3> {
  static Mat<R, 3> apply(const R th[kComps], int tau, bool full) {
    return full ? exp_full(th, tau) : exp_one(th, tau);
  }
};

// magnetic quantum numbers m = s, ..., -s of the basis states
template <class R> R mval(int N, int i) { return N == 2 ? (i == 0 ? R(0.5) : R(-0.5)) : R(1 - i); }

// ---- one output interval -----------------------------------------------------
template <class R, int N>
Mat<R, N> interval_operator(const OProblem& p, const R* params, int64_t k) {
  const R sq3 = sqrt(R(3));
  const R c1 = (R(1) - R(1) / sq3) / R(2);
  const R c2 = (R(1) + R(1) / sq3) / R(2);
  const R wp = (R(3) + R(2) * sq3) / R(12);
  const R wm = (R(3) - R(2) * sq3) / R(12);
  const R Dt = R(p.dt_out);
  const R dt = Dt / R(p.n_fine);
  const R tk = R(p.t_start) + R(k) * Dt;
  R wr = R(0);
  if (p.rotating_frame) {
    R f[kComps];
    field<R>(p, params, tk + Dt / R(2), f);
    wr = two_pi<R>() * f[2];
  }
  const bool full = full_basis(p);
  Mat<R, N> U = Mat<R, N>::identity();
  // sampling nodes (fractions of the fine step) and number of exponentials
  // per step: CF4 two Gauss nodes and two exponentials; the Euler-family
  // comparison methods one exponential of H sampled at the midpoint, or of
  // the average of H at both ends of the step (Sec. "Evaluation of accuracy").
  const int nn = p.method == 1 ? 1 : 2;
  R cnode[2] = {c1, c2};
  if (p.method == 1) cnode[0] = R(1) / R(2);
  if (p.method == 2) {
    cnode[0] = R(0);
    cnode[1] = R(1);
  }
  for (int l = 0; l < p.n_fine; ++l) {
    R w[2][kComps];
    for (int i = 0; i < nn; ++i) {
      const R tau_i = (R(l) + cnode[i]) * dt;
      R f[kComps];
      field<R>(p, params, tk + tau_i, f);
      for (int j = 0; j < kComps; ++j) w[i][j] = two_pi<R>() * f[j];
      // rotating frame: transverse field rotated by exp(-i omega_r (t - t_k))
      cx<R> xy = cx<R>(w[i][0], w[i][1]) * expi(-(wr * tau_i));
      w[i][0] = xy.real();
      w[i][1] = xy.imag();
      w[i][2] = w[i][2] - wr;
      if (full) {
        // Delta m = 2 pair by exp(-2i omega_r (t - t_k)), Delta m = 1 pair by exp(-i ...)
        cx<R> u = cx<R>(w[i][4], w[i][5]) * expi(-(R(2) * (wr * tau_i)));
        cx<R> v = cx<R>(w[i][6], w[i][7]) * expi(-(wr * tau_i));
        w[i][4] = u.real();
        w[i][5] = u.imag();
        w[i][6] = v.real();
        w[i][7] = v.imag();
      }
    }
    R th1[kComps], th2[kComps];
    if (p.method == 0) {
      for (int j = 0; j < kComps; ++j) {
        th1[j] = (wp * w[0][j] + wm * w[1][j]) * dt;
        th2[j] = (wm * w[0][j] + wp * w[1][j]) * dt;
      }
      Mat<R, N> E1 = Exp<R, N>::apply(th1, p.n_squares, full);
      Mat<R, N> E2 = Exp<R, N>::apply(th2, p.n_squares, full);
      U = matmul(E2, matmul(E1, U));
    } else {
      for (int j = 0; j < kComps; ++j)
        th1[j] = (p.method == 1 ? w[0][j] : (w[0][j] + w[1][j]) / R(2)) * dt;
      U = matmul(Exp<R, N>::apply(th1, p.n_squares, full), U);
    }
  }
  // leave the rotating frame: U_k = diag(exp(-i m omega_r Dt)) U_k^r
  for (int i = 0; i < N; ++i) {
    cx<R> ph = expi(-(mval<R>(N, i) * (wr * Dt)));
    for (int j = 0; j < N; ++j) U.m[i][j] = ph * U.m[i][j];
  }
  return U;
}

template <class R, int N>
void store(const Mat<R, N>& M, R* out) {
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      out[2 * (i * N + j)] = M.m[i][j].real();
      out[2 * (i * N + j) + 1] = M.m[i][j].imag();
    }
}

template <class R, int N>
Mat<R, N> load(const R* in) {
  Mat<R, N> M;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) M.m[i][j] = cx<R>(in[2 * (i * N + j)], in[2 * (i * N + j) + 1]);
  return M;
}

template <class R, int N>
void operators(const OProblem& p, const R* params, int64_t k0, int64_t count, R* U) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t c = 0; c < count; ++c) {
    Mat<R, N> M = interval_operator<R, N>(p, params, k0 + c);
    store<R, N>(M, U + 2 * N * N * c);
  }
}

// psi_0 = psi0, psi_{k+1} = U_k psi_k, psi_final = U_{K-1} psi_{K-1}
template <class R, int N>
void states(int64_t K, const R* U, const R* psi0, R* psi, R* psi_final) {
  cx<R> v[N];
  for (int i = 0; i < N; ++i) v[i] = cx<R>(psi0[2 * i], psi0[2 * i + 1]);
  for (int64_t k = 0; k < K; ++k) {
    if (psi) {
      for (int i = 0; i < N; ++i) {
        psi[2 * (N * k + i)] = v[i].real();
        psi[2 * (N * k + i) + 1] = v[i].imag();
      }
    }
    Mat<R, N> M = load<R, N>(U + 2 * N * N * k);
    cx<R> w[N];
    for (int i = 0; i < N; ++i) {
      cx<R> s(0, 0);
      for (int j = 0; j < N; ++j) s += M.m[i][j] * v[j];
      w[i] = s;
    }
    for (int i = 0; i < N; ++i) v[i] = w[i];
  }
  if (psi_final)
    for (int i = 0; i < N; ++i) {
      psi_final[2 * i] = v[i].real();
      psi_final[2 * i + 1] = v[i].imag();
    }
}

template <class R>
int solve(const OProblem* p, const R* params, const R* psi0, R* U, R* psi, R* psi_final) {
  if (!p || p->n_samples < 1 || p->n_fine < 1) return 1;
  const int N = p->spin_twice + 1;
  if (N != 2 && N != 3) return 1;
  std::vector<R> tmp;
  if (!U) {
    tmp.resize((size_t)p->n_samples * 2 * N * N);
    U = tmp.data();
  }
  if (N == 2) {
    operators<R, 2>(*p, params, 0, p->n_samples, U);
    states<R, 2>(p->n_samples, U, psi0, psi, psi_final);
  } else {
    operators<R, 3>(*p, params, 0, p->n_samples, U);
    states<R, 3>(p->n_samples, U, psi0, psi, psi_final);
  }
  return 0;
}


// ---- adjoint: gradient of a final-state population -------------------------
// loss = |psi_final[m]|^2 is differentiated through the same discrete map:
// the costate lambda_final = e_m psi_final[m] (so that dloss = 2 Re lambda^H
// dpsi_final) is pulled back through every operator (lambda_k = U_k^H
// lambda_{k+1}); inside an interval each exponential E contributes
// dloss/dtheta_a = 2 Re(lambda_after^H dE/dtheta_a psi_before), with dE from
// the dual-number exponentiator; the chain rule then runs through the CF4
// weights, the frame rotation of the transverse field and the field terms.
// Gradients exist for parameters used by x and y terms.

template <int N>
void exp_tangents(const double th[4], int tau, Mat<double, N>& E, Mat<double, N>& Ex,
                  Mat<double, N>& Ey) {
  Dual<double> t[kComps] = {Dual<double>(th[0], 1, 0), Dual<double>(th[1], 0, 1),
                            Dual<double>(th[2]), Dual<double>(th[3]), Dual<double>(0.0),
                            Dual<double>(0.0), Dual<double>(0.0), Dual<double>(0.0)};
  Mat<Dual<double>, N> M = Exp<Dual<double>, N>::apply(t, tau, false);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      const cx<Dual<double>>& z = M.m[i][j];
      E.m[i][j] = cx<double>(z.real().v, z.imag().v);
      Ex.m[i][j] = cx<double>(z.real().dx, z.imag().dx);
      Ey.m[i][j] = cx<double>(z.real().dy, z.imag().dy);
    }
}

template <int N>
void matvec(const Mat<double, N>& A, const cx<double>* x, cx<double>* y) {
  for (int i = 0; i < N; ++i) {
    cx<double> s(0, 0);
    for (int j = 0; j < N; ++j) s += A.m[i][j] * x[j];
    y[i] = s;
  }
}

template <int N>
void matvec_h(const Mat<double, N>& A, const cx<double>* x, cx<double>* y) {  // A^H x
  for (int i = 0; i < N; ++i) {
    cx<double> s(0, 0);
    for (int j = 0; j < N; ++j) s += std::conj(A.m[j][i]) * x[j];
    y[i] = s;
  }
}

// 2 Re(l^H A x)
template <int N>
double bilinear(const cx<double>* l, const Mat<double, N>& A, const cx<double>* x) {
  cx<double> Ax[N];
  matvec<N>(A, x, Ax);
  cx<double> s(0, 0);
  for (int i = 0; i < N; ++i) s += std::conj(l[i]) * Ax[i];
  return 2.0 * s.real();
}

// d field-term value / d parameter slots at time t, scaled by G = dloss/df.
void field_param_grad(const OProblem& p, const double* params, double t, double Gx, double Gy,
                      double* grad) {
  for (int i = 0; i < p.n_terms; ++i) {
    const OTerm& tm = p.terms[i];
    if (tm.comp > 1) continue;
    if (!(tm.t_on < t && t < tm.t_off)) continue;
    const double G = tm.comp == 0 ? Gx : Gy;
    int a_slot = tm.a_slot, phi_slot = tm.phi_slot;
    double amp = param_or(params, tm.a_slot, tm.a);
    double ph = param_or(params, tm.phi_slot, tm.phi);
    const double fr = param_or(params, tm.f_slot, tm.f);
    if (tm.kind == K_PWC || tm.kind == K_PWC_COS || tm.kind == K_PWC_SIN) {
      const int64_t s = segment(tm, t);
      if (tm.seg_a_slot >= 0) {
        a_slot = (int)(tm.seg_a_slot + s);
        amp = params[a_slot];
      }
      if (tm.seg_phi_slot >= 0) {
        phi_slot = (int)(tm.seg_phi_slot + s);
        ph = params[phi_slot];
      }
    }
    if (tm.kind == K_CONST || tm.kind == K_PWC) {
      if (a_slot >= 0) grad[a_slot] += G;
      continue;
    }
    const double arg = phase(fr, t, ph);
    const bool is_cos = tm.kind == K_COS || tm.kind == K_PWC_COS;
    const double val = is_cos ? cos(arg) : sin(arg);       // d value / d amp
    const double dar = is_cos ? -amp * sin(arg) : amp * cos(arg);  // d value / d arg
    if (a_slot >= 0) grad[a_slot] += G * val;
    if (phi_slot >= 0) grad[phi_slot] += G * dar;
    if (tm.f_slot >= 0) grad[tm.f_slot] += G * dar * two_pi<double>() * t;
  }
}

template <int N>
void interval_adjoint(const OProblem& p, const double* params, int64_t k, const cx<double>* psi_k,
                      const cx<double>* lam_next, double* grad) {
  const double sq3 = sqrt(3.0);
  const double c1 = (1.0 - 1.0 / sq3) / 2.0;
  const double c2 = (1.0 + 1.0 / sq3) / 2.0;
  const double wp = (3.0 + 2.0 * sq3) / 12.0;
  const double wm = (3.0 - 2.0 * sq3) / 12.0;
  const double Dt = p.dt_out;
  const double dt = Dt / (double)p.n_fine;
  const double tk = p.t_start + (double)k * Dt;
  double wr = 0.0;
  if (p.rotating_frame) {
    double f[kComps];
    field<double>(p, params, tk + Dt / 2.0, f);
    wr = two_pi<double>() * f[2];
  }
  struct Step {
    double tau[2];
    Mat<double, N> E[2], Ex[2], Ey[2];
    cx<double> before[2][N];
  };
  std::vector<Step> steps(p.n_fine);
  cx<double> v[N];
  for (int i = 0; i < N; ++i) v[i] = psi_k[i];
  const double cnode[2] = {c1, c2};
  for (int l = 0; l < p.n_fine; ++l) {
    Step& st = steps[l];
    double w[2][4];
    for (int i = 0; i < 2; ++i) {
      const double tau_i = ((double)l + cnode[i]) * dt;
      st.tau[i] = tau_i;
      double f[kComps];
      field<double>(p, params, tk + tau_i, f);
      for (int j = 0; j < 4; ++j) w[i][j] = two_pi<double>() * f[j];
      cx<double> xy = cx<double>(w[i][0], w[i][1]) * expi(-(wr * tau_i));
      w[i][0] = xy.real();
      w[i][1] = xy.imag();
      w[i][2] = w[i][2] - wr;
    }
    double th[2][4];
    for (int j = 0; j < 4; ++j) {
      th[0][j] = (wp * w[0][j] + wm * w[1][j]) * dt;
      th[1][j] = (wm * w[0][j] + wp * w[1][j]) * dt;
    }
    for (int e = 0; e < 2; ++e) {
      exp_tangents<N>(th[e], p.n_squares, st.E[e], st.Ex[e], st.Ey[e]);
      for (int i = 0; i < N; ++i) st.before[e][i] = v[i];
      cx<double> nv[N];
      matvec<N>(st.E[e], v, nv);
      for (int i = 0; i < N; ++i) v[i] = nv[i];
    }
  }
  // costate at the end of the interval in frame coordinates: R^H lambda_{k+1}
  cx<double> lam[N];
  for (int i = 0; i < N; ++i) lam[i] = expi(mval<double>(N, i) * (wr * Dt)) * lam_next[i];
  for (int l = p.n_fine - 1; l >= 0; --l) {
    Step& st = steps[l];
    double gx[2], gy[2];
    for (int e = 1; e >= 0; --e) {
      gx[e] = bilinear<N>(lam, st.Ex[e], st.before[e]);
      gy[e] = bilinear<N>(lam, st.Ey[e], st.before[e]);
      cx<double> nl[N];
      matvec_h<N>(st.E[e], lam, nl);
      for (int i = 0; i < N; ++i) lam[i] = nl[i];
    }
    // dloss / d omega'_{x,y} at the two nodes
    const double Gp[2][2] = {{dt * (wp * gx[0] + wm * gx[1]), dt * (wp * gy[0] + wm * gy[1])},
                             {dt * (wm * gx[0] + wp * gx[1]), dt * (wm * gy[0] + wp * gy[1])}};
    for (int i = 0; i < 2; ++i) {
      const double a = wr * st.tau[i];
      const double c = cos(a), s = sin(a);
      const double gwx = Gp[i][0] * c - Gp[i][1] * s;
      const double gwy = Gp[i][0] * s + Gp[i][1] * c;
      field_param_grad(p, params, tk + st.tau[i], two_pi<double>() * gwx,
                       two_pi<double>() * gwy, grad);
    }
  }
}

template <int N>
int adjoint_population(const OProblem& p, const double* params, const double* psi0, int m,
                       double* loss, double* grad) {
  const int64_t K = p.n_samples;
  const int P = p.n_params;
  std::vector<double> Ub((size_t)K * 2 * N * N);
  operators<double, N>(p, params, 0, K, Ub.data());
  std::vector<double> psib((size_t)K * 2 * N);
  double fin[2 * N];
  states<double, N>(K, Ub.data(), psi0, psib.data(), fin);
  *loss = fin[2 * m] * fin[2 * m] + fin[2 * m + 1] * fin[2 * m + 1];
  std::vector<cx<double>> lam((size_t)(K + 1) * N, cx<double>(0, 0));
  lam[(size_t)K * N + m] = cx<double>(fin[2 * m], fin[2 * m + 1]);
  for (int64_t k = K - 1; k >= 0; --k) {
    Mat<double, N> Uk = load<double, N>(Ub.data() + (size_t)k * 2 * N * N);
    matvec_h<N>(Uk, &lam[(size_t)(k + 1) * N], &lam[(size_t)k * N]);
  }
  std::vector<double> part((size_t)K * P, 0.0);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t k = 0; k < K; ++k) {
    cx<double> pk[N];
    for (int i = 0; i < N; ++i) pk[i] = cx<double>(psib[(size_t)(k * N + i) * 2], psib[(size_t)(k * N + i) * 2 + 1]);
    interval_adjoint<N>(p, params, k, pk, &lam[(size_t)(k + 1) * N], &part[(size_t)k * P]);
  }
  for (int q = 0; q < P; ++q) {
    double s = 0.0;
    for (int64_t k = 0; k < K; ++k) s += part[(size_t)k * P + q];
    grad[q] = s;
  }
  return 0;
}

}  // namespace

extern "C" {

void oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int oracle_get_threads(void) { return omp_get_max_threads(); }

void oracle_field(const OProblem* p, const double* params, double t, double* out8) {
  field<double>(*p, params, t, out8);
}

void oracle_exp_half(const double* th3, double* out8) {
  store<double, 2>(exp_half<double>(th3), out8);
}

void oracle_exp_one(const double* th4, int tau, double* out18) {
  store<double, 3>(exp_one<double>(th4, tau), out18);
}

void oracle_lie_trotter_residual(const double* th4, int tau, double* out18) {
  store<double, 3>(lie_trotter_residual<double>(th4, tau), out18);
}

void oracle_exp_full(const double* th8, int tau, double* out18) {
  store<double, 3>(exp_full<double>(th8, tau), out18);
}

void oracle_basis_operator(int j, double* out18) {
  store<double, 3>(basis_operator<double>(j), out18);
}

int oracle_operators(const OProblem* p, const double* params, int64_t k0, int64_t count,
                     double* U) {
  if (!p || k0 < 0 || count < 0 || k0 + count > p->n_samples) return 1;
  if (p->spin_twice == 1) operators<double, 2>(*p, params, k0, count, U);
  else if (p->spin_twice == 2) operators<double, 3>(*p, params, k0, count, U);
  else return 1;
  return 0;
}

int oracle_states(int spin_twice, int64_t K, const double* U, const double* psi0, double* psi,
                  double* psi_final) {
  if (spin_twice == 1) states<double, 2>(K, U, psi0, psi, psi_final);
  else if (spin_twice == 2) states<double, 3>(K, U, psi0, psi, psi_final);
  else return 1;
  return 0;
}

// Expected spin projection <J_a>_k = psi_k^H J_a psi_k, a = x, y, z, with the
// spin matrices written out (Sec. "Quantum mechanics background").
int oracle_spin_projection(int spin_twice, int64_t K, const double* psi, double* out) {
  const int N = spin_twice + 1;
  if (N != 2 && N != 3) return 1;
  const double h = 0.5, r = 1.0 / std::sqrt(2.0);
  cx<double> J[3][3][3] = {};
  if (N == 2) {
    J[0][0][1] = h; J[0][1][0] = h;
    J[1][0][1] = cx<double>(0, -h); J[1][1][0] = cx<double>(0, h);
    J[2][0][0] = h; J[2][1][1] = -h;
  } else {
    J[0][0][1] = r; J[0][1][0] = r; J[0][1][2] = r; J[0][2][1] = r;
    J[1][0][1] = cx<double>(0, -r); J[1][1][0] = cx<double>(0, r);
    J[1][1][2] = cx<double>(0, -r); J[1][2][1] = cx<double>(0, r);
    J[2][0][0] = 1; J[2][2][2] = -1;
  }
  for (int64_t k = 0; k < K; ++k) {
    cx<double> v[3];
    for (int i = 0; i < N; ++i) v[i] = cx<double>(psi[2 * (k * N + i)], psi[2 * (k * N + i) + 1]);
    for (int a = 0; a < 3; ++a) {
      cx<double> s(0, 0);
      for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) s += std::conj(v[i]) * J[a][i][j] * v[j];
      out[3 * k + a] = s.real();
    }
  }
  return 0;
}

// loss = |psi_final[m]|^2 and grad[q] = dloss/dparams[q] for q < n_params.
// Returns 1 on bad arguments, 2 if a z or q term uses a parameter slot, 3 for
// a method other than CF4, 4 for a field function (no parameter derivatives).
int oracle_adjoint_population(const OProblem* p, const double* params, const double* psi0, int m,
                              double* loss, double* grad) {
  if (!p || p->n_samples < 1 || p->n_fine < 1 || m < 0 || m > p->spin_twice) return 1;
  if (p->method != 0) return 3;
  if (p->field_fn) return 4;
  if (full_basis(*p)) return 5;
  for (int i = 0; i < p->n_terms; ++i) {
    const OTerm& t = p->terms[i];
    const bool slots = t.a_slot >= 0 || t.f_slot >= 0 || t.phi_slot >= 0 || t.seg_a_slot >= 0 ||
                       t.seg_phi_slot >= 0;
    if (slots && t.comp > 1) return 2;
  }
  if (p->spin_twice == 1) return adjoint_population<2>(*p, params, psi0, m, loss, grad);
  if (p->spin_twice == 2) return adjoint_population<3>(*p, params, psi0, m, loss, grad);
  return 1;
}

int oracle_solve(const OProblem* p, const double* params, const double* psi0, double* U,
                 double* psi, double* psi_final) {
  return solve<double>(p, params, psi0, U, psi, psi_final);
}

// Extended-precision instance (x86 80-bit long double), used for finite
// differences whose step must sit far above the rounding floor.
int oracle_solve_ld(const OProblem* p, const long double* params, const long double* psi0,
                    long double* psi_final) {
  if (p && p->field_fn) return 4;
  return solve<long double>(p, params, psi0, nullptr, nullptr, psi_final);
}

}  // extern "C"
