// Adjoint (C ABI, include/mss.h): gradient of a final-state population
// loss_i = |psi_final_i[m]|^2 with respect to the field parameters of each
// simulation of a batch, by a discrete adjoint of the whole path.
//
//   1. forward: the batch integrator (operators kept) and scan (states);
//   2. seed: loss and the costate lambda_K = e_m psi_final[m] (so that
//      dloss = 2 Re lambda^H dpsi_final), gradients cleared;
//   3. costates lambda_k = U_k^H lambda_{k+1} for all k: the segmented scan
//      run over the reversed, conjugate-transposed operators;
//   4. one lane per (simulation, interval): replay the interval backward
//      from (psi_{k+1}, lambda_{k+1}) in frame coordinates, recovering the
//      state before each exponential as E^H psi (E is unitary), take
//      dloss/dtheta = 2 Re(lambda^H dE/dtheta psi_before) with dE/dtheta
//      from tangent residual squarings (the derivative of exactly the
//      computed exponential), then apply the chain rule through the CF4
//      weights, the frame rotation of the transverse field and the field
//      terms; gradients are summed per segment in registers and added to
//      the output with FP64 atomics.
// Parameters may be used by x and y terms (any kind); a z or q term with a
// parameter slot is rejected (MSS_E_UNSUPPORTED).
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "mss_work.h"

namespace mss {

// ---------------------------------------------------------------------------
// spin-1 exponential with its derivatives along theta_x and theta_y.
//
// E = P(phi) E'(rho) P(phi)^H (exp_one): the symmetric factor E' depends on
// theta_x, theta_y only through rho = |theta_xy| and the phases only through
// phi.  So one tangent direction, d/d rho, goes through the squarings (the
// tangent of a symmetric residual is symmetric too), the phi derivative is
// closed form, dE_jk/d phi = -i (m_j - m_k) E_jk, and
//   dE/dtheta_x = cos(phi) dE/drho - (sin(phi) / rho) dE/dphi,
//   dE/dtheta_y = sin(phi) dE/drho + (cos(phi) / rho) dE/dphi.
// At rho = 0 phi has no derivative, but E is analytic in theta_x, theta_y:
// along +theta_x (phi = 0) dE/dtheta_x = dE/drho = G, and along +theta_y
// dE/dtheta_y = P(pi/2) G P(pi/2)^H, whose entries are -i (m_j - m_k) G_jk
// (the limit of (1 / rho) dE/dphi; G has a zero diagonal and G_13 = 0 there).
// ---------------------------------------------------------------------------

// d a' / d rho of the residual of lie_trotter_residual, term by term from
// the same expressions (a' depends on rho only through Phi = rho / n).
__device__ __forceinline__ void lie_trotter_residual_drho(const double th[4], int tau, Sym3& da) {
  const double ninv = ldexp(1.0, -tau);
  const double z = th[2] * ninv;
  const double q = th[3] * ninv;
  const double rho = sqrt(fma(th[0], th[0], th[1] * th[1]));
  const double Phi = rho * ninv;
  double S, C;
  sincos_small(0.5 * Phi, &S, &C);
  const double dS = 0.5 * ninv * C, dC = -0.5 * ninv * S;
  const double dS2 = 2.0 * S * dS;
  const double drs = kRsqrt2 * (2.0 * fma(dS, C, S * dC));
  double sz, cz, sq, cq;
  sincos_small(0.5 * z, &sz, &cz);
  sincos_small(q * (1.0 / 6.0), &sq, &cq);
  const double gr = fma(cq, cz, sq * sz), gi = fma(sq, cz, -cq * sz);
  const double hr = fma(cq, cz, -sq * sz), hi = fma(sq, cz, cq * sz);
  da.r[3] = drs * gi;  da.i[3] = -drs * gr;
  da.r[5] = drs * hi;  da.i[5] = -drs * hr;
  const double e3r = fma(cq, cq, -sq * sq), e3i = -2.0 * sq * cq;
  da.r[4] = -dS2 * e3r;
  da.i[4] = -dS2 * e3i;
  // diagonals (e^{i b} - 1) - k S^2 e^{i b}: only k S^2 depends on rho
  const double shv[3] = {-hi, -e3i, -gi};
  const double chv[3] = {hr, e3r, gr};
  const double dk[3] = {dS2, 2.0 * dS2, dS2};
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const double sh = shv[j], ch = chv[j];
    const double mr = -2.0 * sh * sh;
    const double mi = 2.0 * sh * ch;
    da.r[j] = -dk[j] * (1.0 + mr);
    da.i[j] = -dk[j] * mi;
  }
}

// index of entry (j, k) of a Sym3
__device__ __forceinline__ constexpr int sym_index(int j, int k) { return j == k ? j : 2 + j + k; }

// Tangent of one residual squaring: for a' <- (a' + 2I) a', the tangent d
// goes to d (a' + I) + (a' + I) d = M + M^T with M = d (a' + I), which is
// symmetric like d: entries M_jk + M_kj, and 2 M_jj on the diagonal.
__device__ __forceinline__ void tangent_square(const Sym3& a, const Sym3& d, Sym3& dn) {
  double br[6], bi[6];  // a' + I
#pragma unroll
  for (int n = 0; n < 6; ++n) {
    br[n] = n < 3 ? a.r[n] + 1.0 : a.r[n];
    bi[n] = a.i[n];
  }
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int k = j; k < 3; ++k) {
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        const int x = sym_index(j, l), y = sym_index(l, k);
        re = fma(d.r[x], br[y], re);
        re = fma(-d.i[x], bi[y], re);
        im = fma(d.r[x], bi[y], im);
        im = fma(d.i[x], br[y], im);
      }
      const int o = sym_index(j, k);
      if (j == k) {
        dn.r[o] = 2.0 * re;
        dn.i[o] = 2.0 * im;
      } else {
#pragma unroll
        for (int l = 0; l < 3; ++l) {
          const int x = sym_index(k, l), y = sym_index(l, j);
          re = fma(d.r[x], br[y], re);
          re = fma(-d.i[x], bi[y], re);
          im = fma(d.r[x], bi[y], im);
          im = fma(d.i[x], br[y], im);
        }
        dn.r[o] = re;
        dn.i[o] = im;
      }
    }
}

// E = exp of the step angles (Lie-Trotter, tau residual squarings) with
// G = dE/drho, the derivative of exactly the computed E, and the chain
// coefficients c = (d rho / d theta_x, d rho / d theta_y, d phi / d theta_x,
// d phi / d theta_y).  Returns false at rho = 0, where c is not defined and
// the angle derivatives come from G alone.
__device__ __forceinline__ bool exp_one_tangent(const double th[4], int tau, Mat<3>& E, Mat<3>& G,
                                                double c[4]) {
  // Three register sets rotate: a step reads (a, d) and writes the new
  // tangent over the free set, then the new residual over d, which the
  // tangent no longer needs; three steps bring the roles back.
  Sym3 X, Y, Z;
  double epr, epi;
  lie_trotter_residual(th, tau, X, &epr, &epi);
  lie_trotter_residual_drho(th, tau, Y);
  int s = 0;
  for (; s + 3 <= tau; s += 3) {
    tangent_square(X, Y, Z);  // (a, d) = (X, Y)
    residual_square(X, Y);
    tangent_square(Y, Z, X);  // (a, d) = (Y, Z)
    residual_square(Y, Z);
    tangent_square(Z, X, Y);  // (a, d) = (Z, X)
    residual_square(Z, X);
  }
  const int r = tau - s;
  if (r == 0) {
    sym_to_full(X, 1.0, epr, epi, E);
    sym_to_full(Y, 0.0, epr, epi, G);
  } else if (r == 1) {
    tangent_square(X, Y, Z);
    residual_square(X, Y);
    sym_to_full(Y, 1.0, epr, epi, E);
    sym_to_full(Z, 0.0, epr, epi, G);
  } else {
    tangent_square(X, Y, Z);
    residual_square(X, Y);
    tangent_square(Y, Z, X);
    residual_square(Y, Z);
    sym_to_full(Z, 1.0, epr, epi, E);
    sym_to_full(X, 0.0, epr, epi, G);
  }
  const double rho = sqrt(fma(th[0], th[0], th[1] * th[1]));
  c[0] = c[1] = c[2] = c[3] = 0.0;
  if (!(rho > 0.0)) return false;
  const double inv = 1.0 / rho;
  c[0] = epr;
  c[1] = epi;
  c[2] = -epi * inv;
  c[3] = epr * inv;
  return true;
}

// Spin-1/2: E = cos(|theta|/2) I - i (sin(|theta|/2)/|theta|) theta.sigma and
// dE/dtheta_dir for dir = x, y.
__device__ __forceinline__ void exp_half_tangent(const double th[4], int /*tau*/, Mat<2>& E,
                                                 Mat<2>& dEx, Mat<2>& dEy) {
  exp_half(th, 0, E);
  const double t2 = fma(th[0], th[0], fma(th[1], th[1], th[2] * th[2]));
  const double big = sqrt(t2);
  const double x = 0.5 * big;
  // c = cos(T/2), S = sin(T/2)/T with T = |theta|:
  //   dc/dtheta_a = -(S/2) theta_a,  dS/dtheta_a = (c/2 - S)/T^2 theta_a,
  // the latter by its series (1/8)(-1/3 + x^2/30 - x^4/840), x = T/2, when small.
  double c, S, dS_over;
  if (x < 0x1p-7) {
    const double x2 = x * x;
    c = fma(x2, fma(x2, fma(x2, -1.0 / 720.0, 1.0 / 24.0), -0.5), 1.0);
    S = 0.5 * fma(x2, fma(x2, 1.0 / 120.0, -1.0 / 6.0), 1.0);
    dS_over = 0.125 * fma(x2, fma(x2, -1.0 / 840.0, 1.0 / 30.0), -1.0 / 3.0);
  } else {
    double s;
    sincos_cw(x, &s, &c);
    S = s / big;
    dS_over = (0.5 * c - S) / t2;
  }
  const double dc_over = -0.5 * S;
#pragma unroll
  for (int dir = 0; dir < 2; ++dir) {
    Mat<2>& dE = dir == 0 ? dEx : dEy;
    const double td = th[dir];
    const double dc = dc_over * td;
    const double dS = dS_over * td;
    const double ex = dir == 0 ? 1.0 : 0.0, ey = dir == 1 ? 1.0 : 0.0;
    // d(S theta_j) = dS theta_j + S e_j
    const double dx = fma(dS, th[0], S * ex), dy = fma(dS, th[1], S * ey), dz = dS * th[2];
    dE.r[0][0] = dc;   dE.i[0][0] = -dz;
    dE.r[0][1] = -dy;  dE.i[0][1] = -dx;
    dE.r[1][0] = dy;   dE.i[1][0] = -dx;
    dE.r[1][1] = dc;   dE.i[1][1] = dz;
  }
}

// ---------------------------------------------------------------------------
// small vector helpers
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void mat_h_vec(const Mat<N>& A, const double* xr, const double* xi,
                                          double* yr, double* yi) {  // y = A^H x
#pragma unroll
  for (int a = 0; a < N; ++a) {
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int b = 0; b < N; ++b) {
      // conj(A[b][a]) x[b]
      re = fma(A.r[b][a], xr[b], re);
      re = fma(A.i[b][a], xi[b], re);
      im = fma(A.r[b][a], xi[b], im);
      im = fma(-A.i[b][a], xr[b], im);
    }
    yr[a] = re;
    yi[a] = im;
  }
}

// 2 Re(l^H A x)
template <int N>
__device__ __forceinline__ double bilinear(const double* lr, const double* li, const Mat<N>& A,
                                           const double* xr, const double* xi) {
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < N; ++a) {
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int b = 0; b < N; ++b) {
      re = fma(A.r[a][b], xr[b], re);
      re = fma(-A.i[a][b], xi[b], re);
      im = fma(A.r[a][b], xi[b], im);
      im = fma(A.i[a][b], xr[b], im);
    }
    // Re(conj(l) (re + i im)) = lr re + li im
    acc = fma(lr[a], re, fma(li[a], im, acc));
  }
  return 2.0 * acc;
}

// 2 Re(l^H (dE/dphi) x) with dE/dphi = -i w E, w_jk = m_j - m_k = k - j:
// Re(conj(l_j) (-i) w E_jk x_k) = w (lr Im(E_jk x_k) - li Re(E_jk x_k)).
__device__ __forceinline__ double bilinear_phi(const double* lr, const double* li, const Mat<3>& E,
                                               const double* xr, const double* xi) {
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (a == b) continue;
      const double er = fma(E.r[a][b], xr[b], -E.i[a][b] * xi[b]);
      const double ei = fma(E.r[a][b], xi[b], E.i[a][b] * xr[b]);
      acc = fma((double)(b - a), fma(lr[a], ei, -li[a] * er), acc);
    }
  return 2.0 * acc;
}

// One exponential of the backward replay: from the state after it (p) and
// the costate after it (l), the state before it b = E^H p, the costate
// before it nl = E^H l, and g = dloss/dtheta_{x,y} = 2 Re(l^H dE/dtheta b).
template <int N> struct TangentStep;
template <> struct TangentStep<2> {
  static __device__ __forceinline__ void apply(const double th[4], int tau, const double* lr,
                                               const double* li, const double* pr,
                                               const double* pi, double* br, double* bi,
                                               double* nlr, double* nli, double* gx, double* gy) {
    Mat<2> E, dEx, dEy;
    exp_half_tangent(th, tau, E, dEx, dEy);
    mat_h_vec<2>(E, pr, pi, br, bi);
    *gx = bilinear<2>(lr, li, dEx, br, bi);
    *gy = bilinear<2>(lr, li, dEy, br, bi);
    mat_h_vec<2>(E, lr, li, nlr, nli);
  }
};
template <> struct TangentStep<3> {
  static __device__ __forceinline__ void apply(const double th[4], int tau, const double* lr,
                                               const double* li, const double* pr,
                                               const double* pi, double* br, double* bi,
                                               double* nlr, double* nli, double* gx, double* gy) {
    Mat<3> E, G;
    double c[4];
    const bool polar = exp_one_tangent(th, tau, E, G, c);
    mat_h_vec<3>(E, pr, pi, br, bi);
    const double grho = bilinear<3>(lr, li, G, br, bi);
    if (polar) {
      const double gphi = bilinear_phi(lr, li, E, br, bi);
      *gx = fma(c[0], grho, c[2] * gphi);
      *gy = fma(c[1], grho, c[3] * gphi);
    } else {  // rho = 0: dE/dtheta_x = G, dE/dtheta_y = -i (m_j - m_k) G_jk
      *gx = grho;
      *gy = bilinear_phi(lr, li, G, br, bi);
    }
    mat_h_vec<3>(E, lr, li, nlr, nli);
  }
};

// ---------------------------------------------------------------------------
// adjoint kernel
// ---------------------------------------------------------------------------
constexpr int kMaxGradTerms = 4;

struct AdjDesc {
  double t_start, dt_out, dt;
  int64_t K;
  int64_t wave_off;            // first wave (64 intervals per wave)
  const double* params;
  double* grad;
  const double* psi;           // forward states [K][N]
  const double* psi_final;     // [N]
  const double* lam_before;    // costates: entry j = lambda_{K-j}, j < K
  int32_t spin_twice, n_terms, term_off, n_fine;
  int32_t tau, frame, n_gterms, pad;
  int32_t gterm[kMaxGradTerms];  // indices (within the simulation's terms) of terms with slots
};

struct AdjArgs {
  const AdjDesc* sims;
  const mss_term* terms;
  int64_t n_waves;
  int32_t n_sims;
};

struct GradAcc {
  int seg;          // current segment (PWC kinds), -1: none yet
  double a, f, ph;  // d loss / d (amplitude, frequency, phase) of the current segment
};

__device__ __forceinline__ void flush(const mss_term& tm, GradAcc& g, double* grad) {
  int a_slot = tm.a_slot, phi_slot = tm.phi_slot;
  if (tm.kind >= MSS_TERM_PWC && g.seg >= 0) {
    if (tm.seg_a_slot >= 0) a_slot = tm.seg_a_slot + g.seg;
    if (tm.seg_phi_slot >= 0) phi_slot = tm.seg_phi_slot + g.seg;
  }
  if (a_slot >= 0 && g.a != 0.0) atomicAdd(grad + a_slot, g.a);
  if (phi_slot >= 0 && g.ph != 0.0) atomicAdd(grad + phi_slot, g.ph);
  if (tm.f_slot >= 0 && g.f != 0.0) atomicAdd(grad + tm.f_slot, g.f);
  g.a = g.f = g.ph = 0.0;
}

// Contribution of one node (time t, d loss / d f_x, f_y = Gx, Gy) to the
// gradient accumulators of the simulation's parameterised terms.
__device__ __forceinline__ void node_grad(const AdjDesc& s, const mss_term* __restrict__ terms,
                                          double t, double Gx, double Gy, GradAcc* acc) {
#pragma clang fp contract(off)
  const double* __restrict__ params = s.params;
#pragma unroll
  for (int g = 0; g < kMaxGradTerms; ++g) {
    if (g >= s.n_gterms) break;
    const mss_term& tm = terms[s.term_off + s.gterm[g]];
    if (!(tm.t_on < t && t < tm.t_off)) continue;
    const double G = tm.comp == MSS_X ? Gx : Gy;
    double amp = tm.a_slot >= 0 ? params[tm.a_slot] : tm.a;
    double ph = tm.phi_slot >= 0 ? params[tm.phi_slot] : tm.phi;
    const double fr = tm.f_slot >= 0 ? params[tm.f_slot] : tm.f;
    if (tm.kind >= MSS_TERM_PWC) {
      const double x = (t - tm.seg_t0) / tm.seg_len;
      const double fl = floor(x);
      const int seg = fl < 0.0 ? 0 : (fl > (double)(tm.n_seg - 1) ? tm.n_seg - 1 : (int)fl);
      if (seg != acc[g].seg) {
        if (acc[g].seg >= 0) flush(tm, acc[g], s.grad);
        acc[g].seg = seg;
      }
      if (tm.seg_a_slot >= 0) amp = params[tm.seg_a_slot + seg];
      if (tm.seg_phi_slot >= 0) ph = params[tm.seg_phi_slot + seg];
    }
    if (tm.kind == MSS_TERM_CONST || tm.kind == MSS_TERM_PWC) {
      acc[g].a += G;
      continue;
    }
    const double ft = fr * t;
    const double arg = kTwoPi * ft + ph;
    double sn, cs;
    sincos_cw(arg, &sn, &cs);
    const bool is_cos = tm.kind == MSS_TERM_COS || tm.kind == MSS_TERM_PWC_COS;
    const double val = is_cos ? cs : sn;
    const double dar = is_cos ? -amp * sn : amp * cs;
    acc[g].a += G * val;
    acc[g].ph += G * dar;
    acc[g].f += G * dar * kTwoPi * t;
  }
}

template <int N>
__device__ __forceinline__ void adjoint_interval(const AdjArgs& A, const AdjDesc& s, int64_t k) {
  const TableTerms terms{A.terms + s.term_off, s.n_terms};
  double tk, wr;
  interval_setup(terms, s.params, s.t_start, s.dt_out, k, s.frame, &tk, &wr);  // CF4 only
  // psi_{k+1}, lambda_{k+1} into frame coordinates: R^H x, R = diag(e^{-i m wr Dt})
  const double* pn = (k + 1 < s.K) ? s.psi + (size_t)(k + 1) * 2 * N : s.psi_final;
  const double* ln = s.lam_before + (size_t)(s.K - 1 - k) * 2 * N;
  double pr[N], pi[N], lr[N], li[N];
  const double beta = wr * s.dt_out;
#pragma unroll
  for (int a = 0; a < N; ++a) {
    const double m = (N == 2) ? (a == 0 ? 0.5 : -0.5) : (double)(1 - a);
    double sn, cs;
    sincos_cw(m * beta, &sn, &cs);
    pr[a] = fma(cs, pn[2 * a], -sn * pn[2 * a + 1]);
    pi[a] = fma(cs, pn[2 * a + 1], sn * pn[2 * a]);
    lr[a] = fma(cs, ln[2 * a], -sn * ln[2 * a + 1]);
    li[a] = fma(cs, ln[2 * a + 1], sn * ln[2 * a]);
  }
  GradAcc acc[kMaxGradTerms];
#pragma unroll
  for (int g = 0; g < kMaxGradTerms; ++g) acc[g] = {-1, 0.0, 0.0, 0.0};
  const double wgt[2][2] = {{kWPlus, kWMinus}, {kWMinus, kWPlus}};  // [node][exponential]
  for (int l = s.n_fine - 1; l >= 0; --l) {
    double th[2][4];
    NodeRotations rot;
    if (wr != 0.0) rot.at(wr, l, s.dt);
    cf4_angles(terms, s.params, tk, l, s.dt, wr, rot, th[0], th[1]);
    double gx[2], gy[2];
    for (int e = 1; e >= 0; --e) {
      // the state before E, the new costate and the angle derivatives
      double br[N], bi[N], nlr[N], nli[N];
      TangentStep<N>::apply(th[e], s.tau, lr, li, pr, pi, br, bi, nlr, nli, &gx[e], &gy[e]);
#pragma unroll
      for (int a = 0; a < N; ++a) {
        pr[a] = br[a];
        pi[a] = bi[a];
        lr[a] = nlr[a];
        li[a] = nli[a];
      }
    }
    // node sensitivities: d loss / d omega'_{x,y}(t_i), rotated back to the lab
    // field, times 2 pi for d / d f
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const double Gxp = s.dt * (wgt[i][0] * gx[0] + wgt[i][1] * gx[1]);
      const double Gyp = s.dt * (wgt[i][0] * gy[0] + wgt[i][1] * gy[1]);
      const double tau_i = ((double)l + (i == 0 ? kNode1 : kNode2)) * s.dt;
      double sn = 0.0, cs = 1.0;
      if (wr != 0.0) sincos_cw(wr * tau_i, &sn, &cs);
      const double Gx = kTwoPi * fma(Gxp, cs, -Gyp * sn);
      const double Gy = kTwoPi * fma(Gxp, sn, Gyp * cs);
      node_grad(s, A.terms, tk + tau_i, Gx, Gy, acc);
    }
  }
#pragma unroll
  for (int g = 0; g < kMaxGradTerms; ++g)
    if (g < s.n_gterms) flush(A.terms[s.term_off + s.gterm[g]], acc[g], s.grad);
}

__global__ void __launch_bounds__(256) adjoint_kernel(const AdjArgs A) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (wave >= A.n_waves) return;
  int lo = 0, hi = A.n_sims - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (A.sims[mid].wave_off <= wave) lo = mid;
    else hi = mid - 1;
  }
  const AdjDesc& s = A.sims[lo];
  const int64_t k = (wave - s.wave_off) * 64 + lane;
  if (k >= s.K) return;
  if (s.spin_twice == 2) adjoint_interval<3>(A, s, k);
  else adjoint_interval<2>(A, s, k);
}

// loss_i and the seed costate lambda_K = e_m psi_final[m]; gradients cleared.
struct SeedArgs {
  const AdjDesc* sims;
  const int64_t* psi0_off;  // complex offsets of psi_final / lambda_K per simulation
  const double* psi_final;
  double* lamK;
  double* loss;
  double* grad;
  int64_t n_grad;
  int32_t n_sims;
  int32_t m;
};

__global__ void adjoint_seed_kernel(const SeedArgs A) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < A.n_grad) A.grad[gid] = 0.0;
  if (gid < A.n_sims) {
    const int N = A.sims[gid].spin_twice + 1;
    const double* f = A.psi_final + 2 * A.psi0_off[gid];
    double* l = A.lamK + 2 * A.psi0_off[gid];
    for (int a = 0; a < N; ++a) {
      l[2 * a] = a == A.m ? f[2 * a] : 0.0;
      l[2 * a + 1] = a == A.m ? f[2 * a + 1] : 0.0;
    }
    A.loss[gid] = f[2 * A.m] * f[2 * A.m] + f[2 * A.m + 1] * f[2 * A.m + 1];
  }
}

// W[j] = U[K - 1 - j]^H within each simulation (operators packed by op_off).
struct ReverseArgs {
  const AdjDesc* sims;
  const int64_t* op_off;    // complex offsets per simulation (n + 1)
  const int64_t* mat_off;   // matrix-count prefix per simulation (n + 1)
  const double* U;
  double* W;
  int64_t n_mats;
  int32_t n_sims;
};

__global__ void adjoint_reverse_kernel(const ReverseArgs A) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= A.n_mats) return;
  int lo = 0, hi = A.n_sims - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (A.mat_off[mid] <= gid) lo = mid;
    else hi = mid - 1;
  }
  const int64_t j = gid - A.mat_off[lo];
  const int64_t K = A.sims[lo].K;
  const int N = A.sims[lo].spin_twice + 1;
  const double* src = A.U + 2 * (A.op_off[lo] + (K - 1 - j) * N * N);
  double* dst = A.W + 2 * (A.op_off[lo] + j * N * N);
  for (int a = 0; a < N; ++a)
    for (int b = 0; b < N; ++b) {
      dst[2 * (a * N + b)] = src[2 * (b * N + a)];
      dst[2 * (a * N + b) + 1] = -src[2 * (b * N + a) + 1];
    }
}

}  // namespace mss

using namespace mss;

// ---------------------------------------------------------------------------
// host
// ---------------------------------------------------------------------------
struct mss_adjoint_plan {
  int32_t n = 0;
  int32_t m = 0;
  std::vector<mss_problem> probs;
  std::vector<std::vector<mss_term>> term_store;
  std::vector<int64_t> psi0_off, state_off, op_off, mat_off, param_off;
  std::vector<size_t> scan_off;
  int64_t n_params_total = 0, n_mats = 0, n_waves = 0;
  size_t scan_bytes = 0;
  WorkSet fwd, bwd;
  std::vector<AdjDesc> adj;
  std::vector<mss_term> terms;
  // workspace layout (bytes)
  size_t o_counter = 0, o_U = 0, o_W = 0, o_psi = 0, o_fin = 0, o_lamK = 0, o_lam = 0,
         o_lam0 = 0, o_scan = 0, ws_bytes = 0;
  int grid_blocks = 0;
  // device descriptors: [fwd image | bwd image | adj | terms | offsets]
  void* desc = nullptr;
  std::vector<char> image;
  size_t f_sims = 0, f_terms = 0, b_sims = 0, b_terms = 0, a_sims = 0, a_terms = 0, a_psi0 = 0,
         a_op = 0, a_mat = 0;
  std::vector<size_t> f_red, f_app, b_red, b_app;
  size_t f_base = 0, b_base = 0;
  DevWork dfwd, dbwd;
  const void* bound[5] = {};
  bool have_bind = false;
  hipEvent_t last_run = nullptr;
  mss_sampler forward = nullptr;  // the shared field compiled in, for the forward pass
};

namespace {

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

void release(mss_adjoint_plan* P) {
  if (!P) return;
  if (P->last_run) (void)hipEventSynchronize(P->last_run);
  if (P->last_run) (void)hipEventDestroy(P->last_run);
  if (P->desc) (void)hipFree(P->desc);
  delete P;
}

void pack_all(mss_adjoint_plan* P) {
  std::vector<char>& img = P->image;
  size_t off = 0;
  auto reserve = [&](size_t b) {
    const size_t o = off;
    off = a256(off + b);
    return o;
  };
  P->f_base = reserve(P->fwd.packed_bytes());
  P->b_base = reserve(P->bwd.packed_bytes());
  P->a_sims = reserve(P->adj.size() * sizeof(AdjDesc));
  P->a_terms = reserve(std::max<size_t>(1, P->terms.size()) * sizeof(mss_term));
  P->a_psi0 = reserve(P->psi0_off.size() * 8);
  P->a_op = reserve(P->op_off.size() * 8);
  P->a_mat = reserve(P->mat_off.size() * 8);
  img.assign(off, 0);
  P->fwd.pack(img.data() + P->f_base, &P->f_sims, &P->f_terms, &P->f_red, &P->f_app);
  P->bwd.pack(img.data() + P->b_base, &P->b_sims, &P->b_terms, &P->b_red, &P->b_app);
  memcpy(img.data() + P->a_sims, P->adj.data(), P->adj.size() * sizeof(AdjDesc));
  if (!P->terms.empty()) memcpy(img.data() + P->a_terms, P->terms.data(), P->terms.size() * sizeof(mss_term));
  memcpy(img.data() + P->a_psi0, P->psi0_off.data(), P->psi0_off.size() * 8);
  memcpy(img.data() + P->a_op, P->op_off.data(), P->op_off.size() * 8);
  memcpy(img.data() + P->a_mat, P->mat_off.data(), P->mat_off.size() * 8);
}

template <class T>
T* shift(T* base, int64_t off) {
  return base ? base + off : nullptr;
}

mss_status bind(mss_adjoint_plan* P, const double* params, const double* psi0, double* grad,
                double* loss, void* ws) {
  const void* key[5] = {params, psi0, grad, loss, ws};
  bool same = P->have_bind;
  for (int i = 0; i < 5 && same; ++i) same = P->bound[i] == key[i];
  if (same) return MSS_OK;
  if (P->have_bind) {
    hipError_t e = hipEventSynchronize(P->last_run);
    if (e != hipSuccess) return api_hip_fail(e, "adjoint wait");
  }
  char* w = (char*)ws;
  double* U = (double*)(w + P->o_U);
  double* W = (double*)(w + P->o_W);
  double* psi = (double*)(w + P->o_psi);
  double* fin = (double*)(w + P->o_fin);
  double* lamK = (double*)(w + P->o_lamK);
  double* lam = (double*)(w + P->o_lam);
  double* lam0 = (double*)(w + P->o_lam0);
  for (int i = 0; i < P->n; ++i) {
    SimDesc& f = P->fwd.sims[i];
    f.params = shift(params, P->param_off[i]);
    f.psi0 = psi0 + 2 * P->psi0_off[i];
    f.psi = psi + 2 * P->state_off[i];
    f.psi_final = fin + 2 * P->psi0_off[i];
    f.U = U + 2 * P->op_off[i];
    f.scan_ws = (double*)(w + P->o_scan + P->scan_off[i]);
    SimDesc& b = P->bwd.sims[i];
    b.params = f.params;
    b.psi0 = lamK + 2 * P->psi0_off[i];
    b.psi = lam + 2 * P->state_off[i];
    b.psi_final = lam0 + 2 * P->psi0_off[i];
    b.U = W + 2 * P->op_off[i];
    b.scan_ws = f.scan_ws;
    AdjDesc& a = P->adj[i];
    a.params = f.params;
    a.grad = grad + P->param_off[i];
    a.psi = f.psi;
    a.psi_final = f.psi_final;
    a.lam_before = b.psi;
  }
  pack_all(P);
  hipError_t e = hipMemcpy(P->desc, P->image.data(), P->image.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return api_hip_fail(e, "adjoint descriptor upload");
  const char* d = (const char*)P->desc;
  P->dfwd = device_view(P->fwd, d + P->f_base, P->f_sims, P->f_terms, P->f_red, P->f_app);
  P->dbwd = device_view(P->bwd, d + P->b_base, P->b_sims, P->b_terms, P->b_red, P->b_app);
  for (int i = 0; i < 5; ++i) P->bound[i] = key[i];
  P->have_bind = true;
  return MSS_OK;
}

}  // namespace

extern "C" {

mss_status mss_adjoint_plan_create_compiled(int32_t n, const mss_problem* problems,
                                            const int64_t* param_off, int32_t level_m,
                                            mss_sampler forward, mss_adjoint_plan** out) {
  if (!out) return api_fail(MSS_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!forward) return api_fail(MSS_E_INVALID, "forward sampler is NULL");
  if (n < 1 || !problems) return api_fail(MSS_E_INVALID, "need at least one problem");
  for (int i = 0; i < n; ++i) {
    mss_status s = api_validate_problem(&problems[i]);
    if (s != MSS_OK) {
      std::string msg = api_last_error_copy();
      return api_fail(s, "simulation %d: %s", i, msg.c_str());
    }
    if (!api_sampler_is_for_terms(forward, problems[i].terms, problems[i].n_terms))
      return api_fail(MSS_E_INVALID,
                      "simulation %d: the forward sampler was not generated from its terms", i);
  }
  mss_status s = mss_adjoint_plan_create(n, problems, param_off, level_m, out);
  if (s != MSS_OK) return s;
  (*out)->forward = forward;
  return api_ok();
}

mss_status mss_adjoint_plan_create(int32_t n, const mss_problem* problems, const int64_t* param_off,
                                   int32_t level_m, mss_adjoint_plan** out) {
  if (!out) return api_fail(MSS_E_INVALID, "out is NULL");
  *out = nullptr;
  if (n < 1 || !problems) return api_fail(MSS_E_INVALID, "need at least one problem");
  for (int i = 0; i < n; ++i) {
    const mss_problem& q = problems[i];
    mss_status s = api_validate_problem(&q);
    if (s != MSS_OK) {
      std::string msg = api_last_error_copy();
      return api_fail(s, "simulation %d: %s", i, msg.c_str());
    }
    if (q.method != MSS_CF4)
      return api_fail(MSS_E_UNSUPPORTED, "simulation %d: gradients need the CF4 method", i);
    if (api_full_basis(&q))
      return api_fail(MSS_E_UNSUPPORTED,
                      "simulation %d: gradients are not defined for the full su(3) basis", i);
    if (level_m < 0 || level_m > q.spin_twice)
      return api_fail(MSS_E_INVALID, "simulation %d: level %d outside 0..%d", i, level_m,
                      q.spin_twice);
    if (q.n_params > 0 && (!param_off || param_off[i] < 0))
      return api_fail(MSS_E_INVALID, "simulation %d has parameters but no valid param_off", i);
    int ng = 0;
    for (int t = 0; t < q.n_terms; ++t) {
      const mss_term& tm = q.terms[t];
      const bool slots = tm.a_slot >= 0 || tm.f_slot >= 0 || tm.phi_slot >= 0 ||
                         tm.seg_a_slot >= 0 || tm.seg_phi_slot >= 0;
      if (!slots) continue;
      if (tm.comp != MSS_X && tm.comp != MSS_Y)
        return api_fail(MSS_E_UNSUPPORTED,
                        "simulation %d, term %d: gradients need parameter slots on x and y terms only",
                        i, t);
      ++ng;
    }
    if (ng > kMaxGradTerms)
      return api_fail(MSS_E_UNSUPPORTED, "simulation %d: more than %d parameterised terms", i,
                      kMaxGradTerms);
  }
  mss_adjoint_plan* P = new (std::nothrow) mss_adjoint_plan();
  if (!P) return api_fail(MSS_E_NOMEM, "host allocation failed");
  P->n = n;
  P->m = level_m;
  P->psi0_off.assign(n + 1, 0);
  P->state_off.assign(n + 1, 0);
  P->op_off.assign(n + 1, 0);
  P->mat_off.assign(n + 1, 0);
  P->param_off.assign(n, 0);
  P->scan_off.assign(n, 0);
  size_t scan = 0;
  int64_t waves = 0, pend = 0;
  for (int i = 0; i < n; ++i) {
    const mss_problem& q = problems[i];
    const int N = q.spin_twice + 1;
    P->psi0_off[i + 1] = P->psi0_off[i] + N;
    P->state_off[i + 1] = P->state_off[i] + q.n_samples * N;
    P->op_off[i + 1] = P->op_off[i] + q.n_samples * N * N;
    P->mat_off[i + 1] = P->mat_off[i] + q.n_samples;
    P->param_off[i] = q.n_params > 0 ? param_off[i] : 0;
    pend = std::max<int64_t>(pend, P->param_off[i] + q.n_params);
    P->scan_off[i] = scan;
    scan += scan_scratch_bytes(N, q.n_samples);
    P->fwd.add(q, 0, 0, q.n_samples, true);
    P->bwd.add(q, 0, 0, 0, true);
    AdjDesc a;
    memset(&a, 0, sizeof a);
    a.t_start = q.t_start;
    a.dt_out = q.dt_out;
    a.dt = q.dt_out / (double)q.n_fine;
    a.K = q.n_samples;
    a.wave_off = waves;
    waves += (q.n_samples + 63) / 64;
    a.spin_twice = q.spin_twice;
    a.n_terms = q.n_terms;
    a.term_off = (int32_t)P->terms.size();
    a.n_fine = q.n_fine;
    a.tau = q.spin_twice == 2 ? q.n_squares : 0;
    a.frame = q.rotating_frame;
    for (int t = 0; t < q.n_terms; ++t) {
      const mss_term& tm = q.terms[t];
      P->terms.push_back(tm);
      if (tm.a_slot >= 0 || tm.f_slot >= 0 || tm.phi_slot >= 0 || tm.seg_a_slot >= 0 ||
          tm.seg_phi_slot >= 0)
        a.gterm[a.n_gterms++] = t;
    }
    P->adj.push_back(a);
  }
  P->fwd.finalize();
  P->bwd.finalize();
  P->n_params_total = pend;
  P->n_mats = P->mat_off[n];
  P->n_waves = waves;
  P->scan_bytes = scan;
  // workspace layout
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off = a256(off + b);
    return o;
  };
  P->o_counter = take(256);
  P->o_U = take((size_t)P->op_off[n] * 16);
  P->o_W = take((size_t)P->op_off[n] * 16);
  P->o_psi = take((size_t)P->state_off[n] * 16);
  P->o_fin = take((size_t)P->psi0_off[n] * 16);
  P->o_lamK = take((size_t)P->psi0_off[n] * 16);
  P->o_lam = take((size_t)P->state_off[n] * 16);
  P->o_lam0 = take((size_t)P->psi0_off[n] * 16);
  P->o_scan = take(scan);
  P->ws_bytes = off;
  pack_all(P);
  hipError_t e = hipMalloc(&P->desc, P->image.size());
  if (e == hipSuccess) e = hipEventCreateWithFlags(&P->last_run, hipEventDisableTiming);
  if (e != hipSuccess) {
    release(P);
    return api_hip_fail(e, "adjoint plan");
  }
  const int cu = api_device_cu_count();
  P->grid_blocks = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)cu * 2, (P->fwd.n_items + 3) / 4));
  *out = P;
  return api_ok();
}

mss_status mss_adjoint_workspace_size(const mss_adjoint_plan* P, size_t* bytes) {
  if (!P || !bytes) return api_fail(MSS_E_INVALID, "plan and bytes are required");
  *bytes = P->ws_bytes;
  return api_ok();
}

mss_status mss_adjoint_param_count(const mss_adjoint_plan* P, int64_t* count) {
  if (!P || !count) return api_fail(MSS_E_INVALID, "plan and count are required");
  *count = P->n_params_total;
  return api_ok();
}

mss_status mss_adjoint_run(mss_adjoint_plan* P, const double* params, const double* psi0,
                           double* loss, double* grad, double* psi_final, void* ws,
                           size_t ws_bytes, void* stream) {
  if (!P) return api_fail(MSS_E_INVALID, "plan is NULL");
  if (!psi0 || !loss || (!grad && P->n_params_total > 0))
    return api_fail(MSS_E_INVALID, "psi0, loss and grad are required");
  if (P->n_params_total > 0 && !params) return api_fail(MSS_E_INVALID, "params is NULL");
  if (!ws || ws_bytes < P->ws_bytes)
    return api_fail(MSS_E_NOMEM, "workspace too small: need %zu bytes, got %zu", P->ws_bytes,
                    ws ? ws_bytes : (size_t)0);
  mss_status s = bind(P, params, psi0, grad, loss, ws);
  if (s != MSS_OK) return s;
  hipFunction_t fwd_fn = nullptr;
  if (P->forward && (s = api_sampler_work_function(P->forward, &fwd_fn)) != MSS_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)ws;
  const char* d = (const char*)P->desc;
  hipError_t e = launch_work_integrate(P->dfwd, (unsigned long long*)(w + P->o_counter),
                                       P->grid_blocks, st, fwd_fn);
  if (e == hipSuccess) e = launch_work_scan(P->dfwd, st);
  if (e == hipSuccess) {
    SeedArgs sa{(const AdjDesc*)(d + P->a_sims), (const int64_t*)(d + P->a_psi0),
                (const double*)(w + P->o_fin), (double*)(w + P->o_lamK), loss, grad,
                P->n_params_total, P->n, P->m};
    const int64_t n = std::max<int64_t>(P->n_params_total, P->n);
    hipLaunchKernelGGL(adjoint_seed_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sa);
    ReverseArgs ra{(const AdjDesc*)(d + P->a_sims), (const int64_t*)(d + P->a_op),
                   (const int64_t*)(d + P->a_mat), (const double*)(w + P->o_U),
                   (double*)(w + P->o_W), P->n_mats, P->n};
    hipLaunchKernelGGL(adjoint_reverse_kernel, dim3((unsigned)((P->n_mats + 255) / 256)), dim3(256),
                       0, st, ra);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = launch_work_scan(P->dbwd, st);
  if (e == hipSuccess) {
    AdjArgs aa{(const AdjDesc*)(d + P->a_sims), (const mss_term*)(d + P->a_terms), P->n_waves, P->n};
    hipLaunchKernelGGL(adjoint_kernel, dim3((unsigned)((P->n_waves + 3) / 4)), dim3(256), 0, st, aa);
    e = hipGetLastError();
  }
  if (e == hipSuccess && psi_final)
    e = hipMemcpyAsync(psi_final, w + P->o_fin, (size_t)P->psi0_off[P->n] * 16,
                       hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipEventRecord(P->last_run, st);
  if (e != hipSuccess) return api_hip_fail(e, "adjoint launch");
  return api_ok();
}

void mss_adjoint_plan_destroy(mss_adjoint_plan* P) { release(P); }

mss_status mss_adjoint_population(int32_t n, const mss_problem* problems,
                                  const int64_t* param_off, int32_t level_m,
                                  const double* params, const double* psi0, double* loss,
                                  double* grad, double* psi_final, void* stream) {
  mss_adjoint_plan* P = nullptr;
  mss_status s = mss_adjoint_plan_create(n, problems, param_off, level_m, &P);
  if (s != MSS_OK) return s;
  void* ws = nullptr;
  hipError_t e = hipMalloc(&ws, std::max<size_t>(P->ws_bytes, 256));
  if (e != hipSuccess)
    s = e == hipErrorOutOfMemory ? api_fail(MSS_E_NOMEM, "workspace allocation failed")
                                 : api_hip_fail(e, "workspace allocation");
  if (s == MSS_OK)
    s = mss_adjoint_run(P, params, psi0, loss, grad, psi_final, ws, P->ws_bytes, stream);
  if (s == MSS_OK) {
    e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) s = api_hip_fail(e, "adjoint wait");
  }
  if (ws) (void)hipFree(ws);
  release(P);
  return s == MSS_OK ? api_ok() : s;
}

}  // extern "C"
