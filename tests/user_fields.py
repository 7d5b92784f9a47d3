"""User field functions for the sampler route, each written twice: as a
Python function for the oracle's field-function callback (the paper's
calling convention: time, sweep parameters, field sample to fill) and as
HIP source for the GPU sampler.  They are problem inputs, like a field
program, and carry none of the solver's arithmetic.

* Landau-Zener ramp: f_z = beta t, f_x = delta (a linear sweep through
  resonance; the term kinds cannot express a ramp).  params: beta, delta, f_q.
* Chirped circular drive: bias F0 on z, drive (f_x, f_y) = A (cos, sin) of
  2 pi (F0 t + beta (t - t_c)^2 / 2): an adiabatic passage through F0 at
  t_c, with phases far from zero.  params: F0, beta, t_c, A, f_q.
"""
import math

TWO_PI = 2.0 * math.pi


def lz_field(t, p, f):
    f[0] = p[1]
    f[2] = p[0] * t
    f[3] = p[2]


LZ_SOURCE = r"""
__device__ void mss_user_field(double t, const double* p, double* f) {
  f[0] = p[1];
  f[2] = p[0] * t;
  f[3] = p[2];
}
"""


def chirp_field(t, p, f):
    dt = t - p[2]
    ph = TWO_PI * (p[0] * t + 0.5 * p[1] * dt * dt)
    f[0] = p[3] * math.cos(ph)
    f[1] = p[3] * math.sin(ph)
    f[2] = p[0]
    f[3] = p[4]


CHIRP_SOURCE = r"""
__device__ void mss_user_field(double t, const double* p, double* f) {
#pragma clang fp contract(off)
  const double dt = t - p[2];
  const double ph = 6.283185307179586 * (p[0] * t + 0.5 * p[1] * dt * dt);
  double s, c;
  mss::sincos_cw(ph, &s, &c);
  f[0] = p[3] * c;
  f[1] = p[3] * s;
  f[2] = p[0];
  f[3] = p[4];
}
"""


def lz_probability(beta, delta):
    """Landau-Zener probability of staying in the diabatic state for
    H = 2 pi (beta t J_z + delta J_x), spin-1/2: exp(-pi^2 delta^2 / beta)."""
    return math.exp(-math.pi ** 2 * delta ** 2 / beta)
