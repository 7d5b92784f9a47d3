"""Seeded synthetic workloads for the spin-1/2 / spin-1 CF4 solver.

This module only *describes* problems: field programs (lists of additive
terms per field component), time grids, initial states and per-simulation
parameter tables, drawn with ``numpy.random.default_rng`` (PCG64) in a fixed
order.  It contains none of the solver's arithmetic, so both the GPU path and
the CPU oracle take their inputs from here.

Field model (paper, Sec. "Quantum mechanics background"): the Hamiltonian is a
real linear combination of a fixed traceless basis,
H(t) = 2*pi * (f_x(t) J_x + f_y(t) J_y + f_z(t) J_z [+ f_q(t) Q]),
with the field functions f_j given in Hz.  The paper lets the user write the
field functions as compiled Python code with a ``sweep_parameters`` array
(Sec. "Compilation of integrator"); here a field function is a *field
program*: a list of terms, each of one of the kinds below, whose numeric
coefficients are either literals or slots into a per-simulation parameter
vector (the analogue of ``sweep_parameters``).

Term kinds (value contributed to component ``comp`` at time t, only while
t_on < t < t_off):
  CONST    a
  COS      a * cos(2*pi*f*t + phi)
  SIN      a * sin(2*pi*f*t + phi)
  PWC      a_s                               s = segment index of t
  PWC_COS  a_s * cos(2*pi*f*t + phi_s)
  PWC_SIN  a_s * sin(2*pi*f*t + phi_s)
The segment index is s = clamp(floor((t - seg_t0) / seg_len), 0, n_seg - 1);
a_s = params[seg_a_slot + s] (or the literal a when seg_a_slot < 0) and
phi_s = params[seg_phi_slot + s] (or the literal phi).  Literal a, f, phi are
replaced by params[a_slot], params[f_slot], params[phi_slot] when the slot is
non-negative.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# term kinds
CONST, COS, SIN, PWC, PWC_COS, PWC_SIN = 0, 1, 2, 3, 4, 5
# field components
X, Y, Z, Q = 0, 1, 2, 3
# spin-1 full su(3) basis: the Delta m = +-2 quadrupoles U_1 = J_x^2 - J_y^2,
# U_2 = J_x J_y + J_y J_x and the Delta m = +-1 quadrupoles V_1 = J_z J_x + J_x J_z,
# V_2 = J_y J_z + J_z J_y
U1, U2, V1, V2 = 4, 5, 6, 7
# integration methods: commutator-free fourth-order Magnus (the solver's), and
# the two Euler-family sampling methods the paper compares it with
CF4, MIDPOINT, HEUN = 0, 1, 2

INF = float("inf")


@dataclass
class Term:
    kind: int
    comp: int
    a: float = 0.0
    f: float = 0.0
    phi: float = 0.0
    a_slot: int = -1
    f_slot: int = -1
    phi_slot: int = -1
    t_on: float = -INF
    t_off: float = INF
    n_seg: int = 0
    seg_t0: float = 0.0
    seg_len: float = 0.0
    seg_a_slot: int = -1
    seg_phi_slot: int = -1


@dataclass
class Problem:
    """One simulation: spin, field program, time grid, initial state."""

    spin_twice: int                 # 1 -> spin-1/2 (N=2), 2 -> spin-1 (N=3)
    terms: List[Term]
    t_start: float
    dt_out: float                   # output step (Delta t)
    n_samples: int                  # K output intervals
    n_fine: int                     # L fine CF4 steps per interval
    n_squares: int = 28             # tau (spin-1 Lie-Trotter squarings)
    rotating_frame: bool = True
    params: np.ndarray = field(default_factory=lambda: np.zeros(0))
    psi0: Optional[np.ndarray] = None
    name: str = ""
    method: int = CF4

    def __post_init__(self):
        self.params = np.ascontiguousarray(np.asarray(self.params, dtype=np.float64))
        if self.psi0 is None:
            self.psi0 = np.zeros(self.dim, dtype=np.complex128)
            self.psi0[0] = 1.0
        self.psi0 = np.ascontiguousarray(np.asarray(self.psi0, dtype=np.complex128))

    @property
    def dim(self) -> int:
        return self.spin_twice + 1

    @property
    def fine_steps(self) -> int:
        return int(self.n_samples) * int(self.n_fine)

    def replace(self, **kw) -> "Problem":
        d = {f.name: getattr(self, f.name) for f in dataclasses.fields(self)}
        d["terms"] = [dataclasses.replace(t) for t in self.terms]
        d.update(kw)
        return Problem(**d)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def spin_half_rabi(n_samples: int = 10_000, n_fine: int = 100, dt_out: float = 1e-5,
                   rotating_frame: bool = True) -> Problem:
    """Spin-1/2 Rabi drive: f_z = 1000 Hz, f_x = 200 cos(2 pi 1000 t) Hz,
    psi0 = |+1/2>, t in [0, K dt_out); default 1e4 samples x 100 fine steps
    (1e6 CF4 steps over 0.1 s)."""
    terms = [Term(COS, X, a=200.0, f=1000.0), Term(CONST, Z, a=1000.0)]
    return Problem(1, terms, 0.0, dt_out, n_samples, n_fine, 0, rotating_frame,
                   name="spin_half_rabi")


def neural_pulse_terms(f_bias: float = 700e3, amp: float = 2000.0, f_pulse: float = 1000.0,
                       f_quad: float = 2.3, pulse_amp: float = 20.0,
                       t_on: float = 0.05, t_off: float = 0.051) -> List[Term]:
    """Spin-1 sensing drive in the shape of the paper's benchmark Hamiltonian
    (Sec. "Evaluation of accuracy", eq. neural_pulse): a bias along z, a
    resonant linear drive along x and a one-cycle 1 kHz signal on x."""
    return [Term(COS, X, a=amp, f=f_bias),
            Term(SIN, X, a=pulse_amp, f=f_pulse, t_on=t_on, t_off=t_off),
            Term(CONST, Z, a=f_bias),
            Term(CONST, Q, a=f_quad)]


def spin_one_sensing(n_samples: int = 200_000, n_fine: int = 10, dt_out: float = 5e-7,
                     n_squares: int = 28, rotating_frame: bool = True,
                     t_start: float = 0.0) -> Problem:
    """Spin-1 single simulation: f_z = 700 kHz, f_q = 2.3 Hz,
    f_x = 2000 cos(2 pi 700e3 t) + 20 sin(2 pi 1000 t) [0.05 < t < 0.051],
    psi0 = |+1>, default 2e5 samples of 5e-7 s x 10 fine steps (2e6 CF4 steps
    over 0.1 s), tau = 28."""
    return Problem(2, neural_pulse_terms(), t_start, dt_out, n_samples, n_fine,
                   n_squares, rotating_frame, name="spin_one_sensing")


def batched_sensing(seed: int = 2, n_sims: int = 4096, dt_out: float = 5e-7, n_fine: int = 10,
                    n_squares: int = 28, dur_lo: float = 0.010, dur_hi: float = 0.100) -> List[Problem]:
    """4096 spin-1 sensing simulations with seeded bias, Rabi amplitude,
    pulse frequency and duration (uneven sample counts).  Draw order:
    f_z ~ U(690e3, 710e3), A ~ U(500, 2000), f_p ~ U(500, 2000),
    dur ~ U(dur_lo, dur_hi), each as a vector of n_sims; K_i = floor(dur_i / dt_out).
    The per-simulation values live in a 3-slot parameter vector
    (f_z, A, f_p), exercising the sweep-parameter path."""
    rng = np.random.default_rng(seed)
    fz = rng.uniform(690e3, 710e3, n_sims)
    amp = rng.uniform(500.0, 2000.0, n_sims)
    fp = rng.uniform(500.0, 2000.0, n_sims)
    dur = rng.uniform(dur_lo, dur_hi, n_sims)
    terms = [Term(COS, X, a_slot=1, f_slot=0),
             Term(SIN, X, a=20.0, f_slot=2, t_on=0.05, t_off=0.051),
             Term(CONST, Z, a_slot=0),
             Term(CONST, Q, a=2.3)]
    out = []
    for i in range(n_sims):
        k = max(1, int(math.floor(dur[i] / dt_out)))
        out.append(Problem(2, [dataclasses.replace(t) for t in terms], 0.0, dt_out, k, n_fine,
                           n_squares, True, params=np.array([fz[i], amp[i], fp[i]]),
                           name=f"batched_sensing[{i}]"))
    return out


@dataclass
class Request:
    arrival: float          # seconds after stream start
    problem: Problem


def serving_stream(rate: float, n_requests: int = 2000, seed: Optional[int] = None,
                   rate_index: int = 0, n_fine: int = 10, k_lo: float = 1e3,
                   k_hi: float = 1e6) -> List[Request]:
    """Poisson request stream of mixed spin-1/2 (30 %) and spin-1 (70 %)
    simulations.  Per request, in order: gap ~ Exp(1/rate); spin-1 with
    probability 0.7; K = floor(exp(U(ln k_lo, ln k_hi))); then the field
    parameters.  Spin-1: f_z ~ U(690e3, 710e3), A ~ U(500, 2000),
    f_p ~ U(500, 2000), dt_out = 5e-7.  Spin-1/2: f_z ~ U(500, 2000),
    A ~ U(100, 400), f_x = A cos(2 pi f_z t), dt_out = 1e-5.  L = n_fine."""
    rng = np.random.default_rng(3 + rate_index if seed is None else seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        spin_one = rng.uniform() < 0.7
        k = int(math.floor(math.exp(rng.uniform(math.log(k_lo), math.log(k_hi)))))
        if spin_one:
            fz = rng.uniform(690e3, 710e3)
            amp = rng.uniform(500.0, 2000.0)
            fp = rng.uniform(500.0, 2000.0)
            p = Problem(2, neural_pulse_terms(f_bias=fz, amp=amp, f_pulse=fp), 0.0, 5e-7, k,
                        n_fine, 28, True, name=f"serve[{i}]")
        else:
            fz = rng.uniform(500.0, 2000.0)
            amp = rng.uniform(100.0, 400.0)
            p = Problem(1, [Term(COS, X, a=amp, f=fz), Term(CONST, Z, a=fz)], 0.0, 1e-5, k,
                        n_fine, 0, True, name=f"serve[{i}]")
        out.append(Request(t, p))
    return out


N_SEGMENTS = 256


def control_problem_terms(n_seg: int = N_SEGMENTS, seg_t0: float = 0.0,
                          seg_len: float = 1e-3 / N_SEGMENTS, f_bias: float = 700e3) -> List[Term]:
    """Piecewise-constant resonant control: in segment s,
    f_x = A_s cos(2 pi f_bias t + phi_s), f_y = A_s sin(2 pi f_bias t + phi_s),
    f_z = f_bias.  Parameters: A_s at slots [0, n_seg), phi_s at
    [n_seg, 2 n_seg)."""
    return [Term(PWC_COS, X, f=f_bias, n_seg=n_seg, seg_t0=seg_t0, seg_len=seg_len,
                 seg_a_slot=0, seg_phi_slot=n_seg),
            Term(PWC_SIN, Y, f=f_bias, n_seg=n_seg, seg_t0=seg_t0, seg_len=seg_len,
                 seg_a_slot=0, seg_phi_slot=n_seg),
            Term(CONST, Z, a=f_bias)]


def control_batch(seed: int = 4, n_inst: int = 1024, n_seg: int = N_SEGMENTS,
                  n_samples: int = 1000, n_fine: int = 100, dt_out: float = 1e-6,
                  n_squares: int = 28) -> List[Problem]:
    """Differentiation workload: n_inst spin-1 instances over 1 ms with
    A ~ N(1000, 200) Hz and phi ~ U(0, 2 pi) per segment (drawn as two
    [n_inst, n_seg] arrays in that order), psi0 = |+1>, frame on."""
    rng = np.random.default_rng(seed)
    amp = rng.normal(1000.0, 200.0, (n_inst, n_seg))
    phi = rng.uniform(0.0, 2.0 * math.pi, (n_inst, n_seg))
    seg_len = n_samples * dt_out / n_seg
    out = []
    for i in range(n_inst):
        out.append(Problem(2, control_problem_terms(n_seg, 0.0, seg_len), 0.0, dt_out, n_samples,
                           n_fine, n_squares, True,
                           params=np.concatenate([amp[i], phi[i]]), name=f"control[{i}]"))
    return out


def random_state(dim: int, rng: np.random.Generator) -> np.ndarray:
    v = rng.normal(size=dim) + 1j * rng.normal(size=dim)
    return v / np.linalg.norm(v)


def random_problem(rng: np.random.Generator, spin_twice: int, n_samples: int, n_fine: int,
                   n_squares: int = 28, rotating_frame: bool = True,
                   bias: float = 5e4) -> Problem:
    """A random problem for property tests: bias along z, cosine and sine
    drives on x and y, a windowed term and a quadrupole term (spin-1)."""
    fz = rng.uniform(0.5, 1.5) * bias
    dt_out = rng.uniform(0.5, 2.0) / bias
    terms = [Term(CONST, Z, a=fz),
             Term(COS, X, a=rng.uniform(0.01, 0.1) * bias, f=fz * rng.uniform(0.98, 1.02),
                  phi=rng.uniform(0, 6.0)),
             Term(SIN, Y, a=rng.uniform(0.01, 0.05) * bias, f=fz * rng.uniform(0.9, 1.1)),
             Term(COS, Z, a=rng.uniform(0.0, 0.02) * bias, f=rng.uniform(0.001, 0.01) * bias,
                  t_on=0.25 * n_samples * dt_out, t_off=0.75 * n_samples * dt_out)]
    if spin_twice == 2:
        terms.append(Term(CONST, Q, a=rng.uniform(-0.01, 0.01) * bias))
    return Problem(spin_twice, terms, rng.uniform(0.0, 1e-3), dt_out, n_samples, n_fine,
                   n_squares, rotating_frame, psi0=random_state(spin_twice + 1, rng),
                   name="random")
