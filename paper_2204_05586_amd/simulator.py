"""Python mirror of the paper's user API (Sec. "Compilation of integrator"):
a ``Simulator`` built once from the user's choices (spin, field program,
rotating frame, squaring count) and reused across ``evaluate`` calls with
different sweep parameters, returning ``Results`` (time, state, time
evolution operators).

The field is either a field program (a list of ``workloads.Term``,
interpreted by the precompiled integrator, or with ``specialize=True``
compiled once into its own integrator at construction, as the paper compiles
its field function) or, like the paper's user field function, code: HIP
source defining ``mss_user_field(t, params, field)``, compiled at run time
into its own integrator (``native.Sampler``).  ``params`` plays the role of
sweep_parameters.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import native
from .workloads import Problem, Term


@dataclass
class Results:
    time: "object"             # torch float64 [K] on the device
    state: "object"            # torch complex128 [K, N]: psi(t_k)
    time_evolution: "object"   # torch complex128 [K, N, N] or None: U_k
    state_final: "object"      # torch complex128 [N]: psi(t_start + K Dt)
    _spin: "object" = None

    @property
    def spin(self):
        """Expected spin projection [K, 3] (<J_x>, <J_y>, <J_z>), computed on
        first use, as the paper's Results.spin."""
        if self._spin is None:
            self._spin = native.spin_projection(self.state)
        return self._spin


def grid_from_times(t_start: float, t_end: float, dt_integration: float, dt_output: float):
    """Number of output intervals K and fine steps per interval L for a time
    range (Sec. "Discretization and parallelization": t_k = t_0 + k Dt,
    dt = Dt / L)."""
    if not (dt_output > 0 and dt_integration > 0 and t_end > t_start):
        raise ValueError("need t_end > t_start and positive time steps")
    K = int(math.floor((t_end - t_start) / dt_output + 1e-9))
    ratio = dt_output / dt_integration
    L = int(round(ratio))
    if L < 1 or abs(ratio - L) > 1e-9 * max(L, 1):
        raise ValueError("dt_output must be an integer multiple of dt_integration")
    if K < 1:
        raise ValueError("time range shorter than one output step")
    return K, L


class Simulator:
    """Spin-1/2 or spin-1 solver configured once, evaluated many times.

    spin: 0.5 or 1.  terms: field program, or HIP source of a field function
    (str), or a compiled ``native.Sampler``; sampler_options: extra compiler
    options for a source.  specialize: compile a field program into its own
    integrator at construction (about a second; the operators are bit for bit
    the interpreter's, and each evaluation is faster).  rotating_frame: per-interval
    rotating frame (paper default: on).  n_squares: Lie-Trotter squaring
    count tau for spin-1 (paper default 24).  method: "cf4" (default), or
    the Euler-family comparison samplings "midpoint" and "heun"."""

    METHODS = {"cf4": 0, "midpoint": 1, "heun": 2}

    def __init__(self, terms, spin: float = 1, rotating_frame: bool = True,
                 n_squares: int = 24, method: str = "cf4", device: str = "cuda",
                 sampler_options: Sequence[str] = (), specialize: bool = False):
        if spin not in (0.5, 1, 1.0):
            raise ValueError("spin must be 0.5 or 1")
        if method not in self.METHODS:
            raise ValueError(f"method must be one of {sorted(self.METHODS)}")
        self.method = self.METHODS[method]
        self.spin_twice = 1 if spin == 0.5 else 2
        self.sampler: Optional[native.Sampler] = None
        if isinstance(terms, str):
            self.sampler = native.Sampler(terms, sampler_options)
            terms = []
        elif isinstance(terms, native.Sampler):
            self.sampler, terms = terms, []
        self.terms: List[Term] = list(terms)
        if specialize and self.sampler is None:
            self.sampler = native.Sampler.for_terms(self.terms)
        self.rotating_frame = bool(rotating_frame)
        self.n_squares = int(n_squares)
        self.device = device

    def problem(self, t_start, t_end, dt_integration, dt_output, params=None, psi0=None) -> Problem:
        K, L = grid_from_times(t_start, t_end, dt_integration, dt_output)
        return Problem(self.spin_twice, self.terms, float(t_start), float(dt_output), K, L,
                       self.n_squares, self.rotating_frame,
                       params=np.zeros(0) if params is None else params, psi0=psi0,
                       method=self.method)

    def evaluate(self, psi0, t_start: float, t_end: float, dt_integration: float,
                 dt_output: float, params=None, keep_operators: bool = True,
                 stream=None, want_spin: bool = False) -> Results:
        """One simulation.  want_spin: also form <J> of every state in the
        last pass of the state product (``Results.spin`` ready, no second
        read of the states)."""
        prob = self.problem(t_start, t_end, dt_integration, dt_output, params, psi0)
        native.validate(prob)
        if self.sampler is not None:
            prob = prob.replace(terms=[])
        r = native.solve(prob, store_u=keep_operators, want_time=True, device=self.device,
                         stream=stream, sampler=self.sampler, want_spin=want_spin)
        return Results(r["time"], r["psi"], r["U"], r["psi_final"], r["spin"])
