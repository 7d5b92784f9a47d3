"""Pins of the oracle's field-function route (a caller-supplied field
function in place of terms, the counterpart of the paper's user field
function, Sec. "Compilation of integrator"), against facts other than the
oracle: closed-form exponentials, an adaptive ODE solution, the
Landau-Zener formula, and the term route on the same field."""
import math

import numpy as np
import pytest

from paper_2204_05586_amd import workloads as W
from tests import spin_algebra as SA
from tests import user_fields as F
from tests.test_oracle_pins import _circular_problem

RNG = np.random.default_rng(77)

DELTA = 1.0e3
BETA = math.pi ** 2 * DELTA ** 2 / 1.2   # Landau-Zener exponent 1.2
T_HALF = 40 * DELTA / BETA               # sweep to 40 x delta on each side
DT_OUT = 5e-6
K_LZ = int(round(2 * T_HALF / DT_OUT))


def _lz_problem(spin_twice, L, psi0, frame=True):
    return W.Problem(spin_twice, [], -K_LZ * DT_OUT / 2, DT_OUT, K_LZ, L, 28, frame,
                     params=np.array([BETA, DELTA, 0.0]), psi0=psi0)


def _hamiltonian(fn, params, t, dim):
    f = np.zeros(4)
    fn(t, params, f)
    return 2 * math.pi * SA.generator(list(f[:3]) if dim == 2 else list(f), dim)


def _dop853(fn, params, dim, t_eval, psi0):
    from scipy.integrate import solve_ivp

    def rhs(t, y):
        psi = y[:dim] + 1j * y[dim:]
        d = -1j * (_hamiltonian(fn, params, t, dim) @ psi)
        return np.concatenate([d.real, d.imag])

    y0 = np.concatenate([np.real(psi0), np.imag(psi0)])
    sol = solve_ivp(rhs, (t_eval[0], t_eval[-1]), y0, method="DOP853", t_eval=t_eval,
                    rtol=1e-12, atol=1e-13)
    return (sol.y[:dim] + 1j * sol.y[dim:]).T


@pytest.mark.parametrize("spin_twice", [1, 2])
def test_constant_field_function_is_exact(oracle, spin_twice):
    """A constant field function: U = exp(-i H Dt) (eq. exp_sol_of_constant)."""
    fv = [310.0, -170.0, 520.0, 90.0]
    dim = spin_twice + 1

    def fn(t, p, f):
        f[:] = fv

    p = W.Problem(spin_twice, [], 0.0, 1e-4, 50, 3, 28, False)
    r = oracle.solve(p, want_U=True, field_fn=fn)
    H = SA.generator([2 * math.pi * x for x in (fv[:3] if dim == 2 else fv)], dim)
    assert np.max(np.abs(r["U"] - SA.expmh(H * 1e-4))) < 1e-13


@pytest.mark.parametrize("spin_twice", [1, 2])
def test_field_function_equals_term_route(oracle, spin_twice):
    """The circular drive as a field function gives the term route's result:
    same node times, parameters and component order."""
    dim = spin_twice + 1
    psi0 = W.random_state(dim, RNG)
    fz, fd, amp, fq = 2.1e5, 2.0e5, 3.0e3, 700.0
    p = _circular_problem(spin_twice, fz, fd, amp, fq, 120, 5, 3.1e-6, True, psi0, t_start=2.3e-5)
    ref = oracle.solve(p, want_U=True)
    prm = np.array([fz, fd, amp, fq])

    def fn(t, q, f):
        ph = 2 * math.pi * (q[1] * t)
        f[0] = q[2] * math.cos(ph)
        f[1] = q[2] * math.sin(ph)
        f[2] = q[0]
        f[3] = q[3]

    got = oracle.solve(p.replace(terms=[], params=prm), want_U=True, field_fn=fn)
    assert np.max(np.abs(got["U"] - ref["U"])) < 1e-14
    assert np.max(np.abs(got["psi"] - ref["psi"])) < 1e-13


def test_landau_zener_ramp_matches_adaptive_ode(oracle):
    """Linear sweep f_z = beta t through resonance with f_x = delta (spin-1/2):
    states vs scipy's DOP853 at rtol 1e-12."""
    p = _lz_problem(1, 40, [1.0, 0.0])
    r = oracle.solve(p, field_fn=F.lz_field)
    idx = np.arange(0, K_LZ, K_LZ // 8)
    ref = _dop853(F.lz_field, p.params, 2, p.t_start + idx * DT_OUT, np.array([1.0, 0.0]))
    assert np.max(np.abs(r["psi"][idx] - ref)) < 1e-9


@pytest.mark.parametrize("spin_twice", [1, 2])
def test_landau_zener_probability(oracle, spin_twice):
    """Start in the lowest adiabatic state at -T; the population of the
    highest adiabatic state at +T is the Landau-Zener probability
    P = exp(-pi^2 delta^2 / beta) for spin-1/2 and P^2 for spin-1 (the
    spin-1 representation of the same SU(2) evolution).  Finite-sweep
    corrections are O(1 / 40^2)."""
    dim = spin_twice + 1
    t0 = -K_LZ * DT_OUT / 2
    t1 = t0 + K_LZ * DT_OUT
    prm = np.array([BETA, DELTA, 0.0])
    _, V0 = np.linalg.eigh(_hamiltonian(F.lz_field, prm, t0, dim))
    _, V1 = np.linalg.eigh(_hamiltonian(F.lz_field, prm, t1, dim))
    r = oracle.solve(_lz_problem(spin_twice, 10, V0[:, 0]), field_fn=F.lz_field)
    P = abs(np.vdot(V1[:, -1], r["psi_final"])) ** 2
    P_lz = F.lz_probability(BETA, DELTA) ** (1 if spin_twice == 1 else 2)
    assert abs(P - P_lz) < 2e-4, (P, P_lz)


def test_chirped_drive_matches_adaptive_ode(oracle):
    """Chirped circular drive around a 50 kHz bias (phases up to ~1.6e3 rad),
    rotating frame on: states vs DOP853."""
    A = 1.0e3
    beta = math.pi ** 2 * A ** 2 / 1.2
    Tc = 40 * A / beta
    K = int(round(2 * Tc / DT_OUT))
    prm = np.array([5.0e4, beta, 0.0, A, 0.0])
    p = W.Problem(1, [], -K * DT_OUT / 2, DT_OUT, K, 40, 28, True, params=prm, psi0=[1.0, 0.0])
    r = oracle.solve(p, field_fn=F.chirp_field)
    idx = np.arange(0, K, K // 8)
    ref = _dop853(F.chirp_field, prm, 2, p.t_start + idx * DT_OUT, np.array([1.0, 0.0]))
    assert np.max(np.abs(r["psi"][idx] - ref)) < 1e-9


def test_field_function_errors_propagate(oracle):
    def bad(t, p, f):
        raise ZeroDivisionError("planted")

    with pytest.raises(ZeroDivisionError):
        oracle.solve(W.Problem(1, [], 0.0, 1e-4, 5, 2, 28, True), field_fn=bad)
    with pytest.raises(ValueError):
        oracle.solve(W.Problem(1, [W.Term(W.CONST, W.Z, a=1.0)], 0.0, 1e-4, 5, 2, 28, True),
                     field_fn=F.lz_field)
