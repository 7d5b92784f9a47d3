"""Oracle pinned to constants the paper prints (tests/golden/): one CF4 fine
step of the oracle equals exp(-i H2 dt) exp(-i H1 dt) built by scipy's expm
from the printed sample times and weights, for spin-1/2 and for spin-1 with
the printed quadrupole Q (Sec. "Unitary time evolution and the Magnus
expansion", eqs. cf4_sample_1/2 and cf4_implementation; Sec. "Quantum
mechanics background")."""
import math
import os

import numpy as np
import pytest

from paper_2204_05586_amd import workloads as W

scipy_linalg = pytest.importorskip("scipy.linalg")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_printed_constants.txt")


def _golden():
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = (x.strip() for x in line.split("="))
                out[k] = float(v)
    return out


G = _golden()


def _spin_ops(spin_twice):
    if spin_twice == 1:
        sx = np.array([[0, 1], [1, 0]], dtype=complex) / 2
        sy = np.array([[0, -1j], [1j, 0]], dtype=complex) / 2
        sz = np.array([[1, 0], [0, -1]], dtype=complex) / 2
        return [sx, sy, sz]
    r = 1 / math.sqrt(2)
    jx = np.array([[0, r, 0], [r, 0, r], [0, r, 0]], dtype=complex)
    jy = np.array([[0, -1j * r, 0], [1j * r, 0, -1j * r], [0, 1j * r, 0]], dtype=complex)
    jz = np.diag([1.0, 0.0, -1.0]).astype(complex)
    q = np.diag([G["q_diag_0"], G["q_diag_1"], G["q_diag_2"]]).astype(complex)
    return [jx, jy, jz, q]


def _random_terms(rng, spin_twice):
    """A field with non-commuting, time-dependent components; returns the
    terms and a numpy function of t giving (f_x, f_y, f_z[, f_q]) in Hz.
    f_z has a part that turns over in a few tens of microseconds, so it
    varies within an interval and the rotating frame's rate depends on
    where in the interval it is sampled."""
    T = W.Term
    ax, fx, px = rng.uniform(2e3, 6e3), rng.uniform(5e3, 2e4), rng.uniform(0, 6)
    ay, fy = rng.uniform(1e3, 5e3), rng.uniform(5e3, 2e4)
    az = rng.uniform(-8e3, 8e3)
    bz, gz, pz = rng.uniform(2e3, 8e3), rng.uniform(2e4, 1e5), rng.uniform(0, 6)
    aq = rng.uniform(-4e3, 4e3)
    terms = [T(W.COS, W.X, a=ax, f=fx, phi=px), T(W.SIN, W.Y, a=ay, f=fy), T(W.CONST, W.Z, a=az),
             T(W.COS, W.Z, a=bz, f=gz, phi=pz)]
    if spin_twice == 2:
        terms.append(T(W.CONST, W.Q, a=aq))

    def field(t):
        f = [ax * math.cos(2 * math.pi * fx * t + px), ay * math.sin(2 * math.pi * fy * t),
             az + bz * math.cos(2 * math.pi * gz * t + pz)]
        return f + ([aq] if spin_twice == 2 else [])
    return terms, field


@pytest.mark.parametrize("spin_twice", [1, 2])
def test_one_cf4_step_from_printed_constants(oracle, spin_twice):
    rng = np.random.default_rng(70 + spin_twice)
    ops = _spin_ops(spin_twice)
    for trial in range(6):
        terms, field = _random_terms(rng, spin_twice)
        t0, dt = rng.uniform(0, 1e-3), rng.uniform(2e-6, 2e-5)
        # one interval of one fine step, lab frame; spin-1 with many squarings so
        # its Lie-Trotter factor is the exact exponential to rounding
        p = W.Problem(spin_twice, terms, t0, dt, 1, 1, 40, False)
        got = oracle.operators(p)[0]

        def H(t):
            return 2 * math.pi * sum(f * A for f, A in zip(field(t), ops))
        h1, h2 = H(t0 + G["c1"] * dt), H(t0 + G["c2"] * dt)
        hb1 = G["w_plus"] * h1 + G["w_minus"] * h2
        hb2 = G["w_minus"] * h1 + G["w_plus"] * h2
        ref = scipy_linalg.expm(-1j * hb2 * dt) @ scipy_linalg.expm(-1j * hb1 * dt)
        assert np.max(np.abs(got - ref)) < 5e-14, (spin_twice, trial)


def test_printed_constants_are_consistent():
    """The printed weights sum to one and the nodes are symmetric about the
    step's midpoint (the Gauss-Legendre structure the paper cites)."""
    assert abs(G["w_plus"] + G["w_minus"] - 0.5) < 1e-15
    assert abs(G["c1"] + G["c2"] - 1.0) < 1e-15
    assert abs(G["q_diag_0"] + G["q_diag_1"] + G["q_diag_2"]) < 1e-15
    assert G["tau_default"] == 24


def _frame_interval(field, ops, t0, Dt, L):
    """exp(-i w_r Dt J_z) times L printed CF4 steps of the frame Hamiltonian
    exp(i w_r s J_z) H exp(-i w_r s J_z) - w_r J_z, s measured from t0,
    w_r = 2 pi f_z(t0 + Dt/2) (Sec. "Dynamically rotating frame")."""
    jz = ops[2]
    N = jz.shape[0]
    wr = 2 * math.pi * field(t0 + Dt / 2)[2]
    dt = Dt / L
    Ur = np.eye(N, dtype=complex)
    for l in range(L):
        t = t0 + l * dt

        def Hrot(s):
            H = 2 * math.pi * sum(f * A for f, A in zip(field(s), ops))
            R = scipy_linalg.expm(-1j * wr * (s - t0) * jz)
            return R.conj().T @ H @ R - wr * jz
        h1, h2 = Hrot(t + G["c1"] * dt), Hrot(t + G["c2"] * dt)
        hb1 = G["w_plus"] * h1 + G["w_minus"] * h2
        hb2 = G["w_minus"] * h1 + G["w_plus"] * h2
        Ur = scipy_linalg.expm(-1j * hb2 * dt) @ scipy_linalg.expm(-1j * hb1 * dt) @ Ur
    return scipy_linalg.expm(-1j * wr * Dt * jz) @ Ur


@pytest.mark.parametrize("spin_twice", [1, 2])
def test_rotating_frame_interval_from_printed_constants(oracle, spin_twice):
    """The oracle's interval operator with the frame on equals the frame
    built independently from its definition with scipy's expm (a wrong sign
    of the frame phase, of w_r, or of the exit rotation fails this at O(1);
    w_r taken at the start or the end of the interval instead of its
    midpoint fails it through the different discretisation error of the
    time-varying f_z, 5e-11 and above here against the 5e-14 bound)."""
    rng = np.random.default_rng(95 + spin_twice)
    ops = _spin_ops(spin_twice)
    for L in (1, 5, 12):
        terms, field = _random_terms(rng, spin_twice)
        t0, Dt = rng.uniform(0, 1e-3), rng.uniform(2e-6, 2e-5)
        got = oracle.operators(W.Problem(spin_twice, terms, t0, Dt, 1, L, 40, True))[0]
        ref = _frame_interval(field, ops, t0, Dt, L)
        assert np.max(np.abs(got - ref)) < 5e-14, (spin_twice, L)
