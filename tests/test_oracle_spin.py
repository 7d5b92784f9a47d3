"""Pins of the oracle's expected spin projection <J> = psi^H J psi
(Sec. "Quantum mechanics background") to closed forms."""
import math

import numpy as np
import pytest

from paper_2204_05586_amd import workloads as W
from tests import spin_algebra as SA


def test_bloch_vector_of_coherent_states(oracle):
    """Spin-1/2 state (cos(t/2), e^{ip} sin(t/2)) has <J> = (sin t cos p,
    sin t sin p, cos t)/2; its spin-1 coherent state has twice that."""
    rng = np.random.default_rng(0)
    th, ph = rng.uniform(0, math.pi, 50), rng.uniform(0, 2 * math.pi, 50)
    half = np.stack([np.cos(th / 2), np.exp(1j * ph) * np.sin(th / 2)], axis=1)
    ref = 0.5 * np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)
    assert np.max(np.abs(oracle.spin_projection(half) - ref)) < 1e-15
    assert np.max(np.abs(oracle.spin_projection(SA.d1_state(half)) - 2 * ref)) < 2e-15


def test_larmor_precession(oracle):
    """Under a constant field (frame off, exact for CF4), <J> precesses about
    the field direction at |omega|: Rodrigues rotation of the initial vector."""
    f = np.array([300.0, -200.0, 500.0])
    p = W.Problem(1, [W.Term(W.CONST, c, a=v) for c, v in enumerate(f)], 0.0, 1e-4, 200, 5, 0,
                  False, psi0=np.array([1.0, 0.0]))
    r = oracle.solve(p)
    J = oracle.spin_projection(r["psi"])
    w = 2 * math.pi * f
    n = w / np.linalg.norm(w)
    v0 = np.array([0.0, 0.0, 0.5])
    for k in (0, 7, 120, 199):
        a = np.linalg.norm(w) * k * 1e-4
        # d<J>/dt = i<[H, J]> = omega x <J>: right-handed rotation by a about n
        rot = (v0 * math.cos(a) + np.cross(n, v0) * math.sin(a) + n * np.dot(n, v0) * (1 - math.cos(a)))
        assert np.max(np.abs(J[k] - rot)) < 1e-12, k


def test_spin_length_conserved(oracle):
    """|<J>| = s for coherent spin-1 states evolved under J-only fields."""
    rng = np.random.default_rng(3)
    p2 = W.random_problem(rng, 1, 100, 4, rotating_frame=True)
    p3 = p2.replace(spin_twice=2, psi0=SA.d1_state(p2.psi0))
    J = oracle.spin_projection(oracle.solve(p3)["psi"])
    assert np.max(np.abs(np.linalg.norm(J, axis=1) - 1.0)) < 1e-12


def _rot(axis, a):
    c, s = math.cos(a), math.sin(a)
    if axis == "x":
        return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


@pytest.mark.parametrize("spin_twice", [1, 2])
def test_circular_drive_closed_form(oracle, spin_twice):
    """Resonant circular drive f_x + i f_y = A e^{i w0 t}, f_z = F0, w0 = 2 pi F0:
    in the frame rotating at w0 about z the Hamiltonian is the constant
    2 pi A J_x, so <J>(t) = R_z(w0 t) R_x(2 pi A t) <J>(0) (right-handed
    rotations of the vector).  With the rotating frame on, each interval's
    frame Hamiltonian is constant and the method is exact to rounding."""
    F0, A = 2.0e4, 900.0
    T = W.Term
    terms = [T(W.COS, W.X, a=A, f=F0), T(W.SIN, W.Y, a=A, f=F0), T(W.CONST, W.Z, a=F0)]
    th, ph = 1.1, 0.4
    half = np.array([math.cos(th / 2), np.exp(1j * ph) * math.sin(th / 2)])
    psi0 = half if spin_twice == 1 else SA.d1_state(half[None])[0]
    p = W.Problem(spin_twice, terms, 0.0, 3e-6, 500, 6, 28, True, psi0=psi0)
    J = oracle.spin_projection(oracle.solve(p)["psi"])
    s = spin_twice / 2
    v0 = s * np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
    assert np.max(np.abs(J[0] - v0)) < 1e-15
    for k in (1, 77, 250, 499):
        t = k * 3e-6
        ref = _rot("z", 2 * math.pi * F0 * t) @ _rot("x", 2 * math.pi * A * t) @ v0
        assert np.max(np.abs(J[k] - ref)) < 2e-12, (k, J[k], ref)
