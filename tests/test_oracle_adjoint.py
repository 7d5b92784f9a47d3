"""Pins of the oracle's adjoint (gradient of a final-state population with
respect to field parameters) to extended-precision central differences of
the forward map and to a closed-form Rabi gradient."""
import math

import numpy as np
import pytest

from paper_2204_05586_amd import workloads as W


def _control_problem(spin_twice, n_seg=6, K=40, L=6, frame=True, tau=24, seed=0,
                     extra=("cos", "sin", "pwc")):
    """Piecewise-constant controls on x and y plus cos/sin terms whose
    amplitude, frequency and phase come from slots (`extra` picks which)."""
    rng = np.random.default_rng(seed)
    f_bias = 3.0e4
    T = K * 2e-5
    terms = W.control_problem_terms(n_seg=n_seg, seg_t0=0.0, seg_len=T / n_seg, f_bias=f_bias)
    more = {"cos": W.Term(W.COS, W.X, a_slot=2 * n_seg, f_slot=2 * n_seg + 1,
                          phi_slot=2 * n_seg + 2),
            "sin": W.Term(W.SIN, W.Y, a_slot=2 * n_seg + 3, f=2.1e3, phi=0.3),
            "pwc": W.Term(W.PWC, W.Y, n_seg=3, seg_t0=0.0, seg_len=T / 3,
                          seg_a_slot=2 * n_seg + 4)}
    terms += [more[k] for k in extra]
    if spin_twice == 2:
        terms.append(W.Term(W.CONST, W.Q, a=150.0))
    params = np.concatenate([rng.normal(2000.0, 400.0, n_seg), rng.uniform(0, 2 * math.pi, n_seg),
                             [700.0, 1.3e3, 0.4, 500.0], rng.normal(300.0, 50.0, 3)])
    psi0 = W.random_state(spin_twice + 1, rng)
    return W.Problem(spin_twice, terms, 0.0, 2e-5, K, L, tau, frame, params=params, psi0=psi0)


@pytest.mark.parametrize("spin_twice,frame", [(2, True), (2, False), (1, True)])
def test_adjoint_matches_extended_precision_differences(oracle, spin_twice, frame):
    """Central differences of the same discrete map in x87 extended precision
    (step 1e-6 relative): truncation ~1e-12, rounding ~1e-12, far below the
    tolerance.  Catches a wrong chain-rule factor (CF4 weight, frame
    rotation, 2 pi, field-term derivative) or a wrong costate."""
    prob = _control_problem(spin_twice, frame=frame, seed=spin_twice + 10 * frame)
    m = 1
    loss, g = oracle.adjoint_population(prob, m)
    p = np.asarray(prob.params, dtype=np.longdouble)
    assert abs(loss - float(oracle.population_ld(prob, m, p))) < 1e-14
    fd = np.zeros(p.size)
    for q in range(p.size):
        h = np.longdouble(1e-6) * max(np.longdouble(1.0), abs(p[q]))
        pp, pm = p.copy(), p.copy()
        pp[q] += h
        pm[q] -= h
        fd[q] = float((oracle.population_ld(prob, m, pp) - oracle.population_ld(prob, m, pm))
                      / (2 * h))
    scale = np.max(np.abs(fd))
    assert scale > 1e-8
    assert np.max(np.abs(g - fd)) <= 1e-9 * scale, np.max(np.abs(g - fd)) / scale


def test_adjoint_resonant_rabi_closed_form(oracle):
    """Spin-1 from |+1> under a resonant circular drive of amplitude A (one
    segment): the |0> population is sin^2(2 pi A T) / 2, so
    dP/dA = 2 pi T sin(2 pi A T) cos(2 pi A T) and dP/dphi = 0."""
    A, phi, T, K = 1234.0, 0.7, 2e-4, 200
    terms = W.control_problem_terms(n_seg=1, seg_t0=0.0, seg_len=T, f_bias=5e4)
    prob = W.Problem(2, terms, 0.0, T / K, K, 4, 28, True, params=np.array([A, phi]))
    loss, g = oracle.adjoint_population(prob, 1)
    th = 2 * math.pi * A * T
    assert loss == pytest.approx(math.sin(th) ** 2 / 2, abs=1e-13)
    assert g[0] == pytest.approx(2 * math.pi * T * math.sin(th) * math.cos(th), abs=1e-12)
    assert abs(g[1]) < 1e-12


def test_adjoint_rejects_z_slots(oracle):
    prob = W.Problem(2, [W.Term(W.CONST, W.Z, a_slot=0)], 0.0, 1e-5, 4, 2, 20, True,
                     params=np.array([1e4]))
    with pytest.raises(ValueError, match="x and y"):
        oracle.adjoint_population(prob, 0)
