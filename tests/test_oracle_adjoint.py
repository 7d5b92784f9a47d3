"""Pins of the oracle's adjoint (gradient of a final-state population with
respect to field parameters) to extended-precision central differences of
the forward map and to a closed-form Rabi gradient."""
import math
import os

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


def _zero_field_problem(spin_twice, frame, seed, K=40, L=6, tau=24):
    """Four segments of controls: a resonant drive with amplitudes
    (A0, 0, A2, 0) and phases (slots 0-7), and static x and y fields with
    amplitudes (b0, 0, b2, 0) and (c0, 0, c2, 0) (slots 8-15); the z bias is
    switched off after half the run.  Segment 1 has no transverse field
    (rho = 0 at every node: all of theta is 0 in the frame, only theta_z is
    left without it); segment 3 has no field at all (theta = 0 with the frame
    on or off).  The bias frequency puts a non-integer number of turns in a
    segment, so no first-order effect averages out.  Random psi0."""
    rng = np.random.default_rng(seed)
    n_seg, dt_out, f_bias = 4, 2e-5, 3.13e4
    T = K * dt_out
    seg = dict(n_seg=n_seg, seg_t0=0.0, seg_len=T / n_seg)
    terms = W.control_problem_terms(f_bias=f_bias, **seg)
    terms[2] = W.Term(W.CONST, W.Z, a=f_bias, t_off=T / 2)
    terms += [W.Term(W.PWC, W.X, seg_a_slot=2 * n_seg, **seg),
              W.Term(W.PWC, W.Y, seg_a_slot=3 * n_seg, **seg)]
    on = np.array([1.0, 0.0, 1.0, 0.0])
    params = np.concatenate([on * rng.uniform(1000.0, 2000.0, n_seg),
                             rng.uniform(0.0, 2 * math.pi, n_seg),
                             on * rng.uniform(-800.0, 800.0, n_seg),
                             on * rng.uniform(-800.0, 800.0, n_seg)])
    return W.Problem(spin_twice, terms, 0.0, dt_out, K, L, tau, frame, params=params,
                     psi0=W.random_state(spin_twice + 1, rng))


def _central_differences(oracle, prob, m, h_rel=1e-6):
    """dloss/dparams by central differences of the x87 extended-precision
    forward map, step h_rel * max(1, |p|)."""
    p = np.asarray(prob.params, dtype=np.longdouble)
    fd = np.zeros(p.size)
    for q in range(p.size):
        h = np.longdouble(h_rel) * max(np.longdouble(1.0), abs(p[q]))
        pp, pm = p.copy(), p.copy()
        pp[q] += h
        pm[q] -= h
        fd[q] = float((oracle.population_ld(prob, m, pp) - oracle.population_ld(prob, m, pm))
                      / (2 * h))
    return fd


def per_component_ok(g, fd, rel=1e-6, floor=1e-12):
    """|g - fd| <= rel |fd| on every component, and |g - fd| <= floor * max|fd|
    where the difference is itself 0 (the phase of a zero-amplitude segment)."""
    bound = np.maximum(rel * np.abs(fd), floor * np.max(np.abs(fd)))
    return bool(np.all(np.abs(g - fd) <= bound)), float(np.max(np.abs(g - fd) / bound))


@pytest.mark.parametrize("spin_twice,frame", [(2, True), (2, False), (1, True), (1, False)])
def test_adjoint_at_zero_transverse_field(oracle, spin_twice, frame):
    """Where a segment's amplitude is 0 the transverse angle rho is 0 and
    phi = atan2(0, 0) is only a convention (Sec. "Lie-Trotter based
    exponentiator"), but each exponential is analytic in theta_x, theta_y,
    so the gradient exists and is not 0.  Oracle adjoint vs extended-precision
    central differences, per component, both spins, frame on and off, random
    psi0 (a zero, NaN or dropped derivative at rho = 0 or theta = 0 fails)."""
    prob = _zero_field_problem(spin_twice, frame, seed=3 * spin_twice + frame)
    m = 1 if spin_twice == 2 else 0
    loss, g = oracle.adjoint_population(prob, m)
    assert np.all(np.isfinite(g))
    fd = _central_differences(oracle, prob, m)
    ok, worst = per_component_ok(g, fd)
    print(f"spin_twice={spin_twice} frame={frame}: grad {g[:4]} worst/bound {worst:.2e}")
    assert ok, (g, fd)
    # the amplitude derivatives of the segments without a transverse field
    # are not 0
    amp = np.max(np.abs(fd[[0, 2, 8, 10, 12, 14]]))
    for q in (1, 3, 9, 11, 13, 15):
        assert abs(fd[q]) > 1e-3 * amp, (q, fd)


@pytest.mark.parametrize("spin_twice", [2, 1])
def test_adjoint_continuous_at_zero_amplitude(oracle, spin_twice):
    """The gradient at A_s = 0 is the limit of the gradients at small
    nonzero A_s of either sign (the generic polar path), frame on."""
    prob = _zero_field_problem(spin_twice, True, seed=40 + spin_twice)
    m = 1 if spin_twice == 2 else 0
    _, g0 = oracle.adjoint_population(prob, m)
    scale = np.max(np.abs(g0))
    for eps in (1e-7, -1e-7, 1e-30):
        p = prob.params.copy()
        p[[1, 9]] = eps
        p[[3, 15]] = -eps
        _, g = oracle.adjoint_population(prob.replace(params=p), m)
        assert np.max(np.abs(g - g0)) <= 1e-9 * scale + 1e-5 * abs(eps) * scale, eps


CONTROL_FD = os.path.join(os.path.dirname(__file__), "golden", "control_gradients_fd.txt")


def control_fd_cases():
    """The stored extended-precision central differences of the control
    workload (tests/golden/control_gradients_fd.py wrote them with the
    oracle): {(label, instance): (params, slots, values)} with the full
    parameter vector rebuilt from the seeded workload and checked against
    the stored parameter values."""
    probs = W.control_batch(seed=4)
    rows = {}
    with open(CONTROL_FD) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            label, i, q, pv, fd = line.split()
            rows.setdefault((label, int(i)), []).append((int(q), float(pv), float(fd)))
    out = {}
    for (label, i), r in rows.items():
        params = probs[i].params.copy()
        if label == "zeroed":
            params[0:W.N_SEGMENTS:4] = 0.0
        slots = np.array([q for q, _, _ in r])
        assert np.array_equal(params[slots], [pv for _, pv, _ in r]), (label, i)
        out[(label, i)] = (params, slots, np.array([fd for _, _, fd in r]))
    return probs, out


def test_control_workload_gradients_vs_stored_differences(oracle):
    """The oracle's adjoint on the full-size control workload (256 segments,
    1e5 CF4 steps, tau = 28, loss = population of |0>) against central
    differences (h = 1e-6 relative) of its own extended-precision forward
    map: 8 seeded instances x (16 amplitudes + 16 phases), and one instance
    with every fourth amplitude set to 0, per component within 1e-6
    relative.  Two of the stored differences are recomputed here, so the
    file cannot drift from the oracle."""
    probs, cases = control_fd_cases()
    assert len(cases) == 9 and sum(len(s) for _, s, _ in cases.values()) == 9 * 32
    worst = 0.0
    for (label, i), (params, slots, fd) in cases.items():
        prob = probs[i].replace(params=params)
        _, g = oracle.adjoint_population(prob, 1)
        ok, w = per_component_ok(g[slots], fd)
        worst = max(worst, w)
        assert ok, (label, i, np.max(np.abs(g[slots] - fd) / np.abs(fd)))
    print(f"control workload: worst |adjoint - differences| / bound = {worst:.2e}")
    (label, i), (params, slots, fd) = next(iter(cases.items()))
    prob = probs[i].replace(params=params)
    for j in (0, len(slots) - 1):
        p = np.asarray(params, dtype=np.longdouble)
        h = np.longdouble(1e-6) * max(np.longdouble(1.0), abs(p[slots[j]]))
        pp, pm = p.copy(), p.copy()
        pp[slots[j]] += h
        pm[slots[j]] -= h
        live = float((oracle.population_ld(prob, 1, pp) - oracle.population_ld(prob, 1, pm))
                     / (2 * h))
        assert live == fd[j], (slots[j], live, fd[j])


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
