"""Pins of the CPU oracle to facts it does not compute itself.

Each test names the passage of arXiv:2204.05586 it pins and the kind of
mistake in the oracle it would catch.  None of these tests needs a GPU.
"""
import math

import numpy as np
import pytest

from paper_2204_05586_amd import workloads as W
from tests import spin_algebra as SA

RNG = np.random.default_rng(12345)


def _rand_theta(scale, n, dim):
    d = 3 if dim == 2 else 4
    v = RNG.normal(size=(n, d))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v * scale * RNG.uniform(0.5, 1.0, size=(n, 1))


# --------------------------------------------------------------------------
# exponentiators (Sec. "Lie-Trotter based exponentiator")
# --------------------------------------------------------------------------

@pytest.mark.parametrize("scale", [1e-9, 1e-4, 0.2, 1.0, 3.0])
def test_exp_half_is_exact_su2_exponential(oracle, scale):
    """Spin-1/2 analytic exponential vs eigh-based exp(-i theta.sigma/2).
    Catches a wrong sign, a swapped x/y entry or a missing factor 1/2."""
    for th in _rand_theta(scale, 50, 2):
        E = oracle.exp_half(th)
        assert np.max(np.abs(E - SA.exact_exp(th, 2))) < 3e-15


def test_exp_half_zero_angle_is_identity(oracle):
    assert np.array_equal(oracle.exp_half([0.0, 0.0, 0.0]), np.eye(2))


@pytest.mark.parametrize("tau", [24, 28])
@pytest.mark.parametrize("scale", [6e-4, 0.22, 1.0])
def test_exp_one_matches_exact_exponential(oracle, tau, scale):
    """Spin-1 Lie-Trotter exponentiator with residual squaring vs the exact
    exponential of theta_x J_x + theta_y J_y + theta_z J_z + theta_q Q.  At
    n = 2^24..2^28 the Trotter error is below 1e-18, so only rounding is
    left (the paper reports its error minimised near tau = 24)."""
    for th in _rand_theta(scale, 60, 3):
        E = oracle.exp_one(th, tau)
        assert np.max(np.abs(E - SA.exact_exp(th, 3))) < 5e-15


def _factor_product(th):
    """T for n = 1 as the product of its three factors (symmetric split):
    exp(-i D/2) exp(-i Phi J_phi) exp(-i D/2), D = theta_z J_z + theta_q Q."""
    D = th[2] * SA.SZ3 + th[3] * SA.Q3
    Phi = math.hypot(th[0], th[1])
    phi = math.atan2(th[1], th[0])
    Jphi = math.cos(phi) * SA.SX3 + math.sin(phi) * SA.SY3
    half = SA.expmh(D / 2)
    return half @ SA.expmh(Phi * Jphi) @ half


def test_elementwise_T_equals_factor_product(oracle):
    """tau = 0 gives T itself; it must equal the product of the three factor
    exponentials.  This pins the corrected element-wise T (the printed
    T_13 and T_22 entries carry misprints)."""
    for th in _rand_theta(1.5, 100, 3):
        T = oracle.exp_one(th, 0)
        assert np.max(np.abs(T - _factor_product(th))) < 2e-15


def test_transverse_angle_enters_only_through_jz_phases(oracle):
    """The transverse direction phi enters the split factor only through
    P = exp(-i phi J_z) = diag(e^{-i phi}, 1, e^{i phi}): rotating about z
    carries J_x to J_phi and commutes with D, so T(theta) = P T0 P^H with T0
    the factor at phi = 0, which is complex symmetric (J_x real symmetric, D
    diagonal).  Squarings keep both properties.  Fails on a wrong sign or
    power of e^{i phi} in any entry, or a transposed off-diagonal pair."""
    m = np.array([1.0, 0.0, -1.0])
    for th in _rand_theta(1.5, 60, 3):
        rho = math.hypot(th[0], th[1])
        phi = math.atan2(th[1], th[0])
        th0 = np.array([rho, 0.0, th[2], th[3]])
        P = np.diag(np.exp(-1j * phi * m))
        for tau in (0, 1, 5, 28):
            T0 = oracle.exp_one(th0, tau)
            T = oracle.exp_one(th, tau)
            assert np.max(np.abs(T0 - T0.T)) < 1e-14
            assert np.max(np.abs(T - P @ T0 @ P.conj().T)) < 1e-14
        a0 = oracle.lie_trotter_residual(th0, 28)
        a = oracle.lie_trotter_residual(th, 28)
        scale = np.max(np.abs(a0))
        assert np.max(np.abs(a0 - a0.T)) / scale < 1e-15
        assert np.max(np.abs(a - P @ a0 @ P.conj().T)) / scale < 1e-14


def test_printed_T_entries_are_misprinted():
    """Documents the reading of the two garbled entries: with q != 0 the
    printed T_13 = -(sin(Phi/2) e^{iq/6} e^{-i phi})^2 and
    T_22 = cos(Phi) e^{i4q} disagree with the factor product, while the
    corrected ones (e^{-iq/6} inside the square, e^{2iq/3}) agree."""
    th = np.array([0.3, -0.2, 0.4, 0.7])
    T = _factor_product(th)
    Phi = math.hypot(th[0], th[1])
    phi = math.atan2(th[1], th[0])
    q = th[3]
    printed_13 = -(math.sin(Phi / 2) * np.exp(1j * q / 6) * np.exp(-1j * phi)) ** 2
    fixed_13 = -(math.sin(Phi / 2) * np.exp(-1j * q / 6) * np.exp(-1j * phi)) ** 2
    printed_22 = math.cos(Phi) * np.exp(4j * q)
    fixed_22 = math.cos(Phi) * np.exp(2j * q / 3)
    assert abs(printed_13 - T[0, 2]) > 1e-2 and abs(fixed_13 - T[0, 2]) < 1e-15
    assert abs(printed_22 - T[1, 1]) > 1e-2 and abs(fixed_22 - T[1, 1]) < 1e-15


def test_residual_has_no_cancellation(oracle):
    """a = T - I at n = 2^28 is ~1e-9: computing it as T - I would keep only
    ~7 digits.  Compare with T - I evaluated at 50 digits (mpmath).  Catches
    a diagonal built by subtracting the identity from T."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    J = [mp.matrix(SA.SX3.tolist()), mp.matrix(SA.SY3.tolist()),
         mp.matrix(SA.SZ3.tolist()), mp.matrix(SA.Q3.tolist())]
    for th in _rand_theta(0.5, 8, 3):
        tau = 28
        n = mp.mpf(2) ** tau
        t = [mp.mpf(float(x)) / n for x in th]
        D = t[2] * J[2] + t[3] * J[3]
        Phi = mp.sqrt(t[0] ** 2 + t[1] ** 2)
        phi = mp.atan2(t[1], t[0])
        Jphi = mp.cos(phi) * J[0] + mp.sin(phi) * J[1]
        half = mp.expm(-1j * D / 2)
        Tm = half * mp.expm(-1j * Phi * Jphi) * half - mp.eye(3)
        ref = np.array([[complex(Tm[i, j]) for j in range(3)] for i in range(3)])
        a = oracle.lie_trotter_residual(th, tau)
        scale = np.max(np.abs(ref))
        assert np.max(np.abs(a - ref)) / scale < 1e-14


def test_tau_sweep_minimum(oracle):
    """The paper chose tau by sweeping the squaring count against a reference
    exponential and found the error minimised at tau = 24.  The symmetric
    split is second order, so below the rounding floor the error falls by
    4x per extra squaring (16x per two); with residual squaring it then
    stays at the floor instead of growing from over-squaring."""
    ths = _rand_theta(1.0, 40, 3)

    def err(tau):
        return max(np.max(np.abs(oracle.exp_one(th, tau) - SA.exact_exp(th, 3))) for th in ths)

    e = {tau: err(tau) for tau in (4, 6, 8, 10, 12, 20, 22, 24, 28, 32, 40)}
    for tau in (4, 6, 8, 10):
        assert 12.0 < e[tau] / e[tau + 2] < 20.0, e
    assert e[20] > 1e-14 and e[22] > e[24]
    for tau in (24, 28, 32, 40):
        assert e[tau] < 3e-15, e


# --------------------------------------------------------------------------
# field programs (data format of the sweep-parameter field functions)
# --------------------------------------------------------------------------

def test_field_program_values(oracle):
    """Hand-evaluated field-program values: literal and slot coefficients,
    strict time windows, piecewise-constant segments with clamping."""
    T = W.Term
    terms = [T(W.CONST, W.Z, a=5.0),
             T(W.COS, W.X, a=2.0, f=0.25, phi=0.0),             # 2 cos(pi t / 2)
             T(W.SIN, W.Y, a_slot=0, f=0.5, phi_slot=1),         # p0 sin(pi t + p1)
             T(W.CONST, W.Z, a=1.0, t_on=1.0, t_off=2.0),
             T(W.PWC, W.Q, n_seg=3, seg_t0=0.0, seg_len=1.0, seg_a_slot=2),
             T(W.PWC_COS, W.X, f=0.0, n_seg=3, seg_t0=0.0, seg_len=1.0, seg_a_slot=2,
               seg_phi_slot=5)]
    params = np.array([3.0, math.pi / 2, 10.0, 20.0, 30.0, 0.0, math.pi, math.pi / 3])
    p = W.Problem(2, terms, 0.0, 1.0, 1, 1, 0, False, params=params)
    # t = 1.0: the window (1, 2) is open at both ends, so the z bump is off
    f = oracle.field(p, 1.0)
    assert f[2] == pytest.approx(5.0, abs=0)
    # 2 cos(pi/2) ~ 0; segment 1 -> 20 cos(pi) = -20
    assert f[0] == pytest.approx(-20.0, abs=1e-12)
    assert f[1] == pytest.approx(3.0 * math.sin(math.pi + math.pi / 2), abs=1e-12)
    assert f[3] == 20.0
    f = oracle.field(p, 1.5)
    assert f[2] == 6.0
    assert f[0] == pytest.approx(2 * math.cos(math.pi * 0.75) - 20.0, abs=1e-12)
    # clamping below and above the segment range
    assert oracle.field(p, -4.0)[3] == 10.0
    f = oracle.field(p, 7.0)
    assert f[3] == 30.0
    assert f[0] == pytest.approx(2 * math.cos(math.pi * 3.5) + 30 * math.cos(math.pi / 3),
                                 abs=1e-12)


# --------------------------------------------------------------------------
# whole trajectories
# --------------------------------------------------------------------------

def _const_problem(spin_twice, f, K, L, dt_out, frame=False, psi0=None):
    T = W.Term
    terms = [T(W.CONST, c, a=v) for c, v in enumerate(f) if v != 0.0]
    if spin_twice == 1:
        terms = [t for t in terms if t.comp != W.Q]
    return W.Problem(spin_twice, terms, 0.0, dt_out, K, L, 28, frame, psi0=psi0)


@pytest.mark.parametrize("spin_twice", [1, 2])
def test_constant_field_is_exact(oracle, spin_twice):
    """Constant H: both CF4 stages average to H/2, so CF4 is exact and
    psi_k = exp(-i H k Dt) psi_0 (eq. exp_sol_of_constant).  Catches wrong
    2 pi factors, a wrong fine step, or wrong exponentiators / Q."""
    f = [310.0, -170.0, 520.0, 90.0]
    dim = spin_twice + 1
    psi0 = W.random_state(dim, RNG)
    K, L, dt_out = 400, 7, 1e-4
    p = _const_problem(spin_twice, f, K, L, dt_out, psi0=psi0)
    r = oracle.solve(p, want_U=True)
    H = SA.generator([2 * math.pi * x for x in (f[:3] if dim == 2 else f)], dim)
    Uex = SA.expmh(H * dt_out)
    assert np.max(np.abs(r["U"] - Uex)) < 1e-13
    for k in (0, 1, 17, K - 1):
        ref = SA.expmh(H * dt_out * k) @ psi0
        assert np.max(np.abs(r["psi"][k] - ref)) < 1e-12
    assert np.max(np.abs(r["psi_final"] - SA.expmh(H * dt_out * K) @ psi0)) < 1e-12


def _circular_problem(spin_twice, fz, fd, amp, fq, K, L, dt_out, frame, psi0, t_start=0.0):
    T = W.Term
    terms = [T(W.CONST, W.Z, a=fz), T(W.COS, W.X, a=amp, f=fd), T(W.SIN, W.Y, a=amp, f=fd)]
    if spin_twice == 2 and fq:
        terms.append(T(W.CONST, W.Q, a=fq))
    return W.Problem(spin_twice, terms, t_start, dt_out, K, L, 28, frame, psi0=psi0)


def _circular_exact(spin_twice, fz, fd, amp, fq, t, psi0, t0=0.0):
    """psi(t) for a circular drive at f_d: exact solution from the frame
    rotating at omega_d from t = 0 (Sec. "Dynamically rotating frame")."""
    dim = spin_twice + 1
    wd = 2 * math.pi * fd
    Hr = SA.generator([2 * math.pi * amp, 0.0, 2 * math.pi * (fz - fd), 2 * math.pi * fq], dim)
    Jz = SA.SZ2 if dim == 2 else SA.SZ3
    Rt = SA.expmh(wd * t * Jz)
    R0 = SA.expmh(wd * t0 * Jz)
    return Rt @ SA.expmh(Hr * (t - t0)) @ R0.conj().T @ psi0


@pytest.mark.parametrize("spin_twice", [1, 2])
def test_resonant_circular_drive_in_frame_is_exact(oracle, spin_twice):
    """Circular drive at f_d = f_z with the frame on: omega_r = omega_z and
    the frame Hamiltonian is constant within every interval, so CF4 is
    exact.  Pins the frame entry (time origin t - t_k, sign of the rotation)
    and the exit R(-Dt)."""
    fz = fd = 2.0e5
    amp, fq = 3.0e3, 700.0
    dim = spin_twice + 1
    psi0 = W.random_state(dim, RNG)
    K, L, dt_out, t0 = 300, 5, 3.1e-6, 2.3e-5
    p = _circular_problem(spin_twice, fz, fd, amp, fq, K, L, dt_out, True, psi0, t_start=t0)
    r = oracle.solve(p)
    for k in (0, 1, 5, 99, K - 1):
        ref = _circular_exact(spin_twice, fz, fd, amp, fq, t0 + k * dt_out, psi0, t0)
        assert np.max(np.abs(r["psi"][k] - ref)) < 1e-12, k
    ref = _circular_exact(spin_twice, fz, fd, amp, fq, t0 + K * dt_out, psi0, t0)
    assert np.max(np.abs(r["psi_final"] - ref)) < 1e-12


@pytest.mark.parametrize("frame", [False, True])
def test_fourth_order_convergence(oracle, frame):
    """CF4 is fourth order (eq. cf4_implementation: local error O(dt^5)):
    halving dt divides the global error by ~16.  Detuned circular drive,
    compared with its exact solution.  Catches swapped Gauss weights, wrong
    nodes or a wrong product order."""
    fz, fd, amp = 5.0e3, 5.6e3, 1.2e3
    psi0 = np.array([1.0, 0.0], dtype=complex)
    K, dt_out = 20, 1e-4
    errs = []
    Ls = [2, 4, 8, 16]
    for L in Ls:
        p = _circular_problem(1, fz, fd, amp, 0.0, K, L, dt_out, frame, psi0)
        r = oracle.solve(p)
        ref = _circular_exact(1, fz, fd, amp, 0.0, K * dt_out, psi0)
        errs.append(np.max(np.abs(r["psi_final"] - ref)))
    slopes = np.diff(np.log(errs)) / np.diff(np.log(1.0 / np.array(Ls)))
    assert np.all(np.array(errs) > 1e-12), errs
    assert np.all((slopes > 3.8) & (slopes < 4.2)), (errs, slopes)


@pytest.mark.parametrize("frame", [False, True])
def test_spin_one_is_d1_of_spin_half(oracle, frame):
    """With f_q = 0 the spin-1 problem is the spin-1 representation of the
    spin-1/2 one: U^(1) = D^1(U^(1/2)) through every step (exponentials of
    Lie-algebra elements, products, frame).  Catches inconsistent basis
    order, J_y sign or m values between the two exponentiators."""
    rng = np.random.default_rng(7)
    p2 = W.random_problem(rng, 1, 200, 6, rotating_frame=frame)
    p3 = p2.replace(spin_twice=2, psi0=SA.d1_state(p2.psi0))
    r2 = oracle.solve(p2, want_U=True)
    r3 = oracle.solve(p3, want_U=True)
    assert np.max(np.abs(r3["U"] - SA.d1(r2["U"]))) < 1e-12
    assert np.max(np.abs(r3["psi"] - SA.d1_state(r2["psi"]))) < 1e-12


@pytest.mark.parametrize("spin_twice", [1, 2])
def test_unitarity(oracle, spin_twice):
    """Exponentials of anti-Hermitian generators are unitary by construction
    (Sec. "Lie-Trotter based exponentiator", last paragraph)."""
    rng = np.random.default_rng(11)
    p = W.random_problem(rng, spin_twice, 300, 10, rotating_frame=False)
    U = oracle.solve(p, want_U=True)["U"]
    dev = np.einsum("kji,kjl->kil", U.conj(), U) - np.eye(spin_twice + 1)
    assert np.max(np.abs(dev)) < 1e-12


def test_state_compilation_convention(oracle):
    """psi_0 = psi_init, psi_{k+1} = U_k psi_k, psi_final = U_{K-1} psi_{K-1}
    (eq. integration_compilation), on diagonal phases with a closed form."""
    K = 50
    alpha = RNG.uniform(-1, 1, K)
    U = np.zeros((K, 2, 2), dtype=complex)
    U[:, 0, 0] = np.exp(-1j * alpha)
    U[:, 1, 1] = np.exp(1j * alpha)
    psi0 = np.array([0.6, 0.8j])
    psi, fin = oracle.states(U, psi0)
    cum = np.concatenate([[0.0], np.cumsum(alpha)])
    ref = np.stack([psi0[0] * np.exp(-1j * cum), psi0[1] * np.exp(1j * cum)], axis=1)
    assert np.max(np.abs(psi - ref[:K])) < 1e-14
    assert np.max(np.abs(fin - ref[K])) < 1e-14


def test_brute_force_50_digits(oracle):
    """Tiny problems: the same discrete scheme (nodes, weights, frame, exit,
    ordered products) in 50-digit arithmetic with exact matrix exponentials
    in place of the exponentiators.  Pins the oracle's arithmetic and its
    evaluation order to ~1e-14."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    for spin_twice, frame in [(1, True), (2, True), (2, False)]:
        rng = np.random.default_rng(100 + spin_twice)
        p = W.random_problem(rng, spin_twice, 4, 3, rotating_frame=frame)
        ref = _mp_solve(mp, p)
        r = oracle.solve(p)
        assert np.max(np.abs(r["psi"] - ref[:-1])) < 1e-13
        assert np.max(np.abs(r["psi_final"] - ref[-1])) < 1e-13


def _mp_field(mp, p, t):
    f = [mp.mpf(0)] * 4
    for tm in p.terms:
        if not (tm.t_on < t < tm.t_off):
            continue
        a = mp.mpf(p.params[tm.a_slot]) if tm.a_slot >= 0 else mp.mpf(tm.a)
        fr = mp.mpf(p.params[tm.f_slot]) if tm.f_slot >= 0 else mp.mpf(tm.f)
        ph = mp.mpf(p.params[tm.phi_slot]) if tm.phi_slot >= 0 else mp.mpf(tm.phi)
        arg = 2 * mp.pi * fr * t + ph
        v = {W.CONST: a, W.COS: a * mp.cos(arg), W.SIN: a * mp.sin(arg)}[tm.kind]
        f[tm.comp] += v
    return f


def _mp_solve(mp, p):
    dim = p.dim
    if dim == 2:
        J = [mp.matrix(SA.SX2.tolist()), mp.matrix(SA.SY2.tolist()), mp.matrix(SA.SZ2.tolist()),
             mp.zeros(2, 2)]
        m = [mp.mpf(1) / 2, -mp.mpf(1) / 2]
    else:
        J = [mp.matrix(M.tolist()) for M in (SA.SX3, SA.SY3, SA.SZ3, SA.Q3)]
        m = [1, 0, -1]
    s3 = mp.sqrt(3)
    c = [(1 - 1 / s3) / 2, (1 + 1 / s3) / 2]
    wp, wm = (3 + 2 * s3) / 12, (3 - 2 * s3) / 12
    Dt = mp.mpf(p.dt_out)
    dt = Dt / p.n_fine
    v = mp.matrix([[complex(x)] for x in p.psi0])
    out = [v]
    for k in range(p.n_samples):
        tk = mp.mpf(p.t_start) + k * Dt
        wr = 2 * mp.pi * _mp_field(mp, p, tk + Dt / 2)[2] if p.rotating_frame else mp.mpf(0)
        U = mp.eye(dim)
        for l in range(p.n_fine):
            w = []
            for i in range(2):
                ti = (l + c[i]) * dt
                f = _mp_field(mp, p, tk + ti)
                om = [2 * mp.pi * x for x in f]
                xy = (om[0] + 1j * om[1]) * mp.exp(-1j * wr * ti)
                w.append([mp.re(xy), mp.im(xy), om[2] - wr, om[3]])
            H1 = sum(((wp * w[0][j] + wm * w[1][j]) * J[j] for j in range(4)), mp.zeros(dim, dim))
            H2 = sum(((wm * w[0][j] + wp * w[1][j]) * J[j] for j in range(4)), mp.zeros(dim, dim))
            U = mp.expm(-1j * H2 * dt) * (mp.expm(-1j * H1 * dt) * U)
        R = mp.diag([mp.exp(-1j * m[i] * wr * Dt) for i in range(dim)])
        v = R * U * v
        out.append(v)
    return np.array([[complex(x[i]) for i in range(dim)] for x in out])


def test_rabi_rotating_wave_sanity(oracle):
    """Spin-1/2 Rabi drive (f_z = 1 kHz, f_x = 200 cos(2 pi 1 kHz t)) vs the
    rotating-wave closed form.  The RWA drops the counter-rotating term, so
    agreement is only to a few 1e-2 (Bloch-Siegert shift, micromotion)."""
    p = W.spin_half_rabi(n_samples=2000)
    r = oracle.solve(p)
    t = np.arange(p.n_samples) * p.dt_out
    w0, Om = 2 * math.pi * 1000, 2 * math.pi * 100
    ref = np.stack([np.exp(-1j * w0 * t / 2) * np.cos(Om * t / 2),
                    -1j * np.exp(1j * w0 * t / 2) * np.sin(Om * t / 2)], axis=1)
    assert np.max(np.abs(r["psi"] - ref)) < 6e-2
    assert np.max(np.abs(np.abs(r["psi"]) ** 2 - np.abs(ref) ** 2)) < 4e-2


def test_rabi_matches_adaptive_ode_solver(oracle):
    """The paper's own accuracy baseline: a tight-tolerance adaptive
    Runge-Kutta solution of the Schroedinger equation (scipy solve_ivp,
    DOP853).  CF4 at dt = 1e-7 s is far below the ODE tolerance here."""
    from scipy.integrate import solve_ivp
    p = W.spin_half_rabi(n_samples=1000)
    r = oracle.solve(p)
    t_eval = np.arange(p.n_samples) * p.dt_out

    def rhs(t, y):
        fx = 200.0 * math.cos(2 * math.pi * 1000.0 * t)
        H = 2 * math.pi * (fx * SA.SX2 + 1000.0 * SA.SZ2)
        psi = y[:2] + 1j * y[2:]
        d = -1j * (H @ psi)
        return np.concatenate([d.real, d.imag])

    sol = solve_ivp(rhs, (0.0, t_eval[-1]), [1.0, 0.0, 0.0, 0.0], method="DOP853",
                    t_eval=t_eval, rtol=1e-12, atol=1e-13)
    ref = (sol.y[:2] + 1j * sol.y[2:]).T
    assert np.max(np.abs(r["psi"] - ref)) < 1e-9
