"""Oracle pins for spin-1 in the full su(3) basis (the paper's extension
H = w_x J_x + w_y J_y + w_z J_z + w_q Q + w_u1 U_1 + w_u2 U_2 + w_v1 V_1 + w_v2 V_2,
Sec. "Spin-one").  The paper takes U_1, U_2, V_1, V_2 from a reference it does
not print; the reading pinned here is the Cartesian quadrupoles with
Delta m = +-2 (U) and +-1 (V).  The exponentiator (scaling and squaring with a
degree-4 Taylor residual) is pinned against scipy's expm, and the rotating
frame of the new components against a closed-form resonant solution."""
import math

import numpy as np
import pytest

from paper_2204_05586_amd import workloads as W

scipy_linalg = pytest.importorskip("scipy.linalg")

RNG = np.random.default_rng(2024)


def _ops(oracle):
    return [oracle.basis_operator(j) for j in range(8)]


def test_basis_spans_su3(oracle):
    A = _ops(oracle)
    for M in A:
        assert np.allclose(M, M.conj().T, atol=0) and abs(np.trace(M)) < 1e-15
    # real coordinates of the 8 Hermitian operators are linearly independent
    V = np.array([np.concatenate([M.real.ravel(), M.imag.ravel()]) for M in A])
    assert np.linalg.matrix_rank(V, tol=1e-12) == 8
    Jx, Jy, Jz = A[0], A[1], A[2]
    assert np.allclose(Jx @ Jy - Jy @ Jx, 1j * Jz, atol=1e-15)
    # spin-1 Casimir
    assert np.allclose(Jx @ Jx + Jy @ Jy + Jz @ Jz, 2 * np.eye(3), atol=1e-15)


def test_quadrupoles_carry_delta_m_two_and_one(oracle):
    """[J_z, U_1 + i U_2] = 2 (U_1 + i U_2) and [J_z, V_1 + i V_2] = V_1 + i V_2:
    the orientation the rotating frame relies on (U rotates at 2 omega_r,
    V at omega_r, both like x + i y).  The U's are orthogonal to the J's and
    to Q, as quadrupoles are."""
    A = _ops(oracle)
    Jz = A[2]
    Up = A[4] + 1j * A[5]
    Vp = A[6] + 1j * A[7]
    assert np.allclose(Jz @ Up - Up @ Jz, 2 * Up, atol=1e-15)
    assert np.allclose(Jz @ Vp - Vp @ Jz, Vp, atol=1e-15)
    Jp = A[0] + 1j * A[1]
    assert np.allclose(Jz @ Jp - Jp @ Jz, Jp, atol=1e-15)
    for u in (A[4], A[5], A[6], A[7]):
        for j in (A[0], A[1], A[2], A[3]):
            assert abs(np.trace(u @ j)) < 1e-15


def _generator(A, th):
    return sum(t * M for t, M in zip(th, A))


@pytest.mark.parametrize("tau", [16, 24, 28])
@pytest.mark.parametrize("scale", [1e-6, 0.3, 2.0])
def test_exp_full_matches_expm(oracle, tau, scale):
    A = _ops(oracle)
    for _ in range(40):
        th = RNG.normal(size=8)
        th *= scale / np.linalg.norm(th)
        ref = scipy_linalg.expm(-1j * _generator(A, th))
        got = oracle.exp_full(th, tau)
        assert np.max(np.abs(got - ref)) < 6e-15, (tau, scale)


@pytest.mark.parametrize("tau", [3, 5, 8])
def test_exp_full_truncation_bound(oracle, tau):
    """The degree-4 residual of the 2^-tau step leaves ~||G||^5 / (120 n^5)
    per step, n steps: the error is bounded by ||G||^5 / (120 n^4) (spectral
    norm), and is not far below it (the truncation is really degree 4)."""
    A = _ops(oracle)
    ratios = []
    for _ in range(30):
        th = RNG.normal(size=8)
        th *= 2.0 / np.linalg.norm(th)
        G = _generator(A, th)
        g = np.linalg.norm(G, 2)
        bound = g ** 5 / (120 * 2.0 ** (4 * tau))
        err = np.linalg.norm(oracle.exp_full(th, tau) - scipy_linalg.expm(-1j * G), 2)
        assert err <= 1.05 * bound + 1e-14, (tau, err, bound)
        ratios.append(err / bound)
    assert max(ratios) > 0.05


def test_exp_full_is_the_taylor_polynomial_at_tau_zero(oracle):
    """tau = 0: the degree-4 Taylor polynomial of exp(-i G); tau = 1: its
    square at G / 2 (the scaling and squaring of the definition)."""
    A = _ops(oracle)
    for _ in range(20):
        th = RNG.normal(size=8) * 0.3
        X = -1j * _generator(A, th)
        P = np.eye(3) + X + X @ X / 2 + X @ X @ X / 6 + X @ X @ X @ X / 24
        assert np.max(np.abs(oracle.exp_full(th, 0) - P)) < 1e-15
        Xh = X / 2
        Ph = np.eye(3) + Xh + Xh @ Xh / 2 + Xh @ Xh @ Xh / 6 + Xh @ Xh @ Xh @ Xh / 24
        assert np.max(np.abs(oracle.exp_full(th, 1) - Ph @ Ph)) < 1e-15


def test_exp_full_agrees_with_lie_trotter_without_quadrupoles(oracle):
    """With u = v = 0 both spin-1 exponentiators approximate the same
    exponential; at tau = 28 they agree to rounding."""
    for _ in range(40):
        th4 = RNG.normal(size=4) * 0.8
        th8 = np.concatenate([th4, np.zeros(4)])
        assert np.max(np.abs(oracle.exp_full(th8, 28) - oracle.exp_one(th4, 28))) < 5e-15


def _resonant_problem(frame, K=400, L=40, Dt=2e-6):
    F0, A, B, fq = 2.0e4, 700.0, 400.0, 90.0
    T = W.Term
    terms = [T(W.CONST, W.Z, a=F0), T(W.CONST, W.Q, a=fq),
             T(W.COS, W.V1, a=A, f=F0), T(W.SIN, W.V2, a=A, f=F0),
             T(W.COS, W.U1, a=B, f=2 * F0), T(W.SIN, W.U2, a=B, f=2 * F0)]
    psi0 = np.array([0.6, 0.48 + 0.36j, 0.0j + 0.52])
    psi0 = psi0 / np.linalg.norm(psi0)
    return W.Problem(2, terms, 0.0, Dt, K, L, 28, frame, psi0=psi0), (F0, A, B, fq)


def test_resonant_quadrupole_drive_closed_form(oracle):
    """Bias w0 = 2 pi F0 on z, (v1 + i v2) = A e^{i w0 t} and
    (u1 + i u2) = B e^{2 i w0 t}: in the frame rotating at w0 about z the
    Hamiltonian is the constant 2 pi (A V_1 + B U_1 + f_q Q), so
    psi(t) = exp(-i w0 t J_z) exp(-i 2 pi (A V_1 + B U_1 + f_q Q) t) psi0.
    With the rotating frame on, each interval's frame Hamiltonian is
    constant and CF4 is exact; with it off the result is 4th-order accurate."""
    A_ = _ops(oracle)
    for frame, tol in ((True, 2e-12), (False, 2e-6)):
        prob, (F0, A, B, fq) = _resonant_problem(frame)
        r = oracle.solve(prob)
        H0 = 2 * math.pi * (A * A_[6] + B * A_[4] + fq * A_[3])
        worst = 0.0
        for k in (0, 57, 199, prob.n_samples - 1):
            t = k * prob.dt_out
            ref = scipy_linalg.expm(-1j * 2 * math.pi * F0 * t * A_[2]) @ \
                scipy_linalg.expm(-1j * H0 * t) @ prob.psi0
            worst = max(worst, np.max(np.abs(r["psi"][k] - ref)))
        assert worst < tol, (frame, worst)


def test_full_basis_frame_on_matches_frame_off(oracle):
    """Random full-basis fields: frame on and off solve the same lab-frame
    problem, so they agree to the integrator's accuracy (a wrong frame
    phase on any of the new components breaks this at O(1))."""
    rng = np.random.default_rng(5)
    T = W.Term
    F0 = 1.5e4
    comps = [W.X, W.Y, W.U1, W.U2, W.V1, W.V2]
    terms = [T(W.CONST, W.Z, a=F0), T(W.CONST, W.Q, a=120.0)]
    for c in comps:
        terms.append(T(W.COS if rng.random() < 0.5 else W.SIN, c, a=rng.uniform(100, 500),
                       f=F0 * rng.choice([1.0, 2.0]) * rng.uniform(0.98, 1.02),
                       phi=rng.uniform(0, 6)))
    psi0 = np.array([0.6, 0.0, 0.8], dtype=complex)
    out = []
    for frame in (False, True):
        p = W.Problem(2, terms, 0.0, 2e-6, 300, 40, 28, frame, psi0=psi0)
        out.append(oracle.solve(p)["psi"])
    assert np.max(np.abs(out[0] - out[1])) < 5e-7


def test_adjoint_refuses_full_basis(oracle):
    prob, _ = _resonant_problem(True, K=4, L=2)
    with pytest.raises(ValueError, match="su\\(3\\)"):
        oracle.adjoint_population(prob, 0)
