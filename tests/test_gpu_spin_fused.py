"""GPU: <J> formed in the last pass of the state product
(mss_propagate_spin) equals the projection kernel on the stored states bit for
bit, and leaves the states themselves as mss_propagate writes them, on every
scan shape (no level, one level, the fused two-level top, two levels in
separate launches, three levels); and the Simulator's want_spin path agrees
with the oracle."""
import numpy as np
import pytest

from paper_2204_05586_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_05586_amd import native
    native.lib()
    return torch


def _unitaries(torch, N, K, seed):
    """U_k = D_k V: one random unitary V and per-interval diagonal phases,
    built on the device (unitary, and cheap at tens of millions)."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    rng = np.random.default_rng(seed)
    V, _ = np.linalg.qr(rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N)))
    Vd = torch.from_numpy(V).cuda()
    ang = torch.rand((K, N), generator=g, device="cuda", dtype=torch.float64) * 6.283185307179586
    D = torch.polar(torch.ones_like(ang), ang)
    return (D[:, :, None] * Vd[None]).contiguous()


# K: 1 and 200 (one tile), 3000 (one level), 200000 (two levels, fused top),
# 1200000 (two levels, separate launches), 256^3 + 1 (three levels)
SHAPES = [(N, K) for N in (2, 3) for K in (1, 200, 3000, 200_000, 1_200_000)] + \
    [(3, 256 ** 3 + 1)]


@pytest.mark.parametrize("N,K", SHAPES, ids=[f"N{n}-K{k}" for n, k in SHAPES])
def test_fused_spin_equals_projection(dev, N, K):
    torch = dev
    from paper_2204_05586_amd import native
    print(f"[gpu] fused spin N={N} K={K}", flush=True)
    U = _unitaries(torch, N, K, seed=N * 1000 + K % 997)
    rng = np.random.default_rng(K)
    psi0 = native.device_state(W.random_state(N, rng))
    ws = native.alloc_workspace(native.propagate_workspace_size(N - 1, K))
    psi_a = torch.empty((K, N), dtype=torch.complex128, device="cuda")
    fin_a = torch.empty((N,), dtype=torch.complex128, device="cuda")
    psi_b, fin_b = torch.empty_like(psi_a), torch.empty_like(fin_a)
    spin = torch.full((K, 3), float("nan"), dtype=torch.float64, device="cuda")
    native.propagate(N - 1, U, psi0, psi_a, fin_a, ws)
    native.propagate(N - 1, U, psi0, psi_b, fin_b, ws, spin=spin)
    ref = native.spin_projection(psi_a)
    torch.cuda.synchronize()
    assert torch.equal(psi_a, psi_b) and torch.equal(fin_a, fin_b)
    assert torch.equal(spin, ref), float((spin - ref).abs().max())
    # norm is kept: |<J>| <= j for a unit state
    assert float(spin.norm(dim=1).max()) <= (N - 1) / 2 + 1e-9


@pytest.mark.parametrize("spin", [0.5, 1])
def test_simulator_want_spin(dev, oracle, spin):
    from paper_2204_05586_amd import Simulator
    terms = W.neural_pulse_terms() if spin == 1 else W.neural_pulse_terms()[:3]
    sim = Simulator(terms, spin=spin, rotating_frame=True, n_squares=28)
    args = ([0.6, 0.8j, 0] if spin == 1 else [0.6, 0.8j], 0.0495, 0.0505, 5e-8, 5e-7)
    a = sim.evaluate(*args, want_spin=True)
    b = sim.evaluate(*args)
    assert a._spin is not None and b._spin is None
    assert float((a.state - b.state).abs().max()) == 0.0
    assert float((a.spin - b.spin).abs().max()) == 0.0
    prob = sim.problem(0.0495, 0.0505, 5e-8, 5e-7, psi0=args[0])
    ref = oracle.solve(prob)
    assert np.max(np.abs(a.spin.cpu().numpy() - oracle.spin_projection(ref["psi"]))) <= TOL


@pytest.mark.parametrize("spin_twice", [1, 2])
def test_fused_spin_circular_drive_closed_form(dev, spin_twice):
    """The resonant circular drive of the oracle pins, on the GPU with <J>
    fused into the scan: <J>(t) = R_z(w0 t) R_x(2 pi A t) <J>(0)."""
    import math
    from paper_2204_05586_amd import native
    from tests import spin_algebra as SA
    F0, A, th, ph = 2.0e4, 900.0, 1.1, 0.4
    T = W.Term
    terms = [T(W.COS, W.X, a=A, f=F0), T(W.SIN, W.Y, a=A, f=F0), T(W.CONST, W.Z, a=F0)]
    half = np.array([math.cos(th / 2), np.exp(1j * ph) * math.sin(th / 2)])
    psi0 = half if spin_twice == 1 else SA.d1_state(half[None])[0]
    p = W.Problem(spin_twice, terms, 0.0, 3e-6, 70_000, 6, 28, True, psi0=psi0)
    print(f"[gpu] circular drive spin_twice={spin_twice}", flush=True)
    J = native.solve(p, want_spin=True)["spin"].cpu().numpy()

    def rot(axis, a):
        c, s = math.cos(a), math.sin(a)
        if axis == "x":
            return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
        return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])
    v0 = spin_twice / 2 * np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph),
                                    math.cos(th)])
    for k in (0, 1, 999, 35_000, 69_999):
        t = k * 3e-6
        ref = rot("z", 2 * math.pi * F0 * t) @ rot("x", 2 * math.pi * A * t) @ v0
        # over 4.2e5 fine steps and frame phases up to 2.6e4 rad, rounding
        # leaves the oracle itself 6.3e-11 from this closed form
        assert np.max(np.abs(J[k] - ref)) < 2e-10, (k, J[k], ref)
