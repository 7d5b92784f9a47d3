"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  Bar: max |delta psi| <= 1e-10 (FP64), unitarity of U_k
to 1e-12, launch-shape invariance to 1e-13."""
import math

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


def _gpu(prob, store_u=True, launch=None):
    import torch
    from paper_2204_05586_amd import native
    print(f"[gpu] {prob.name} spin2={prob.spin_twice} K={prob.n_samples} L={prob.n_fine} "
          f"tau={prob.n_squares} frame={prob.rotating_frame} launch={launch}", flush=True)
    if launch is None:
        r = native.solve(prob, store_u=store_u, want_time=True)
    else:
        K, N = prob.n_samples, prob.dim
        U = torch.empty((K, N, N), dtype=torch.complex128, device="cuda")
        psi = torch.empty((K, N), dtype=torch.complex128, device="cuda")
        fin = torch.empty((N,), dtype=torch.complex128, device="cuda")
        ws = native.alloc_workspace(native.propagate_workspace_size(prob.spin_twice, K))
        native.integrate(prob, native.device_params(prob), U, launch=launch)
        native.propagate(prob.spin_twice, U, native.device_state(prob.psi0), psi, fin, ws)
        r = {"U": U, "psi": psi, "psi_final": fin, "time": None}
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in r.items()}


def _compare(g, ref, tol=TOL, name=""):
    dpsi = np.max(np.abs(g["psi"] - ref["psi"]))
    dfin = np.max(np.abs(g["psi_final"] - ref["psi_final"]))
    msg = f"{name}: max|dpsi|={dpsi:.3e} max|dfinal|={dfin:.3e}"
    if g.get("U") is not None and ref.get("U") is not None:
        dU = np.max(np.abs(g["U"] - ref["U"]))
        msg += f" max|dU|={dU:.3e}"
        assert dU <= tol, msg
    print(msg, flush=True)
    assert dpsi <= tol and dfin <= tol, msg


def test_spin_half_rabi_full(dev, oracle):
    """Spin-1/2 Rabi drive, 1e4 samples x 100 fine steps (1e6 CF4 steps)."""
    prob = W.spin_half_rabi()
    _compare(_gpu(prob), oracle.solve(prob, want_U=True), name=prob.name)


def test_spin_one_sensing_full(dev, oracle):
    """Spin-1 sensing drive, 2e5 samples x 10 fine steps (2e6 CF4 steps),
    tau = 28, across the 1 ms pulse window."""
    prob = W.spin_one_sensing()
    g = _gpu(prob, store_u=False)
    ref = oracle.solve(prob)
    _compare(g, ref, name=prob.name)
    t = g["time"]
    assert np.array_equal(t, prob.t_start + np.arange(prob.n_samples) * prob.dt_out)


@pytest.mark.parametrize("spin_twice", [1, 2])
@pytest.mark.parametrize("frame", [True, False])
@pytest.mark.parametrize("K", [1, 255, 256, 257, 3001])
def test_random_problems(dev, oracle, spin_twice, frame, K):
    rng = np.random.default_rng(1000 * spin_twice + K + (7 if frame else 0))
    prob = W.random_problem(rng, spin_twice, K, int(rng.integers(1, 13)), rotating_frame=frame)
    _compare(_gpu(prob), oracle.solve(prob, want_U=True), name=f"random K={K}")


@pytest.mark.parametrize("K", [65537, 300001])
def test_multilevel_scan(dev, oracle, K):
    """K above 256^2 needs three scan levels."""
    rng = np.random.default_rng(5)
    prob = W.random_problem(rng, 2, K, 2, n_squares=12)
    _compare(_gpu(prob), oracle.solve(prob, want_U=True), name=f"K={K}")


@pytest.mark.parametrize("slices", [1, 2, 4, 8, 16])
def test_launch_shapes_agree(dev, oracle, slices):
    """Any lane-slice count gives the same operators (product association
    only changes rounding)."""
    prob = W.spin_one_sensing(n_samples=1500, n_fine=16, t_start=0.0499)
    ref = oracle.solve(prob, want_U=True)
    g = _gpu(prob, launch=(slices, 256))
    _compare(g, ref, name=f"slices={slices}")
    base = _gpu(prob, launch=(1, 256))
    assert np.max(np.abs(g["U"] - base["U"])) < 1e-13


def test_unitarity(dev):
    prob = W.random_problem(np.random.default_rng(9), 2, 4000, 10, rotating_frame=False)
    U = _gpu(prob)["U"]
    dev_ = np.einsum("kji,kjl->kil", U.conj(), U) - np.eye(3)
    assert np.max(np.abs(dev_)) < 1e-12


@pytest.mark.parametrize("tau", [0, 1, 24, 40])
def test_squaring_counts(dev, oracle, tau):
    prob = W.spin_one_sensing(n_samples=300, n_squares=tau, t_start=0.05)
    _compare(_gpu(prob), oracle.solve(prob, want_U=True), name=f"tau={tau}")


def test_piecewise_constant_controls(dev, oracle):
    """Control-problem field program (PWC cos/sin with per-segment slots)."""
    prob = W.control_batch(n_inst=1, n_samples=400, n_fine=20)[0]
    _compare(_gpu(prob), oracle.solve(prob, want_U=True), name="pwc controls")


def test_free_evolution_is_identity(dev):
    prob = W.Problem(2, [], 0.0, 1e-3, 100, 3, 28, True)
    g = _gpu(prob)
    assert np.max(np.abs(g["U"] - np.eye(3))) == 0.0
    assert np.max(np.abs(g["psi"] - prob.psi0)) == 0.0


def test_propagate_matches_sequential_product(dev, oracle):
    """Scan alone on random unitaries vs the oracle's sequential product."""
    import torch
    from paper_2204_05586_amd import native
    rng = np.random.default_rng(3)
    for N, K in [(2, 1), (3, 700), (3, 70_000)]:
        X = rng.normal(size=(K, N, N)) + 1j * rng.normal(size=(K, N, N))
        Uh, _ = np.linalg.qr(X)
        psi0 = W.random_state(N, rng)
        ref_psi, ref_fin = oracle.states(Uh, psi0)
        U = torch.from_numpy(Uh).cuda()
        psi = torch.empty((K, N), dtype=torch.complex128, device="cuda")
        fin = torch.empty((N,), dtype=torch.complex128, device="cuda")
        ws = native.alloc_workspace(native.propagate_workspace_size(N - 1, K))
        print(f"[gpu] propagate N={N} K={K}", flush=True)
        native.propagate(N - 1, U, native.device_state(psi0), psi, fin, ws)
        torch.cuda.synchronize()
        assert np.max(np.abs(psi.cpu().numpy() - ref_psi)) < 1e-11
        assert np.max(np.abs(fin.cpu().numpy() - ref_fin)) < 1e-11


def test_simulator_front_end(dev, oracle):
    from paper_2204_05586_amd import Simulator
    sim = Simulator(W.neural_pulse_terms(), spin=1, rotating_frame=True, n_squares=24)
    res = sim.evaluate([1, 0, 0], 0.0495, 0.0505, 5e-8, 5e-7)
    prob = sim.problem(0.0495, 0.0505, 5e-8, 5e-7, psi0=[1, 0, 0])
    ref = oracle.solve(prob, want_U=True)
    assert res.state.shape == (2000, 3)
    assert np.max(np.abs(res.state.cpu().numpy() - ref["psi"])) <= TOL
    assert np.max(np.abs(res.time_evolution.cpu().numpy() - ref["U"])) <= TOL


def test_simulator_specialised_field(dev, oracle):
    """A Simulator that compiles its field program at construction gives the
    interpreting Simulator's states (same lane plan) and the oracle's."""
    from paper_2204_05586_amd import Simulator
    args = ([0.6, 0.8j, 0], 0.0495, 0.0505, 5e-8, 5e-7)
    a = Simulator(W.neural_pulse_terms(), spin=1, n_squares=28, specialize=True)
    b = Simulator(W.neural_pulse_terms(), spin=1, n_squares=28)
    ra, rb = a.evaluate(*args), b.evaluate(*args)
    ref = oracle.solve(a.problem(0.0495, 0.0505, 5e-8, 5e-7, psi0=args[0]), want_U=True)
    assert np.max(np.abs(ra.state.cpu().numpy() - ref["psi"])) <= TOL
    assert np.max(np.abs(ra.time_evolution.cpu().numpy() - ref["U"])) <= TOL
    print(f"[gpu] specialised vs interpreted simulator: "
          f"{float((ra.state - rb.state).abs().max()):.3e}", flush=True)
    a.sampler.close()


def test_spin_projection(dev, oracle):
    """<J> of the GPU states vs the oracle's <J> of the oracle's states, and
    the projection kernel alone on identical inputs."""
    import torch
    from paper_2204_05586_amd import Simulator, native
    sim = Simulator(W.neural_pulse_terms(), spin=1, rotating_frame=True, n_squares=28)
    res = sim.evaluate([0.6, 0.8j, 0], 0.0495, 0.0505, 5e-8, 5e-7)
    prob = sim.problem(0.0495, 0.0505, 5e-8, 5e-7, psi0=[0.6, 0.8j, 0])
    ref = oracle.solve(prob)
    J = res.spin.cpu().numpy()
    assert np.max(np.abs(J - oracle.spin_projection(ref["psi"]))) <= TOL
    for N in (2, 3):
        rng = np.random.default_rng(N)
        psi = rng.normal(size=(1001, N)) + 1j * rng.normal(size=(1001, N))
        got = native.spin_projection(torch.from_numpy(psi).cuda()).cpu().numpy()
        assert np.max(np.abs(got - oracle.spin_projection(psi))) < 1e-14


@pytest.mark.parametrize("method", [W.MIDPOINT, W.HEUN])
@pytest.mark.parametrize("spin_twice,frame", [(1, True), (2, True), (2, False)])
def test_euler_methods(dev, oracle, method, spin_twice, frame):
    rng = np.random.default_rng(50 + method + 10 * spin_twice + frame)
    prob = W.random_problem(rng, spin_twice, 777, 5, rotating_frame=frame).replace(method=method)
    _compare(_gpu(prob), oracle.solve(prob, want_U=True), name=f"method={method}")
