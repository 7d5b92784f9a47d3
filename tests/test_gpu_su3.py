"""GPU parity of spin-1 in the full su(3) basis (terms on U_1, U_2, V_1, V_2)
against the oracle: single simulations (CF4 and the Euler-family methods,
frame on and off, several tau and lane-slice shapes), batches and the
serving loop bit for bit against the single-simulation path, and the
entry points that refuse the basis."""
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


def _su3_problem(seed, K=700, L=6, tau=28, frame=True, method=W.CF4, slots=False):
    """Bias on z, a quadrupole shift, and sinusoidal drives on all of x, y,
    u1, u2, v1, v2 near the Delta m = 1 and 2 resonances, one of them
    windowed and one a piecewise-constant control."""
    rng = np.random.default_rng(seed)
    F0 = rng.uniform(1.0e4, 2.0e4)
    T = W.Term
    terms = [T(W.CONST, W.Z, a=F0), T(W.CONST, W.Q, a=rng.uniform(-300, 300))]
    for c, h in ((W.X, 1), (W.Y, 1), (W.U1, 2), (W.U2, 2), (W.V1, 1), (W.V2, 1)):
        terms.append(T(W.COS if rng.random() < 0.5 else W.SIN, c, a=rng.uniform(50, 600),
                       f=h * F0 * rng.uniform(0.97, 1.03), phi=rng.uniform(0, 6)))
    Dt = rng.uniform(0.5, 2.0) / F0
    terms.append(T(W.SIN, W.U1, a=200.0, f=3 * F0, t_on=0.3 * K * Dt, t_off=0.6 * K * Dt))
    params = np.zeros(0)
    if slots:
        params = rng.uniform(-400, 400, 6)
        terms.append(T(W.PWC, W.V2, n_seg=6, seg_a_slot=0, seg_t0=0.0, seg_len=K * Dt / 6))
    psi0 = W.random_state(3, rng)
    return W.Problem(2, terms, rng.uniform(0, 1e-4), Dt, K, L, tau, frame, params=params,
                     psi0=psi0, name=f"su3[{seed}]", method=method)


def _compare(g, ref, name):
    d = max(np.max(np.abs(g["psi"].cpu().numpy() - ref["psi"])),
            np.max(np.abs(g["psi_final"].cpu().numpy() - ref["psi_final"])),
            np.max(np.abs(g["U"].cpu().numpy() - ref["U"])))
    print(f"[gpu] {name}: max |d| = {d:.3e}", flush=True)
    assert d <= TOL, (name, d)


CASES = [dict(seed=1), dict(seed=2, frame=False), dict(seed=3, tau=0, K=200),
         dict(seed=4, tau=5), dict(seed=5, method=W.MIDPOINT), dict(seed=6, method=W.HEUN),
         dict(seed=7, K=1, L=3), dict(seed=8, K=3001, L=4, slots=True),
         dict(seed=9, frame=False, method=W.HEUN, slots=True)]


@pytest.mark.parametrize("case", CASES, ids=[str(c) for c in CASES])
def test_su3_matches_oracle(dev, oracle, case):
    from paper_2204_05586_amd import native
    prob = _su3_problem(**case)
    print(f"[gpu] su3 case {case}", flush=True)
    _compare(native.solve(prob, store_u=True), oracle.solve(prob, want_U=True), str(case))


@pytest.mark.parametrize("slices", [1, 2, 4])
def test_su3_lane_slices(dev, oracle, slices):
    import torch
    from paper_2204_05586_amd import native
    prob = _su3_problem(11, K=500, L=8)
    U = torch.empty((prob.n_samples, 3, 3), dtype=torch.complex128, device="cuda")
    print(f"[gpu] su3 slices={slices}", flush=True)
    native.integrate(prob, native.device_params(prob), U, launch=(slices, 256))
    torch.cuda.synchronize()
    assert np.max(np.abs(U.cpu().numpy() - oracle.operators(prob))) <= TOL


def test_su3_resonant_closed_form(dev, oracle):
    """The resonant quadrupole drive of the oracle pins, on the GPU: frame
    on, exact per interval, against exp(-i w0 t J_z) exp(-i H0 t) psi0."""
    import math
    scipy_linalg = pytest.importorskip("scipy.linalg")
    from paper_2204_05586_amd import native
    F0, A, B, fq = 2.0e4, 700.0, 400.0, 90.0
    T = W.Term
    terms = [T(W.CONST, W.Z, a=F0), T(W.CONST, W.Q, a=fq),
             T(W.COS, W.V1, a=A, f=F0), T(W.SIN, W.V2, a=A, f=F0),
             T(W.COS, W.U1, a=B, f=2 * F0), T(W.SIN, W.U2, a=B, f=2 * F0)]
    psi0 = np.array([0.6, 0.48 + 0.36j, 0.52], dtype=complex)
    psi0 /= np.linalg.norm(psi0)
    prob = W.Problem(2, terms, 0.0, 2e-6, 400, 40, 28, True, psi0=psi0)
    g = native.solve(prob)["psi"].cpu().numpy()
    ops = [oracle.basis_operator(j) for j in range(8)]
    H0 = 2 * math.pi * (A * ops[6] + B * ops[4] + fq * ops[3])
    for k in (0, 199, 399):
        t = k * prob.dt_out
        ref = scipy_linalg.expm(-1j * 2 * math.pi * F0 * t * ops[2]) @ \
            scipy_linalg.expm(-1j * H0 * t) @ psi0
        assert np.max(np.abs(g[k] - ref)) < 2e-12


def _alone(p, slices=1):
    """The single-simulation path with slices lanes per interval (one: the
    lane mapping of the batch plan below)."""
    import torch
    from paper_2204_05586_amd import native
    K, N = p.n_samples, p.dim
    out = {"U": torch.empty((K, N, N), dtype=torch.complex128, device="cuda"),
           "psi": torch.empty((K, N), dtype=torch.complex128, device="cuda"),
           "psi_final": torch.empty((N,), dtype=torch.complex128, device="cuda")}
    ws = native.alloc_workspace(native.propagate_workspace_size(p.spin_twice, K))
    native.integrate(p, native.device_params(p), out["U"], launch=(slices, 256))
    native.propagate(p.spin_twice, out["U"], native.device_state(p.psi0), out["psi"],
                     out["psi_final"], ws)
    torch.cuda.synchronize()
    return out


def test_su3_batch_and_server_equal_alone(dev, oracle):
    """Full-basis simulations mixed with ordinary spin-1 and spin-1/2 ones in
    one batch plan and one server: each equals its single-simulation
    result bit for bit."""
    import torch
    from paper_2204_05586_amd import native
    rng = np.random.default_rng(40)
    probs = [_su3_problem(20 + i, K=int(rng.integers(1, 900)), L=4) for i in range(5)]
    probs += [W.random_problem(rng, 2, 333, 4), W.random_problem(rng, 1, 257, 4)]
    plan = native.BatchPlan(probs, slices_spin_one=1, slices_spin_half=1)
    bufs = plan.allocate(store_u=True)
    print(f"[gpu] su3 batch info={plan.info()}", flush=True)
    plan.run(bufs)
    torch.cuda.synchronize()
    srv = native.Server(iteration_steps=2e5)
    tickets = [srv.submit(p) for p in probs]
    for i, p in enumerate(probs):
        got = plan.split(bufs, i)
        alone = _alone(p)
        alone_srv = _alone(p, srv.request_slices(p))
        info = srv.wait(tickets[i], 60.0)
        assert info["state"] == native.MSS_REQ_DONE
        served = srv.fetch(tickets[i], p, want_u=True)
        torch.cuda.synchronize()
        for k in ("psi", "psi_final", "U"):
            assert float((got[k] - alone[k]).abs().max()) == 0.0, (i, k)
            assert float((served[k] - alone_srv[k]).abs().max()) == 0.0, (i, k)
        if i < 5:
            ref = oracle.solve(p, want_U=True)
            assert np.max(np.abs(got["psi"].cpu().numpy() - ref["psi"])) <= TOL
        srv.release(tickets[i])
    srv.close()
    plan.close()


def test_su3_refused_by_adjoint_and_specialisation(dev):
    from paper_2204_05586_amd import native
    prob = _su3_problem(30, K=20, L=2, slots=True)
    with pytest.raises(native.MssError, match="su\\(3\\)") as e:
        native.AdjointPlan([prob], 0)
    assert e.value.status == native.MSS_E_UNSUPPORTED
    plan = native.BatchPlan([prob], specialize=True)
    assert not plan.specialized
    plan.close()
