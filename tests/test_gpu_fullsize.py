"""Parity at the full sizes of the batched, serving and control workloads,
on outputs the oracle can compute one simulation at a time."""
import time

import numpy as np
import pytest

from paper_2204_05586_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def torch_dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _unitarity_defect(prob) -> float:
    """max_k ||U_k^H U_k - I||_F over one simulation's operators, integrated
    alone with its field program compiled in (bit for bit the batch's)."""
    import torch
    from paper_2204_05586_amd import native
    K, N = prob.n_samples, prob.dim
    s = native.Sampler.for_terms(prob.terms)
    U = torch.empty((K, N, N), dtype=torch.complex128, device="cuda")
    s.integrate(prob.replace(terms=[]), native.device_params(prob), U)
    eye = torch.eye(N, dtype=torch.complex128, device="cuda")
    G = torch.matmul(U.conj().transpose(1, 2).contiguous(), U) - eye
    out = float(torch.linalg.matrix_norm(G).max())
    s.close()
    return out


def test_batched_sensing_full(torch_dev, oracle):
    """All 4096 uneven spin-1 simulations (4.5e9 CF4 steps) in one batch,
    states only, the bench's configuration (one captured graph of the
    chained integrator with the shared field program compiled in, autotuned
    launch); the longest, the shortest and 64 seeded simulations against the
    oracle, every state's norm against its rounding bound, and every state
    against the separate-scan plan on the same batch."""
    import torch
    from paper_2204_05586_amd import autotune, native
    probs = W.batched_sensing(seed=2)
    opts = autotune.tune(probs, cache_path=None, reps=2, specialize=True)
    plan = native.BatchPlan(probs, specialize=True, chained=True, use_graph=True, **opts)
    assert plan.specialized
    bufs = plan.allocate(store_u=False)
    print(f"[gpu] full batched sensing {plan.info()} options {opts}", flush=True)
    plan.run(bufs)
    torch.cuda.synchronize()
    ks = np.array([p.n_samples for p in probs])
    rng = np.random.default_rng(2024)
    pick = sorted({int(ks.argmax()), int(ks.argmin()), *rng.choice(len(probs), 64, replace=False)})
    # every one of the 4.5e8 states keeps unit norm (a property at any size).
    # One interval changes |psi|^2 by at most ||U^H U - I||_2 <= eps (the
    # Frobenius defect, measured on the longest simulation's operators) plus
    # the rounding of applying it, <= 12 u (a length-6 real dot product per
    # component, twice for the square); the chained form multiplies up to 64
    # operators in a tree of depth 6 before applying them, which stays within
    # the same 12 u per interval.  So |(|psi_k|^2 - 1)| <= K_max (eps + 12 u).
    eps = _unitarity_defect(probs[int(ks.argmax())])
    bound = int(ks.max()) * (eps + 12 * 2.0 ** -53)
    psi = bufs["psi"]
    worst_norm = 0.0
    step = 3 << 26  # whole spin-1 states per chunk
    for a in range(0, psi.numel(), step):
        chunk = psi[a:a + step]
        sq = (chunk.real.square() + chunk.imag.square()).view(-1, 3).sum(dim=1)
        worst_norm = max(worst_norm, float((sq - 1.0).abs().max()))
    print(f"batch: max | |psi_k|^2 - 1 | over all states = {worst_norm:.3e}; operator defect "
          f"{eps:.3e}, bound K_max (eps + 12 u) = {bound:.3e}", flush=True)
    assert worst_norm <= bound
    for i in pick:
        ref = oracle.solve(probs[i])
        got = plan.split(bufs, i)
        d = max(np.max(np.abs(got["psi"].cpu().numpy() - ref["psi"])),
                np.max(np.abs(got["psi_final"].cpu().numpy() - ref["psi_final"])))
        print(f"sim {i} K={probs[i].n_samples}: max |d| = {d:.3e}", flush=True)
        assert d <= TOL, (i, d)
    plan.close()
    # the separate-scan plan (operators in the workspace, then the segmented
    # scan): the same operators, the product in another order
    sep = native.BatchPlan(probs, specialize=True, **opts)
    sbufs = sep.allocate(store_u=False)
    sep.run(sbufs)
    torch.cuda.synchronize()
    d_all = max(float((sbufs["psi"] - bufs["psi"]).abs().max()),
                float((sbufs["psi_final"] - bufs["psi_final"]).abs().max()))
    print(f"chained vs separate scan over all states: max |d| = {d_all:.3e}", flush=True)
    assert d_all <= TOL
    sep.close()


def test_plain_sensing_full_compiled_field(torch_dev, oracle):
    """The bench's plain leg at full size: 2e5 intervals x 10 CF4 steps with
    the field program compiled into the integrator, the library's default
    launch, then the scan; every state and operator against the oracle."""
    import torch
    from paper_2204_05586_amd import native
    prob = W.spin_one_sensing()
    s = native.Sampler.for_terms(prob.terms)
    K, N = prob.n_samples, prob.dim
    U = torch.empty((K, N, N), dtype=torch.complex128, device="cuda")
    psi = torch.empty((K, N), dtype=torch.complex128, device="cuda")
    fin = torch.empty((N,), dtype=torch.complex128, device="cuda")
    ws = native.alloc_workspace(native.propagate_workspace_size(prob.spin_twice, K))
    print(f"[gpu] plain sensing, compiled field, K={K}", flush=True)
    s.integrate(prob.replace(terms=[]), native.device_params(prob), U)
    native.propagate(prob.spin_twice, U, native.device_state(prob.psi0), psi, fin, ws)
    torch.cuda.synchronize()
    ref = oracle.solve(prob, want_U=True)
    d = max(np.max(np.abs(psi.cpu().numpy() - ref["psi"])),
            np.max(np.abs(fin.cpu().numpy() - ref["psi_final"])),
            np.max(np.abs(U.cpu().numpy() - ref["U"])))
    print(f"plain sensing, compiled field: max |d| = {d:.3e}", flush=True)
    assert d <= TOL
    # every interval operator unitary: max |U^H U - I| over all 2e5 of them
    uh = U.conj().transpose(-1, -2).contiguous()
    eye = torch.eye(N, dtype=torch.complex128, device="cuda")
    dev_u = float((torch.matmul(uh, U) - eye).abs().max())
    print(f"plain sensing: max |U^H U - I| = {dev_u:.3e}", flush=True)
    assert dev_u < 1e-12
    s.close()


def test_serving_stream_full(torch_dev, oracle):
    """A seeded 200-request Poisson stream at 1000 req/s (30 % spin-1/2,
    K log-uniform in [1e3, 1e6]) submitted on schedule: every result equals
    the same simulation run alone and every one is checked against the
    oracle; latencies are reported."""
    import torch
    from paper_2204_05586_amd import native
    stream = W.serving_stream(1000.0, n_requests=200, rate_index=4)
    srv = native.Server()
    base = srv.clock() + 0.05
    tickets = []
    for r in stream:
        delay = base + r.arrival - srv.clock()
        if delay > 0:
            time.sleep(delay)
        tickets.append(srv.submit(r.problem))
    lat, worst, worst_ref = [], 0.0, 0.0
    for j, (t, r) in enumerate(zip(tickets, stream)):
        info = srv.wait(t, 300.0)
        lat.append(info["t_done"] - (base + r.arrival))
        p = r.problem
        got = srv.fetch(t, p)
        K, N = p.n_samples, p.dim
        U = torch.empty((K, N, N), dtype=torch.complex128, device="cuda")
        psi = torch.empty((K, N), dtype=torch.complex128, device="cuda")
        fin = torch.empty((N,), dtype=torch.complex128, device="cuda")
        ws = native.alloc_workspace(native.propagate_workspace_size(p.spin_twice, K))
        native.integrate(p, native.device_params(p), U, launch=(srv.request_slices(p), 256))
        native.propagate(p.spin_twice, U, native.device_state(p.psi0), psi, fin, ws)
        torch.cuda.synchronize()
        d = float((got["psi"] - psi).abs().max())
        worst = max(worst, d)
        assert d == 0.0, (j, d)
        ref = oracle.solve(p)
        d_ref = max(np.max(np.abs(got["psi"].cpu().numpy() - ref["psi"])),
                    np.max(np.abs(got["psi_final"].cpu().numpy() - ref["psi_final"])))
        worst_ref = max(worst_ref, d_ref)
        assert d_ref <= TOL, (j, d_ref)
        if j % 20 == 19:
            print(f"served {j + 1}: max |d| vs oracle so far {worst_ref:.3e}", flush=True)
        srv.release(t)
        del U, psi, ws
    lat = np.array(lat) * 1e3
    print(f"served 200: max |d| vs alone {worst:.3e}, vs the oracle {worst_ref:.3e}; latency "
          f"p50 {np.percentile(lat, 50):.3f} ms p99 {np.percentile(lat, 99):.3f} ms", flush=True)
    srv.close()


def test_control_gradients_full(torch_dev, oracle):
    """All 1024 control instances (512 gradients each), the shared field
    compiled into the forward pass as the bench runs them: 64 seeded
    instances and those of least and largest loss against the oracle's
    adjoint (1e-9 of the largest entry); the 8 instances with stored
    extended-precision central differences against them per component
    (1e-6 relative)."""
    import torch
    from paper_2204_05586_amd import native
    from tests.test_oracle_adjoint import control_fd_cases, per_component_ok
    probs, fd_cases = control_fd_cases()
    plan = native.AdjointPlan(probs, 1, specialize=True)
    assert plan.specialized
    bufs = plan.allocate()
    print(f"[gpu] full control gradients n={len(probs)}", flush=True)
    plan.run(bufs)
    torch.cuda.synchronize()
    loss = bufs["loss"].cpu().numpy()
    rng = np.random.default_rng(4096)
    pick = sorted({int(loss.argmin()), int(loss.argmax()),
                   *(int(i) for i in rng.choice(len(probs), 64, replace=False))})
    assert len(pick) >= 64
    worst = 0.0
    for i in pick:
        l_ref, g_ref = oracle.adjoint_population(probs[i], 1)
        g = plan.grad_of(bufs, i).cpu().numpy()
        r = float(np.max(np.abs(g - g_ref)) / np.max(np.abs(g_ref)))
        worst = max(worst, r)
        assert abs(loss[i] - l_ref) <= 1e-11 and r <= 1e-9, (i, loss[i], l_ref, r)
    print(f"{len(pick)} instances (loss {loss.min():.4f} .. {loss.max():.4f}) vs the oracle "
          f"adjoint: max rel grad err {worst:.2e}", flush=True)
    worst = 0.0
    for (label, i), (params, slots, fd) in fd_cases.items():
        if label != "drawn":
            continue
        ok, w = per_component_ok(plan.grad_of(bufs, i).cpu().numpy()[slots], fd)
        worst = max(worst, w)
        assert ok, (i, w)
    print(f"8 instances x 32 controls vs extended-precision differences: worst / bound "
          f"{worst:.2e}", flush=True)
    # every instance: the gradient along a seeded direction v against the
    # central difference of the GPU's own losses at params +- h v (amplitude
    # steps of ~0.1 Hz, phase steps of ~1e-4 rad).  On the oracle the
    # difference's truncation falls as h^2 (3.5e-7 relative at h = 1, 3.0e-9
    # at h = 0.1) down to its rounding floor near 1e-9 at h = 0.03.
    n_inst, per = len(probs), 512
    grad = bufs["grad"][:n_inst * per].clone()
    p0 = bufs["params"].clone()
    rng = np.random.default_rng(77)
    v = rng.normal(size=(n_inst, per))
    v[:, per // 2:] *= 1e-3
    vt = torch.from_numpy(v.ravel()).cuda()
    ad = (grad * vt).view(n_inst, per).sum(dim=1)
    h = 0.1
    losses = []
    for sgn in (1.0, -1.0):
        bufs["params"].copy_(p0 + sgn * h * vt)
        plan.run(bufs)
        torch.cuda.synchronize()
        losses.append(bufs["loss"].clone())
    fd = (losses[0] - losses[1]) / (2 * h)
    rel = float((fd - ad).abs().max() / ad.abs().max())
    print(f"all {n_inst} instances: directional gradient vs central difference, max rel {rel:.2e}",
          flush=True)
    assert rel <= 1e-6
    plan.close()


def test_control_gradients_zero_amplitudes_full(torch_dev, oracle):
    """A full-size control instance with every fourth segment's amplitude 0
    (no transverse field there): GPU gradients against the oracle adjoint
    (1e-9) and, per component, against the stored extended-precision
    central differences at the zeroed amplitudes and phases (1e-6)."""
    import torch
    from paper_2204_05586_amd import native
    from tests.test_oracle_adjoint import control_fd_cases, per_component_ok
    probs, fd_cases = control_fd_cases()
    (params, slots, fd), = [v for (label, _), v in fd_cases.items() if label == "zeroed"]
    prob = probs[0].replace(params=params)
    plan = native.AdjointPlan([prob], 1, specialize=True)
    bufs = plan.allocate()
    print("[gpu] control instance 0 with zeroed amplitudes", flush=True)
    plan.run(bufs)
    torch.cuda.synchronize()
    g = plan.grad_of(bufs, 0).cpu().numpy()
    assert np.all(np.isfinite(g))
    l_ref, g_ref = oracle.adjoint_population(prob, 1)
    r = float(np.max(np.abs(g - g_ref)) / np.max(np.abs(g_ref)))
    ok, w = per_component_ok(g[slots], fd)
    print(f"zeroed amplitudes: rel vs oracle {r:.2e}, worst / bound vs differences {w:.2e}",
          flush=True)
    assert abs(float(bufs["loss"][0]) - l_ref) <= 1e-11 and r <= 1e-9
    assert ok
    plan.close()
