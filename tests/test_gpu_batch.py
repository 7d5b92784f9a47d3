"""GPU parity of the batched path (persistent integrator + segmented scan)
against the oracle, batch-vs-alone invariance and graph replays."""
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


def _mixed_batch(seed=21):
    rng = np.random.default_rng(seed)
    probs = []
    for K in [1, 7, 255, 256, 257, 1000, 3001, 70000]:
        for spin_twice in (1, 2):
            frame = bool(rng.integers(0, 2))
            L = int(rng.integers(1, 9))
            probs.append(W.random_problem(rng, spin_twice, K, L, n_squares=int(rng.integers(8, 29)),
                                          rotating_frame=frame))
    probs += W.batched_sensing(seed=2, n_sims=6, dur_lo=0.0499, dur_hi=0.0515)
    probs += W.control_batch(n_inst=3, n_samples=300, n_fine=20)
    rng.shuffle(probs)
    return probs


def _run(plan, store_u=True, stream=None):
    import torch
    bufs = plan.allocate(store_u=store_u)
    print(f"[gpu] batch n={plan.n} info={plan.info()}", flush=True)
    plan.run(bufs, stream=stream)
    torch.cuda.synchronize()
    return bufs


def test_batch_matches_oracle(torch_dev, oracle):
    from paper_2204_05586_amd import native
    probs = _mixed_batch()
    plan = native.BatchPlan(probs)
    bufs = _run(plan)
    worst = 0.0
    for i, p in enumerate(probs):
        ref = oracle.solve(p, want_U=True)
        got = {k: v.cpu().numpy() for k, v in plan.split(bufs, i).items()}
        d = max(np.max(np.abs(got["psi"] - ref["psi"])),
                np.max(np.abs(got["psi_final"] - ref["psi_final"])),
                np.max(np.abs(got["U"] - ref["U"])))
        worst = max(worst, d)
        assert d <= TOL, (i, p.name, p.n_samples, d)
    print(f"batch vs oracle: max |d| = {worst:.3e}", flush=True)
    plan.close()


def test_batch_equals_alone(torch_dev):
    """Each simulation's result is the same alone (single-simulation path,
    same lane-slice count) and inside the batch."""
    from paper_2204_05586_amd import native
    probs = _mixed_batch(seed=5)
    plan = native.BatchPlan(probs, slices_spin_half=1, slices_spin_one=1)
    bufs = _run(plan)
    import torch
    worst, bitwise = 0.0, 0
    for i, p in enumerate(probs):
        K, N = p.n_samples, p.dim
        U = torch.empty((K, N, N), dtype=torch.complex128, device="cuda")
        psi = torch.empty((K, N), dtype=torch.complex128, device="cuda")
        fin = torch.empty((N,), dtype=torch.complex128, device="cuda")
        ws = native.alloc_workspace(native.propagate_workspace_size(p.spin_twice, K))
        native.integrate(p, native.device_params(p), U, launch=(1, 256))
        native.propagate(p.spin_twice, U, native.device_state(p.psi0), psi, fin, ws)
        torch.cuda.synchronize()
        got = plan.split(bufs, i)
        d = max(float((got["psi"] - psi).abs().max()), float((got["U"] - U).abs().max()),
                float((got["psi_final"] - fin).abs().max()))
        worst = max(worst, d)
        bitwise += d == 0.0
        assert d <= 1e-13, (i, d)
    print(f"batch vs alone: max |d| = {worst:.3e}, bitwise equal {bitwise}/{len(probs)}",
          flush=True)
    plan.close()


def test_batch_states_only_and_slices(torch_dev, oracle):
    """U kept in the workspace (states only) with forced lane-slicing."""
    from paper_2204_05586_amd import native
    probs = W.batched_sensing(seed=7, n_sims=12, dur_lo=0.0005, dur_hi=0.004)
    for S in (1, 2, 8):
        plan = native.BatchPlan(probs, slices_spin_one=S)
        bufs = _run(plan, store_u=False)
        for i in (0, 5, 11):
            ref = oracle.solve(probs[i])
            got = plan.split(bufs, i)
            d = np.max(np.abs(got["psi"].cpu().numpy() - ref["psi"]))
            assert d <= TOL, (S, i, d)
        plan.close()


def test_batch_graph_replays(torch_dev):
    """The captured graph replayed several times, with eager work and
    synchronisations in between, reproduces the eager result each time."""
    import torch
    from paper_2204_05586_amd import native
    probs = _mixed_batch(seed=9)[:12]
    eager = native.BatchPlan(probs)
    be = _run(eager)
    graph = native.BatchPlan(probs, use_graph=True)
    bufs = graph.allocate(store_u=True)
    s = torch.cuda.Stream()
    for rep in range(3):
        bufs["psi"].fill_(float("nan"))
        with torch.cuda.stream(s):
            graph.run(bufs, stream=s)
        s.synchronize()
        x = torch.randn(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        d = float((bufs["psi"] - be["psi"]).abs().max())
        print(f"[gpu] graph replay {rep}: max |d| = {d:.3e}", flush=True)
        assert d == 0.0, (rep, d)
    eager.close()
    graph.close()


def test_batch_rejects_bad_members(torch_dev):
    from paper_2204_05586_amd import native
    probs = W.batched_sensing(n_sims=3)
    probs[1] = probs[1].replace(n_samples=0)
    with pytest.raises(native.MssError, match="simulation 1"):
        native.BatchPlan(probs)


def test_autotuned_plan_matches_oracle(torch_dev, oracle, tmp_path):
    """The autotuner picks valid options (cached on disk, reused on the
    second call) and the tuned plan still matches the oracle."""
    from paper_2204_05586_amd import autotune, native
    probs = W.batched_sensing(seed=8, n_sims=40, dur_lo=0.001, dur_hi=0.004)
    cache = str(tmp_path / "tune.json")
    opts = autotune.tune(probs, cache_path=cache, reps=2, target_fine_steps=2e7, verbose=True)
    assert opts["scan_per_lane"] in (2, 4, 8) and opts["waves_per_simd"] in (1, 2, 4)
    assert autotune.tune(probs, cache_path=cache) == opts
    plan = native.BatchPlan(probs, **opts)
    bufs = _run(plan, store_u=False)
    for i in (0, 17, 39):
        ref = oracle.solve(probs[i])
        got = plan.split(bufs, i)
        assert np.max(np.abs(got["psi"].cpu().numpy() - ref["psi"])) <= TOL
    plan.close()
