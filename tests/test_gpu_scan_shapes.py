"""The single-sequence scan (mss_propagate) across its shapes: bitwise the
result of the batch plan's segmented scan on the same operators, within
rounding of the oracle's sequential product, and bitwise repeatable through
one workspace and in replays of a captured graph.  Shapes cover one level
above the operators (K <= 65536), two levels with the upper two in one
workgroup (at most 8 level-1 tiles) and beyond it, and three levels."""
import numpy as np
import pytest

from paper_2204_05586_amd import workloads as W

pytestmark = pytest.mark.gpu

SHAPES = [(2, 257), (3, 3000), (2, 10_000), (3, 65_536), (3, 65_537), (2, 200_000),
          (3, 200_000), (3, 262_144), (3, 262_145), (2, 458_752), (3, 524_288),
          (2, 524_289), (3, 1 << 20), (2, (1 << 20) + 1)]


@pytest.fixture(scope="module")
def dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_05586_amd import native
    native.lib()
    return torch


def _unitaries(torch, N, K, seed):
    """K random unitaries built on the device: a fixed unitary times random
    diagonal phases."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    rng = np.random.default_rng(seed)
    V, _ = np.linalg.qr(rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N)))
    Vd = torch.from_numpy(V).cuda()
    ang = torch.rand((K, N), generator=g, device="cuda", dtype=torch.float64) * 6.283185307179586
    D = torch.polar(torch.ones_like(ang), ang)
    return (D[:, :, None] * Vd[None]).contiguous()


@pytest.mark.parametrize("N,K", SHAPES, ids=[f"N{n}-K{k}" for n, k in SHAPES])
def test_scan_equals_batch_scan_and_oracle(dev, oracle, N, K):
    torch = dev
    from paper_2204_05586_amd import native
    print(f"[gpu] scan N={N} K={K}", flush=True)
    U = _unitaries(torch, N, K, seed=7 * K + N)
    rng = np.random.default_rng(K + N)
    psi0 = W.random_state(N, rng)
    ws = native.alloc_workspace(native.propagate_workspace_size(N - 1, K))
    # the workspace starts out holding operator bits
    junk = U.view(-1).view(torch.uint8)
    n = min(ws.numel(), junk.numel())
    ws[:n].copy_(junk[:n])
    psi = torch.empty((K, N), dtype=torch.complex128, device="cuda")
    fin = torch.empty((N,), dtype=torch.complex128, device="cuda")
    native.propagate(N - 1, U, native.device_state(psi0), psi, fin, ws)
    # the batch plan's level-by-level scan on the same operators
    prob = W.Problem(N - 1, [], 0.0, 1e-6, K, 1, 0, False, psi0=psi0)
    plan = native.BatchPlan([prob])
    bufs = plan.allocate(store_u=True)
    bufs["U"].copy_(U.view(-1))
    plan.propagate(bufs)
    torch.cuda.synchronize()
    assert torch.equal(psi.view(-1), bufs["psi"]), float((psi.view(-1) - bufs["psi"]).abs().max())
    assert torch.equal(fin, bufs["psi_final"])
    plan.close()
    ref_psi, ref_fin = oracle.states(U.cpu().numpy(), psi0)
    d = max(np.max(np.abs(psi.cpu().numpy() - ref_psi)), np.max(np.abs(fin.cpu().numpy() - ref_fin)))
    print(f"N={N} K={K}: max |d| vs the oracle's sequential product {d:.2e}", flush=True)
    assert d < 1e-11


@pytest.mark.parametrize("N,K", [(2, 10_000), (3, 200_000)])
def test_scan_repeated_calls_and_graph_replays(dev, N, K):
    """Calls through one workspace, then a captured graph replayed three
    times with eager work (other operators through the same workspace) in
    between: all bitwise equal."""
    torch = dev
    from paper_2204_05586_amd import native
    U = _unitaries(torch, N, K, seed=N * 31 + K)
    U2 = _unitaries(torch, N, K, seed=N * 37 + K)
    psi0 = native.device_state(W.random_state(N, np.random.default_rng(K)))
    ws = native.alloc_workspace(native.propagate_workspace_size(N - 1, K))
    ref = torch.empty((K, N), dtype=torch.complex128, device="cuda")
    other = torch.empty_like(ref)
    print(f"[gpu] scan repeated N={N} K={K}", flush=True)
    native.propagate(N - 1, U, psi0, ref, None, ws)
    for i in range(3):
        native.propagate(N - 1, U2 if i % 2 else U, psi0, other, None, ws)
    native.propagate(N - 1, U, psi0, other, None, ws)
    torch.cuda.synchronize()
    assert torch.equal(other, ref)
    out = torch.empty_like(ref)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    print(f"[gpu] scan graph capture N={N} K={K}", flush=True)
    with torch.cuda.graph(g, stream=s):
        native.propagate(N - 1, U, psi0, out, None, ws)
    torch.cuda.synchronize()
    for r in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), r
        native.propagate(N - 1, U2, psi0, other, None, ws)  # eager work between replays
        torch.cuda.synchronize()
