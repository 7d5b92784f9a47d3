"""The single-sequence scan in one launch (mss_propagate with one or two
levels above the operators): bitwise the result of the batch plan's
level-by-level scan on the same operators, within rounding of the oracle's
sequential product, correct on repeated calls through one workspace and in
replays of a captured graph, and its bounded waits never run out.  Shapes
cover both sides of every switch: one level (K <= 65536), two levels,
the largest grid it takes for spin-1 (262144) and the first it leaves to
separate launches, and three levels."""
import numpy as np
import pytest

from paper_2204_05586_amd import workloads as W

pytestmark = pytest.mark.gpu

SHAPES = [(2, 257), (3, 3000), (2, 10_000), (3, 65_536), (3, 65_537), (2, 200_000),
          (3, 200_000), (3, 262_144), (3, 262_145), (2, 458_752), (3, 1 << 20),
          (2, (1 << 20) + 1)]


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


M64 = (1 << 64) - 1


def call_tag(c):
    """The SplitMix64 finalizer the kernel tags a call with."""
    c &= M64
    c ^= c >> 30
    c = (c * 0xBF58476D1CE4E5B9) & M64
    c ^= c >> 27
    c = (c * 0x94D049BB133111EB) & M64
    c ^= c >> 31
    return c


def _header(ws):
    """(epoch, whether the call numbered epoch ran out of a wait) of a
    one-launch scan workspace."""
    import torch
    h = ws[:256].view(dtype=torch.int64).cpu().numpy().astype(np.uint64)
    epoch = int(h[0])
    return epoch, int(h[2]) == call_tag(epoch)


@pytest.mark.parametrize("N,K", SHAPES, ids=[f"N{n}-K{k}" for n, k in SHAPES])
def test_one_pass_equals_level_scan_and_oracle(dev, oracle, N, K):
    torch = dev
    from paper_2204_05586_amd import native
    print(f"[gpu] one-pass scan N={N} K={K}", flush=True)
    U = _unitaries(torch, N, K, seed=7 * K + N)
    rng = np.random.default_rng(K + N)
    psi0 = W.random_state(N, rng)
    ws = native.alloc_workspace(native.propagate_workspace_size(N - 1, K))
    # the workspace starts out holding operator bits (near-identical doubles)
    junk = U.view(-1).view(torch.uint8)
    n = min(ws.numel(), junk.numel())
    ws[:n].copy_(junk[:n])
    e_before = int(ws[:8].view(torch.int64).item()) & M64
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
    epoch, failed = _header(ws)
    one_pass = epoch == (e_before + 1) & M64
    print(f"N={N} K={K}: one launch {one_pass}", flush=True)
    if 256 < K <= 262_144:
        assert one_pass and not failed


@pytest.mark.parametrize("N,K", [(2, 10_000), (3, 200_000)])
def test_one_pass_repeated_calls_and_graph_replays(dev, N, K):
    """Calls through one workspace each see their own call number: eager
    calls, then a captured graph replayed three times with eager work in
    between, all bitwise equal; the workspace's call counter advances by one
    per call or replay and no wait runs out."""
    torch = dev
    from paper_2204_05586_amd import native
    U = _unitaries(torch, N, K, seed=N * 31 + K)
    U2 = _unitaries(torch, N, K, seed=N * 37 + K)
    psi0 = native.device_state(W.random_state(N, np.random.default_rng(K)))
    ws = native.alloc_workspace(native.propagate_workspace_size(N - 1, K))
    ref = torch.empty((K, N), dtype=torch.complex128, device="cuda")
    other = torch.empty_like(ref)
    print(f"[gpu] one-pass repeated N={N} K={K}", flush=True)
    native.propagate(N - 1, U, psi0, ref, None, ws)
    torch.cuda.synchronize()
    e0, failed = _header(ws)
    assert not failed
    for i in range(3):
        native.propagate(N - 1, U2 if i % 2 else U, psi0, other, None, ws)
    torch.cuda.synchronize()
    e1, failed = _header(ws)
    assert e1 == e0 + 3 and not failed
    native.propagate(N - 1, U, psi0, other, None, ws)
    torch.cuda.synchronize()
    assert torch.equal(other, ref)
    out = torch.empty_like(ref)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    print(f"[gpu] one-pass graph capture N={N} K={K}", flush=True)
    with torch.cuda.graph(g, stream=s):
        native.propagate(N - 1, U, psi0, out, None, ws)
    torch.cuda.synchronize()
    e2, _ = _header(ws)
    for r in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), r
        native.propagate(N - 1, U2, psi0, other, None, ws)  # eager work between replays
        torch.cuda.synchronize()
    e3, failed = _header(ws)
    assert e3 == e2 + 6 and not failed
