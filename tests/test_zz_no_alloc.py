"""mss_propagate_noalloc (the ordered product with the library's static
scan scratch, no allocation) against mss_propagate with an allocated
workspace: calls in a row through the same scratch, each smaller than the
one before, across the scan's shapes and both
spins, plus the size limit.""" 
import numpy as np
import pytest

from paper_2204_05586_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _operators(spin_twice, K, seed):
    import torch
    from paper_2204_05586_amd import native
    rng = np.random.default_rng(seed)
    p = W.random_problem(rng, spin_twice, K, 1, n_squares=12)
    N = spin_twice + 1
    U = torch.empty((K, N, N), dtype=torch.complex128, device="cuda")
    native.integrate(p, native.device_params(p), U)
    return U, native.device_state(p.psi0)


def test_noalloc_matches_propagate(torch_dev):
    import torch
    from paper_2204_05586_amd import native
    # 5e6 spin-1: three levels; 300,001: two levels, the upper two in one
    # workgroup; then spin-1/2 with one level, and single tiles (no scratch)
    cases = [(2, 5_000_001), (2, 300_001), (1, 70_001), (1, 1000), (2, 200)]
    for i, (spin_twice, K) in enumerate(cases):
        print(f"[gpu] noalloc case spin_twice={spin_twice} K={K}", flush=True)
        U, psi0 = _operators(spin_twice, K, seed=100 + i)
        N = spin_twice + 1
        psi_a = torch.empty((K, N), dtype=torch.complex128, device="cuda")
        fin_a = torch.empty((N,), dtype=torch.complex128, device="cuda")
        ws = native.alloc_workspace(native.propagate_workspace_size(spin_twice, K))
        native.propagate(spin_twice, U, psi0, psi_a, fin_a, ws)
        psi_b = torch.full((K, N), float("nan"), dtype=torch.complex128, device="cuda")
        fin_b = torch.full((N,), float("nan"), dtype=torch.complex128, device="cuda")
        native.propagate_noalloc(spin_twice, U, psi0, psi_b, fin_b)
        torch.cuda.synchronize()
        d = max(float((psi_b - psi_a).abs().max()), float((fin_b - fin_a).abs().max()))
        print(f"[gpu] noalloc vs propagate: max |d| = {d:.3e}", flush=True)
        assert d <= 1e-10
        assert bool((psi_b == psi_a).all()) and bool((fin_b == fin_a).all())
        del U, psi_a, psi_b, ws


def test_noalloc_rejects_oversize(torch_dev):
    """Beyond the scratch: an error before any launch (the pointers are not
    read, so small buffers stand in)."""
    import torch
    from paper_2204_05586_amd import native
    U = torch.zeros((1, 3, 3), dtype=torch.complex128, device="cuda")
    psi = torch.zeros((1, 3), dtype=torch.complex128, device="cuda")
    psi0 = torch.zeros((3,), dtype=torch.complex128, device="cuda")
    for spin_twice, kmax in ((2, 11_141_120), (1, 22_280_192)):
        with pytest.raises(native.MssError, match="scan scratch"):
            native.propagate_noalloc(spin_twice, U, psi0, psi, n_samples=kmax + 1)
        assert native.propagate_workspace_size(spin_twice, kmax) <= 8 << 20
        assert native.propagate_workspace_size(spin_twice, kmax + 1) > 8 << 20
    torch.cuda.synchronize()
