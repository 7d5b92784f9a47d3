"""GPU tests of the continuous-batching server: results in the mix equal
results alone (and the oracle), admission under an HBM budget with
back-pressure, and overlap of requests within rounds."""
import threading
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


def _alone(p, slices=1):
    """The single-simulation path with the server's lane mapping (slices
    lanes per interval)."""
    import torch
    from paper_2204_05586_amd import native
    K, N = p.n_samples, p.dim
    U = torch.empty((K, N, N), dtype=torch.complex128, device="cuda")
    psi = torch.empty((K, N), dtype=torch.complex128, device="cuda")
    fin = torch.empty((N,), dtype=torch.complex128, device="cuda")
    ws = native.alloc_workspace(native.propagate_workspace_size(p.spin_twice, K))
    native.integrate(p, native.device_params(p), U, launch=(slices, 256))
    native.propagate(p.spin_twice, U, native.device_state(p.psi0), psi, fin, ws)
    torch.cuda.synchronize()
    return psi, fin, U


def _mix(n, seed, k_hi=2e4):
    reqs = W.serving_stream(rate=1000.0, n_requests=n, seed=seed, k_lo=1e2, k_hi=k_hi)
    return [r.problem for r in reqs]


def test_server_results_equal_alone_and_oracle(torch_dev, oracle):
    """Requests split over several rounds (small round budget) give exactly
    the operators and states of the same simulation run alone with the lane
    slicing the server chose for it (several requests here are short enough
    to get more than one lane per interval)."""
    from paper_2204_05586_amd import native
    probs = _mix(40, seed=31)
    srv = native.Server(iteration_steps=2e5)
    print(f"[gpu] server mix of {len(probs)}", flush=True)
    tickets = [srv.submit(p) for p in probs]
    worst, bitwise, n_sliced = 0.0, 0, 0
    for i, (t, p) in enumerate(zip(tickets, probs)):
        info = srv.wait(t, 120.0)
        assert info["state"] == native.MSS_REQ_DONE
        got = srv.fetch(t, p, want_u=True)
        import torch
        torch.cuda.synchronize()
        sl = srv.request_slices(p)
        n_sliced += sl > 1
        psi, fin, U = _alone(p, sl)
        d = max(float((got["psi"] - psi).abs().max()), float((got["U"] - U).abs().max()),
                float((got["psi_final"] - fin).abs().max()))
        worst = max(worst, d)
        bitwise += d == 0.0
        assert d == 0.0, (i, sl, d)
        if i % 8 == 0:
            ref = oracle.solve(p)
            assert np.max(np.abs(got["psi"].cpu().numpy() - ref["psi"])) <= TOL
            assert np.max(np.abs(got["psi_final"].cpu().numpy() - ref["psi_final"])) <= TOL
        srv.release(t)
    st = srv.stats()
    print(f"served vs alone: max |d| = {worst:.3e}, bitwise {bitwise}/{len(probs)}, "
          f"{n_sliced} with more than one lane per interval, stats {st}", flush=True)
    assert st["rounds"] > 1 and st["completed"] == len(probs) and n_sliced > 0
    srv.close()


def test_server_back_pressure(torch_dev):
    """A budget that holds only a few requests: the rest wait in the queue
    and are admitted as finished requests are released."""
    from paper_2204_05586_amd import native
    probs = [W.spin_one_sensing(n_samples=20000, t_start=0.001 * i) for i in range(10)]
    per = 20000 * (9 + 3) * 16
    srv = native.Server(hbm_budget=int(3.5 * per) + (1 << 20))
    tickets = [srv.submit(p) for p in probs]
    seen_queued = srv.stats()["queued"] > 0
    for t in tickets:
        srv.wait(t, 120.0)
        st = srv.stats()
        seen_queued = seen_queued or st["queued"] > 0
        assert st["bytes_peak"] <= st["budget"]
        srv.release(t)
    st = srv.stats()
    print(f"[gpu] back-pressure stats {st}", flush=True)
    assert seen_queued and st["completed"] == len(probs) and st["bytes_in_use"] == 0
    srv.close()


def test_server_overlaps_requests(torch_dev):
    """Continuous batching: short requests arriving while a long one runs
    are admitted into the running rounds and finish before it, instead of
    waiting behind it."""
    from paper_2204_05586_amd import native
    long_p = W.spin_one_sensing(n_samples=3_000_000, t_start=0.0)
    short = _mix(20, seed=32, k_hi=5e3)
    srv = native.Server(iteration_steps=2e5)
    t_long = srv.submit(long_p)
    time.sleep(0.002)
    tickets = [srv.submit(p) for p in short]
    infos = [srv.wait(t, 120.0) for t in tickets]
    big = srv.wait(t_long, 120.0)
    st = srv.stats()
    admitted_during = sum(1 for i in infos if i["t_admit"] < big["t_done"])
    finished_before = sum(1 for i in infos if i["t_done"] < big["t_done"])
    print(f"[gpu] rounds {st['rounds']}; short requests admitted while the long one ran: "
          f"{admitted_during}/{len(short)}, finished before it: {finished_before}", flush=True)
    assert admitted_during == len(short) and finished_before >= len(short) // 2
    for t in tickets + [t_long]:
        srv.release(t)
    srv.close()


def test_server_fixed_slices(torch_dev):
    """options.slices fixes the lanes per interval (capped at a request's
    fine steps) and the results follow it bit for bit."""
    import torch
    from paper_2204_05586_amd import native
    probs = _mix(6, seed=33, k_hi=3e3)
    for slices in (1, 4):
        srv = native.Server(slices=slices, iteration_steps=1e5)
        tickets = [srv.submit(p) for p in probs]
        for t, p in zip(tickets, probs):
            assert srv.request_slices(p) == min(slices, 1 << (int(p.n_fine).bit_length() - 1))
            srv.wait(t, 120.0)
            got = srv.fetch(t, p, want_u=True)
            psi, fin, U = _alone(p, srv.request_slices(p))
            torch.cuda.synchronize()
            assert float((got["U"] - U).abs().max()) == 0.0
            assert float((got["psi"] - psi).abs().max()) == 0.0
            srv.release(t)
        srv.close()


def test_server_grows_round_image(torch_dev, oracle):
    """Requests with 2048 parameters each (control instances with 1024
    segments) on a server whose round image starts with room for 32 per
    request (about 30 KB for 6 active requests, against 6 x 16 KB of
    parameters here): the image grows and every result still equals the
    request alone."""
    import torch
    from paper_2204_05586_amd import native
    probs = W.control_batch(seed=9, n_inst=12, n_seg=1024, n_samples=200, n_fine=20)
    assert all(len(p.params) == 2048 for p in probs)
    srv = native.Server(max_active=6, iteration_steps=5e4)
    tickets = [srv.submit(p) for p in probs]
    print(f"[gpu] server with 512-parameter requests: {len(probs)}", flush=True)
    for i, (t, p) in enumerate(zip(tickets, probs)):
        info = srv.wait(t, 120.0)
        assert info["state"] == native.MSS_REQ_DONE
        got = srv.fetch(t, p, want_u=True)
        psi, fin, U = _alone(p, srv.request_slices(p))
        torch.cuda.synchronize()
        assert float((got["U"] - U).abs().max()) == 0.0, i
        assert float((got["psi"] - psi).abs().max()) == 0.0, i
        if i == 0:
            ref = oracle.solve(p)
            assert np.max(np.abs(got["psi"].cpu().numpy() - ref["psi"])) <= TOL
        srv.release(t)
    assert srv.stats()["rounds"] > 1
    srv.close()


def test_server_rejects_oversized(torch_dev):
    from paper_2204_05586_amd import native
    srv = native.Server(hbm_budget=1 << 24)
    with pytest.raises(native.MssError, match="budget"):
        srv.submit(W.spin_one_sensing(n_samples=200_000))
    srv.close()
