"""GPU parity of chained batch runs: the states formed inside the
integrator's launch (each work item's operators multiplied in registers and
its leaving state passed to the next item of its simulation), against the
oracle and against the separate-scan plan on the same batch."""
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


def _mixed_batch(seed):
    """Both spins, lengths from one interval to several thousand units'
    worth (single-unit simulations, exact multiples of 64 and of the 192
    intervals of a one-slice unit, ragged tails), frame on and off, both
    method families and the full su(3) basis."""
    rng = np.random.default_rng(seed)
    probs = []
    for K in [1, 2, 63, 64, 65, 127, 128, 129, 191, 192, 193, 383, 384, 385, 1000, 4097,
              70001]:
        for spin_twice in (1, 2):
            probs.append(W.random_problem(rng, spin_twice, K, int(rng.integers(1, 9)),
                                          n_squares=int(rng.integers(8, 29)),
                                          rotating_frame=bool(rng.integers(0, 2))))
    probs += W.batched_sensing(seed=2, n_sims=6, dur_lo=0.0499, dur_hi=0.0515)
    probs += W.control_batch(n_inst=3, n_samples=300, n_fine=20)
    probs.append(W.random_problem(rng, 2, 3001, 3, n_squares=20, rotating_frame=True)
                 .replace(method=W.HEUN))
    probs.append(W.random_problem(rng, 1, 2999, 4, rotating_frame=False)
                 .replace(method=W.MIDPOINT))
    full = W.spin_one_sensing(n_samples=777, t_start=0.0499)
    probs.append(full.replace(terms=list(full.terms) + [W.Term(W.COS, W.V1, a=300.0, f=700e3)]))
    rng.shuffle(probs)
    return probs


def _run(plan, store_u):
    import torch
    bufs = plan.allocate(store_u=store_u)
    bufs["psi"].fill_(float("nan"))
    bufs["psi_final"].fill_(float("nan"))
    print(f"[gpu] batch n={plan.n} chained={plan.chained} store_u={store_u} "
          f"info={plan.info()}", flush=True)
    plan.run(bufs)
    torch.cuda.synchronize()
    return bufs


@pytest.mark.parametrize("slices", [(0, 0), (1, 1), (16, 2), (4, 8)])
def test_chained_matches_separate_scan_and_oracle(torch_dev, oracle, slices):
    """Same operators bit for bit (U written by the chained launch too),
    states within rounding of the separate scan and within 1e-10 of the
    oracle, for every simulation of a mixed batch."""
    from paper_2204_05586_amd import native
    probs = _mixed_batch(seed=31)
    half, one = slices
    sep = native.BatchPlan(probs, slices_spin_half=half, slices_spin_one=one)
    ch = native.BatchPlan(probs, slices_spin_half=half, slices_spin_one=one, chained=True)
    assert ch.workspace_size(True) == ch.workspace_size(False)
    assert ch.workspace_size(False) <= 256 + 128 * len(probs) + 256
    if half and one:
        # a unit is 64 / S groups of three consecutive intervals
        units = 0
        for p in probs:
            S = half if p.spin_twice == 1 else one
            while S > p.n_fine:
                S >>= 1
            span = 3 * (64 // S)
            units += -(-p.n_samples // span)
        assert ch.info()["n_items"] == units
    bs = _run(sep, store_u=True)
    bc = _run(ch, store_u=True)
    assert bool((bc["U"] == bs["U"]).all())
    d_sep = float((bc["psi"] - bs["psi"]).abs().max())
    d_fin = float((bc["psi_final"] - bs["psi_final"]).abs().max())
    print(f"chained vs separate scan: max |dpsi| = {d_sep:.3e}, |dpsi_final| = {d_fin:.3e}",
          flush=True)
    assert d_sep <= 1e-12 and d_fin <= 1e-12
    worst = 0.0
    for i, p in enumerate(probs):
        ref = oracle.solve(p)
        got = ch.split(bc, i)
        d = max(np.max(np.abs(got["psi"].cpu().numpy() - ref["psi"])),
                np.max(np.abs(got["psi_final"].cpu().numpy() - ref["psi_final"])))
        worst = max(worst, d)
        assert d <= TOL, (i, p.name, p.n_samples, d)
    print(f"chained vs oracle: max |d| = {worst:.3e}", flush=True)
    # states only: no operator buffer anywhere, same states bit for bit
    bo = _run(ch, store_u=False)
    assert bool((bo["psi"] == bc["psi"]).all()) and bool((bo["psi_final"] == bc["psi_final"]).all())
    sep.close()
    ch.close()


def test_chained_repeats_and_graph_replays(torch_dev):
    """Calls through one workspace (the call number advances on the device)
    and replays of the captured graph, with eager work and synchronisations
    between them, give the eager result bit for bit each time."""
    import torch
    from paper_2204_05586_amd import native
    probs = _mixed_batch(seed=9)[:14]
    eager = native.BatchPlan(probs, chained=True)
    be = _run(eager, store_u=False)
    for rep in range(2):
        eager.run(be)
        torch.cuda.synchronize()
    ref = _run(eager, store_u=False)
    assert bool((ref["psi"] == be["psi"]).all())
    graph = native.BatchPlan(probs, chained=True, use_graph=True)
    bufs = graph.allocate(store_u=False)
    s = torch.cuda.Stream()
    for rep in range(3):
        bufs["psi"].fill_(float("nan"))
        bufs["psi_final"].fill_(float("nan"))
        with torch.cuda.stream(s):
            graph.run(bufs, stream=s)
        s.synchronize()
        torch.randn(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        d = float((bufs["psi"] - be["psi"]).abs().max())
        df = float((bufs["psi_final"] - be["psi_final"]).abs().max())
        print(f"[gpu] chained graph replay {rep}: max |d| = {d:.3e} {df:.3e}", flush=True)
        assert d == 0.0 and df == 0.0, (rep, d, df)
    eager.close()
    graph.close()


def test_chained_compiled_field_and_one_long_simulation(torch_dev, oracle):
    """The field program compiled into the chained integrator gives the
    interpreter's states bit for bit; a batch of one simulation (every item
    waits for the one before) matches the oracle."""
    from paper_2204_05586_amd import native
    probs = W.batched_sensing(seed=3, n_sims=40, dur_lo=0.001, dur_hi=0.006)
    interp = native.BatchPlan(probs, chained=True)
    comp = native.BatchPlan(probs, chained=True, specialize=True)
    assert comp.specialized
    bi = _run(interp, store_u=False)
    bc = _run(comp, store_u=False)
    assert bool((bi["psi"] == bc["psi"]).all())
    for i in (0, 13, 39):
        ref = oracle.solve(probs[i])
        assert np.max(np.abs(comp.split(bc, i)["psi"].cpu().numpy() - ref["psi"])) <= TOL
    interp.close()
    comp.close()
    one = [W.spin_one_sensing(n_samples=20011, t_start=0.0495)]
    plan = native.BatchPlan(one, chained=True, specialize=True)
    b = _run(plan, store_u=False)
    ref = oracle.solve(one[0])
    got = plan.split(b, 0)
    d = max(np.max(np.abs(got["psi"].cpu().numpy() - ref["psi"])),
            np.max(np.abs(got["psi_final"].cpu().numpy() - ref["psi_final"])))
    print(f"one long chained simulation vs oracle: {d:.3e}", flush=True)
    assert d <= TOL
    plan.close()


def test_chained_plan_api(torch_dev):
    """A chained plan has no separate scan and keeps no operators; a normal
    run passes mss_batch_check; a negative wait bound is refused."""
    from paper_2204_05586_amd import native
    probs = W.batched_sensing(n_sims=3, dur_lo=0.001, dur_hi=0.002)
    plan = native.BatchPlan(probs, chained=True)
    bufs = plan.allocate(store_u=False)
    with pytest.raises(native.MssError, match="chained"):
        plan.propagate(bufs)
    with pytest.raises(native.MssError, match="needs U"):
        plan.integrate(bufs)
    plan.run(bufs)
    plan.check(bufs)  # a normal run passes its check
    plan.close()
    with pytest.raises(native.MssInvalidError, match="chain_wait_us"):
        native.BatchPlan(probs, chained=True, chain_wait_us=-1)
    # a CU holds two chained workgroups: a plan asking for four per CU launches
    # two, and one asking for one launches one; all give the same states
    cu = torch_dev.cuda.get_device_properties(0).multi_processor_count
    many = W.batched_sensing(n_sims=2 * cu, dur_lo=0.002, dur_hi=0.004)
    four = native.BatchPlan(many, chained=True, waves_per_simd=4)
    two = native.BatchPlan(many, chained=True)
    one = native.BatchPlan(many, chained=True, waves_per_simd=1)
    assert four.info()["grid_blocks"] == two.info()["grid_blocks"] == 2 * cu
    assert one.info()["grid_blocks"] == cu
    b4, b2 = _run(four, store_u=False), _run(two, store_u=False)
    assert torch_dev.equal(b4["psi"], b2["psi"])
    # one workgroup per CU: every resident wave goes round the queue more
    # often; units still wait only for units taken before them
    b1 = _run(one, store_u=False)
    one.check(b1)
    assert torch_dev.equal(b1["psi"], b2["psi"])
    assert torch_dev.equal(b1["psi_final"], b2["psi_final"])
    four.close()
    two.close()
    one.close()
    # unit tags are 32-bit: a simulation of 2^31 units or more is refused
    # (before anything is allocated), one just below is planned
    huge = W.spin_one_sensing(n_samples=2 ** 39)
    with pytest.raises(native.MssError, match="too long for a chained plan"):
        native.BatchPlan([huge], chained=True, slices_spin_one=1)
    ok = native.BatchPlan([W.spin_one_sensing(n_samples=192 * (2 ** 31 - 1))], chained=True,
                          slices_spin_one=1)
    assert ok.info()["n_items"] == 2 ** 31 - 1
    ok.close()


def test_chained_wait_bound_reports_failure(torch_dev, oracle):
    """A wait bound far below the real waits (one simulation: every unit
    waits for the one before) makes the run give up: the launch still drains
    and ends, and mss_batch_check reports the failure.  The same problem
    without the bound checks clean and matches the oracle."""
    from paper_2204_05586_amd import native
    one = [W.spin_one_sensing(n_samples=20011, t_start=0.0495)]
    bounded = native.BatchPlan(one, chained=True, chain_wait_us=1)
    b = _run(bounded, store_u=False)
    with pytest.raises(native.MssError, match="waited longer"):
        bounded.check(b)
    print(f"[gpu] bounded chained run reported: {native.last_error()}", flush=True)
    bounded.close()
    plain = native.BatchPlan(one, chained=True)
    b = _run(plain, store_u=False)
    plain.check(b)
    ref = oracle.solve(one[0])
    d = np.max(np.abs(plain.split(b, 0)["psi"].cpu().numpy() - ref["psi"]))
    print(f"[gpu] unbounded run after it: check ok, max |d| vs oracle {d:.3e}", flush=True)
    assert d <= TOL
    plain.close()


def test_one_shot_calls_match_plans(torch_dev, oracle):
    """mss_solve_batch gives the chained plan's results bit for bit (and the
    oracle's); mss_adjoint_population gives the adjoint plan's losses and
    gradients (gradients summed with FP64 atomics: within 1e-12 relative)."""
    import torch
    from paper_2204_05586_amd import native
    probs = _mixed_batch(seed=44)[:16]
    print(f"[gpu] one-shot solve_batch n={len(probs)}", flush=True)
    one = native.solve_batch(probs, store_u=True)
    plan = native.BatchPlan(probs, chained=True)
    b = _run(plan, store_u=True)
    for key in ("psi", "psi_final", "U"):
        assert bool((one[key] == b[key]).all()), key
    for i in (0, 7, 15):
        ref = oracle.solve(probs[i])
        got = plan.split(b, i)
        assert np.max(np.abs(got["psi"].cpu().numpy() - ref["psi"])) <= TOL
    plan.close()
    ctl = W.control_batch(seed=5, n_inst=6, n_samples=200, n_fine=20)
    print(f"[gpu] one-shot adjoint_population n={len(ctl)}", flush=True)
    res = native.adjoint_population(ctl, 1)
    ap = native.AdjointPlan(ctl, 1)
    bufs = ap.allocate()
    ap.run(bufs)
    torch.cuda.synchronize()
    assert bool((res["loss"] == bufs["loss"]).all())
    g1, g2 = res["grad"], bufs["grad"][:res["grad"].numel()]
    rel = float((g1 - g2).abs().max() / g2.abs().max())
    print(f"[gpu] one-shot adjoint vs plan: loss equal, grad rel {rel:.3e}", flush=True)
    assert rel <= 1e-12
    ap.close()
