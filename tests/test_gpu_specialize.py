"""GPU: field programs compiled into their own integrator
(mss_sampler_create_for_terms) give the interpreter's operators bit for bit,
alone (with the same lane slicing) and in batch plans, and the oracle's within
the parity tolerance."""
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
    from paper_2204_05586_amd import native
    native.lib()
    return torch


def _all_kinds(spin_twice, frame, method=0, K=1200, L=7, tau=28):
    """Every term kind, literal and slot operands, finite, one-sided and
    empty windows, piecewise segments with clamping at both ends."""
    T = W.Term
    terms = [T(W.CONST, W.Z, a=1.2e4),
             T(W.COS, W.X, a=3.0e3, f=1.1e4, phi=0.3),
             T(W.SIN, W.Y, a_slot=0, f_slot=1, phi_slot=2, t_on=2e-4, t_off=6e-4),
             T(W.PWC, W.X, n_seg=4, seg_a_slot=3, seg_t0=1e-4, seg_len=2.5e-4),
             T(W.PWC_COS, W.Y, f=9.0e3, n_seg=3, seg_a_slot=7, seg_phi_slot=10, seg_t0=1e-4,
               seg_len=3e-4, t_off=8e-4),
             T(W.PWC_SIN, W.X, a=1.5e3, f=7.0e3, n_seg=2, seg_phi_slot=13, seg_t0=-1e-4,
               seg_len=5e-4, t_on=-0.1),
             T(W.COS, W.Z, a=50.0, f=30.0, t_on=1.0, t_off=1.0)]
    if spin_twice == 2:
        terms += [T(W.CONST, W.Q, a=-0.0), T(W.SIN, W.Q, a=400.0, f=2e3)]
    rng = np.random.default_rng(7)
    params = np.concatenate([[800.0, 1.3e4, 0.7], rng.uniform(-4e3, 4e3, 4),
                             rng.uniform(500, 5e3, 3), rng.uniform(-3, 3, 3),
                             rng.uniform(-3, 3, 2)])
    return W.Problem(spin_twice, terms, 0.0, 1e-6, K, L, tau, frame, params=params,
                     psi0=W.random_state(spin_twice + 1, rng), name="all_kinds", method=method)


def _cases():
    rng = np.random.default_rng(31)
    out = []
    for s in (1, 2):
        for frame in (False, True):
            out.append((f"all_kinds s{s} frame{int(frame)}", _all_kinds(s, frame)))
            out.append((f"random s{s} frame{int(frame)}",
                        W.random_problem(rng, s, 777, 5, n_squares=int(rng.integers(8, 29)),
                                         rotating_frame=frame)))
        out.append((f"all_kinds s{s} midpoint", _all_kinds(s, True, method=1)))
        out.append((f"all_kinds s{s} heun", _all_kinds(s, True, method=2)))
        out.append((f"all_kinds s{s} tau0", _all_kinds(s, True, tau=0, K=300)))
    out.append(("sensing window", W.spin_one_sensing(n_samples=3000, t_start=0.0499)))
    out.append(("control pwc", W.control_batch(n_inst=1, n_samples=300, n_fine=20)[0]))
    out.append(("no terms", W.Problem(2, [], 0.0, 1e-6, 100, 4, 28, True)))
    return out


CASES = _cases()


@pytest.mark.parametrize("name,prob", CASES, ids=[c[0] for c in CASES])
def test_specialised_equals_interpreter(torch_dev, oracle, name, prob):
    import torch
    from paper_2204_05586_amd import native
    K, N = prob.n_samples, prob.spin_twice + 1
    s = native.Sampler.for_terms(prob.terms)
    bare = prob.replace(terms=[])
    params = native.device_params(prob)
    for launch in ((1, 256), (2, 256), (4, 128)):
        print(f"[gpu] specialise {name} K={K} launch={launch}", flush=True)
        Ui = torch.empty((K, N, N), dtype=torch.complex128, device="cuda")
        Us = torch.empty_like(Ui)
        native.integrate(prob, params, Ui, launch=launch)
        s.integrate(bare, params, Us, launch=launch)
        torch.cuda.synchronize()
        d = float((Ui - Us).abs().max())
        assert d == 0.0, (name, launch, d)
    ref = oracle.operators(prob)
    assert float(np.max(np.abs(Us.cpu().numpy() - ref))) <= TOL
    s.close()


def test_specialised_batch_equals_interpreted(torch_dev):
    import torch
    from paper_2204_05586_amd import native
    probs = W.batched_sensing(seed=5, n_sims=40, dur_lo=0.0495, dur_hi=0.052)
    opts = dict(slices_spin_one=2, scan_per_lane=2)
    res = []
    for spec in (False, True):
        plan = native.BatchPlan(probs, specialize=spec, **opts)
        assert plan.specialized == spec
        bufs = plan.allocate(store_u=True)
        print(f"[gpu] batch specialise={spec} info={plan.info()}", flush=True)
        plan.run(bufs)
        torch.cuda.synchronize()
        res.append({k: bufs[k].cpu().numpy() for k in ("psi", "psi_final", "U")})
        plan.close()
    for k in ("psi", "psi_final", "U"):
        assert float(np.max(np.abs(res[0][k] - res[1][k]))) == 0.0, k


def test_specialise_needs_one_term_list(torch_dev):
    """Problems with different term lists stay interpreted."""
    from paper_2204_05586_amd import native
    rng = np.random.default_rng(3)
    probs = [W.random_problem(rng, 2, 50, 2) for _ in range(3)]
    plan = native.BatchPlan(probs, specialize=True)
    assert not plan.specialized
    plan.close()
