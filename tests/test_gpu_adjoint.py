"""GPU adjoint (gradients of a final population w.r.t. field parameters)
against the oracle's adjoint and extended-precision central differences."""
import numpy as np
import pytest

from paper_2204_05586_amd import workloads as W
from tests.test_oracle_adjoint import (_central_differences, _control_problem,
                                       _zero_field_problem, per_component_ok)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _gpu_adjoint(probs, m, specialize=False):
    import torch
    from paper_2204_05586_amd import native
    plan = native.AdjointPlan(probs, m, specialize=specialize)
    assert plan.specialized == specialize
    bufs = plan.allocate()
    print(f"[gpu] adjoint n={len(probs)} grads={plan.n_grad} ws={plan.ws_bytes}", flush=True)
    plan.run(bufs)
    torch.cuda.synchronize()
    out = {"loss": bufs["loss"].cpu().numpy(),
           "grad": [plan.grad_of(bufs, i).cpu().numpy() for i in range(len(probs))],
           "psi_final": bufs["psi_final"].cpu().numpy()}
    plan.close()
    return out


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def test_adjoint_matches_oracle_small(torch_dev, oracle):
    """Mixed spins, frame on/off, all term kinds with slots."""
    cs, pw = ("cos", "sin"), ("pwc",)
    probs = [_control_problem(2, frame=True, seed=1, extra=cs),
             _control_problem(2, frame=False, seed=2, extra=pw),
             _control_problem(1, frame=True, seed=3, extra=cs),
             _control_problem(1, frame=False, seed=4, extra=pw),
             _control_problem(2, frame=True, seed=5, K=301, L=3, extra=cs)]
    m = 1
    g = _gpu_adjoint(probs, m)
    for i, p in enumerate(probs):
        loss, grad = oracle.adjoint_population(p, m)
        assert abs(g["loss"][i] - loss) < 1e-12, (i, g["loss"][i], loss)
        r = _rel(g["grad"][i], grad)
        print(f"adjoint {i}: loss {loss:.6f} rel grad err {r:.2e}", flush=True)
        assert r <= 1e-9, (i, r)


def test_adjoint_at_zero_transverse_field(torch_dev, oracle):
    """Segments with no transverse field (rho = 0) and no field at all
    (theta = 0), both spins, frame on and off, random psi0, in one adjoint
    plan: the GPU gradients against the oracle adjoint (rel 1e-9 of the
    largest entry) and, per component, against extended-precision central
    differences (rel 1e-6)."""
    cases = [(2, True), (2, False), (1, True), (1, False)]
    probs = [_zero_field_problem(s, f, seed=3 * s + f) for s, f in cases]
    for m in (1, 0):
        g = _gpu_adjoint(probs, m)
        for i, p in enumerate(probs):
            assert np.all(np.isfinite(g["grad"][i]))
            loss, grad = oracle.adjoint_population(p, m)
            assert abs(g["loss"][i] - loss) < 1e-12
            r = _rel(g["grad"][i], grad)
            fd = _central_differences(oracle, p, m)
            ok, worst = per_component_ok(g["grad"][i], fd)
            print(f"zero field {cases[i]} m={m}: rel vs oracle {r:.2e}, "
                  f"worst/bound vs differences {worst:.2e}", flush=True)
            assert r <= 1e-9, (cases[i], m, r)
            assert ok, (cases[i], m, g["grad"][i], fd)


def test_adjoint_control_workload_subset(torch_dev, oracle):
    """Full-size control instances (256 segments x (amplitude, phase), 1 ms,
    1e5 CF4 steps, tau = 28): GPU vs oracle adjoint on every gradient
    entry, and vs extended-precision central differences (h = 1e-6) on a
    seeded subset of the controls."""
    probs = W.control_batch(n_inst=4)
    m = 1
    g = _gpu_adjoint(probs, m)
    for i in (0, 3):
        loss, grad = oracle.adjoint_population(probs[i], m)
        assert abs(g["loss"][i] - loss) < 1e-11
        r = _rel(g["grad"][i], grad)
        print(f"control {i}: loss {loss:.6f} rel grad err vs oracle adjoint {r:.2e}", flush=True)
        assert r <= 1e-9
    rng = np.random.default_rng(44)
    p = probs[0]
    par = np.asarray(p.params, dtype=np.longdouble)
    for q in rng.choice(par.size, 4, replace=False):
        h = np.longdouble(1e-6) * max(np.longdouble(1.0), abs(par[q]))
        pp, pm = par.copy(), par.copy()
        pp[q] += h
        pm[q] -= h
        fd = float((oracle.population_ld(p, m, pp) - oracle.population_ld(p, m, pm)) / (2 * h))
        scale = np.max(np.abs(g["grad"][0]))
        print(f"control 0 slot {q}: adjoint {g['grad'][0][q]:.10e} fd {fd:.10e}", flush=True)
        assert abs(g["grad"][0][q] - fd) <= 1e-6 * scale


def test_autograd_function_matches_oracle(torch_dev, oracle):
    """torch.autograd through PopulationModel: d(sum_i w_i loss_i)/dparams
    equals w_i times the oracle adjoint of instance i, and repeated calls
    at new parameters give new losses and gradients."""
    torch = torch_dev
    from paper_2204_05586_amd.autograd import PopulationModel
    probs = [_control_problem(2, frame=True, seed=11, extra=("cos",)),
             _control_problem(1, frame=True, seed=12, extra=("pwc",)),
             _control_problem(2, frame=False, seed=13, extra=("cos", "sin"))]
    m = 1
    model = PopulationModel(probs, m)
    w = torch.tensor([0.7, -1.3, 2.0], dtype=torch.float64, device="cuda")
    for it in range(2):
        params = model.initial_params()
        if it == 1:
            params = params * 1.05
        params.requires_grad_(True)
        print(f"[gpu] autograd call {it}", flush=True)
        loss = model(params)
        (w * loss).sum().backward()
        torch.cuda.synchronize()
        g = params.grad.cpu().numpy()
        pv = params.detach().cpu().numpy()
        off = model.plan.param_off
        for i, p in enumerate(probs):
            n = model.plan.packed[i].n_params
            q = p.replace(params=pv[off[i]:off[i] + n])
            ref_loss, ref_grad = oracle.adjoint_population(q, m)
            assert abs(loss[i].item() - ref_loss) < 1e-12
            r = _rel(g[off[i]:off[i] + n], w[i].item() * ref_grad)
            print(f"autograd call {it} instance {i}: rel err {r:.2e}", flush=True)
            assert r <= 1e-9
    model.close()


def test_autograd_gradcheck_small(torch_dev):
    """torch.autograd.gradcheck (central differences on the GPU forward) on a
    short spin-1 control problem."""
    torch = torch_dev
    from paper_2204_05586_amd.autograd import PopulationModel
    p = _control_problem(2, frame=True, seed=21, K=40, L=5, extra=("cos", "pwc"))
    model = PopulationModel([p], 1)
    params = model.initial_params().requires_grad_(True)
    print("[gpu] gradcheck", flush=True)
    assert torch.autograd.gradcheck(lambda x: model(x), (params,), eps=1e-4, atol=1e-7,
                                    rtol=1e-4, nondet_tol=1e-12)
    model.close()


def test_autograd_descent_lowers_loss(torch_dev):
    """Steps along minus the autograd gradient, sized for a 1 % predicted
    decrease, lower the population each time (a wrong sign or scale of the
    gradient would not)."""
    torch = torch_dev
    from paper_2204_05586_amd.autograd import PopulationModel
    p = _control_problem(2, frame=True, seed=31, extra=("cos",))
    model = PopulationModel([p], 1)
    x = model.initial_params().requires_grad_(True)
    losses = []
    for _ in range(4):
        x.grad = None
        loss = model(x).sum()
        loss.backward()
        losses.append(loss.item())
        with torch.no_grad():
            g = x.grad
            x -= 0.01 * loss.item() / float((g * g).sum()) * g
    print(f"descent losses {losses}", flush=True)
    assert all(b < a for a, b in zip(losses, losses[1:])), losses
    model.close()


def test_compiled_forward_gives_the_same_gradients(torch_dev):
    """The shared field program compiled into the forward pass: losses and
    final states bit for bit those of the interpreted forward, gradients
    equal up to the order of their FP64 atomic sums."""
    probs = W.control_batch(seed=6, n_inst=16, n_samples=300, n_fine=40)
    a = _gpu_adjoint(probs, 1)
    b = _gpu_adjoint(probs, 1, specialize=True)
    assert np.array_equal(a["loss"], b["loss"])
    assert np.array_equal(a["psi_final"], b["psi_final"])
    for ga, gb in zip(a["grad"], b["grad"]):
        assert _rel(gb, ga) <= 1e-13


def test_compiled_forward_needs_its_own_terms(torch_dev):
    from paper_2204_05586_amd import native
    probs = W.control_batch(seed=6, n_inst=2, n_samples=50, n_fine=10)
    other = native.Sampler.for_terms(probs[0].terms[:1])
    plan = native.AdjointPlan(probs, 1, specialize=False)
    with pytest.raises(native.MssError, match="not generated from its terms"):
        native.check(native.lib().mss_adjoint_plan_create_compiled(
            2, plan._arr, plan.param_off.ctypes.data_as(native.C.POINTER(native.C.c_int64)), 1,
            other._h, native.C.byref(native.C.c_void_p())))
    plan.close()
    other.close()
