"""GPU parity of user field samplers (HIP source compiled at run time into
its own integrator, through mss_sampler_*) against the oracle's
field-function route on the same field (tests/user_fields.py).
Bar: max |delta| <= 1e-10 on U, psi and psi_final."""
import math

import numpy as np
import pytest

from paper_2204_05586_amd import workloads as W
from tests import user_fields as F

pytestmark = pytest.mark.gpu

TOL = 1e-10
DT = 5e-6
DELTA = 1.0e3
BETA = math.pi ** 2 * DELTA ** 2 / 1.2
K_LZ = int(round(2 * 40 * DELTA / BETA / DT))

SENSING_SOURCE = r"""
__device__ void mss_user_field(double t, const double* p, double* f) {
#pragma clang fp contract(off)
  double s, c;
  mss::sincos_cw(mss::kTwoPi * (700e3 * t) + 0.0, &s, &c);
  double fx = 0.0 + 2000.0 * c;
  if (0.05 < t && t < 0.051) {
    mss::sincos_cw(mss::kTwoPi * (1000.0 * t) + 0.0, &s, &c);
    fx = fx + 20.0 * s;
  }
  f[0] = fx;
  f[2] = 0.0 + 700e3;
  f[3] = 0.0 + 2.3;
}
"""


@pytest.fixture(scope="module")
def dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_05586_amd import native
    native.lib()
    return torch


@pytest.fixture(scope="module")
def samplers(dev):
    from paper_2204_05586_amd import native
    s = {"lz": native.Sampler(F.LZ_SOURCE), "chirp": native.Sampler(F.CHIRP_SOURCE),
         "sensing": native.Sampler(SENSING_SOURCE)}
    yield s
    for v in s.values():
        v.close()


def _lz(spin_twice, frame, L=10, psi0=None, fq=0.0):
    return W.Problem(spin_twice, [], -K_LZ * DT / 2, DT, K_LZ, L, 28, frame,
                     params=np.array([BETA, DELTA, fq]), psi0=psi0)


def _chirp(spin_twice, frame, fq=0.0, K=1500, L=10):
    A = 1.0e3
    beta = math.pi ** 2 * A ** 2 / 1.2
    prm = np.array([5.0e4, beta, 1.0e-3, A, fq])
    return W.Problem(spin_twice, [], 1.0e-3 - K * DT / 2, DT, K, L, 28, frame, params=prm)


def _run(sampler, prob, launch=None):
    import torch
    from paper_2204_05586_amd import native
    print(f"[gpu] sampler spin2={prob.spin_twice} K={prob.n_samples} L={prob.n_fine} "
          f"frame={prob.rotating_frame} launch={launch}", flush=True)
    if launch is None:
        r = native.solve(prob, store_u=True, want_time=True, sampler=sampler)
    else:
        K, N = prob.n_samples, prob.dim
        U = torch.empty((K, N, N), dtype=torch.complex128, device="cuda")
        psi = torch.empty((K, N), dtype=torch.complex128, device="cuda")
        fin = torch.empty((N,), dtype=torch.complex128, device="cuda")
        ws = native.alloc_workspace(native.propagate_workspace_size(prob.spin_twice, K))
        sampler.integrate(prob, native.device_params(prob), U, launch=launch)
        native.propagate(prob.spin_twice, U, native.device_state(prob.psi0), psi, fin, ws)
        r = {"U": U, "psi": psi, "psi_final": fin, "time": None}
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in r.items()}


def _compare(g, ref, tol=TOL, name=""):
    d = {k: float(np.max(np.abs(g[k] - ref[k]))) for k in ("U", "psi", "psi_final")}
    print(f"{name}: " + " ".join(f"max|d{k}|={v:.3e}" for k, v in d.items()), flush=True)
    assert max(d.values()) <= tol, (name, d)


@pytest.mark.parametrize("spin_twice", [1, 2])
@pytest.mark.parametrize("frame", [True, False])
def test_landau_zener_ramp(dev, oracle, samplers, spin_twice, frame):
    prob = _lz(spin_twice, frame, fq=(150.0 if spin_twice == 2 else 0.0))
    ref = oracle.solve(prob, want_U=True, field_fn=F.lz_field)
    g = _run(samplers["lz"], prob)
    _compare(g, ref, name=f"LZ spin2={spin_twice} frame={frame}")
    assert np.array_equal(g["time"], prob.t_start + np.arange(prob.n_samples) * prob.dt_out)


@pytest.mark.parametrize("spin_twice", [1, 2])
@pytest.mark.parametrize("frame", [True, False])
def test_chirped_drive(dev, oracle, samplers, spin_twice, frame):
    prob = _chirp(spin_twice, frame, fq=(80.0 if spin_twice == 2 else 0.0))
    _compare(_run(samplers["chirp"], prob), oracle.solve(prob, want_U=True, field_fn=F.chirp_field),
             name=f"chirp spin2={spin_twice} frame={frame}")


@pytest.mark.parametrize("method", [W.MIDPOINT, W.HEUN])
def test_sampler_with_euler_methods(dev, oracle, samplers, method):
    prob = _chirp(2, True, fq=80.0, K=400).replace(method=method)
    _compare(_run(samplers["chirp"], prob), oracle.solve(prob, want_U=True, field_fn=F.chirp_field),
             name=f"chirp method={method}")


def test_sampler_reproduces_field_program(dev, samplers):
    """The sensing field written as a sampler with the interpreter's own
    arithmetic gives the precompiled field-program path's operators."""
    from paper_2204_05586_amd import native
    prob = W.spin_one_sensing(n_samples=3000, t_start=0.0499)
    g = _run(samplers["sensing"], prob.replace(terms=[]))
    r = native.solve(prob, store_u=True)
    dU = float(np.max(np.abs(g["U"] - r["U"].cpu().numpy())))
    print(f"sampler vs field program: max|dU| = {dU:.3e} (bitwise: {dU == 0.0})", flush=True)
    assert dU <= 1e-13


@pytest.mark.parametrize("slices", [1, 2, 4, 8])
def test_sampler_launch_shapes(dev, oracle, samplers, slices):
    prob = _chirp(2, True, K=777, L=16)
    ref = oracle.solve(prob, want_U=True, field_fn=F.chirp_field)
    g = _run(samplers["chirp"], prob, launch=(slices, 256))
    _compare(g, ref, name=f"chirp slices={slices}")


def test_sampler_sweep_and_lifetimes(dev, oracle):
    """One compiled sampler evaluated over a parameter sweep (the paper's
    reuse of a compiled simulator), with a second sampler created and
    destroyed in between."""
    from paper_2204_05586_amd import native
    s = native.Sampler(F.LZ_SOURCE)
    for i, delta in enumerate((500.0, 1000.0, 2000.0)):
        prob = W.Problem(1, [], -2e-3, DT, 800, 8, 28, True,
                         params=np.array([BETA, delta, 0.0]))
        _compare(_run(s, prob), oracle.solve(prob, want_U=True, field_fn=F.lz_field),
                 name=f"sweep delta={delta}")
        if i == 0:
            other = native.Sampler(F.CHIRP_SOURCE)
            _run(other, _chirp(1, True, K=64))
            other.close()
    s.close()


def test_sampler_edge_cases(dev, oracle):
    """K = 1, L = 1, no parameters (params NULL), and a K spanning several
    scan levels."""
    from paper_2204_05586_amd import native
    src = r"""
__device__ void mss_user_field(double t, const double* p, double* f) {
  f[0] = 250.0 * cos(2000.0 * t);
  f[2] = 1.0e3 + 4.0e5 * t;
}
"""

    def fn(t, p, f):
        f[0] = 250.0 * math.cos(2000.0 * t)
        f[2] = 1.0e3 + 4.0e5 * t

    s = native.Sampler(src)
    for K, L in ((1, 1), (1, 7), (70_001, 2)):
        prob = W.Problem(2, [], 0.0, 1e-6, K, L, 28, True)
        _compare(_run(s, prob), oracle.solve(prob, want_U=True, field_fn=fn), name=f"edge K={K} L={L}")
    s.close()


def test_simulator_with_source(dev, oracle):
    from paper_2204_05586_amd import Simulator
    sim = Simulator(F.CHIRP_SOURCE, spin=1, rotating_frame=True, n_squares=28)
    prm = _chirp(2, True).params
    res = sim.evaluate([0.6, 0.8j, 0.0], 0.0, 2e-3, 5e-7, 5e-6, params=prm)
    prob = sim.problem(0.0, 2e-3, 5e-7, 5e-6, params=prm, psi0=[0.6, 0.8j, 0.0])
    ref = oracle.solve(prob, want_U=True, field_fn=F.chirp_field)
    assert np.max(np.abs(res.state.cpu().numpy() - ref["psi"])) <= TOL
    assert np.max(np.abs(res.time_evolution.cpu().numpy() - ref["U"])) <= TOL
    assert np.max(np.abs(res.spin.cpu().numpy() - oracle.spin_projection(ref["psi"]))) <= TOL


def _sweep(seed=8):
    """A sweep of the Landau-Zener field over (beta, delta, f_q) with uneven
    lengths, both spins and both frame settings."""
    rng = np.random.default_rng(seed)
    probs = []
    for K in (1, 63, 64, 65, 700, 2049, 9000):
        for spin_twice in (1, 2):
            beta = BETA * rng.uniform(0.5, 2.0)
            delta = DELTA * rng.uniform(0.5, 2.0)
            fq = rng.uniform(-300.0, 300.0) if spin_twice == 2 else 0.0
            L = int(rng.integers(1, 13))
            frame = bool(rng.integers(0, 2))
            psi0 = W.random_state(spin_twice + 1, rng)
            probs.append(W.Problem(spin_twice, [], -K * DT / 2, DT, K, L, int(rng.integers(12, 29)),
                                   frame, params=np.array([beta, delta, fq]), psi0=psi0))
    return probs


def test_sampled_batch_matches_oracle_and_alone(dev, oracle, samplers):
    """One persistent launch over a parameter sweep of one compiled field
    function: every simulation vs the oracle, and vs the single-simulation
    sampler path with the same lane-slice count."""
    from paper_2204_05586_amd import native
    probs = _sweep()
    plan = native.BatchPlan(probs, slices_spin_half=1, slices_spin_one=1, sampler=samplers["lz"])
    bufs = plan.allocate(store_u=True)
    print(f"[gpu] sampled batch n={plan.n} info={plan.info()}", flush=True)
    plan.run(bufs)
    dev.cuda.synchronize()
    worst_ref = worst_alone = 0.0
    for i, p in enumerate(probs):
        got = {k: v.cpu().numpy() for k, v in plan.split(bufs, i).items()}
        ref = oracle.solve(p, want_U=True, field_fn=F.lz_field)
        d = max(float(np.max(np.abs(got[k] - ref[k]))) for k in ("U", "psi", "psi_final"))
        assert d <= TOL, (i, p.n_samples, d)
        alone = _run(samplers["lz"], p, launch=(1, 256))
        worst_alone = max(worst_alone, float(np.max(np.abs(got["U"] - alone["U"]))))
        worst_ref = max(worst_ref, d)
    print(f"sampled batch: vs oracle {worst_ref:.3e}, vs alone {worst_alone:.3e}", flush=True)
    assert worst_alone <= 1e-13
    plan.close()


def test_sampled_batch_graph_replays(dev, samplers):
    from paper_2204_05586_amd import native
    probs = _sweep(seed=9)
    eager = native.BatchPlan(probs, sampler=samplers["lz"])
    e = eager.allocate(store_u=True)
    eager.run(e)
    graph = native.BatchPlan(probs, use_graph=True, sampler=samplers["lz"])
    g = graph.allocate(store_u=True)
    for rep in range(3):
        print(f"[gpu] sampled batch graph replay {rep}", flush=True)
        g["psi"].zero_()
        graph.run(g)
        dev.cuda.synchronize()
        assert dev.equal(g["psi"], e["psi"]) and dev.equal(g["U"], e["U"])
    eager.close()
    graph.close()


def test_sampled_batch_autotuned(dev, oracle, samplers, tmp_path):
    from paper_2204_05586_amd import autotune
    probs = _sweep(seed=10)
    plan = autotune.tuned_plan(probs, sampler=samplers["lz"], cache_path=str(tmp_path / "t.json"),
                               reps=1)
    bufs = plan.allocate(store_u=False)
    print(f"[gpu] autotuned sampled batch {plan.options}", flush=True)
    plan.run(bufs)
    dev.cuda.synchronize()
    for i in (0, len(probs) // 2, len(probs) - 1):
        got = plan.split(bufs, i)
        ref = oracle.solve(probs[i], field_fn=F.lz_field)
        assert np.max(np.abs(got["psi"].cpu().numpy() - ref["psi"])) <= TOL
    plan.close()


def test_sampled_batch_rejects_terms(dev, samplers):
    from paper_2204_05586_amd import native
    probs = _sweep()[:2] + [W.spin_half_rabi(n_samples=10)]
    with pytest.raises(native.MssError, match="no terms"):
        native.BatchPlan(probs, sampler=samplers["lz"])
