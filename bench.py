#!/usr/bin/env python3
"""Throughput benchmark of the solver path on one MI355X.

Default workload: 4096 spin-1 sensing simulations of uneven length (10-100
ms at 5e-7 s output steps, 10 CF4 steps per interval, tau = 28, rotating
frame) run as one batch: one captured HIP graph of the chained persistent
integrator, which builds every interval operator from its CF4 fine steps
and forms the states psi_k in the same launch (work items pass their
leaving state on to the next item of their simulation), through the C ABI.
The simulations share one field program (their parameters differ), which
the plan compiles into the integrator at creation
(mss_sampler_create_for_terms; the interpreter's time is reported beside
it).  One step = one replay of the graph over the whole batch.  Inputs and
outputs stay resident in HBM; the timed region starts after they are
allocated.

Also measured in the same run: the separate-scan form of the batch
(operators kept in HBM, then the segmented scan), the plain path (one
simulation per launch sequence) on the single spin-1 sensing simulation and
the spin-1/2 Rabi simulation, the rows beyond the hot path, the adjoint and
the serving sweep.

Prints one JSON line: CF4 fine steps/s, the integrator's roofline figures
(algorithmic FP64 flops / measured kernel time vs the 78.6 TFLOP/s FP64
vector peak) and the CPU oracle's rate on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6  # 256 CU x 2.4 GHz x 128 FP64 flop/clk

# HBM traffic per launch of the batched integrators from rocprofv3 FETCH_SIZE /
# WRITE_SIZE passes, calibrated against a 1 GiB copy (FETCH x 2.000, WRITE x 1.000),
# keyed by the hash of the kernel sources they were taken with: reported only while
# the sources are unchanged.
MEASURED_TRAFFIC = {
    ("mss_user_work_chained", "batched_sensing"): {
        "src": "3cddbfb6a0a9c8eb",
        "fetch_kib": 284383.0, "write_kib": 24306971.7,
        "bytes": int(round((284383.0 * 2.000 + 24306971.7 * 1.000) * 1024)),
    },
    ("mss_user_work_integrate", "batched_sensing"): {
        "src": "3cddbfb6a0a9c8eb",
        "fetch_kib": 3700.7, "write_kib": 64036245.0,
        "bytes": int(round((3700.7 * 2.000 + 64036245.0 * 1.000) * 1024)),
    },
}


# sources that define the batched integrators: the field program compiled into
# the persistent work-queue kernels at run time (mss_user_work_chained and
# mss_user_work_integrate: the generated field function, the device headers they
# are compiled with, the compile options, the work tables and the launch)
INTEGRATOR_SOURCES = ("mss_device.h", "mss_work.h", "mss_work_device.h", "mss_work.hip",
                      "mss_user_kernels.h", "mss_sampler.hip")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2204_05586_amd", "csrc")
    for name in INTEGRATOR_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


# The paper's own speed figure, quoted as context (another GPU; not the
# target): Sec. "Parallelization performance" runs its 100 ms spin-1 sensing
# simulation at 100 ns steps (1e6 CF4 steps) almost twice as fast as real
# time on an RTX 3080, about 50 ms, i.e. about 2e7 fine steps/s.
PAPER_CONTEXT = {"workload": "one 100 ms spin-1 sensing simulation, 1e6 CF4 steps",
                 "hardware": "GeForce RTX 3080", "ms": 50.0, "fine_steps_per_s": 2.0e7}


def spin_one_flops_per_fine_step(tau: int) -> int:
    """Algorithmic FP64 flops of one spin-1 CF4 fine step as computed: two
    Lie-Trotter exponentials of tau residual squarings of a complex symmetric
    3x3 matrix (six entries: 96 flops each, counting a fused multiply-add as
    two) plus two general 3x3 complex products into the interval operator
    (27 complex multiply-adds = 216 flops each).  Angle set-up and the
    phases put back once per exponential are not counted."""
    return 2 * tau * 96 + 2 * 216


# Algorithmic FP64 flops of one state update psi_{k+1} = U_k psi_k (spin-1:
# 9 complex multiply-adds of 8 flops each).
STATE_UPDATE_FLOPS = 72


def cpu_baseline(problems, seconds: float) -> dict:
    """The CPU oracle on a bounded sample of the workload's simulations."""
    from oracle import oracle
    threads = oracle.get_threads()
    done_steps, used, t0 = 0, 0, time.perf_counter()
    for p in problems:
        oracle.solve(p)
        done_steps += p.fine_steps
        used += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    # one thread, on the same simulations in the same order, for a third of the time
    oracle.set_threads(1)
    one_steps, one_used, t1 = 0, 0, time.perf_counter()
    try:
        for p in problems:
            oracle.solve(p)
            one_steps += p.fine_steps
            one_used += 1
            if time.perf_counter() - t1 >= seconds / 3:
                break
    finally:
        oracle.set_threads(threads)
    dt1 = time.perf_counter() - t1
    return {"value": round(done_steps / dt, 1), "unit": "fine_steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{used} of {len(problems)} simulations ({done_steps} fine steps, "
                      f"{dt:.1f} s, {threads} OpenMP threads over intervals)",
            "single_thread": {"value": round(one_steps / dt1, 1),
                              "sample": f"{one_used} simulations ({one_steps} fine steps, "
                                        f"{dt1:.1f} s)"},
            "host": {"cpu_count": os.cpu_count(), "model": _cpu_model()}}


def cpu_serving_baseline(seconds: float) -> dict:
    """The CPU oracle on the serving workload's requests (the 10 req/s
    stream, in arrival order), solved one after another for a bounded
    time: the rate a CPU server would sustain on the same mix."""
    from oracle import oracle
    from paper_2204_05586_amd import workloads as W
    stream = W.serving_stream(10.0, n_requests=600, rate_index=0)
    threads = oracle.get_threads()
    steps, used, t0 = 0, 0, time.perf_counter()
    for r in stream:
        oracle.solve(r.problem)
        steps += r.problem.fine_steps
        used += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": round(steps / dt, 1), "unit": "fine_steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"the first {used} of the 10 req/s stream's {len(stream)} requests in "
                      f"arrival order ({steps} fine steps, {dt:.1f} s, {threads} OpenMP threads "
                      f"over intervals)"}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_plain(prob, steps: int, warmup: int, specialise: bool = True) -> dict:
    """One simulation per launch sequence: the integrator (the field program
    compiled into it, unless specialise is off) and the scan; the
    interpreter's integrator is timed too."""
    import torch
    from paper_2204_05586_amd import native
    K, N = prob.n_samples, prob.dim
    params = native.device_params(prob)
    sampler = native.Sampler.for_terms(prob.terms) if specialise else None
    bare = prob.replace(terms=[])
    psi0 = native.device_state(prob.psi0)
    U = torch.empty((K, N, N), dtype=torch.complex128, device="cuda")
    psi = torch.empty((K, N), dtype=torch.complex128, device="cuda")
    fin = torch.empty((N,), dtype=torch.complex128, device="cuda")
    ws = native.alloc_workspace(native.propagate_workspace_size(prob.spin_twice, K))
    launch = native.plan_launch(prob)  # reported; the launch itself is the library's default
    stream = torch.cuda.current_stream()

    def integrate(interpret=False):
        if sampler is None or interpret:
            native.integrate(prob, params, U, stream=stream)
        else:
            sampler.integrate(bare, params, U, stream=stream)

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        integrate()
        if ev:
            ev[1].record(stream)
        native.propagate(prob.spin_twice, U, psi0, psi, fin, ws, stream=stream)
        if ev:
            ev[2].record(stream)

    # at least `warmup` steps and 0.2 s, so the clock has ramped up
    t_warm = time.perf_counter()
    done = 0
    while done < warmup or time.perf_counter() - t_warm < 0.2:
        step()
        done += 1
        if done % 16 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    # the step's wall time over `steps` back-to-back steps, with nothing else
    # on the stream (an event record per launch adds its own cost)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the integrator / scan split from HIP events, in a pass of its own
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for e in evs:
        step(e)
    torch.cuda.synchronize()
    integ = [e[0].elapsed_time(e[1]) for e in evs]
    prop = [e[1].elapsed_time(e[2]) for e in evs]
    interp = []
    for _ in range(max(steps, 1)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        integrate(interpret=True)
        e1.record(stream)
        interp.append((e0, e1))
    torch.cuda.synchronize()
    if sampler is not None:
        sampler.close()
    return {"workload": prob.name, "fine_steps": prob.fine_steps,
            "value": prob.fine_steps * steps / wall, "ms_per_step": wall / steps * 1e3,
            "integrate_ms": statistics.mean(integ), "propagate_ms": statistics.mean(prop),
            "integrate_ms_interpreter": statistics.mean(a.elapsed_time(b) for a, b in interp),
            "field": "compiled in" if sampler is not None else "interpreted",
            "launch": {"slices": launch[0], "block": launch[1]}, "tau": prob.n_squares}


def states_to_host(psi, stream, max_bytes: int = 2 << 30) -> dict:
    """The states' copy to the host, outside every timed step: a prefix of
    at most max_bytes into pinned host memory (allocated pinned), three
    copies between HIP events; the rate and the time it gives for all the
    states."""
    import torch
    flat = psi.view(-1)
    n = min(flat.numel(), max_bytes // flat.element_size())
    host = torch.empty(n, dtype=flat.dtype, pin_memory=True)
    ms = []
    for _ in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        with torch.cuda.stream(stream):
            host.copy_(flat[:n], non_blocking=True)
        b.record(stream)
        b.synchronize()
        ms.append(a.elapsed_time(b))
    nbytes = n * flat.element_size()
    rate = nbytes / (min(ms) * 1e-3)
    total = flat.numel() * flat.element_size()
    del host
    return {"bytes": nbytes, "ms": round(min(ms), 3), "gb_per_s": round(rate / 1e9, 2),
            "states_bytes": total, "states_ms_at_that_rate": round(total / rate * 1e3, 1)}


def bench_batched(problems, steps: int, warmup: int, tune: bool, specialise: bool = True,
                  separate_reps: int = 3) -> dict:
    """The batch as one captured HIP graph of a chained plan (the shared
    field program compiled into the persistent integrator, which also forms
    the states; no operator buffer), replayed `steps` times after at least
    3 warm-up replays, each replay between HIP events on the stream it runs
    on (with more replays after the timed ones when `steps` < 10, so that
    the replay statistics cover at least 10).  Then the separate-scan plan (operators kept in the workspace, then
    the segmented scan) eagerly, integrator and scan timed apart, and the
    interpreter's integrator on its buffers."""
    import torch
    from paper_2204_05586_amd import autotune, native
    t0 = time.perf_counter()
    opts = autotune.tune(problems, cache_path=None, specialize=specialise) if tune else {}
    tune_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    plan = native.BatchPlan(problems, specialize=specialise, chained=True, use_graph=True, **opts)
    compile_s = time.perf_counter() - t0
    bufs = plan.allocate(store_u=False)
    stream = torch.cuda.current_stream()
    fine = sum(p.fine_steps for p in problems)
    for _ in range(max(warmup, 3)):  # the first run captures the graph
        plan.run(bufs, stream=stream)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        plan.run(bufs, stream=stream)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the replay statistics cover at least 10 replays: when fewer steps are
    # timed, the rest run after the timed region
    extra = [[torch.cuda.Event(enable_timing=True) for _ in range(2)]
             for _ in range(max(0, 10 - steps))]
    for a, b in extra:
        a.record(stream)
        plan.run(bufs, stream=stream)
        b.record(stream)
    torch.cuda.synchronize()
    replay = [a.elapsed_time(b) for a, b in evs + extra]
    info = plan.info()
    specialized = plan.specialized
    ws_bytes = int(bufs["ws"].numel())
    psi_chained = bufs["psi"]
    d2h = states_to_host(psi_chained, stream)
    plan.close()
    del bufs["ws"]
    # the separate-scan plan: integrator then scan, eager
    sep = native.BatchPlan(problems, specialize=specialise, **opts)
    sbufs = sep.allocate(store_u=False)
    integ, prop = [], []
    for rep in range(separate_reps + 1):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(stream)
        sep.integrate(sbufs, stream=stream)
        e[1].record(stream)
        sep.propagate(sbufs, stream=stream)
        e[2].record(stream)
        torch.cuda.synchronize()
        if rep:  # the first is a warm-up
            integ.append(e[0].elapsed_time(e[1]))
            prop.append(e[1].elapsed_time(e[2]))
    d_sep = float((sbufs["psi"] - psi_chained).abs().max())
    sep_ws = int(sbufs["ws"].numel())
    sep.close()
    iplan = native.BatchPlan(problems, **opts)
    interp = []
    for _ in range(2):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        iplan.integrate(sbufs, stream=stream)
        e1.record(stream)
        interp.append((e0, e1))
    torch.cuda.synchronize()
    iplan.close()
    del sbufs, psi_chained
    torch.cuda.empty_cache()
    return {"value": fine * steps / wall, "ms_per_step": wall / steps * 1e3,
            "replay_ms_mean": statistics.mean(replay),
            "replay_ms_median": statistics.median(replay),
            "replay_ms_min": min(replay), "replay_ms_max": max(replay),
            "workspace_bytes": ws_bytes, "d2h": d2h,
            "separate_scan": {"integrate_ms": statistics.mean(integ),
                              "propagate_ms": statistics.mean(prop),
                              "ms_per_step": statistics.mean(integ) + statistics.mean(prop),
                              "workspace_bytes": sep_ws,
                              "max_abs_diff_vs_chained": d_sep},
            "integrate_ms_interpreter": statistics.mean(a.elapsed_time(b) for a, b in interp),
            "specialized": specialized, "compile_s": compile_s,
            "fine_steps": fine, "info": info, "options": opts, "tune_s": tune_s}


def bench_serving(rates, seconds_per_rate: float, max_requests: int, budget_gib: float,
                  burst: int = 0, min_requests: int = 600) -> dict:
    """Poisson request streams (70 % spin-1, 30 % spin-1/2, K log-uniform in
    [1e3, 1e6], 10 CF4 steps per interval) submitted at their arrival times
    to one server; latency = completion - scheduled arrival.  Each rate gets
    rate x seconds_per_rate requests, at least min_requests (so that p99 rests
    on several samples) and at most max_requests.  With burst > 0,
    also `burst` requests of the same mix submitted at once: the server's
    capacity (fine steps/s from the first submission to the last
    completion), with latency = completion - submission."""
    import queue
    import threading
    import numpy as np
    from paper_2204_05586_amd import native, workloads as W
    all_rates = [10.0, 30.0, 100.0, 300.0, 1000.0]
    srv = native.Server(hbm_budget=int(budget_gib * (1 << 30)))
    out = {}
    for rate in rates:
        n = int(min(max_requests, max(min_requests, rate * seconds_per_rate)))
        idx = all_rates.index(rate) if rate in all_rates else len(all_rates)
        stream = W.serving_stream(rate, n_requests=n, rate_index=idx)
        q, records = queue.Queue(), []

        def collect():
            while True:
                item = q.get()
                if item is None:
                    return
                t, arrival, steps = item
                info = srv.wait(t, 600.0)
                records.append((arrival, info["t_submit"], info["t_done"], steps))
                srv.release(t)

        th = threading.Thread(target=collect)
        th.start()
        base = srv.clock() + 0.05
        for r in stream:
            # sleep to within 2 ms of the arrival, then spin on the server
            # clock: the load generator's own lateness stays out of the latency
            due = base + r.arrival
            delay = due - srv.clock()
            if delay > 0.002:
                time.sleep(delay - 0.002)
            while srv.clock() < due:
                pass
            q.put((srv.submit(r.problem), due, r.problem.fine_steps))
        q.put(None)
        th.join()
        lat = np.array([d - a for a, _, d, _ in records]) * 1e3
        lag = np.array([sub - a for a, sub, _, _ in records]) * 1e3
        span = max(d for _, _, d, _ in records) - base
        steps = sum(st for *_, st in records)
        out[str(int(rate))] = {"requests": n, "p50_ms": round(float(np.percentile(lat, 50)), 3),
                               "p99_ms": round(float(np.percentile(lat, 99)), 3),
                               "mean_ms": round(float(lat.mean()), 3),
                               "submit_lag_p99_ms": round(float(np.percentile(lag, 99)), 3),
                               "fine_steps_per_s": round(steps / span, 1)}
    if burst > 0:
        reqs = W.serving_stream(1000.0, n_requests=burst, rate_index=len(all_rates) + 1)
        t0 = srv.clock()
        tickets = [(srv.submit(r.problem), r.problem.fine_steps) for r in reqs]
        spin_one_steps = sum(r.problem.fine_steps for r in reqs if r.problem.spin_twice == 2)
        lat, steps, last = [], 0, t0
        for t, st_ in tickets:
            info = srv.wait(t, 600.0)
            lat.append(info["t_done"] - info["t_submit"])
            last = max(last, info["t_done"])
            steps += st_
            srv.release(t)
        lat = np.array(lat) * 1e3
        out["burst"] = {"requests": burst, "fine_steps": steps, "spin_one_fine_steps": spin_one_steps,
                        "p50_ms": round(float(np.percentile(lat, 50)), 3),
                        "p99_ms": round(float(np.percentile(lat, 99)), 3),
                        "span_s": round(last - t0, 4),
                        "fine_steps_per_s": round(steps / (last - t0), 1)}
    st = srv.stats()
    out["server"] = {"rounds": st["rounds"], "bytes_peak": st["bytes_peak"],
                     "budget": st["budget"]}
    srv.close()
    return out


def bench_adjoint(n_inst: int, steps: int, warmup: int, specialise: bool = True) -> dict:
    """Gradients of the |0> population w.r.t. 512 piecewise-constant
    controls (256 amplitudes, 256 phases) for n_inst spin-1 instances of 1
    ms (1e3 intervals x 100 CF4 steps, tau = 28, resonant rotating frame).
    The instances share one field program, compiled into the forward pass
    unless specialise is off."""
    import torch
    from paper_2204_05586_amd import native, workloads as W
    probs = W.control_batch(seed=4, n_inst=n_inst)
    plan = native.AdjointPlan(probs, 1, specialize=specialise)
    forward = "field compiled in" if plan.specialized else "interpreted"
    bufs = plan.allocate()
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.run(bufs, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.run(bufs, stream=stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    fine = sum(p.fine_steps for p in probs)
    plan.close()
    del bufs
    torch.cuda.empty_cache()
    return {"instances": n_inst, "controls_per_instance": 512, "forward": forward,
            "ms_per_gradient_batch": round(dt * 1e3, 3),
            "gradients_per_s": round(n_inst * 512 / dt, 1),
            "forward_plus_adjoint_fine_steps_per_s": round(fine / dt, 1)}


# The spin-1 sensing field written as a user field function (HIP source),
# the way the paper's users write theirs: the f3 row's input.
SENSING_USER_SOURCE = r"""
__device__ void mss_user_field(double t, const double* p, double* f) {
  double s, c;
  mss::sincos_cw(mss::kTwoPi * (700e3 * t), &s, &c);
  double fx = 2000.0 * c;
  if (0.05 < t && t < 0.051) {
    mss::sincos_cw(mss::kTwoPi * (1000.0 * t), &s, &c);
    fx += 20.0 * s;
  }
  f[0] = fx;
  f[2] = 700e3;
  f[3] = 2.3;
}
"""


def bench_next_rows(reps: int = 20) -> dict:
    """The rows beyond the batched path, each timed with HIP events on the
    2e5-interval spin-1 sensing simulation (inputs resident on the device):
    f1 <J> of its states; f2 its midpoint and Heun samplings (field program
    compiled in); f3 its field written as a user sampler; f4 the same problem
    in the full su(3) basis (a resonant V_1 drive added; interpreted)."""
    import torch
    from paper_2204_05586_amd import native, workloads as W
    prob = W.spin_one_sensing()
    K, N, tau = prob.n_samples, prob.dim, prob.n_squares
    fine = prob.fine_steps
    stream = torch.cuda.current_stream()
    params = native.device_params(prob)
    U = torch.empty((K, N, N), dtype=torch.complex128, device="cuda")

    def timed(fn) -> float:
        # back-to-back launches between one pair of events: the per-launch
        # time of short kernels without an event pair's own overhead.  At
        # least 0.2 s of warm-up first: a run-time compile just before leaves
        # the GPU idle and its clock low.
        t_warm, done = time.perf_counter(), 0
        while done < 3 or time.perf_counter() - t_warm < 0.2:
            fn()
            done += 1
            if done % 16 == 0:
                torch.cuda.synchronize()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    def alu(flops_per_step: int, ms: float) -> dict:
        tf = flops_per_step * fine / (ms * 1e-3) / 1e12
        return {"fine_steps_per_s": round(fine / (ms * 1e-3), 1), "integrate_ms": round(ms, 4),
                "roofline": {"bound": "alu", "achieved": round(tf, 3),
                             "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                             "frac": round(tf / FP64_VECTOR_PEAK_TFLOPS, 4),
                             "flops_per_fine_step": flops_per_step}}

    out = {}
    smp = native.Sampler.for_terms(prob.terms)
    for name, method in (("midpoint", W.MIDPOINT), ("heun", W.HEUN)):
        bare = prob.replace(terms=[], method=method)
        ms = timed(lambda: smp.integrate(bare, params, U, stream=stream))
        # one exponential of tau symmetric squarings and one product per fine step
        out[f"f2_{name}"] = alu(96 * tau + 216, ms)
    smp.close()
    user = native.Sampler(SENSING_USER_SOURCE)
    bare = prob.replace(terms=[])
    ms = timed(lambda: user.integrate(bare, params, U, stream=stream))
    out["f3_user_sampler"] = alu(spin_one_flops_per_fine_step(tau), ms)
    user.close()
    full = prob.replace(terms=list(prob.terms) + [W.Term(W.COS, W.V1, a=300.0, f=700e3)])
    ms = timed(lambda: native.integrate(full, params, U, stream=stream))
    # per exponential: the Taylor residual (3 products) and tau general
    # squarings (27 complex multiply-adds = 216 flops each); two per step,
    # plus the two products into U
    out["f4_full_su3"] = alu(2 * (3 * 216 + tau * 216) + 2 * 216, ms)
    psi = torch.empty((K, N), dtype=torch.complex128, device="cuda")
    fin = torch.empty((N,), dtype=torch.complex128, device="cuda")
    ws = native.alloc_workspace(native.propagate_workspace_size(prob.spin_twice, K))
    native.integrate(prob, params, U, stream=stream)
    native.propagate(prob.spin_twice, U, native.device_state(prob.psi0), psi, fin, ws,
                     stream=stream)
    ms = timed(lambda: native.spin_projection(psi, stream=stream))
    gbs = K * (16 * N + 24) / (ms * 1e-3) / 1e9  # read the state, write <J_x>, <J_y>, <J_z>
    psi0 = native.device_state(prob.psi0)
    spin = torch.empty((K, 3), dtype=torch.float64, device="cuda")
    ms_scan = timed(lambda: native.propagate(prob.spin_twice, U, psi0, psi, fin, ws,
                                             stream=stream))
    ms_fused = timed(lambda: native.propagate(prob.spin_twice, U, psi0, psi, fin, ws,
                                              stream=stream, spin=spin))
    out["f1_spin_projection"] = {"states_per_s": round(K / (ms * 1e-3), 1), "ms": round(ms, 4),
                                 "roofline": {"bound": "hbm", "achieved": round(gbs, 1),
                                              "peak": 8000.0, "unit": "GB/s",
                                              "frac": round(gbs / 8000.0, 4)},
                                 # the scan alone, then with <J> formed in its last pass
                                 "scan_ms": round(ms_scan, 4),
                                 "scan_with_spin_ms": round(ms_fused, 4)}
    del U, psi, ws, spin
    torch.cuda.empty_cache()
    return out


ACCURACY_FINE_STEPS = (1, 2, 5, 10, 20, 50, 100)  # fine steps per 0.5 us sample


def accuracy_study(ref_fine: int = 500, reps: int = 3) -> dict:
    """The paper's accuracy benchmark (Sec. "Evaluation of accuracy") on
    the GPU: the 0.1 s sensing drive with its 1 ms pulse (2e5 samples of
    0.5 us), spin-1 and spin-1/2, CF4, midpoint and Heun sampling with the
    rotating frame on ("frame") and off ("lab"), over a range of fine steps.
    Each point is [dt in ns, ms per simulation (integrator with the field
    compiled in + scan, inputs resident, HIP events), error of eq. (error)
    against CF4 with the frame at ref_fine fine steps per sample].  The
    paper counts errors above 1e-3 as failures and floors its baseline at
    1e-11."""
    import numpy as np
    import torch
    from paper_2204_05586_amd import native, workloads as W
    stream = torch.cuda.current_stream()
    out = {"reference": f"CF4, rotating frame, {ref_fine} fine steps per sample"}
    for spin_twice in (2, 1):
        base = W.spin_one_sensing()
        if spin_twice == 1:
            base = base.replace(spin_twice=1, psi0=None,
                                terms=[t for t in base.terms if t.comp != W.Q])
        K, N = base.n_samples, base.dim
        smp = native.Sampler.for_terms(base.terms)
        params = native.device_params(base)
        psi0 = native.device_state(base.psi0)
        U = torch.empty((K, N, N), dtype=torch.complex128, device="cuda")
        ws = native.alloc_workspace(native.propagate_workspace_size(spin_twice, K))

        def run(prob, psi):
            smp.integrate(prob.replace(terms=[]), params, U, stream=stream)
            native.propagate(spin_twice, U, psi0, psi, None, ws, stream=stream)

        ref = torch.empty((K, N), dtype=torch.complex128, device="cuda")
        run(base.replace(n_fine=ref_fine), ref)
        psi = torch.empty_like(ref)
        # 0.2 s of work first: the compile above left the GPU idle, its clock low
        t_warm = time.perf_counter()
        while time.perf_counter() - t_warm < 0.2:
            run(base, psi)
            torch.cuda.synchronize()
        series = {}
        for mname, method in (("cf4", W.CF4), ("midpoint", W.MIDPOINT), ("heun", W.HEUN)):
            for frame in (True, False):
                pts = []
                for L in ACCURACY_FINE_STEPS:
                    p = base.replace(n_fine=L, method=method, rotating_frame=frame)
                    run(p, psi)
                    torch.cuda.synchronize()
                    a = torch.cuda.Event(enable_timing=True)
                    b = torch.cuda.Event(enable_timing=True)
                    a.record(stream)
                    for _ in range(reps):
                        run(p, psi)
                    b.record(stream)
                    torch.cuda.synchronize()
                    err = float(torch.sqrt((psi - ref).abs().square().sum())) / K
                    pts.append([round(base.dt_out / L * 1e9, 3),
                                round(a.elapsed_time(b) / reps, 4), float(f"{err:.3e}")])
                series[f"{mname}_{'frame' if frame else 'lab'}"] = pts
        out["spin_one" if spin_twice == 2 else "spin_half"] = series
        smp.close()
        del U, ws, ref, psi
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batched_sensing",
                    choices=["batched_sensing", "spin_one_sensing", "spin_half_rabi"])
    ap.add_argument("--n-sims", type=int, default=4096, help="batch size of batched_sensing")
    ap.add_argument("--plain-steps", type=int, default=200)
    ap.add_argument("--no-tune", action="store_true", help="planner defaults, no autotuning")
    ap.add_argument("--interpret", action="store_true",
                    help="interpret the field program instead of compiling it into the integrator")
    ap.add_argument("--cpu-baseline-seconds", type=float, default=10.0,
                    help="target CPU seconds of the oracle sample (0: skip)")
    ap.add_argument("--serve-rates", default="10,30,100,300,1000",
                    help="request rates (req/s) of the serving sweep, '' to skip")
    ap.add_argument("--serve-burst", type=int, default=300,
                    help="requests submitted at once to measure the server's capacity (0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=6.0,
                    help="target stream length per rate (requests = rate x seconds, "
                         "600 <= requests <= 2000)")
    ap.add_argument("--adjoint-instances", type=int, default=1024,
                    help="instances of the control-gradient workload (0: skip)")
    ap.add_argument("--no-next-rows", action="store_true",
                    help="skip the f1-f4 measurements (spin projection, Euler samplings, "
                         "user sampler, full su(3) basis)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one device copy of this size (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU only; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2204_05586_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.init()
    src_hash = kernel_source_hash()

    if args.workload == "batched_sensing":
        problems = W.batched_sensing(seed=2, n_sims=args.n_sims)
        tau = problems[0].n_squares
        res = bench_batched(problems, args.steps, args.warmup, not args.no_tune,
                            not args.interpret)
        kernel = "mss_user_work_chained" if res["specialized"] else "work_chained_kernel"
        plain = (bench_plain(W.spin_one_sensing(), args.plain_steps, 3, not args.interpret)
                 if args.plain_steps > 0 else None)
        # the spin-1/2 Rabi simulation (1e4 samples x 100 fine steps) the same way
        plain_half = (bench_plain(W.spin_half_rabi(), args.plain_steps, 3, not args.interpret)
                      if args.plain_steps > 0 else None)
        value, ms, integ_ms, fine = res["value"], res["ms_per_step"], res["replay_ms_mean"], \
            res["fine_steps"]
        intervals = res["info"]["total_samples"]
        sep = res["separate_scan"]
        config = {"workload": f"batched_sensing: {len(problems)} spin-1 simulations, seed 2, "
                              f"durations U(10,100) ms, dt_out 5e-7 s",
                  "mode": ("one captured HIP graph of the chained persistent integrator (field "
                           "program " + ("compiled in" if res["specialized"] else "interpreted")
                           + "), states formed in the same launch; replays timed"),
                  "compile_s": round(res["compile_s"], 2),
                  "n_sims": len(problems), "total_intervals": intervals,
                  "n_fine": 10, "fine_steps": fine, "n_squares": tau, "rotating_frame": True,
                  "work_items": res["info"]["n_items"], "grid_blocks": res["info"]["grid_blocks"],
                  "autotuned": res["options"], "autotune_s": round(res["tune_s"], 2),
                  "workspace_bytes": res["workspace_bytes"]}
        extra = {"replay_ms_mean": round(res["replay_ms_mean"], 3),
                 "replay_ms_median": round(res["replay_ms_median"], 3),
                 "replay_ms_min": round(res["replay_ms_min"], 3),
                 "replay_ms_max": round(res["replay_ms_max"], 3),
                 "d2h": res["d2h"],
                 "separate_scan": {k: (round(v, 3) if isinstance(v, float) and k.endswith("ms")
                                       else v) for k, v in sep.items()},
                 "integrate_ms_interpreter": round(res["integrate_ms_interpreter"], 3),
                 "plain": ({k: (round(v, 4) if isinstance(v, float) else v)
                            for k, v in plain.items()} if plain else None),
                 "batched_over_plain": round(value / plain["value"], 3) if plain else None,
                 "plain_spin_half": ({k: (round(v, 4) if isinstance(v, float) else v)
                                      for k, v in plain_half.items() if k != "tau"}
                                     if plain_half else None)}
        base_problems = problems
    else:
        prob = W.spin_one_sensing() if args.workload == "spin_one_sensing" else W.spin_half_rabi()
        tau = prob.n_squares
        res = bench_plain(prob, args.steps, args.warmup, not args.interpret)
        n = prob.spin_twice + 1
        kernel = (f"mss_user_integrate_{n}" if res["field"] == "compiled in"
                  else f"integrate_kernel<{n}>")
        value, ms, integ_ms, fine = res["value"], res["ms_per_step"], res["integrate_ms"], \
            res["fine_steps"]
        config = {"workload": prob.name,
                  "mode": f"plain (one simulation per launch sequence, field program {res['field']})",
                  "n_samples": prob.n_samples, "n_fine": prob.n_fine, "fine_steps": fine,
                  "n_squares": tau, "rotating_frame": prob.rotating_frame,
                  "launch": res["launch"]}
        extra = {"integrate_ms_mean": round(integ_ms, 4),
                 "integrate_ms_interpreter": round(res["integrate_ms_interpreter"], 4),
                 "propagate_ms_mean": round(res["propagate_ms"], 4)}
        base_problems = [prob]

    roofline = None
    if args.workload != "spin_half_rabi":
        flops = spin_one_flops_per_fine_step(tau) * fine
        if args.workload == "batched_sensing":
            flops += STATE_UPDATE_FLOPS * intervals  # the states, formed in the same launch
        achieved = flops / (integ_ms * 1e-3) / 1e12
        traffic = MEASURED_TRAFFIC.get((kernel, args.workload))
        roofline = {"bound": "alu", "achieved": round(achieved, 3),
                    "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(achieved / FP64_VECTOR_PEAK_TFLOPS, 4),
                    "traffic": (traffic["bytes"] if traffic and traffic["src"] == src_hash
                                else None),
                    "kernel": kernel, "flops_per_launch": flops,
                    "kernel_ms_mean": round(integ_ms, 4)}

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    next_rows = None
    if not args.no_next_rows and args.plain_steps > 0:
        next_rows = bench_next_rows()
        next_rows["f2_accuracy"] = accuracy_study()

    adjoint = None
    if args.adjoint_instances > 0:
        adjoint = bench_adjoint(args.adjoint_instances, 3, 1, not args.interpret)

    serving = None
    if args.serve_rates:
        rates = [float(x) for x in args.serve_rates.split(",") if x]
        serving = bench_serving(rates, args.serve_seconds, 2000, budget_gib=64.0,
                                burst=args.serve_burst)

    base = (cpu_baseline(base_problems, args.cpu_baseline_seconds)
            if args.cpu_baseline_seconds > 0 else None)
    if base is not None and serving is not None:
        base["serving"] = cpu_serving_baseline(args.cpu_baseline_seconds / 3)

    out = {
        "metric": "CF4 fine steps/sec (spin-1, FP64) batched vs plain on 1 GPU; p50/p99 latency",
        "value": round(value, 1),
        "unit": "fine_steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": config,
        **extra,
        "latency": serving,
        "adjoint": adjoint,
        "next_rows": next_rows,
        "roofline": roofline,
        "cpu_baseline": base,
        "paper_context": PAPER_CONTEXT,
        "kernel_src": src_hash,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
