#!/usr/bin/env python3
"""Throughput benchmark of the solver path on one MI355X.

One step = the whole path over one simulation: the integrator (interval
operators U_k from CF4 fine steps in the rotating frame, frame exit) and the
ordered product (states psi_k), both through the C ABI.  Inputs and outputs
stay resident in HBM; the timed region starts after they are allocated.

Prints one JSON line: CF4 fine steps/s, the integrator's roofline figures
(algorithmic FP64 flops / measured kernel time vs the 78.6 TFLOP/s FP64
vector peak) and the CPU oracle's rate on a bounded sample.
"""
import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6  # 256 CU x 2.4 GHz x 128 FP64 flop/clk


def spin_one_flops_per_fine_step(tau: int) -> int:
    """Algorithmic FP64 flops of one spin-1 CF4 fine step: two Lie-Trotter
    exponentials of tau residual squarings (27 complex multiply-adds = 216
    flops each) plus two 3x3 complex products into the interval operator."""
    return 2 * tau * 216 + 2 * 216


def make_workload(name: str):
    from paper_2204_05586_amd import workloads as W
    if name == "spin_one_sensing":
        return W.spin_one_sensing()
    if name == "spin_half_rabi":
        return W.spin_half_rabi()
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(prob, seconds: float) -> dict:
    """The CPU oracle on a bounded prefix of the same simulation."""
    from oracle import oracle
    threads = oracle.get_threads()
    k = min(prob.n_samples, 2000)
    t0 = time.perf_counter()
    oracle.solve(prob.replace(n_samples=k))
    dt = time.perf_counter() - t0
    k = int(min(prob.n_samples, max(k, k * seconds / max(dt, 1e-6))))
    sample = prob.replace(n_samples=k)
    t0 = time.perf_counter()
    oracle.solve(sample)
    dt = time.perf_counter() - t0
    return {"value": sample.fine_steps / dt, "unit": "fine_steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {k} of {prob.n_samples} intervals of {prob.name} "
                      f"({sample.fine_steps} fine steps, {dt:.1f} s, {threads} threads)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="spin_one_sensing")
    ap.add_argument("--cpu-baseline-seconds", type=float, default=10.0,
                    help="target CPU seconds of the oracle sample (0: skip)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one device copy of this size (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU only (single-GPU solver path); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2204_05586_amd import native

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    prob = make_workload(args.workload)
    K, N, L = prob.n_samples, prob.dim, prob.n_fine
    dev = "cuda"
    params = native.device_params(prob, dev)
    psi0 = native.device_state(prob.psi0, dev)
    U = torch.empty((K, N, N), dtype=torch.complex128, device=dev)
    psi = torch.empty((K, N), dtype=torch.complex128, device=dev)
    fin = torch.empty((N,), dtype=torch.complex128, device=dev)
    ws = native.alloc_workspace(native.propagate_workspace_size(prob.spin_twice, K), dev)
    launch = native.plan_launch(prob)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        native.integrate(prob, params, U, launch=launch, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        native.propagate(prob.spin_twice, U, psi0, psi, fin, ws, stream=stream)
        if ev is not None:
            ev[2].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(events[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    integ_ms = [e[0].elapsed_time(e[1]) for e in events]
    prop_ms = [e[1].elapsed_time(e[2]) for e in events]
    fine_steps = prob.fine_steps
    value = fine_steps * args.steps / wall

    roofline = None
    if prob.spin_twice == 2:
        flops = spin_one_flops_per_fine_step(prob.n_squares) * fine_steps
        achieved = flops / (statistics.mean(integ_ms) * 1e-3) / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 3),
                    "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(achieved / FP64_VECTOR_PEAK_TFLOPS, 4), "traffic": None,
                    "kernel": "integrate_kernel<3>",
                    "flops_per_launch": flops,
                    "kernel_ms_mean": round(statistics.mean(integ_ms), 4)}

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    base = cpu_baseline(prob, args.cpu_baseline_seconds) if args.cpu_baseline_seconds > 0 else None

    out = {
        "metric": "CF4 fine steps/sec (spin-1, FP64) batched vs plain on 1 GPU; p50/p99 latency",
        "value": round(value, 1),
        "unit": "fine_steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": prob.name, "mode": "plain (one simulation per launch sequence)",
                   "spin": "1" if prob.spin_twice == 2 else "1/2", "n_samples": K,
                   "n_fine": L, "fine_steps": fine_steps, "n_squares": prob.n_squares,
                   "rotating_frame": prob.rotating_frame, "launch": {"slices": launch[0],
                                                                      "block": launch[1]}},
        "integrate_ms_mean": round(statistics.mean(integ_ms), 4),
        "propagate_ms_mean": round(statistics.mean(prop_ms), 4),
        "roofline": roofline,
        "cpu_baseline": base,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
