"""Autotuner of the batched path.

Picks, for a batch of simulations, the launch options of ``BatchPlan``:
lane-slices per interval for each spin class (how many lanes share one
interval's fine steps), the persistent integrator's resident waves per SIMD
(grid size), and the scan tile (operators per lane, tile = 64 x that).  It
times trial runs on a strided sample of the batch (coordinate descent:
integrator options on integrator-only launches, then the scan tile on
scan-only launches, each the median of a few HIP-event-timed repetitions)
and caches the winner on disk, keyed by GPU architecture and the batch's
shape (spins, squaring counts, fine steps per interval, frame, and the
total interval count rounded to a power of two).
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import statistics
from typing import Dict, List, Optional

from . import native

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "mss_autotune.json")


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{getattr(p, 'gcnArchName', p.name)}:{p.multi_processor_count}cu"


def _sampler_id(sampler) -> Optional[str]:
    """Cache identity of a sampler: a hash of its source, or of the term
    list it was compiled from."""
    if sampler is None:
        return None
    if sampler.source is not None:
        return hashlib.sha256(sampler.source.encode()).hexdigest()[:16]
    return "terms:" + hashlib.sha256(repr(native._terms_key(sampler.terms)).encode()).hexdigest()[:16]


def shape_key(problems, sampler=None) -> str:
    spins = sorted({p.spin_twice for p in problems})
    taus = sorted({p.n_squares for p in problems if p.spin_twice == 2})
    fines = sorted({p.n_fine for p in problems})
    frames = sorted({bool(p.rotating_frame) for p in problems})
    total = sum(p.n_samples for p in problems)
    return json.dumps({"arch": _arch(), "spins": spins, "taus": taus, "fines": fines,
                       "frames": frames, "intervals_log2": int(round(math.log2(max(total, 1)))),
                       "sampler": _sampler_id(sampler)},
                      sort_keys=True)


def sample(problems, target_fine_steps: float = 2e8) -> list:
    """Every j-th simulation, j chosen so the sample holds about
    target_fine_steps fine steps (all of them if the batch is smaller)."""
    total = sum(p.fine_steps for p in problems)
    stride = max(1, int(total // max(target_fine_steps, 1.0)))
    return list(problems)[::stride]


def _time(plan: "native.BatchPlan", bufs: dict, what: str, reps: int) -> float:
    import torch
    stream = torch.cuda.current_stream()
    call = plan.integrate if what == "integrate" else plan.propagate
    if what == "propagate":
        plan.integrate(bufs, stream=stream)
    call(bufs, stream=stream)  # warm-up
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        call(bufs, stream=stream)
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b))
    return statistics.median(times)


def tune(problems, cache_path: Optional[str] = DEFAULT_CACHE, reps: int = 3,
         target_fine_steps: float = 2e8, verbose: bool = False,
         sampler: "Optional[native.Sampler]" = None,
         specialize: bool = False) -> Dict[str, int]:
    """Options for BatchPlan(problems, **options), tuned (or read from the cache).
    With a sampler the trials run its integrator and the cache key includes
    a hash of its source.  specialize: tune the plan BatchPlan(problems,
    specialize=True) makes (the shared field program compiled into its own
    integrator), when the problems share one term list."""
    if specialize and sampler is None:
        sp = native.specialise(problems)
        if sp is not None:
            try:
                return tune(sp[1], cache_path, reps, target_fine_steps, verbose, sampler=sp[0])
            finally:
                sp[0].close()
    key = shape_key(problems, sampler)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if key in cache:
        return dict(cache[key]["options"])
    smp = sample(problems, target_fine_steps)
    has_half = any(p.spin_twice == 1 for p in smp)
    has_one = any(p.spin_twice == 2 for p in smp)
    min_l = min(p.n_fine for p in smp)
    slices_one = [s for s in (1, 2, 4) if s <= min_l] if has_one else [0]
    slices_half = [s for s in (1, 4, 16) if s <= min_l] if has_half else [0]
    trials: List[dict] = []

    def run(opts: dict, what: str) -> float:
        plan = native.BatchPlan(smp, sampler=sampler, **opts)
        bufs = plan.allocate(store_u=False)
        ms = _time(plan, bufs, what, reps)
        plan.close()
        trials.append({"options": dict(opts), "what": what, "ms": ms})
        if verbose:
            print(f"autotune {what} {opts}: {ms:.3f} ms", flush=True)
        return ms

    best, best_ms = None, float("inf")
    for s1 in slices_one:
        for sh in slices_half:
            for wps in (1, 2, 4):
                opts = {"slices_spin_one": s1, "slices_spin_half": sh, "waves_per_simd": wps,
                        "scan_per_lane": 4}
                ms = run(opts, "integrate")
                if ms < best_ms:
                    best, best_ms = opts, ms
    scan_best, scan_ms = 4, float("inf")
    for e in (2, 4, 8):
        ms = run({**best, "scan_per_lane": e}, "propagate")
        if ms < scan_ms:
            scan_best, scan_ms = e, ms
    best = {**best, "scan_per_lane": scan_best}
    if cache_path:
        cache[key] = {"options": best, "trials": trials, "sample_sims": len(smp)}
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, cache_path)
    return best


def tuned_plan(problems, use_graph: bool = False, sampler=None, specialize: bool = False,
               **kw) -> "native.BatchPlan":
    opts = tune(problems, sampler=sampler, specialize=specialize, **kw)
    return native.BatchPlan(problems, use_graph=use_graph, sampler=sampler,
                            specialize=specialize, **opts)
