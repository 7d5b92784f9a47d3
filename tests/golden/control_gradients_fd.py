"""Writes control_gradients_fd.txt: central differences of the control
workload's loss in x87 extended precision, computed by the oracle only.

Workload: the differentiation batch (1024 spin-1 instances, 256 segments of
a resonant drive with amplitude A_s and phase phi_s, 1 ms, 1e5 CF4 steps,
tau = 28, frame on, loss = population of |0>; drawn by
workloads.control_batch(seed=4)).  Eight instances are picked with
numpy.random.default_rng(2045); in each, 16 amplitude and 16 phase slots are
picked with the same generator.  A ninth case is instance 0 with the
amplitude of every fourth segment set to 0 (segments without a transverse
field, the usual starting point of a control optimisation), differentiated at
16 zeroed amplitudes, the phases of 8 of those segments (derivative 0) and 8
other amplitudes.

Each value is (loss(p + h e_q) - loss(p - h e_q)) / 2h with
h = 1e-6 * max(1, |p_q|), both losses from the oracle's extended-precision
forward map.  Run from the repository root:
    python tests/golden/control_gradients_fd.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle  # noqa: E402
from paper_2204_05586_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "control_gradients_fd.txt")
M = 1  # loss = |psi_final[m]|^2, m = 1 is |0>
H_REL = 1e-6


def cases():
    """[(label, instance index, params, slots)] in a fixed order."""
    probs = W.control_batch(seed=4)
    n_seg = W.N_SEGMENTS
    rng = np.random.default_rng(2045)
    out = []
    for i in sorted(rng.choice(len(probs), 8, replace=False)):
        slots = np.concatenate([np.sort(rng.choice(n_seg, 16, replace=False)),
                                n_seg + np.sort(rng.choice(n_seg, 16, replace=False))])
        out.append(("drawn", int(i), probs[i].params.copy(), slots))
    p = probs[0].params.copy()
    zero = np.arange(0, n_seg, 4)
    p[zero] = 0.0
    slots = np.concatenate([zero[:16], n_seg + zero[:8], np.arange(1, n_seg, 32)])
    out.append(("zeroed", 0, p, np.sort(slots)))
    return probs, out


def central_difference(prob, params, q):
    p = np.asarray(params, dtype=np.longdouble)
    h = np.longdouble(H_REL) * max(np.longdouble(1.0), abs(p[q]))
    pp, pm = p.copy(), p.copy()
    pp[q] += h
    pm[q] -= h
    return float((oracle.population_ld(prob, M, pp) - oracle.population_ld(prob, M, pm)) / (2 * h))


def main():
    probs, cs = cases()
    t0 = time.time()
    lines = [line.rstrip() for line in __doc__.strip().splitlines()]
    rows = ["# " + line if line else "#" for line in lines]
    rows.append("# columns: case label, instance, slot, parameter value, d loss / d parameter")
    for label, i, params, slots in cs:
        prob = probs[i].replace(params=params)
        for q in slots:
            fd = central_difference(prob, params, int(q))
            rows.append(f"{label} {i} {int(q)} {float(params[q])!r} {fd!r}")
        print(f"{label} {i}: {len(slots)} slots, {time.time() - t0:.0f} s", flush=True)
    with open(OUT, "w") as f:
        f.write("\n".join(rows) + "\n")


if __name__ == "__main__":
    main()
