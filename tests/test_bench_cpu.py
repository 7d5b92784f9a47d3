"""bench.py's contract pieces that need no GPU: one-GPU scope, the
algorithmic flop count it prices the integrator with, and the traffic
table's keys."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout.strip()


def test_flops_per_fine_step():
    """Two exponentials of tau symmetric squarings (6 entries: 3 complex
    squares, 3 diagonal and 3 off-diagonal updates = 96 flops) and two
    27-multiply-add complex products (216 flops each)."""
    adds = 3                      # b_j = x_jj + 2
    squares = 3 * (3 + 2)         # x_jk^2: re = fma(x, x, -y * y), im = 2 x y (mul, add)
    diag = 3 * (2 + 4 + 4)        # the two squares summed, re and im: two fma each
    off = 3 * (2 + 7 + 7)         # c = b_j + x_kk, re and im: mul + 3 fma
    per_square = adds + squares + diag + off
    assert per_square == 96
    for tau in (0, 1, 24, 28):
        assert bench.spin_one_flops_per_fine_step(tau) == 2 * tau * per_square + 2 * 216


def test_traffic_table_names_kernels_the_bench_reports():
    for (kernel, workload), v in bench.MEASURED_TRAFFIC.items():
        assert kernel in ("mss_user_work_chained", "mss_user_work_integrate",
                          "work_integrate_kernel")
        assert workload == "batched_sensing"
        assert v["bytes"] == int(round((v["fetch_kib"] * 2.0 + v["write_kib"]) * 1024))
        assert len(v["src"]) == 16


def test_cpu_serving_baseline_solves_the_request_stream_in_order():
    """The oracle's serving sample: the 10 req/s stream's requests from the
    first, one after another, until the time bound passes."""
    from paper_2204_05586_amd import workloads as W
    r = bench.cpu_serving_baseline(0.05)
    first = W.serving_stream(10.0, n_requests=600, rate_index=0)[0].problem.fine_steps
    assert r["kind"] == "oracle" and r["unit"] == "fine_steps/s" and r["value"] > 0
    assert r["sample"].startswith("the first 1 of the 10 req/s stream's 600 requests")
    assert f"({first} fine steps" in r["sample"]
