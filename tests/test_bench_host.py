"""Host-side parts of the benchmark on the CPU: the one-GPU refusal, and the
oracle baseline whose multi-threaded leg must reproduce the single-thread
integer sums exactly (the sums over sampled edges are order-independent)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.mark.parametrize("n", [0, 2, 8])
def test_bench_refuses_other_gpu_counts(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_cpu_baseline_threads_reproduce_single_thread_sums():
    import bench
    from paper_1701_01772_amd import inputs
    g = inputs.er_2000()
    out = bench.cpu_baseline(g, 0.5, 11, target_s=0.2)
    assert out["kind"] == "oracle" and out["cores"] == 1 and out["value"] > 0
    mt = out["all_cores"]
    assert mt["cores"] >= 1 and mt["value"] > 0
    assert mt["sums_match_single_thread"] is True
