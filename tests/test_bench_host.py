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


def _timing(count_ms, words, alg):
    return {"count_ms": count_ms, "words_read": words, "alg_bytes": alg, "sample_ms": 0.5,
            "global_prep_ms": 1.0}


def test_roofline_takes_the_dominant_kernel_and_its_bytes():
    import bench
    tim = [_timing([2.0, 1.0, 4.0], [10, 20, 1000], [1e9, 2e9, 8e9]),
           _timing([2.0, 1.0, 6.0], [10, 20, 3000], [1e9, 2e9, 8e9])]
    dev, roof = bench.roofline_of(tim, "no_such_workload")
    assert dev["count_global"] == 5.0 and dev["count_wave"] == 2.0 and dev["global_prep"] == 1.0
    assert roof["kernel"].startswith("k_count_global")
    assert roof["launch_ms"] == 5.0
    # achieved: the 4-byte words the kernel read, per launch, over the launch time
    assert roof["bytes_per_launch"] == 4.0 * 2000
    assert roof["achieved"] == 4.0 * 2000 / 5e-3 / 1e9  # GB/s
    assert roof["frac"] == roof["achieved"] / 8000.0
    # effective: the neighbour-iteration bytes of the same launch
    assert roof["effective"]["bytes_per_launch"] == 8e9
    assert roof["effective"]["GBps"] == 8e9 / 5e-3 / 1e9
    assert roof["traffic"] is None  # no counter profile for this workload


def test_roofline_traffic_only_from_a_profile_of_the_same_source():
    import json
    import bench
    for wl in ("chung_lu", "rmat"):
        with open(os.path.join(ROOT, "profiles", "pmc_%s_p0.1_global.json" % wl)) as fh:
            pmc = json.load(fh)
        tim = [_timing([1.0, 1.0, 3.0], [0, 0, 0], [0, 0, 1e9])]
        _, roof = bench.roofline_of(tim, wl, pmc["p"])
        if pmc["kernel_hash"] == bench.kernel_source_hash():
            assert roof["traffic"] == pmc["traffic_bytes_per_launch"]
        else:
            assert roof["traffic"] is None
        # a profile taken at another sampling probability is not used (none
        # is committed at p / 3)
        _, other = bench.roofline_of(tim, wl, pmc["p"] / 3)
        assert other["traffic"] is None


def test_tune_report_times_tuned_and_default_options_alike(monkeypatch):
    # a stand-in for the library: lge_autotune returns fixed options, and an
    # estimate "takes" 2 ms with them and 3 ms with the defaults (opts None);
    # the report must time both with the same steps and seeds and compare
    # the per-step times, the tuning time kept apart
    import types
    import bench
    calls = []

    class R:
        sampled_edges = 100

    def est(ctx, h, p, seed, opts=None, raw=False, out=None):
        calls.append((seed, opts))
        bench.time.sleep(0.002 if opts is not None else 0.003)
        return R()

    fake = types.SimpleNamespace(
        Result=R, lge_estimate=est, lge_last_timing=lambda ctx: {},
        lge_autotune=lambda ctx, h, p: {"probe_ratio": 8},
        opts_dict=lambda o: dict(o))
    import torch  # time_steps brackets the steps with device synchronisations
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    rep = bench.tune_report(fake, None, None, 0.1, 500, 5)
    assert rep["options"] == {"probe_ratio": 8}
    assert [s for s, o in calls if o is not None] == [500 + i for i in range(5)]
    assert [s for s, o in calls if o is None] == [500 + i for i in range(5)]
    assert rep["tuned_ms_per_step"] < rep["default_ms_per_step"]
    assert rep["tuned_vs_default"] == rep["default_ms_per_step"] / rep["tuned_ms_per_step"]
    assert rep["seconds"] >= 0.0
