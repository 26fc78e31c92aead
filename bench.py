"""Benchmark of the sampled-edge graphlet estimator on one MI355X.

A step is one full estimate (sample -> bin -> count -> reduce -> FP64
finalise) on a graph resident in HBM.  Default workload: Chung-Lu power law,
n = 1,000,000, mean expected degree 16, exponent 2.1, degree cap 50,000,
p = 0.1.  Prints one JSON line with the throughput in sampled edges/s, the
roofline of the dominant counting kernel (device time from HIP events the
library records on its own stream), and the CPU oracle timed on a bounded
subsample of the same workload on this host.

    python bench.py [--steps K] [--warmup W] [--workload chung_lu|rmat|er|batch|serve|micro|designs] [--p P]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(msg):
    sys.stderr.write("[bench] %s\n" % msg)
    sys.stderr.flush()


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("lge_kernels.hip", "lge_internal.h", "lge_host.cpp"):
        with open(os.path.join(ROOT, "paper_1701_01772_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def make_workload(name):
    from paper_1701_01772_amd import inputs
    if name == "chung_lu":
        return inputs.chung_lu_1m(), "chung_lu_n1e6_d16_g2.1_cap5e4"
    if name == "rmat":
        return inputs.rmat_22(), "rmat_s22_ef16_a.57_b.19_c.19"
    if name == "er":
        return inputs.er_2000(), "erdos_renyi_n2000_q0.005"
    raise SystemExit("unknown workload %s" % name)


CLASS_KERNELS = ["k_count_lds<64,128> (wavefront per edge)", "k_count_lds<256,1024> (workgroup per edge)",
                 "k_count_global (split hub edges)"]


def cpu_baseline(g, p, seed, target_s=15.0):
    """The oracle, untuned, on every K-th sampled edge of the same workload."""
    import numpy as np
    import oracle
    mask_all = oracle.sample_mask(seed, p, g.m)
    sampled_ids = np.nonzero(mask_all)[0]
    if sampled_ids.size == 0:
        return None
    stride = max(1, sampled_ids.size // 64)
    while True:
        sub = sampled_ids[::stride]
        mask = np.zeros(g.m, dtype=np.uint8)
        mask[sub] = 1
        t0 = time.perf_counter()
        r = oracle.estimate(g.row_ptr, g.col, p, seed, mask=mask)
        dt = time.perf_counter() - t0
        if dt >= target_s * 0.5 or stride == 1:
            break
        stride = max(1, int(stride * dt / target_s))
    out = {"value": r["sampled"] / dt, "unit": "sampled edges/s", "cores": 1, "kind": "oracle",
           "sample": "every %d-th of the %d Philox-sampled edges (%d edges, %.1f s)" % (
               stride, sampled_ids.size, r["sampled"], dt),
           "host_cpus": os.cpu_count(), "host_cpu_model": host_cpu_model()}
    out["all_cores"] = cpu_baseline_threads(g, p, seed, sub, r)
    return out


def cpu_baseline_threads(g, p, seed, sub, whole):
    """The same oracle call on the same sample, split round-robin over one
    thread per usable host core (the C oracle is reentrant and ctypes drops
    the GIL during the call).  The per-thread integer sums must add up to the
    single-thread ones exactly, since the sums are order-independent."""
    import numpy as np
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        threads = os.cpu_count() or 1
    threads = max(1, min(threads, 16, sub.size))
    masks = []
    for i in range(threads):
        mk = np.zeros(g.m, dtype=np.uint8)
        mk[sub[i::threads]] = 1
        masks.append(mk)
    with ThreadPoolExecutor(max_workers=threads) as pool:
        t0 = time.perf_counter()
        parts = list(pool.map(lambda mk: oracle.estimate(g.row_ptr, g.col, p, seed, mask=mk), masks))
        dt = time.perf_counter() - t0
    sampled = sum(x["sampled"] for x in parts)
    same = sampled == whole["sampled"] and all(
        sum(x[k][i] for x in parts) == whole[k][i] for k in ("csum", "qsum") for i in range(18))
    return {"value": sampled / dt, "unit": "sampled edges/s", "cores": threads,
            "seconds": round(dt, 3), "sums_match_single_thread": bool(same)}


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def roofline_of(tim, workload):
    """Roofline of the dominant counting kernel.  achieved = the neighbour-
    iteration bytes of the sampled edges it counts (per edge
    16 + 4(d_u + d_v) + sum over w in Gamma(a)\\{b} of (8 + 4 d_w), summed by
    the sampling kernel) / its mean launch time; the kernel's tables let it
    read far fewer bytes, so this "effective" figure can exceed the HBM peak.
    traffic = HBM-side bytes per launch from the committed rocprofv3 counter
    profile of the same kernel source (null when the source has changed)."""
    k = len(tim)
    cnt_ms = [sum(t["count_ms"][c] for t in tim) / k for c in range(3)]
    words = [sum(t["words_read"][c] for t in tim) / k for c in range(3)]
    alg = [sum(t["alg_bytes"][c] for t in tim) / k for c in range(3)]
    dom = max(range(3), key=lambda c: cnt_ms[c])
    sec = cnt_ms[dom] * 1e-3
    achieved = alg[dom] / sec / 1e9 if sec > 0 else 0.0
    traffic = None
    pmc_path = os.path.join(ROOT, "profiles", "pmc_%s_%s.json" % (workload, ["wave", "block", "global"][dom]))
    if os.path.exists(pmc_path):
        with open(pmc_path) as fh:
            pmc = json.load(fh)
        if pmc.get("kernel_hash") == kernel_source_hash():
            traffic = pmc.get("traffic_bytes_per_launch")
    device_ms = {"sample_bin": sum(t["sample_ms"] for t in tim) / k, "count_wave": cnt_ms[0],
                 "count_block": cnt_ms[1], "global_prep": sum(t["global_prep_ms"] for t in tim) / k,
                 "count_global": cnt_ms[2]}
    roof = {"bound": "hbm", "kernel": CLASS_KERNELS[dom], "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "algorithmic_bytes_per_launch": alg[dom], "issued_bytes_per_launch": 4.0 * words[dom],
            "launch_ms": cnt_ms[dom]}
    if traffic is not None and sec > 0:
        roof["traffic_GBps"] = traffic / sec / 1e9
        roof["traffic_frac"] = traffic / sec / 1e9 / HBM_PEAK_GBS
    return device_ms, roof


def bench_batch(args):
    """4096 small graphs: one lge_estimate_many launch sequence per step vs
    one lge_estimate per graph (the plain path), graphs resident."""
    import torch
    from paper_1701_01772_amd import inputs, lge
    log("generating 4096 graphs")
    graphs = inputs.batch_graphs(4096, 4096)
    tot_m = sum(g.m for g in graphs)
    log("batch: %d graphs, %d vertices, %d edges" % (len(graphs), sum(g.n for g in graphs), tot_m))
    ctx = lge.lge_open(0)
    hs = [lge.lge_graph_create_host(ctx, g.row_ptr, g.col) for g in graphs]
    seeds = [args.seed + i for i in range(len(hs))]
    p = args.p if args.p is not None else 1.0
    lge.lge_estimate_many(ctx, hs, p, seeds)
    for h in hs[:64]:
        lge.lge_estimate(ctx, h, p, 1)
    torch.cuda.synchronize()
    # plain path: one estimate (one launch sequence) per graph; both legs
    # keep the library's result structs (no conversion to Python numbers)
    res = lge.Result()
    t0 = time.perf_counter()
    plain_sampled = 0
    for h, sd in zip(hs, seeds):
        plain_sampled += lge.lge_estimate(ctx, h, p, sd, raw=True, out=res).sampled_edges
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    log("plain: %.3f s" % t_plain)
    sampled = 0
    tim = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        outs = lge.lge_estimate_many(ctx, hs, p, seeds, raw=True)
        sampled += sum(outs[k].sampled_edges for k in range(len(hs)))
        tim.append(lge.lge_last_timing(ctx))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log("batched: %d steps in %.3f s" % (args.steps, dt))
    # end-to-end from host arrays (union upload + preprocessing + one launch)
    t0 = time.perf_counter()
    lge.lge_count_batch(ctx, [(g.row_ptr, g.col) for g in graphs], p, seeds)
    t_e2e = time.perf_counter() - t0
    for h in hs:
        lge.lge_graph_destroy(h)
    lge.lge_close(ctx)
    device_ms, roof = roofline_of(tim, "batch")
    return {
        "metric": "sampled edges/s (all 3/4-node graphlets), batched",
        "value": sampled / dt, "unit": "sampled edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "batch_4096_er_chunglu_n50_5000", "graphs": len(graphs), "m_total": tot_m, "p": p,
                   "path": "batched (one lge_estimate_many per step, graphs resident)"},
        "plain": {"value": plain_sampled / t_plain, "unit": "sampled edges/s", "s": t_plain,
                  "path": "4096 lge_estimate calls, one launch sequence each"},
        "batched_vs_plain": (sampled / dt) / (plain_sampled / t_plain),
        "end_to_end_count_batch_s": t_e2e,
        "device_ms": device_ms, "roofline": roof,
    }


def bench_serve(args):
    """Poisson request stream over resident graphs served by lge_server
    (continuous batching); rates at 50% and 80% of the plain path's measured
    saturation throughput."""
    import threading
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    import torch
    from paper_1701_01772_amd import inputs, lge
    log("generating 64 serving graphs (edge counts log-uniform in [1e3, %.0e])" % args.serve_m_hi)
    graphs = inputs.serving_graphs(64, 64, 1e3, args.serve_m_hi)
    log("serving set: %d edges total" % sum(g.m for g in graphs))
    ctx = lge.lge_open(0)
    # 64 graphs stay resident: compact co-degree rows keep the set's HBM bounded
    hs = [lge.lge_graph_create_host(ctx, g.row_ptr, g.col, lge.LGE_FLAG_COMPACT) for g in graphs]
    rng = np.random.default_rng(args.seed)
    n_req = args.serve_requests

    def draw(k):
        return [(int(rng.integers(0, len(hs))), float(rng.choice([1.0, 0.1, 0.01])), 10_000 + i) for i in range(k)]

    # plain-path saturation: requests back to back, one lge_estimate each
    cal = draw(n_req)
    for gi, p, s in cal[:8]:
        lge.lge_estimate(ctx, hs[gi], p, s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_edges = 0
    for gi, p, s in cal:
        plain_edges += lge.lge_estimate(ctx, hs[gi], p, s)["sampled"]
    t_plain = time.perf_counter() - t0
    sat_qps = len(cal) / t_plain
    log("plain saturation: %.1f requests/s" % sat_qps)
    out = {"plain": {"requests_per_s": sat_qps, "sampled_edges_per_s": plain_edges / t_plain}}
    scfg = lge.lge_server_cfg_default()
    if args.serve_step_us:
        scfg.target_step_us = int(args.serve_step_us)
    srv = lge.lge_server_create(ctx, scfg)
    gids = [lge.lge_server_add_graph(srv, h) for h in hs]
    try:
        # closed loop on the same requests as the plain measurement: all
        # submitted at once, drained by the server
        st0 = lge.lge_server_get_stats(srv)
        t0 = time.perf_counter()
        tk = [lge.lge_submit(srv, gids[gi], p, s) for gi, p, s in cal]
        burst_edges = sum(lge.lge_wait(srv, t, -1)["sampled"] for t in tk)
        t_burst = time.perf_counter() - t0
        st1 = lge.lge_server_get_stats(srv)
        assert burst_edges == plain_edges
        out["burst"] = {"requests_per_s": len(cal) / t_burst, "sampled_edges_per_s": burst_edges / t_burst,
                        "steps": st1["steps"] - st0["steps"], "busy_s": st1["busy_s"] - st0["busy_s"],
                        "vs_plain": t_plain / t_burst}
        log("burst: %.1f requests/s (plain %.1f), %d steps" % (len(cal) / t_burst, sat_qps, out["burst"]["steps"]))
        for frac in (0.5, 0.8):
            reqs = draw(n_req)
            qps = frac * sat_qps
            gaps = rng.exponential(1.0 / qps, len(reqs))
            lat = [None] * len(reqs)
            sampled = [0] * len(reqs)
            pool = ThreadPoolExecutor(64)

            def waiter(i, ticket, t_sub):
                r = lge.lge_wait(srv, ticket, -1)
                lat[i] = time.perf_counter() - t_sub
                sampled[i] = r["sampled"]

            t_start = time.perf_counter()
            t_next = t_start
            futs = []
            for i, ((gi, p, s), gap) in enumerate(zip(reqs, gaps)):
                t_next += gap
                d = t_next - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                t_sub = time.perf_counter()
                ticket = lge.lge_submit(srv, gids[gi], p, s)
                futs.append(pool.submit(waiter, i, ticket, t_sub))
            for f in futs:
                f.result()
            span = time.perf_counter() - t_start
            pool.shutdown()
            la = np.array(lat) * 1e3
            st = lge.lge_server_get_stats(srv)
            key = "served_%d" % int(frac * 100)
            out[key] = {"offered_qps": qps, "requests": len(reqs), "p50_ms": float(np.percentile(la, 50)),
                        "p99_ms": float(np.percentile(la, 99)), "throughput_rps": len(reqs) / span,
                        "sampled_edges_per_s": sum(sampled) / span, "steps_total": st["steps"]}
            log("%s: p50 %.2f ms p99 %.2f ms" % (key, out[key]["p50_ms"], out[key]["p99_ms"]))
    finally:
        lge.lge_server_destroy(srv)
    for h in hs:
        lge.lge_graph_destroy(h)
    lge.lge_close(ctx)
    s80 = out["served_80"]
    return {
        "metric": "served p50/p99 latency and throughput (sampled edges/s)",
        "value": s80["sampled_edges_per_s"], "unit": "sampled edges/s", "n_gpus": 1, "steps": n_req,
        "warmup": 8, "ms_per_step": s80["p50_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "serving_64_graphs_chunglu_rmat_m1e3_%.0e" % args.serve_m_hi,
                   "p_mix": [1.0, 0.1, 0.01], "arrivals": "poisson"},
        "serving": out,
    }


def bench_sweep(args):
    """Times option settings on one resident workload (results never depend
    on them); prints one line per setting to stderr and a JSON summary."""
    import torch
    from paper_1701_01772_amd import lge
    p = args.p if args.p is not None else 0.1
    g, wname = make_workload(args.workload)
    ctx = lge.lge_open(0)
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    settings = []
    for spec in args.sweep.split(";"):
        kw = dict(kv.split("=") for kv in spec.split(",") if kv)
        settings.append({k: int(v) for k, v in kw.items()})
    rows = []
    ref = None
    for kw in settings:
        o = lge.make_opts(**kw)
        lge.lge_estimate(ctx, h, p, args.seed, o)
        tim = []
        t0 = time.perf_counter()
        for i in range(args.steps):
            r = lge.lge_estimate(ctx, h, p, args.seed + i, o)
            tim.append(lge.lge_last_timing(ctx))
            if i == 0:
                key = (r["sampled"], tuple(r["csum"]), tuple(r["qsum"]))
                ref = ref or key
                assert key == ref, "results changed with options %s" % kw
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        dev, roof = roofline_of(tim, args.workload)
        rows.append({"opts": kw, "ms_per_step": 1e3 * dt, "device_ms": dev})
        log("%-60s %8.2f ms/step  global %8.2f  block %7.2f  wave %6.2f" % (
            kw, 1e3 * dt, dev["count_global"], dev["count_block"], dev["count_wave"]))
    lge.lge_graph_destroy(h)
    lge.lge_close(ctx)
    return {"sweep": rows, "workload": wname, "p": p}


def bench_micro(args):
    """Micro-level rows (Sec. 3, Alg. 7 at p_e = 1) of every edge of the
    Chung-Lu 1e6 graph: one lge_micro over all m edges per step, rows in a
    resident m x 17 int64 device buffer."""
    import torch
    from paper_1701_01772_amd import lge
    g, wname = make_workload("chung_lu")
    ctx = lge.lge_open(0)
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    rows = torch.empty((g.m, lge.LGE_MICRO_COLS), dtype=torch.int64, device="cuda:0")
    for i in range(max(1, args.warmup)):
        lge.lge_micro(ctx, h, 0, g.m, out=rows)
        log("micro warmup %d" % (i + 1))
    torch.cuda.synchronize()
    tim = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, cm = lge.lge_micro(ctx, h, 0, g.m, out=rows)
        tim.append(lge.lge_last_timing(ctx))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log("micro: %d steps in %.3f s" % (args.steps, dt))
    k = len(tim)
    device_ms, roof = roofline_of(tim, "micro")
    micro_ms = sum(t["micro_ms"] for t in tim) / k
    device_ms["micro_rows"] = micro_ms
    out_bytes = g.m * lge.LGE_MICRO_COLS * 8
    res = {"metric": "micro rows/s (17 exact per-edge graphlet counts, every edge)", "value": g.m * args.steps / dt,
           "unit": "edges/s", "steps": args.steps, "ms_per_step": 1e3 * dt / args.steps,
           "config": {"workload": wname, "n": g.n, "m": g.m, "p": 1.0},
           "device_ms": device_ms, "roofline": roof,
           "micro_rows_kernel": {"ms": micro_ms, "row_bytes_written": out_bytes,
                                 "write_GBps": out_bytes / (micro_ms * 1e-3) / 1e9 if micro_ms > 0 else None},
           "colmax": cm}
    del rows
    lge.lge_graph_destroy(h)
    lge.lge_close(ctx)
    return res


def bench_adaptive(args):
    """Adaptive estimation (Sec. 4, Alg. 8) on the Chung-Lu 1e6 graph,
    beta = 0.01, phi0 = 1/sqrt(m)."""
    import torch
    from paper_1701_01772_amd import lge
    g, wname = make_workload("chung_lu")
    ctx = lge.lge_open(0)
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    lge.lge_estimate_adaptive(ctx, h, args.seed, beta=0.01)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r, tr = lge.lge_estimate_adaptive(ctx, h, args.seed + 1, beta=0.01)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lge.lge_graph_destroy(h)
    lge.lge_close(ctx)
    return {"workload": wname, "beta": 0.01, "rounds": tr["rounds"], "final_p": tr["p"][-1],
            "sampled": tr["sampled"][-1], "seconds": dt, "sampled_edges_per_s": tr["sampled"][-1] / dt,
            "final_delta": tr["delta"][-1]}


def bench_designs(args):
    """The other sampling designs on the Chung-Lu 1e6 graph: k-core and
    degree weighted Bernoulli samples (mean probability 0.1) and a fixed-size
    sample of 0.1 m edges with the ratio estimator."""
    import torch
    from paper_1701_01772_amd import lge
    g, wname = make_workload("chung_lu")
    ctx = lge.lge_open(0)
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    out = {"workload": wname}
    t0 = time.perf_counter()
    _, mc = lge.lge_core_numbers(ctx, h)
    out["core_numbers_s"] = time.perf_counter() - t0
    out["max_core"] = mc
    steps = max(1, args.steps // 2)
    for name, mode in (("kcore", lge.LGE_WEIGHT_KCORE), ("degree", lge.LGE_WEIGHT_DEGREE)):
        lge.lge_estimate_weighted(ctx, h, mode, 0.1, args.seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sampled = 0
        for i in range(steps):
            r, _ = lge.lge_estimate_weighted(ctx, h, mode, 0.1, args.seed + 100 + i)
            sampled += r["sampled"]
        dt = time.perf_counter() - t0
        out["weighted_" + name] = {"sampled_edges_per_s": sampled / dt, "ms_per_step": 1e3 * dt / steps}
    k = g.m // 10
    lge.lge_estimate_fixed_k(ctx, h, k, args.seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        lge.lge_estimate_fixed_k(ctx, h, k, args.seed + 100 + i)
    dt = time.perf_counter() - t0
    out["fixed_k"] = {"k": k, "sampled_edges_per_s": k * steps / dt, "ms_per_step": 1e3 * dt / steps}
    lge.lge_graph_destroy(h)
    lge.lge_close(ctx)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="chung_lu")
    ap.add_argument("--p", type=float, default=None)
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-m-hi", type=float, default=2e6)
    ap.add_argument("--sweep", default=None,
                    help="';'-separated option settings, e.g. 'flags=0;flags=1,global_chunk=128'")
    ap.add_argument("--serve-requests", type=int, default=300)
    ap.add_argument("--serve-step-us", type=int, default=0, help="server target step time (0: library default)")
    ap.add_argument("--quick", action="store_true", help="headline workload only (no batched / served legs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (known bytes) to scale memory counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (--gpus 1): the estimate shards by canonical edge-id "
              "ranges (lge_estimate_range), but no multi-GPU launcher is implemented",
              file=sys.stderr)
        sys.exit(2)

    if args.sweep:
        print(json.dumps(bench_sweep(args)))
        return
    if args.workload == "batch":
        print(json.dumps(bench_batch(args)))
        return
    if args.workload == "serve":
        print(json.dumps(bench_serve(args)))
        return
    if args.workload == "micro":
        print(json.dumps(bench_micro(args)))
        return
    if args.workload == "designs":
        print(json.dumps(bench_designs(args)))
        return

    import torch
    from paper_1701_01772_amd import lge

    p = args.p if args.p is not None else {"chung_lu": 0.1, "rmat": 0.1, "er": 1.0}.get(args.workload, 0.1)
    log("generating %s" % args.workload)
    g, wname = make_workload(args.workload)
    log("graph n=%d m=%d" % (g.n, g.m))
    ctx = lge.lge_open(0)
    t_create = time.perf_counter()
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    t_create = time.perf_counter() - t_create
    log("graph resident in %.2f s (upload, validation, edge list, hub and co-degree tables)" % t_create)
    for i in range(args.warmup):
        lge.lge_estimate(ctx, h, p, args.seed + i)
        log("warmup %d/%d" % (i + 1, args.warmup))
    torch.cuda.synchronize()
    sampled = 0
    tim = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = lge.lge_estimate(ctx, h, p, args.seed + 100 + i)
        sampled += r["sampled"]
        tim.append(lge.lge_last_timing(ctx))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log("timed %d steps in %.3f s" % (args.steps, dt))
    k = len(tim)
    device_ms, roof = roofline_of(tim, args.workload)
    result = {
        "metric": "sampled edges/s (all 3/4-node graphlets)",
        "value": sampled / dt,
        "unit": "sampled edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": wname, "n": g.n, "m": g.m, "p": p, "seed0": args.seed + 100,
                   "path": "plain (one lge_estimate per step, graph resident)"},
        "device_ms": device_ms,
        "class_edges": [sum(t["class_edges"][c] for t in tim) // k for c in range(3)],
        "graph_create_s": t_create,
        "roofline": roof,
    }
    lge.lge_graph_destroy(h)
    lge.lge_close(ctx)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = {"read": src.numel() * 4, "write": dst.numel() * 4}
        del src, dst
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(g, p, args.seed + 100, args.cpu_seconds)
    if not args.quick and args.workload == "chung_lu" and not args.copy_calibration:
        # the metric's other legs: batched vs plain, and served latency
        bargs = argparse.Namespace(**vars(args))
        bargs.steps, bargs.p = 3, None
        b = bench_batch(bargs)
        result["batched"] = {"workload": b["config"]["workload"], "value": b["value"], "unit": b["unit"],
                             "plain_value": b["plain"]["value"], "batched_vs_plain": b["batched_vs_plain"],
                             "ms_per_step": b["ms_per_step"]}
        sv = bench_serve(bargs)["serving"]
        result["served"] = {"workload": "serving_64_graphs_chunglu_rmat_m1e3_%.0e" % args.serve_m_hi,
                            "plain_requests_per_s": sv["plain"]["requests_per_s"],
                            "burst_vs_plain": sv["burst"]["vs_plain"],
                            "p50_ms_at_50pct": sv["served_50"]["p50_ms"], "p99_ms_at_50pct": sv["served_50"]["p99_ms"],
                            "p50_ms_at_80pct": sv["served_80"]["p50_ms"], "p99_ms_at_80pct": sv["served_80"]["p99_ms"],
                            "throughput_rps_at_80pct": sv["served_80"]["throughput_rps"]}
        mi = bench_micro(bargs)
        result["micro"] = {"workload": mi["config"]["workload"], "value": mi["value"], "unit": mi["unit"],
                           "ms_per_step": mi["ms_per_step"], "device_ms": mi["device_ms"],
                           "micro_rows_kernel": mi["micro_rows_kernel"]}
        result["adaptive"] = bench_adaptive(bargs)
        result["designs"] = bench_designs(bargs)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
