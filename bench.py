"""Benchmark of the sampled-edge graphlet estimator on one MI355X.

A step is one full estimate (sample -> bin -> count -> reduce -> FP64
finalise) on a graph resident in HBM.  Headline workload: Chung-Lu power law,
n = 1,000,000, mean expected degree 16, exponent 2.1, degree cap 50,000,
p = 0.1.  The default run adds the large power-law workload (R-MAT scale 22
at p = 0.1 and 0.01), the batched leg (4,096 graphs in one launch sequence
against one launch sequence per graph), the served leg (64 resident graphs,
edge counts log-uniform in [1e3, 5e7]), micro rows, adaptive estimation and
the other sampling designs.  Prints one JSON line.

Per workload: the roofline of the dominant counting kernel (device time from
HIP events the library records on its own stream; bytes = the 4-byte words
the kernel's algorithm reads, counted by the kernel), the graph build (wall
time, state bytes, one estimate from a cold graph, estimates until the
tables pay for their build against a hub-tables-only graph), and the CPU
oracle timed on a bounded sample of the same workload on this host.

    python bench.py [--steps K] [--warmup W] [--workload chung_lu|rmat|er|batch|serve|micro|designs] [--p P]
"""
import argparse
import hashlib
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(msg):
    sys.stderr.write("[bench] %s\n" % msg)
    sys.stderr.flush()


def kernel_source_hash():
    """First 16 hex digits of the SHA-256 of the device code's sources (the
    kernels and the layouts they share with the host)."""
    h = hashlib.sha256()
    for f in ("lge_kernels.hip", "lge_internal.h", "lge_layout.h"):
        with open(os.path.join(ROOT, "paper_1701_01772_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


WORKLOAD_NAMES = {"chung_lu": "chung_lu_n1e6_d16_g2.1_cap5e4", "rmat": "rmat_s22_ef16_a.57_b.19_c.19",
                  "er": "erdos_renyi_n2000_q0.005"}


def make_workload(name):
    from paper_1701_01772_amd import inputs
    makers = {"chung_lu": inputs.chung_lu_1m, "rmat": inputs.rmat_22, "er": inputs.er_2000}
    if name not in makers:
        raise SystemExit("unknown workload %s" % name)
    return makers[name](), WORKLOAD_NAMES[name]


class Background:
    """A value computed on a host thread (input generation overlapping GPU work)."""

    def __init__(self, fn, *args, **kw):
        self._out, self._err = None, None

        def run():
            try:
                self._out = fn(*args, **kw)
            except BaseException as e:  # re-raised in get()
                self._err = e
        self._t = threading.Thread(target=run, daemon=True)
        self._t.start()

    def get(self):
        self._t.join()
        if self._err is not None:
            raise self._err
        return self._out


CLASS_KERNELS = ["k_count_lds<64,256> (wavefront per edge)", "k_count_lds<256,1024> (workgroup per edge)",
                 "k_count_global (split hub edges)"]
CLASS_TAGS = ["wave", "block", "global"]


# ---------------------------------------------------------------------------
# CPU baseline: the oracle, untuned
# ---------------------------------------------------------------------------

def cpu_baseline(g, p, seed, target_s=15.0):
    """The oracle, untuned, on every K-th sampled edge of the same workload
    (K chosen so the single-thread run takes about target_s), then the same
    sample split over the host's cores."""
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


# ---------------------------------------------------------------------------
# roofline of the dominant counting kernel
# ---------------------------------------------------------------------------

def load_counter_profile(workload, cls_tag, p=None):
    """Counter figures of the kernel (profiles/pmc_<workload>_p<p>_<class>.json),
    or None when absent, taken on another kernel source or at another
    sampling probability."""
    if p is None:
        return None
    path = os.path.join(ROOT, "profiles", "pmc_%s_p%g_%s.json" % (workload, p, cls_tag))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        pmc = json.load(fh)
    if pmc.get("kernel_hash") != kernel_source_hash():
        return None
    if p is not None and pmc.get("p") != p:
        return None
    return pmc


def roofline_of(tim, workload, p=None):
    """Roofline of the counting kernel with the longest mean launch.

    achieved = the bytes the kernel's algorithm reads per launch (4-byte words
    counted by the kernel as it issues them: positions, packed rank words,
    vertex records, co-degree and row entries, walked list entries, table
    probes, bit-row words) / the mean launch time; frac = achieved / peak.
    effective = the same launch priced at the neighbour iteration of
    Alg. 2-4 (per edge 16 + 4(d_u + d_v) + sum over w in Gamma(a)\\{b} of
    (8 + 4 d_w)), which the tables avoid reading, so it may exceed the peak.
    traffic = HBM-side bytes per launch from the committed counter profile of
    the same kernel source (null when there is none)."""
    k = len(tim)
    cnt_ms = [sum(t["count_ms"][c] for t in tim) / k for c in range(3)]
    words = [sum(t["words_read"][c] for t in tim) / k for c in range(3)]
    alg = [sum(t["alg_bytes"][c] for t in tim) / k for c in range(3)]
    dom = max(range(3), key=lambda c: cnt_ms[c])
    sec = cnt_ms[dom] * 1e-3
    read_bytes = 4.0 * words[dom]
    achieved = read_bytes / sec / 1e9 if sec > 0 else 0.0
    eff = alg[dom] / sec / 1e9 if sec > 0 else 0.0
    device_ms = {"sample_bin": sum(t["sample_ms"] for t in tim) / k, "count_wave": cnt_ms[0],
                 "count_block": cnt_ms[1], "global_prep": sum(t["global_prep_ms"] for t in tim) / k,
                 "count_global": cnt_ms[2]}
    roof = {"bound": "hbm", "kernel": CLASS_KERNELS[dom], "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "bytes_per_launch": read_bytes, "launch_ms": cnt_ms[dom],
            "effective": {"bytes_per_launch": alg[dom], "GBps": eff, "vs_peak": eff / HBM_PEAK_GBS,
                          "basis": "neighbour iteration of Alg. 2-4"}}
    pmc = load_counter_profile(workload, CLASS_TAGS[dom], p)
    if pmc is not None:
        roof["traffic"] = pmc["traffic_bytes_per_launch"]
        if sec > 0:
            roof["traffic_GBps"] = pmc["traffic_bytes_per_launch"] / sec / 1e9
            roof["traffic_frac"] = roof["traffic_GBps"] / HBM_PEAK_GBS
        roof["traffic_source"] = pmc.get("source")
    return device_ms, roof


# ---------------------------------------------------------------------------
# timed steps and graph build reports
# ---------------------------------------------------------------------------

def time_steps(lge, ctx, h, p, seed0, steps, opts=None):
    """K timed estimates (device idle before and after); per-step timing."""
    import torch
    r = lge.Result()
    torch.cuda.synchronize()
    sampled, tim = 0, []
    t0 = time.perf_counter()
    for i in range(steps):
        sampled += lge.lge_estimate(ctx, h, p, seed0 + i, opts, raw=True, out=r).sampled_edges
        tim.append(lge.lge_last_timing(ctx))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"seconds": dt, "sampled": sampled, "value": sampled / dt, "ms_per_step": 1e3 * dt / steps, "tim": tim}


def create_timed(lge, ctx, g, flags=0):
    t0 = time.perf_counter()
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col, flags)
    return h, time.perf_counter() - t0


def cold_estimate(lge, ctx, h, p, seed, create_s):
    """The first estimate on a just-created graph (its work lists are sized
    on the way): one estimate's throughput counting the graph build."""
    t0 = time.perf_counter()
    r = lge.lge_estimate(ctx, h, p, seed, raw=True)
    first = time.perf_counter() - t0
    return {"first_estimate_s": first, "create_plus_first_s": create_s + first,
            "sampled_edges_per_s": r.sampled_edges / (create_s + first)}


def build_report(lge, ctx, g, h, create_s, p, seed, step_ms, min_steps=1):
    """Graph build against a hub-tables-only graph of the same CSR: state,
    build time and the number of estimates after which the co-degree table,
    bit rows and co-degree rows have paid for their build."""
    info = lge.lge_graph_query(h)
    hm, create_min = create_timed(lge, ctx, g, lge.LGE_FLAG_NO_TABLES)
    try:
        log("build report: hub-tables-only graph, warm-up estimate at p=%g" % p)
        lge.lge_estimate(ctx, hm, p, seed, raw=True)
        log("build report: %d timed estimate(s)" % min_steps)
        mst = time_steps(lge, ctx, hm, p, seed + 1, min_steps)
        info_min = lge.lge_graph_query(hm)
    finally:
        lge.lge_graph_destroy(hm)
    gain_ms = mst["ms_per_step"] - step_ms
    extra_s = create_s - create_min
    return {"graph_create_s": create_s, "build_ms": info["build_ms"], "state_bytes": info["state_bytes"],
            "csr_bytes": 4 * (g.n + 1 + 2 * g.m), "ranked_vertices": info["ranked"], "codeg_rows": info["rows"],
            "p": p, "ms_per_step": step_ms,
            "hub_tables_only": {"graph_create_s": create_min, "state_bytes": info_min["state_bytes"],
                                "ms_per_step": mst["ms_per_step"]},
            "break_even_estimates": (extra_s / (gain_ms * 1e-3)) if gain_ms > 0 else None}


# ---------------------------------------------------------------------------
# the headline and large power-law legs
# ---------------------------------------------------------------------------

def tune_report(lge, ctx, h, p, seed, steps):
    """lge_autotune's options for this graph class and p (the tuning time
    reported, not timed with the steps), K steps with them against K steps
    with the library defaults."""
    t0 = time.perf_counter()
    opts = lge.lge_autotune(ctx, h, p)
    tune_s = time.perf_counter() - t0
    tuned = time_steps(lge, ctx, h, p, seed, steps, opts)
    base = time_steps(lge, ctx, h, p, seed, steps)
    return {"seconds": tune_s, "options": lge.opts_dict(opts), "tuned_ms_per_step": tuned["ms_per_step"],
            "default_ms_per_step": base["ms_per_step"], "tuned_value": tuned["value"],
            "tuned_vs_default": base["ms_per_step"] / tuned["ms_per_step"]}


def estimate_leg(lge, ctx, g, wname, workload, p, seed, steps, warmup, h=None, create_s=None, cpu_s=0.0,
                 want_build=True, want_tune=False):
    """One workload at one p: cold estimate (if the graph is new), warm-up,
    K timed steps with the default options (the leg's value), roofline,
    autotuned options against the defaults, build report, CPU oracle
    baseline."""
    out = {"workload": wname, "n": g.n, "m": g.m, "p": p}
    own = h is None
    if own:
        h, create_s = create_timed(lge, ctx, g)
        log("%s resident in %.2f s" % (wname, create_s))
        out["cold"] = cold_estimate(lge, ctx, h, p, seed, create_s)
    for i in range(warmup):
        lge.lge_estimate(ctx, h, p, seed + i, raw=True)
    st = time_steps(lge, ctx, h, p, seed + 100, steps)
    log("%s p=%g: %d steps in %.3f s (%.1f M sampled edges/s)" % (wname, p, steps, st["seconds"], st["value"] / 1e6))
    k = len(st["tim"])
    device_ms, roof = roofline_of(st["tim"], workload, p)
    out.update({"value": st["value"], "unit": "sampled edges/s", "steps": steps, "warmup": warmup,
                "ms_per_step": st["ms_per_step"], "seed0": seed + 100, "device_ms": device_ms,
                "class_edges": [sum(t["class_edges"][c] for t in st["tim"]) // k for c in range(3)],
                "host_waits": max(t["host_waits"] for t in st["tim"]), "roofline": roof})
    if want_tune:
        out["autotune"] = tune_report(lge, ctx, h, p, seed + 500, steps)
        log("%s p=%g autotune: %.2f vs %.2f ms per step (%.1f s of tuning)" % (
            wname, p, out["autotune"]["tuned_ms_per_step"], out["autotune"]["default_ms_per_step"],
            out["autotune"]["seconds"]))
    if want_build:
        out["build"] = build_report(lge, ctx, g, h, create_s, p, seed + 200, st["ms_per_step"])
        log("%s build: %.2f s, %.1f GB state, break-even %s estimates" % (
            wname, create_s, out["build"]["state_bytes"] / 1e9, out["build"]["break_even_estimates"]))
    if cpu_s > 0:
        log("%s p=%g: cpu baseline (oracle)" % (wname, p))
        out["cpu_baseline"] = cpu_baseline(g, p, seed + 100, cpu_s)
    if own:
        lge.lge_graph_destroy(h)
    return out


def rmat_leg(lge, ctx, args, g):
    """R-MAT scale 22 (the large power-law configuration) at p = 0.1 and
    0.01: plain path, roofline, build, CPU baseline; autotuned options
    against the defaults."""
    wname = WORKLOAD_NAMES["rmat"]
    h, create_s = create_timed(lge, ctx, g)
    log("%s resident in %.2f s" % (wname, create_s))
    out = {"workload": wname, "n": g.n, "m": g.m, "cold": cold_estimate(lge, ctx, h, 0.1, 7, create_s)}
    try:
        for p, steps in ((0.1, args.rmat_steps), (0.01, 3 * args.rmat_steps)):
            leg = estimate_leg(lge, ctx, g, wname, "rmat", p, args.seed, steps, 1, h=h, create_s=create_s,
                               cpu_s=args.rmat_cpu_seconds if not args.no_cpu_baseline else 0.0,
                               want_build=(p == 0.01), want_tune=True)
            out["p%g" % p] = leg
    finally:
        lge.lge_graph_destroy(h)
    return out


# ---------------------------------------------------------------------------
# batched and served legs
# ---------------------------------------------------------------------------

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
    lge.lge_estimate_many(ctx, hs, p, seeds, raw=True)
    res = lge.Result()
    for h in hs[:64]:
        lge.lge_estimate(ctx, h, p, 1, raw=True, out=res)
    torch.cuda.synchronize()
    # plain path: one estimate (one launch sequence) per graph; both legs
    # keep the library's result structs (no conversion to Python numbers)
    t0 = time.perf_counter()
    plain_sampled = 0
    for h, sd in zip(hs, seeds):
        plain_sampled += lge.lge_estimate(ctx, h, p, sd, raw=True, out=res).sampled_edges
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    log("plain: %.3f s (%.0f us per graph)" % (t_plain, 1e6 * t_plain / len(hs)))
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
                  "us_per_graph": 1e6 * t_plain / len(hs),
                  "path": "4096 lge_estimate calls, one launch sequence each"},
        "batched_vs_plain": (sampled / dt) / (plain_sampled / t_plain),
        "end_to_end_count_batch_s": t_e2e,
        "device_ms": device_ms, "roofline": roof,
    }


def serving_set(args, threads=16):
    from paper_1701_01772_amd import inputs
    return inputs.serving_graphs(64, 64, 1e3, args.serve_m_hi, threads=threads)


def bench_serve(args, graphs=None):
    """Poisson request stream over resident graphs served by lge_server
    (continuous batching); rates at 50% and 80% of the plain path's measured
    saturation throughput, the same requests each time, so every latency has
    its plain latency alone beside it (the slowdown)."""
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    import torch
    from paper_1701_01772_amd import lge
    if graphs is None:
        log("generating 64 serving graphs (edge counts log-uniform in [1e3, %.0e])" % args.serve_m_hi)
        graphs = serving_set(args)
    log("serving set: %d graphs, %d edges in all" % (len(graphs), sum(g.m for g in graphs)))
    ctx = lge.lge_open(0)
    # 64 graphs stay resident: their co-degree tables and rows share
    # args.serve_table_gb of HBM in proportion to their edge counts
    t0 = time.perf_counter()
    m_all = float(sum(g.m for g in graphs))
    hs = []
    for g in graphs:
        share = args.serve_table_gb * 1e9 * g.m / m_all
        lge.lge_set_table_budget(ctx, int(share / 2), int(share / 2))
        hs.append(lge.lge_graph_create_host(ctx, g.row_ptr, g.col))
    lge.lge_set_table_budget(ctx, 0, 0)
    state = sum(lge.lge_graph_query(h)["state_bytes"] for h in hs)
    log("serving set resident in %.1f s (%.1f GB of graph state)" % (time.perf_counter() - t0, state / 1e9))
    rng = np.random.default_rng(args.seed)
    n_req = args.serve_requests

    def draw(k):
        return [(int(rng.integers(0, len(hs))), float(rng.choice([1.0, 0.1, 0.01])), 10_000 + i) for i in range(k)]

    # plain-path saturation: requests back to back, one lge_estimate each
    cal = draw(n_req)
    res = lge.Result()
    for gi, p, s in cal[:8]:
        lge.lge_estimate(ctx, hs[gi], p, s, raw=True, out=res)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_edges = 0
    plain_lat = []
    for i, (gi, p, s) in enumerate(cal):
        t1 = time.perf_counter()
        plain_edges += lge.lge_estimate(ctx, hs[gi], p, s, raw=True, out=res).sampled_edges
        plain_lat.append(time.perf_counter() - t1)
        if (i + 1) % 16 == 0:
            log("plain: %d of %d requests, %.1f s" % (i + 1, len(cal), time.perf_counter() - t0))
    t_plain = time.perf_counter() - t0
    alone = {}  # latency of each (graph, p, seed) alone, for slowdowns
    for (gi, p, s), lt in zip(cal, plain_lat):
        alone[(gi, p, s)] = lt
    sat_qps = len(cal) / t_plain
    log("plain saturation: %.1f requests/s" % sat_qps)
    out = {"graphs": len(graphs), "edges_total": sum(g.m for g in graphs), "graph_state_bytes": state,
           "plain": {"requests_per_s": sat_qps, "sampled_edges_per_s": plain_edges / t_plain,
                     "p50_ms_alone": float(np.percentile(np.array(plain_lat) * 1e3, 50)),
                     "p99_ms_alone": float(np.percentile(np.array(plain_lat) * 1e3, 99))}}
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
        burst_edges = 0
        for i, t in enumerate(tk):
            burst_edges += lge.lge_wait(srv, t, -1)["sampled"]
            if (i + 1) % 16 == 0:
                log("burst: %d of %d requests, %.1f s" % (i + 1, len(tk), time.perf_counter() - t0))
        t_burst = time.perf_counter() - t0
        st1 = lge.lge_server_get_stats(srv)
        assert burst_edges == plain_edges
        out["burst"] = {"requests_per_s": len(cal) / t_burst, "sampled_edges_per_s": burst_edges / t_burst,
                        "steps": st1["steps"] - st0["steps"], "busy_s": st1["busy_s"] - st0["busy_s"],
                        "vs_plain": t_plain / t_burst}
        log("burst: %.1f requests/s (plain %.1f), %d steps" % (len(cal) / t_burst, sat_qps, out["burst"]["steps"]))
        for frac in (0.5, 0.8):
            reqs = cal  # the measured requests again, so each has its latency alone
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
            for i, f in enumerate(futs):
                f.result()
                if (i + 1) % 16 == 0:
                    log("served at %d%%: %d of %d requests, %.1f s" % (
                        int(frac * 100), i + 1, len(futs), time.perf_counter() - t_start))
            span = time.perf_counter() - t_start
            pool.shutdown()
            la = np.array(lat) * 1e3
            slow = np.array([lat[i] / alone[r] for i, r in enumerate(reqs)])
            st = lge.lge_server_get_stats(srv)
            key = "served_%d" % int(frac * 100)
            out[key] = {"offered_qps": qps, "requests": len(reqs), "p50_ms": float(np.percentile(la, 50)),
                        "p99_ms": float(np.percentile(la, 99)), "throughput_rps": len(reqs) / span,
                        "sampled_edges_per_s": sum(sampled) / span, "steps_total": st["steps"],
                        "slowdown_p50": float(np.percentile(slow, 50)), "slowdown_p99": float(np.percentile(slow, 99))}
            log("%s: p50 %.2f ms p99 %.2f ms, slowdown vs alone p50 %.2f p99 %.2f" % (
                key, out[key]["p50_ms"], out[key]["p99_ms"], out[key]["slowdown_p50"], out[key]["slowdown_p99"]))
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
        r = lge.lge_estimate(ctx, h, p, args.seed, o)
        key = (r["sampled"], tuple(r["csum"]), tuple(r["qsum"]))
        ref = ref or key
        assert key == ref, "results changed with options %s" % kw
        st = time_steps(lge, ctx, h, p, args.seed, args.steps, o)
        dev, roof = roofline_of(st["tim"], args.workload, p)
        rows.append({"opts": kw, "ms_per_step": st["ms_per_step"], "device_ms": dev})
        log("%-60s %8.2f ms/step  global %8.2f  block %7.2f  wave %6.2f" % (
            kw, st["ms_per_step"], dev["count_global"], dev["count_block"], dev["count_wave"]))
    lge.lge_graph_destroy(h)
    lge.lge_close(ctx)
    return {"sweep": rows, "workload": wname, "p": p}


def bench_micro(args, g=None):
    """Micro-level rows (Sec. 3, Alg. 7 at p_e = 1) of every edge of the
    Chung-Lu 1e6 graph: one lge_micro over all m edges per step, rows in a
    resident m x 17 int64 device buffer."""
    import torch
    from paper_1701_01772_amd import lge
    if g is None:
        g, _ = make_workload("chung_lu")
    wname = WORKLOAD_NAMES["chung_lu"]
    ctx = lge.lge_open(0)
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    rows = torch.empty((g.m, lge.LGE_MICRO_COLS), dtype=torch.int64, device="cuda:0")
    for i in range(max(1, args.warmup)):
        lge.lge_micro(ctx, h, 0, g.m, out=rows)
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


def bench_adaptive(args, g=None):
    """Adaptive estimation (Sec. 4, Alg. 8) on the Chung-Lu 1e6 graph,
    beta = 0.01, phi0 = 1/sqrt(m)."""
    import torch
    from paper_1701_01772_amd import lge
    if g is None:
        g, _ = make_workload("chung_lu")
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
    return {"workload": WORKLOAD_NAMES["chung_lu"], "beta": 0.01, "rounds": tr["rounds"], "final_p": tr["p"][-1],
            "sampled": tr["sampled"][-1], "seconds": dt, "sampled_edges_per_s": tr["sampled"][-1] / dt,
            "final_delta": tr["delta"][-1]}


def bench_designs(args, g=None):
    """The other sampling designs on the Chung-Lu 1e6 graph: k-core and
    degree weighted Bernoulli samples (mean probability 0.1) and a fixed-size
    sample of 0.1 m edges with the ratio estimator."""
    import torch
    from paper_1701_01772_amd import lge
    if g is None:
        g, _ = make_workload("chung_lu")
    ctx = lge.lge_open(0)
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    out = {"workload": WORKLOAD_NAMES["chung_lu"]}
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


# ---------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="chung_lu")
    ap.add_argument("--p", type=float, default=None)
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--rmat-cpu-seconds", type=float, default=8.0)
    ap.add_argument("--rmat-steps", type=int, default=3, help="timed steps at p = 0.1 (three times that at 0.01)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-m-hi", type=float, default=5e7)
    ap.add_argument("--sweep", default=None,
                    help="';'-separated option settings, e.g. 'flags=0;flags=1,global_chunk=128'")
    ap.add_argument("--serve-requests", type=int, default=128)
    ap.add_argument("--serve-table-gb", type=float, default=120.0,
                    help="HBM the serving set's co-degree tables and rows share (in proportion to edge counts)")
    ap.add_argument("--serve-step-us", type=int, default=0, help="server target step time (0: library default)")
    ap.add_argument("--quick", action="store_true", help="headline workload only (no other legs)")
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

    from paper_1701_01772_amd import inputs, lge
    full = args.workload == "chung_lu" and not args.quick and not args.copy_calibration

    p = args.p if args.p is not None else {"chung_lu": 0.1, "rmat": 0.1, "er": 1.0}.get(args.workload, 0.1)
    log("generating %s" % args.workload)
    g, wname = make_workload(args.workload)
    log("graph n=%d m=%d" % (g.n, g.m))
    ctx = lge.lge_open(0)
    head = estimate_leg(lge, ctx, g, wname, args.workload, p, args.seed, args.steps, args.warmup,
                        cpu_s=0.0, want_build=not args.quick, want_tune=not args.quick)
    # the other legs' inputs are drawn on host threads (not while steps or
    # the CPU baseline are timed: they would compete for host cores)
    bg_rmat = Background(inputs.rmat_22) if full else None
    bg_serve = Background(serving_set, args) if full else None
    result = {
        "metric": "sampled edges/s (all 3/4-node graphlets)",
        "value": head["value"],
        "unit": "sampled edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": wname, "n": g.n, "m": g.m, "p": p, "seed0": head["seed0"],
                   "path": "plain (one lge_estimate per step, graph resident)"},
        "device_ms": head["device_ms"],
        "class_edges": head["class_edges"],
        "host_waits_per_step": head["host_waits"],
        "graph_create_s": head["cold"]["create_plus_first_s"] - head["cold"]["first_estimate_s"],
        "cold": head["cold"],
        "roofline": head["roofline"],
    }
    if "autotune" in head:
        result["autotune"] = head["autotune"]
    if "build" in head:
        result["build"] = head["build"]
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = {"read": src.numel() * 4, "write": dst.numel() * 4}
        del src, dst
    if full:  # the host is quiet again before the CPU baseline is timed
        log("waiting for the input generators")
        g_rmat, g_serve = bg_rmat.get(), bg_serve.get()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(g, p, args.seed + 100, args.cpu_seconds)
    if full:
        result["rmat"] = rmat_leg(lge, ctx, args, g_rmat)
        lge.lge_close(ctx)
        ctx = None
        bargs = argparse.Namespace(**vars(args))
        bargs.steps, bargs.p = 3, None
        b = bench_batch(bargs)
        result["batched"] = {"workload": b["config"]["workload"], "value": b["value"], "unit": b["unit"],
                             "plain_value": b["plain"]["value"], "plain_us_per_graph": b["plain"]["us_per_graph"],
                             "batched_vs_plain": b["batched_vs_plain"], "ms_per_step": b["ms_per_step"],
                             "end_to_end_count_batch_s": b["end_to_end_count_batch_s"]}
        sv = bench_serve(bargs, g_serve)["serving"]
        result["served"] = {"workload": "serving_64_graphs_chunglu_rmat_m1e3_%.0e" % args.serve_m_hi,
                            "edges_total": sv["edges_total"], "graph_state_bytes": sv["graph_state_bytes"],
                            "requests": args.serve_requests,
                            "plain_requests_per_s": sv["plain"]["requests_per_s"],
                            "burst_vs_plain": sv["burst"]["vs_plain"],
                            "p50_ms_alone": sv["plain"]["p50_ms_alone"], "p99_ms_alone": sv["plain"]["p99_ms_alone"],
                            "p50_ms_at_50pct": sv["served_50"]["p50_ms"], "p99_ms_at_50pct": sv["served_50"]["p99_ms"],
                            "p50_ms_at_80pct": sv["served_80"]["p50_ms"], "p99_ms_at_80pct": sv["served_80"]["p99_ms"],
                            "slowdown_p50_at_80pct": sv["served_80"]["slowdown_p50"],
                            "slowdown_p99_at_80pct": sv["served_80"]["slowdown_p99"],
                            "throughput_rps_at_80pct": sv["served_80"]["throughput_rps"]}
        mi = bench_micro(bargs, g)
        result["micro"] = {"workload": mi["config"]["workload"], "value": mi["value"], "unit": mi["unit"],
                           "ms_per_step": mi["ms_per_step"], "device_ms": mi["device_ms"],
                           "micro_rows_kernel": mi["micro_rows_kernel"]}
        result["adaptive"] = bench_adaptive(bargs, g)
        result["designs"] = bench_designs(bargs, g)
    if ctx is not None:
        lge.lge_close(ctx)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
