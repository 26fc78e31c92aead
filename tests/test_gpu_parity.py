"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar: every integer (sampled edge count, the 13 C sums, the 15 Z and 15 Q
sums, the 17 exact counts at p = 1) bit-equal; every FP64 output within a
relative 1e-12 (or both zero).  Inputs are seeded synthetic graphs sized so
the oracle finishes in seconds, chosen to hit all three edge classes
(wavefront, workgroup, split global) and the ragged tails of every loop.
"""
import math
import os
import sys
import time

import numpy as np

import pytest

import oracle
from paper_1701_01772_amd import inputs, lge

pytestmark = pytest.mark.gpu

REL = 1e-12


def _say(msg):
    sys.stdout.write("[gpu-parity] %s\n" % msg)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = lge.lge_open(0)
    yield c
    lge.lge_close(c)


def _close(a, b):
    if a == b:
        return True
    return abs(a - b) <= REL * max(abs(a), abs(b))


def assert_parity(gpu, orc, what=""):
    assert gpu["sampled"] == orc["sampled"], what
    for key in ("csum", "zsum", "qsum"):
        for i in range(3, 18):
            assert gpu[key][i] == orc[key][i], (what, key, i, gpu[key][i], orc[key][i])
    if orc["p"] == 1.0:
        assert gpu["exact"][1:] == orc["exact"][1:], what
    for key in ("estimate", "variance", "lower95", "upper95"):
        for i in range(1, 18):
            assert _close(gpu[key][i], orc[key][i]), (what, key, i, gpu[key][i], orc[key][i])


def run_pair(ctx, g, p, seed, opts=None, what=""):
    _say("%s n=%d m=%d p=%g seed=%d" % (what or g.name, g.n, g.m, p, seed))
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    try:
        got = lge.lge_estimate(ctx, h, p, seed, opts)
    finally:
        lge.lge_graph_destroy(h)
    want = oracle.estimate(g.row_ptr, g.col, p, seed)
    assert_parity(got, want, what or g.name)
    return got


def two_hub_graph(seed=3):
    """Two adjacent hubs (degree > 1024) sharing half their neighbours, a dense
    cluster, and sparse background edges: exercises hub tables and splitting."""
    rng = np.random.default_rng(seed)
    n = 5000
    edges = [(0, 1)]
    n0 = rng.choice(np.arange(2, n), 2600, replace=False)
    n1 = np.concatenate([n0[:1300], rng.choice(np.arange(2, n), 1400, replace=False)])
    edges += [(0, int(x)) for x in n0] + [(1, int(x)) for x in n1]
    cl = rng.choice(np.arange(2, n), 40, replace=False)
    edges += [(int(a), int(b)) for i, a in enumerate(cl) for b in cl[i + 1:]]
    m_bg = 12000
    a = rng.integers(2, n, m_bg)
    b = rng.integers(2, n, m_bg)
    edges += [(int(x), int(y)) for x, y in zip(a, b)]
    # a mid-degree vertex (block class) wired into both hubs' neighbourhoods
    mid = 2
    edges += [(mid, int(x)) for x in rng.choice(n0, 600, replace=False)]
    return inputs.from_edges(n, edges)


# ---------------------------------------------------------------------------


@pytest.mark.parametrize("seed", range(12))
def test_small_random_exact(ctx, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 90))
    q = float(rng.choice([0.02, 0.1, 0.3, 0.6, 0.9]))
    run_pair(ctx, inputs.erdos_renyi(n, q, 100 + seed), 1.0, 0)


def test_degenerate_graphs(ctx):
    for n, es in ((1, []), (5, []), (2, [(0, 1)]), (3, [(0, 1), (1, 2), (0, 2)]), (7, [(0, 1), (5, 6)])):
        g = inputs.from_edges(n, es)
        for p in (1.0, 0.5):
            run_pair(ctx, g, p, 9, what="degenerate n=%d m=%d" % (n, len(es)))


def test_er_config_exact(ctx):
    run_pair(ctx, inputs.er_2000(), 1.0, 0, what="er(2000,0.005)")


@pytest.mark.parametrize("maker,name", [
    (lambda: two_hub_graph(), "two-hub"),
    (lambda: inputs.chung_lu(20000, 10.0, 2.1, 3000.0, 41), "chung-lu-20k"),
    (lambda: inputs.rmat(12, 16, 0.57, 0.19, 0.19, 42), "rmat-12"),
])
def test_all_classes_exact(ctx, maker, name):
    run_pair(ctx, maker(), 1.0, 0, what=name)
    if name != "two-hub":  # the power-law graphs fill all three classes under the default options
        assert all(c > 0 for c in lge.lge_last_timing(ctx)["class_edges"]), name


@pytest.mark.parametrize("p,seed", [(0.5, 1), (0.1, 2), (0.01, 3), (1e-4, 4)])
def test_sampled_powerlaw(ctx, p, seed):
    run_pair(ctx, inputs.chung_lu(20000, 10.0, 2.1, 3000.0, 41), p, seed, what="chung-lu-20k")


@pytest.mark.parametrize("p", [0.3, 0.05])
def test_sampled_two_hub(ctx, p):
    run_pair(ctx, two_hub_graph(), p, 17, what="two-hub")


def test_tuning_invariance(ctx):
    g = inputs.rmat(11, 16, 0.57, 0.19, 0.19, 5)
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    try:
        base = lge.lge_estimate(ctx, h, 0.7, 3)
        for wv in (8, 64, 200, 512):
            for pr in (0, 1, 16, 1000):
                for gpc in (1, 3):
                    o = lge.make_opts(wave_max_deg=wv, probe_ratio=pr, grid_per_cu=gpc)
                    got = lge.lge_estimate(ctx, h, 0.7, 3, o)
                    for k in ("sampled", "csum", "zsum", "qsum"):
                        assert got[k] == base[k], (wv, pr, gpc, k)
        for chunk in (1, 37, 256, 1024):
            for flags in (0, lge.LGE_OPT_SORT_HUB, lge.LGE_OPT_XCD_LOCAL,
                          lge.LGE_OPT_SORT_HUB | lge.LGE_OPT_XCD_LOCAL):
                o = lge.make_opts(global_chunk=chunk, flags=flags)
                got = lge.lge_estimate(ctx, h, 0.7, 3, o)
                for k in ("sampled", "csum", "zsum", "qsum"):
                    assert got[k] == base[k], (chunk, flags, k)
        for share in (5, 25, 75):  # smaller persistent grids
            got = lge.lge_estimate(ctx, h, 0.7, 3, lge.make_opts(grid_share=share))
            for k in ("sampled", "csum", "zsum", "qsum"):
                assert got[k] == base[k], (share, k)
        for bmd in (1, 100, 300, 700):  # block class narrowed or empty
            got = lge.lge_estimate(ctx, h, 0.7, 3, lge.make_opts(block_max_deg=bmd))
            for k in ("sampled", "csum", "zsum", "qsum"):
                assert got[k] == base[k], (bmd, k)
    finally:
        lge.lge_graph_destroy(h)
    assert_parity(base, oracle.estimate(g.row_ptr, g.col, 0.7, 3), "rmat-11 tuned")


def test_range_additivity_and_parity(ctx):
    g = inputs.chung_lu(20000, 10.0, 2.1, 3000.0, 41)
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    try:
        full = lge.lge_estimate(ctx, h, 0.25, 8)
        cuts = [0, 1, 777, g.m // 2, g.m - 3, g.m]
        parts = [lge.lge_estimate_range(ctx, h, 0.25, 8, a, b) for a, b in zip(cuts, cuts[1:])]
        for k in ("sampled",):
            assert sum(pt[k] for pt in parts) == full[k]
        for k in ("csum", "zsum", "qsum"):
            for i in range(3, 18):
                assert sum(pt[k][i] for pt in parts) == full[k][i], (k, i)
        a, b = 1234, 1234 + 3000
        got = lge.lge_estimate_range(ctx, h, 0.25, 8, a, b)
        mask = oracle.sample_mask(8, 0.25, g.m, a, b)
        assert_parity(got, oracle.estimate(g.row_ptr, g.col, 0.25, 8, mask=mask), "range")
    finally:
        lge.lge_graph_destroy(h)


def test_list_budget_pieces_equal_one_sequence(ctx):
    # a 1 MiB bound on the split-class lists makes every call below run its
    # edge-id range in pieces; the exact sums must not change
    g = inputs.chung_lu(20000, 10.0, 2.1, 3000.0, 41)
    g2 = inputs.rmat(12, 16, 0.57, 0.19, 0.19, 4)
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    h2 = lge.lge_graph_create_host(ctx, g2.row_ptr, g2.col)
    small = lge.make_opts(max_list_mib=1)
    keys = ("sampled", "csum", "zsum", "qsum", "exact", "estimate", "variance")
    try:
        for p in (1.0, 0.5):
            base = lge.lge_estimate(ctx, h, p, 12)
            tb = lge.lge_last_timing(ctx)
            got = lge.lge_estimate(ctx, h, p, 12, small)
            t = lge.lge_last_timing(ctx)
            _say("pieces p=%g: %d host waits (one sequence: %d)" % (p, t["host_waits"], tb["host_waits"]))
            assert t["host_waits"] > 2, t["host_waits"]
            assert list(t["class_edges"]) == list(tb["class_edges"])
            for k in keys:
                assert got[k] == base[k], (p, k)
        assert_parity(got, oracle.estimate(g.row_ptr, g.col, 0.5, 12), "pieces")
        many = lge.lge_estimate_many(ctx, [h, h2, h], [1.0, 0.8, 0.3], [5, 6, 7], small)
        for hh, out, p, sd in zip([h, h2, h], many, [1.0, 0.8, 0.3], [5, 6, 7]):
            single = lge.lge_estimate(ctx, hh, p, sd)
            for k in keys:
                assert out[k] == single[k], (p, k)
        a, b = 100, g.m - 100
        rs = lge.lge_estimate_range(ctx, h, 0.9, 3, a, b, small)
        rb = lge.lge_estimate_range(ctx, h, 0.9, 3, a, b)
        for k in ("sampled", "csum", "zsum", "qsum"):
            assert rs[k] == rb[k], k
        ws, _ = lge.lge_estimate_weighted(ctx, h2, lge.LGE_WEIGHT_DEGREE, 0.4, 9, small)
        wb, _ = lge.lge_estimate_weighted(ctx, h2, lge.LGE_WEIGHT_DEGREE, 0.4, 9)
        for k in ("sampled", "csum", "zsum", "qsum", "estimate", "variance"):
            assert ws[k] == wb[k], k
    finally:
        lge.lge_graph_destroy(h2)
        lge.lge_graph_destroy(h)


def test_batch_equals_singles(ctx):
    graphs = inputs.batch_graphs(count=24, seed=77, n_lo=20, n_hi=1500)
    graphs.append(inputs.from_edges(4, []))
    graphs.append(two_hub_graph(5))
    ps = [1.0 if i % 3 else 0.4 for i in range(len(graphs))]
    seeds = [1000 + i for i in range(len(graphs))]
    _say("batch of %d graphs" % len(graphs))
    outs = lge.lge_count_batch(ctx, [(g.row_ptr, g.col) for g in graphs], ps, seeds)
    for g, out, p, s in zip(graphs, outs, ps, seeds):
        want = oracle.estimate(g.row_ptr, g.col, p, s)
        assert_parity(out, want, "batch member n=%d" % g.n)


@pytest.mark.parametrize("p", [0.25])
def test_codeg_pair_beyond_16_bits(ctx, p):
    # two adjacent hubs sharing 70,000 neighbours plus a few hundred mid-degree
    # vertices (ranked, so the co-degree table is built): the hubs'
    # co-degree, 70,000, does not fit a 16-bit entry and must come from
    # walking; their rows count in 32-bit LDS words (degree >= 2^16)
    k = 70000
    rng = np.random.default_rng(9)
    edges = [(0, 1)] + [(0, 2 + i) for i in range(k)] + [(1, 2 + i) for i in range(k)]
    mids = np.arange(2 + k, 2 + k + 300)
    for v in mids:  # each mid vertex: 120 random leaves and one hub
        edges += [(int(v), int(x)) for x in rng.choice(np.arange(2, 2 + k), 120, replace=False)]
        edges.append((0 if v % 2 else 1, int(v)))
    g = inputs.from_edges(2 + k + len(mids), edges)
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    try:
        info = lge.lge_graph_query(h)
        _say("saturated pair: n=%d m=%d ranked %d, p=%g" % (g.n, g.m, info["ranked"], p))
        assert info["ranked"] >= 2
        got = lge.lge_estimate(ctx, h, p, 21)
    finally:
        lge.lge_graph_destroy(h)
    assert_parity(got, oracle.estimate(g.row_ptr, g.col, p, 21), "two hubs of degree > 2^16")


def test_table_budgets_change_state_not_results(ctx):
    # the same graph with the library's tables, with capped tables, with the
    # compact budgets and with hub tables only: identical integers and
    # estimates, state shrinking in that order
    g = inputs.rmat(14, 16, 0.57, 0.19, 0.19, 71)
    made = []
    try:
        made.append(("default", lge.lge_graph_create_host(ctx, g.row_ptr, g.col)))
        lge.lge_set_table_budget(ctx, 1 << 20, 1 << 20)
        made.append(("capped", lge.lge_graph_create_host(ctx, g.row_ptr, g.col)))
        lge.lge_set_table_budget(ctx, 0, 0)
        made.append(("compact", lge.lge_graph_create_host(ctx, g.row_ptr, g.col, lge.LGE_FLAG_COMPACT)))
        made.append(("no tables", lge.lge_graph_create_host(ctx, g.row_ptr, g.col, lge.LGE_FLAG_NO_TABLES)))
        infos = [(name, lge.lge_graph_query(h)) for name, h in made]
        _say("table budgets: " + ", ".join("%s %d ranked %.1f MB" % (n, i["ranked"], i["state_bytes"] / 1e6)
                                           for n, i in infos))
        assert infos[1][1]["state_bytes"] < infos[0][1]["state_bytes"]
        assert infos[1][1]["ranked"] < infos[0][1]["ranked"]
        assert infos[3][1]["ranked"] == 0 and infos[3][1]["rows"] == 0
        assert infos[3][1]["state_bytes"] < infos[1][1]["state_bytes"]
        for p, seed in ((1.0, 3), (0.3, 4)):
            base = lge.lge_estimate(ctx, made[0][1], p, seed)
            for name, h in made[1:]:
                got = lge.lge_estimate(ctx, h, p, seed)
                for k in ("sampled", "csum", "zsum", "qsum", "exact", "estimate", "variance"):
                    assert got[k] == base[k], (name, p, k)
        assert_parity(base, oracle.estimate(g.row_ptr, g.col, 0.3, 4), "rmat-14 with table budgets")
    finally:
        lge.lge_set_table_budget(ctx, 0, 0)
        for _, h in made:
            lge.lge_graph_destroy(h)


def test_row_tiles_in_passes(ctx):
    # co-degree rows over several 65,536-column tiles, built with the
    # segment-end scratch at its minimum (one tile per pass) and in one pass:
    # the same state, and the same integers as a graph with hub tables only
    g = inputs.chung_lu(300000, 16.0, 2.1, 5e4, 77)
    deg = np.diff(np.asarray(g.row_ptr, dtype=np.int64))
    made = []
    try:
        made.append(lge.lge_graph_create_host(ctx, g.row_ptr, g.col))
        lge.lge_set_build_scratch(ctx, 1)
        made.append(lge.lge_graph_create_host(ctx, g.row_ptr, g.col))
        lge.lge_set_build_scratch(ctx, 0)
        made.append(lge.lge_graph_create_host(ctx, g.row_ptr, g.col, lge.LGE_FLAG_NO_TABLES))
        i0, i1 = lge.lge_graph_query(made[0]), lge.lge_graph_query(made[1])
        ncol = int((deg > i0["rows_floor"]).sum()) - i0["ranked"]
        _say("row tiles: %d rows x %d columns (%d tiles), %d ranked" % (i0["rows"], ncol, -(-ncol // 65536),
                                                                        i0["ranked"]))
        assert i0["rows"] > 0 and ncol > 2 * 65536
        for k in ("rows", "ranked", "rows_floor", "rows_width", "state_bytes"):
            assert i1[k] == i0[k], k
        for p, seed in ((1.0, 5), (0.1, 6)):
            base = lge.lge_estimate(ctx, made[0], p, seed)
            for h in made[1:]:
                got = lge.lge_estimate(ctx, h, p, seed)
                for k in ("sampled", "csum", "zsum", "qsum", "exact", "estimate", "variance"):
                    assert got[k] == base[k], (p, k)
    finally:
        lge.lge_set_build_scratch(ctx, 0)
        for h in made:
            lge.lge_graph_destroy(h)


def test_count_batch_large_union(ctx):
    # 16,384 members of up to 5,000 vertices: the union's own n would fail
    # the whole-graph bound on exact sums, but every member's sums use the
    # member's n and m, so the batch must run
    graphs = inputs.batch_graphs(count=16384, seed=16384)
    N = sum(g.n for g in graphs)
    _say("batch of %d graphs, %d vertices, %d edges" % (len(graphs), N, sum(g.m for g in graphs)))
    seeds = [5000 + i for i in range(len(graphs))]
    outs = lge.lge_count_batch(ctx, [(g.row_ptr, g.col) for g in graphs], 1.0, seeds)
    rng = np.random.default_rng(3)
    for k in rng.choice(len(graphs), 12, replace=False):
        g = graphs[int(k)]
        assert_parity(outs[int(k)], oracle.estimate(g.row_ptr, g.col, 1.0, seeds[int(k)]), "member %d" % k)


def test_graph_create_device_matches_host(ctx):
    torch = pytest.importorskip("torch")
    g = inputs.chung_lu(5000, 8.0, 2.3, 800.0, 12)
    rp = torch.from_numpy(g.row_ptr).to("cuda:0")
    cl = torch.from_numpy(g.col).to("cuda:0")
    torch.cuda.synchronize()
    h = lge.lge_graph_create_device(ctx, g.n, rp.data_ptr(), cl.data_ptr(), torch.cuda.current_stream().cuda_stream)
    try:
        got = lge.lge_estimate(ctx, h, 0.6, 21)
    finally:
        lge.lge_graph_destroy(h)
    assert_parity(got, oracle.estimate(g.row_ptr, g.col, 0.6, 21), "device-adopted")


def test_invalid_graph_rejected_on_gpu(ctx):
    # asymmetric: 0->1 without 1->0
    rp = np.array([0, 1, 1], dtype=np.int32)
    cl = np.array([1], dtype=np.int32)
    with pytest.raises(lge.LgeError) as ei:
        lge.lge_graph_create_host(ctx, rp, cl)
    assert ei.value.code in (lge.LGE_EGRAPH,)


# ---------------------------------------------------------------------------
# Full-size configurations: properties at full size, oracle parity on ranges
# the oracle finishes in seconds, in the launch configuration of the bench.
# ---------------------------------------------------------------------------


def _full_size_checks(ctx, g, p, seed, ranges):
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    try:
        _say("full %s p=%g" % (g.name, p))
        full = lge.lge_estimate(ctx, h, p, seed)
        assert full["sampled"] == oracle.sample_count(seed, p, 0, g.m)
        # 4-node counts sum to C(n,4) in every estimate (X17 is the complement)
        tot4 = sum(full["estimate"][7:18])
        assert abs(tot4 - math.comb(g.n, 4)) <= 1e-9 * math.comb(g.n, 4)
        for a, b in ranges:
            _say("range [%d, %d)" % (a, b))
            got = lge.lge_estimate_range(ctx, h, p, seed, a, b)
            mask = oracle.sample_mask(seed, p, g.m, a, b)
            assert_parity(got, oracle.estimate(g.row_ptr, g.col, p, seed, mask=mask), "%s range" % g.name)
    finally:
        lge.lge_graph_destroy(h)


@pytest.mark.parametrize("p", [0.1, 0.01])
def test_full_size_chung_lu(ctx, p):
    g = inputs.chung_lu_1m()
    rng = np.random.default_rng(5)
    starts = rng.integers(0, g.m - 4000, 3)
    _full_size_checks(ctx, g, p, 2024, [(int(s), int(s) + 4000) for s in starts])


def test_estimate_many_equals_singles(ctx):
    graphs = inputs.batch_graphs(count=16, seed=91, n_lo=30, n_hi=2500)
    hs = [lge.lge_graph_create_host(ctx, g.row_ptr, g.col) for g in graphs]
    try:
        ps = [1.0 if i % 2 else 0.35 for i in range(len(hs))]
        seeds = [7 + 3 * i for i in range(len(hs))]
        _say("estimate_many over %d resident graphs" % len(hs))
        many = lge.lge_estimate_many(ctx, hs, ps, seeds)
        for g, h, out, p, s in zip(graphs, hs, many, ps, seeds):
            single = lge.lge_estimate(ctx, h, p, s)
            for k in ("sampled", "csum", "zsum", "qsum", "exact", "estimate", "variance"):
                assert out[k] == single[k], k
            assert_parity(out, oracle.estimate(g.row_ptr, g.col, p, s), "many n=%d" % g.n)
    finally:
        for h in hs:
            lge.lge_graph_destroy(h)


def test_async_estimate_matches_sync(ctx):
    torch = pytest.importorskip("torch")
    g = inputs.chung_lu(20000, 10.0, 2.1, 3000.0, 41)
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    try:
        sync = lge.lge_estimate(ctx, h, 0.3, 5)
        x = torch.ones(1 << 20, device="cuda:0")
        x.mul_(2.0)  # work queued on torch's stream before the estimate
        ev, r = lge.lge_estimate_async(ctx, h, 0.3, 5, torch.cuda.current_stream().cuda_stream)
        lge.lge_event_wait(ev)
        got = lge.result_dict(r)
        for k in ("sampled", "csum", "zsum", "qsum", "estimate", "variance"):
            assert got[k] == sync[k], k
    finally:
        lge.lge_graph_destroy(h)


def test_autotune_changes_speed_not_results(ctx):
    g = inputs.chung_lu(20000, 10.0, 2.1, 3000.0, 41)
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    try:
        _say("autotune on chung-lu-20k")
        o = lge.lge_autotune(ctx, h, 0.4)
        assert 1 <= o.wave_max_deg <= 512 and o.probe_ratio > 0
        assert 1 <= o.block_max_deg <= 1024 and o.global_chunk in (256, 512, 1024)
        tuned = lge.lge_estimate(ctx, h, 0.4, 77, o)
        base = lge.lge_estimate(ctx, h, 0.4, 77)
        for k in ("sampled", "csum", "zsum", "qsum", "estimate", "variance"):
            assert tuned[k] == base[k], k
        # a second graph of the same class (same bit lengths of m and of the
        # maximum degree, same p) gets the cached choice at once
        g2 = inputs.chung_lu(20000, 10.0, 2.1, 3000.0, 42)
        h2 = lge.lge_graph_create_host(ctx, g2.row_ptr, g2.col)
        try:
            same_class = (g2.m.bit_length() == g.m.bit_length()
                          and lge.lge_graph_query(h2)["max_deg"].bit_length()
                          == lge.lge_graph_query(h)["max_deg"].bit_length())
            t0 = time.perf_counter()
            o2 = lge.lge_autotune(ctx, h2, 0.4)
            dt = time.perf_counter() - t0
            if same_class:
                assert lge.opts_dict(o2) == lge.opts_dict(o)
                assert dt < 0.5, dt
            lge.lge_autotune_reset(ctx)
            o3 = lge.lge_autotune(ctx, h2, 0.4)  # timed afresh
            assert lge.lge_estimate(ctx, h2, 0.4, 78, o3)["csum"] == lge.lge_estimate(ctx, h2, 0.4, 78)["csum"]
        finally:
            lge.lge_graph_destroy(h2)
    finally:
        lge.lge_graph_destroy(h)


@pytest.mark.parametrize("beta,phi0", [(0.05, 0.0), (0.0, 0.3), (0.01, 1.0)])
def test_adaptive_equals_oracle_and_plain(ctx, beta, phi0):
    from oracle import adaptive as oadaptive
    g = inputs.chung_lu(8000, 10.0, 2.1, 1500.0, 17)
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    try:
        _say("adaptive beta=%g phi0=%g on n=%d m=%d" % (beta, phi0, g.n, g.m))
        got, tr = lge.lge_estimate_adaptive(ctx, h, 31, beta=beta, t_max=8, phi0=phi0)
        want, otr = oadaptive.adaptive(g.row_ptr, g.col, 31, beta=beta, t_max=8, phi0=phi0)
        assert tr["rounds"] == otr["rounds"]
        assert tr["p"] == otr["p"] and tr["sampled"] == otr["sampled"]
        for a, b in zip(tr["delta"], otr["delta"]):
            assert _close(a, b), (a, b)
        assert_parity(got, want, "adaptive")
        # rounds add disjoint slices [p_{t-1}, p_t): the union is the plain sample at p_T
        plain = lge.lge_estimate(ctx, h, tr["p"][-1], 31)
        for k in ("sampled", "csum", "zsum", "qsum", "estimate", "variance"):
            assert got[k] == plain[k], k
    finally:
        lge.lge_graph_destroy(h)


@pytest.fixture(scope="module")
def rmat22():
    _say("generating R-MAT scale 22")
    return inputs.rmat_22()


@pytest.mark.parametrize("p", [0.01, 0.1])
def test_full_size_rmat(ctx, rmat22, p):
    g = rmat22
    rng = np.random.default_rng(6 if p == 0.1 else 7)
    starts = rng.integers(0, g.m - 4000, 3)
    _full_size_checks(ctx, g, p, 2025, [(int(s), int(s) + 4000) for s in starts])


def test_compact_graph_same_results(ctx, rmat22):
    # R-MAT scale 22 has ~12k vertices of degree > 1024: the compact budget
    # builds co-degree rows for far fewer of them than the default
    g = rmat22
    outs = []
    for flags in (0, lge.LGE_FLAG_COMPACT):
        _say("R-MAT scale 22 flags=%d p=0.005" % flags)
        h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col, flags)
        try:
            outs.append(lge.lge_estimate(ctx, h, 0.005, 99))
        finally:
            lge.lge_graph_destroy(h)
    for k in ("sampled", "csum", "zsum", "qsum", "estimate", "variance"):
        assert outs[0][k] == outs[1][k], k


def wide_t_graph(k):
    """Hubs 0 and 1, adjacent, with k common neighbours joined in a ring
    lattice (48 on each side), so every common neighbour has degree 98 and is
    in the co-degree table: T_e of the hub edge holds k ranked members."""
    e = [(0, 1)] + [(0, 2 + i) for i in range(k)] + [(1, 2 + i) for i in range(k)]
    e += [(2 + i, 2 + (i + s) % k) for i in range(k) for s in range(1, 49)]
    return inputs.from_edges(k + 2, np.array(e, dtype=np.int32))


@pytest.mark.parametrize("k", [20000, 40000])
def test_wide_ranked_t(ctx, k):
    # the ranked members of T_e fill 313 (k = 20000) and 626 (k = 40000)
    # bit-set words, all held in the split kernel's LDS copy
    g = wide_t_graph(k)
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    try:
        for a, b in ((0, 1), (1, 9), (k + 1, k + 9), (2 * k + 1, 2 * k + 40), (g.m - 5, g.m)):
            _say("wide T_e k=%d range [%d, %d)" % (k, a, b))
            got = lge.lge_estimate_range(ctx, h, 1.0, 5, a, b)
            mask = oracle.sample_mask(5, 1.0, g.m, a, b)
            assert_parity(got, oracle.estimate(g.row_ptr, g.col, 1.0, 5, mask=mask), "wide-t k=%d [%d,%d)" % (k, a, b))
    finally:
        lge.lge_graph_destroy(h)


def test_bounds_coverage_matches_oracle(ctx):
    # the statistical pin of the oracle (95 % bounds cover the exact counts
    # near the nominal rate) holds for the GPU path's bounds, run for run
    from test_oracle_estimator import COVERAGE_BAND, COVERAGE_SEEDS, coverage_of
    g = inputs.er_2000()
    exact = oracle.estimate(g.row_ptr, g.col, 1.0, 0)["exact"]
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    try:
        _say("coverage over %d seeds on er(2000, 0.005) at p=0.1" % COVERAGE_SEEDS)
        runs = [lge.lge_estimate(ctx, h, 0.1, 1000 + s) for s in range(COVERAGE_SEEDS)]
    finally:
        lge.lge_graph_destroy(h)
    for s in (0, COVERAGE_SEEDS // 2, COVERAGE_SEEDS - 1):
        assert_parity(runs[s], oracle.estimate(g.row_ptr, g.col, 0.1, 1000 + s), "coverage seed %d" % s)
    cov = coverage_of(runs, exact)
    for i, c in cov.items():
        assert COVERAGE_BAND[0] <= c <= COVERAGE_BAND[1], (i, c)


def test_single_hub_without_co_degree_table(ctx):
    # one vertex above degree 96 (so no co-degree table, no ranks, no rows):
    # a hub of degree 3001, its leaves on a ring, and a vertex of degree 80
    # adjacent to the hub and 79 leaves, whose edge to the hub is a split-class
    # work item; the hub's other edges go to the wavefront kernel via its table
    k = 3000
    e = [(0, i) for i in range(1, k + 1)] + [(i, i % k + 1) for i in range(1, k + 1)]
    e += [(0, k + 1)] + [(k + 1, i) for i in range(1, 80)]
    g = inputs.from_edges(k + 2, np.array(e, dtype=np.int32))
    for p, seed in ((1.0, 0), (0.3, 12)):
        run_pair(ctx, g, p, seed, what="single hub p=%g" % p)
