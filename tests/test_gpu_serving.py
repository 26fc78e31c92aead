"""Serving loop on the GPU: continuous batching returns, for every request,
exactly what the same (graph, p, seed) gives alone; failure paths (timeout,
cancellation, full queue, shutdown with waiters) resolve every ticket."""
import sys
import threading
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_1701_01772_amd import inputs, lge

pytestmark = pytest.mark.gpu


def _say(msg):
    sys.stdout.write("[gpu-serving] %s\n" % msg)
    sys.stdout.flush()


INT_KEYS = ("sampled", "csum", "zsum", "qsum", "exact")


def _same(a, b):
    for k in INT_KEYS:
        assert a[k] == b[k], k
    for k in ("estimate", "variance", "lower95", "upper95"):
        assert a[k] == b[k], k


@pytest.fixture(scope="module")
def graphs():
    gs = [inputs.erdos_renyi(300, 0.05, 1), inputs.chung_lu(6000, 8.0, 2.1, 1500.0, 2),
          inputs.rmat(11, 16, 0.57, 0.19, 0.19, 3), inputs.chung_lu(20000, 10.0, 2.1, 3000.0, 4),
          inputs.from_edges(6, [(0, 1)]), inputs.from_edges(5, [])]
    return gs


def _server(ctx, **kw):
    cfg = lge.lge_server_cfg_default()
    for k, v in kw.items():
        setattr(cfg, k, v)
    return lge.lge_server_create(ctx, cfg)


def test_alone_equals_mix(graphs):
    alone_ctx = lge.lge_open(0)
    ctx = lge.lge_open(0)
    hs = [lge.lge_graph_create_host(ctx, g.row_ptr, g.col) for g in graphs]
    ha = [lge.lge_graph_create_host(alone_ctx, g.row_ptr, g.col) for g in graphs]
    # tiny step budget: every request larger than ~3000 edge ids is chunked
    # across steps and shares steps with others
    srv = _server(ctx, max_inflight=5, hbm_budget_bytes=128 * 6000, min_chunk_edges=500)
    try:
        gids = [lge.lge_server_add_graph(srv, h) for h in hs]
        rng = np.random.default_rng(0)
        reqs = [(int(rng.integers(0, len(gids))), float(rng.choice([1.0, 0.3, 0.01])), 100 + i) for i in range(40)]
        _say("submitting %d requests from 4 threads" % len(reqs))
        tickets = [None] * len(reqs)

        def submit(idx):
            gi, p, s = reqs[idx]
            tickets[idx] = lge.lge_submit(srv, gids[gi], p, s)
            time.sleep(0.001 * (idx % 3))

        with ThreadPoolExecutor(4) as ex:
            list(ex.map(submit, range(len(reqs))))
        with ThreadPoolExecutor(8) as ex:
            results = list(ex.map(lambda t: lge.lge_wait(srv, t, -1), tickets))
        st = lge.lge_server_get_stats(srv)
        _say("stats %s" % st)
        assert st["completed"] == len(reqs)
        assert st["steps"] > 1
        for (gi, p, s), got in zip(reqs, results):
            _same(got, lge.lge_estimate(alone_ctx, ha[gi], p, s))
        # and against the oracle for the small graphs
        for (gi, p, s), got in list(zip(reqs, results))[:12]:
            g = graphs[gi]
            if g.m <= 60000:
                want = oracle.estimate(g.row_ptr, g.col, p, s)
                for k in ("sampled", "csum", "zsum", "qsum"):
                    assert got[k] == want[k], k
    finally:
        lge.lge_server_destroy(srv)
        for h in hs:
            lge.lge_graph_destroy(h)
        for h in ha:
            lge.lge_graph_destroy(h)
        lge.lge_close(ctx)
        lge.lge_close(alone_ctx)


def test_alone_equals_mix_large():
    # a graph of more than 1e7 edges among small ones, default server
    # configuration (work-profile chunks, short lane): every result equals
    # the same request alone
    big = inputs.chung_lu(1_400_000, 16.0, 2.1, 70000.0, 21)
    assert big.m >= 10_000_000
    gs = [big, inputs.rmat(16, 16, 0.57, 0.19, 0.19, 22), inputs.erdos_renyi(500, 0.02, 23),
          inputs.chung_lu(30000, 10.0, 2.1, 3000.0, 24)]
    ctx = lge.lge_open(0)
    alone_ctx = lge.lge_open(0)
    hs = [lge.lge_graph_create_host(ctx, g.row_ptr, g.col) for g in gs]
    ha = [lge.lge_graph_create_host(alone_ctx, g.row_ptr, g.col) for g in gs]
    srv = _server(ctx)
    try:
        gids = [lge.lge_server_add_graph(srv, h) for h in hs]
        rng = np.random.default_rng(5)
        reqs = [(0, 1.0, 900), (0, 0.1, 901), (0, 0.01, 902)]
        reqs += [(int(rng.integers(1, len(gs))), float(rng.choice([1.0, 0.1, 0.01])), 910 + i) for i in range(24)]
        _say("large mix: m=%d plus %d small requests" % (big.m, len(reqs) - 3))
        tickets = [lge.lge_submit(srv, gids[gi], p, s) for gi, p, s in reqs]
        with ThreadPoolExecutor(8) as ex:
            results = list(ex.map(lambda t: lge.lge_wait(srv, t, -1), tickets))
        for (gi, p, s), got in zip(reqs, results):
            _same(got, lge.lge_estimate(alone_ctx, ha[gi], p, s))
        st = lge.lge_server_get_stats(srv)
        _say("stats %s" % st)
        assert st["completed"] == len(reqs)
    finally:
        lge.lge_server_destroy(srv)
        for h in hs:
            lge.lge_graph_destroy(h)
        for h in ha:
            lge.lge_graph_destroy(h)
        lge.lge_close(ctx)
        lge.lge_close(alone_ctx)


def test_step_workspace_within_budget():
    # the HBM budget bounds what a worker's workspace holds: per-id arrays
    # for half of it, split-class lists (run in pieces) for the other half
    budget = 64 << 20
    gs = [inputs.rmat(16, 16, 0.57, 0.19, 0.19, 51), inputs.chung_lu(150000, 14.0, 2.1, 6000.0, 52)]
    ctx = lge.lge_open(0)
    alone_ctx = lge.lge_open(0)
    hs = [lge.lge_graph_create_host(ctx, g.row_ptr, g.col) for g in gs]
    ha = [lge.lge_graph_create_host(alone_ctx, g.row_ptr, g.col) for g in gs]
    srv = _server(ctx, hbm_budget_bytes=budget)
    try:
        gids = [lge.lge_server_add_graph(srv, h) for h in hs]
        reqs = [(0, 1.0, 61), (1, 1.0, 62), (0, 0.3, 63), (1, 0.05, 64)]
        tickets = [lge.lge_submit(srv, gids[gi], p, sd) for gi, p, sd in reqs]
        results = [lge.lge_wait(srv, t, -1) for t in tickets]
        for (gi, p, sd), got in zip(reqs, results):
            _same(got, lge.lge_estimate(alone_ctx, ha[gi], p, sd))
        st = lge.lge_server_get_stats(srv)
        _say("budget %d MiB: largest workspace %.1f MiB over %d steps" % (
            budget >> 20, st["workspace_bytes"] / 2**20, st["steps"]))
        assert 0 < st["workspace_bytes"] <= budget + (4 << 20)
    finally:
        lge.lge_server_destroy(srv)
        for h in hs:
            lge.lge_graph_destroy(h)
        for h in ha:
            lge.lge_graph_destroy(h)
        lge.lge_close(ctx)
        lge.lge_close(alone_ctx)


def test_short_request_not_behind_long_one():
    # with the short lane a small request submitted after a long one
    # finishes while the long one is still running
    ctx = lge.lge_open(0)
    big = inputs.rmat(18, 16, 0.57, 0.19, 0.19, 31)
    small = inputs.erdos_renyi(400, 0.02, 32)
    hb = lge.lge_graph_create_host(ctx, big.row_ptr, big.col)
    hsm = lge.lge_graph_create_host(ctx, small.row_ptr, small.col)
    t0 = time.perf_counter()
    lge.lge_estimate(ctx, hb, 1.0, 40, raw=True)
    alone_s = time.perf_counter() - t0
    srv = _server(ctx)
    try:
        gb = lge.lge_server_add_graph(srv, hb)
        gsm = lge.lge_server_add_graph(srv, hsm)
        for i in range(3):  # let the server measure its work rate
            lge.lge_wait(srv, lge.lge_submit(srv, gsm, 1.0, 50 + i), -1)
        lge.lge_wait(srv, lge.lge_submit(srv, gb, 0.05, 60), -1)
        tl = lge.lge_submit(srv, gb, 1.0, 41)
        time.sleep(min(0.02, alone_s / 10))
        ts = lge.lge_submit(srv, gsm, 1.0, 42)
        t1 = time.perf_counter()
        rs = lge.lge_wait(srv, ts, -1)
        small_s = time.perf_counter() - t1
        rc_long, _ = lge.lge_wait_rc(srv, tl, 0)
        _say("long alone %.1f ms; short done after %.1f ms, long %s" % (
            alone_s * 1e3, small_s * 1e3, "running" if rc_long == lge.LGE_ETIMEDOUT else "done"))
        assert rs["sampled"] == small.m
        if alone_s > 0.2:  # a long request that is long enough to tell
            assert rc_long == lge.LGE_ETIMEDOUT
        rc, rl = lge.lge_wait_rc(srv, tl, -1)
        assert rc == lge.LGE_OK and rl["sampled"] == big.m
    finally:
        lge.lge_server_destroy(srv)
        lge.lge_graph_destroy(hb)
        lge.lge_graph_destroy(hsm)
        lge.lge_close(ctx)


def test_timeout_cancel_busy_and_shutdown():
    ctx = lge.lge_open(0)
    g = inputs.chung_lu(200000, 12.0, 2.1, 6000.0, 9)
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    srv = _server(ctx, max_inflight=1, queue_capacity=4, hbm_budget_bytes=128 * 20000, min_chunk_edges=1000)
    try:
        gid = lge.lge_server_add_graph(srv, h)
        _say("timeout / cancel / busy on n=%d m=%d" % (g.n, g.m))
        t1 = lge.lge_submit(srv, gid, 1.0, 1)      # long: ~60 steps of 20000 ids
        rc, _ = lge.lge_wait_rc(srv, t1, 0)
        assert rc == lge.LGE_ETIMEDOUT             # the ticket stays valid
        t2 = lge.lge_submit(srv, gid, 0.5, 2)
        t3 = lge.lge_submit(srv, gid, 0.5, 3)
        t4 = lge.lge_submit(srv, gid, 0.5, 4)
        with pytest.raises(lge.LgeError) as ei:
            lge.lge_submit(srv, gid, 0.5, 5)
        assert ei.value.code == lge.LGE_EBUSY
        assert lge.lge_cancel(srv, t3) == lge.LGE_OK
        rc3, _ = lge.lge_wait_rc(srv, t3, -1)
        assert rc3 == lge.LGE_ECANCELED
        assert lge.lge_wait_rc(srv, t3, 0)[0] == lge.LGE_ENOTFOUND
        rc1, r1 = lge.lge_wait_rc(srv, t1, -1)
        assert rc1 == lge.LGE_OK and r1["sampled"] == g.m
        rc2, _ = lge.lge_wait_rc(srv, t2, -1)
        assert rc2 == lge.LGE_OK
        # shutdown with a request in flight and a thread blocked on it
        t5 = lge.lge_submit(srv, gid, 1.0, 6)
        out = {}
        w = threading.Thread(target=lambda: out.setdefault("rc", lge.lge_wait_rc(srv, t5, -1)[0]))
        w.start()
        time.sleep(0.05)
        rc4, _ = lge.lge_wait_rc(srv, t4, -1)
        assert rc4 == lge.LGE_OK
        lge.lge_server_destroy(srv)
        srv = None
        w.join(timeout=60)
        assert not w.is_alive()
        assert out["rc"] in (lge.LGE_ECANCELED, lge.LGE_OK)
    finally:
        if srv is not None:
            lge.lge_server_destroy(srv)
        lge.lge_graph_destroy(h)
        lge.lge_close(ctx)


def test_bad_requests():
    ctx = lge.lge_open(0)
    g = inputs.erdos_renyi(50, 0.1, 1)
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    srv = _server(ctx)
    try:
        gid = lge.lge_server_add_graph(srv, h)
        for p in (0.0, 1.5):
            with pytest.raises(lge.LgeError) as ei:
                lge.lge_submit(srv, gid, p, 0)
            assert ei.value.code == lge.LGE_EINVAL
        with pytest.raises(lge.LgeError) as ei:
            lge.lge_submit(srv, gid + 7, 0.5, 0)
        assert ei.value.code == lge.LGE_ENOTFOUND
        assert lge.lge_wait_rc(srv, 123456, 0)[0] == lge.LGE_ENOTFOUND
    finally:
        lge.lge_server_destroy(srv)
        lge.lge_graph_destroy(h)
        lge.lge_close(ctx)
