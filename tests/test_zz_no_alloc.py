"""The allocation-free entry point (lge_estimate_noalloc) through the C ABI.

It must return what lge_estimate returns (every integer and every double
equal), match the oracle to the usual bar, keep doing so on consecutive
calls (the second with a smaller graph, then a larger one, so stale contents
of the shared workspace would show), allocate no device memory, and refuse
graphs beyond its stated limit with LGE_ERANGE while the context stays usable.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1701_01772_amd import inputs, lge

pytestmark = pytest.mark.gpu

REL = 1e-12
MAX_EDGES = 1 << 18


def _say(msg):
    sys.stdout.write("[gpu-noalloc] %s\n" % msg)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = lge.lge_open(0)
    yield c
    lge.lge_close(c)


def _same(a, b, what):
    for k in ("sampled", "csum", "zsum", "qsum", "exact", "estimate", "variance", "lower95", "upper95"):
        assert a[k] == b[k], (what, k)


def _parity(got, want, what):
    assert got["sampled"] == want["sampled"], what
    for key in ("csum", "zsum", "qsum"):
        for i in range(3, 18):
            assert got[key][i] == want[key][i], (what, key, i)
    if want["p"] == 1.0:
        assert got["exact"][1:] == want["exact"][1:], what
    for key in ("estimate", "variance", "lower95", "upper95"):
        for i in range(1, 18):
            a, b = got[key][i], want[key][i]
            assert a == b or abs(a - b) <= REL * max(abs(a), abs(b)), (what, key, i, a, b)


def _hub_graph(seed=3):
    # two hubs of degree > 1024 sharing neighbours: split-class work items
    rng = np.random.default_rng(seed)
    n = 4000
    e = [(0, 1)]
    n0 = rng.choice(np.arange(2, n), 2000, replace=False)
    n1 = np.concatenate([n0[:900], rng.choice(np.arange(2, n), 1200, replace=False)])
    e += [(0, int(x)) for x in n0] + [(1, int(x)) for x in n1]
    a = rng.integers(2, n, 9000)
    b = rng.integers(2, n, 9000)
    e += [(int(x), int(y)) for x, y in zip(a, b)]
    return inputs.from_edges(n, e)


def _free_bytes():
    import torch
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info(0)[0]


def test_noalloc_equals_estimate_on_consecutive_calls(ctx):
    cases = [
        (inputs.chung_lu(30000, 10.0, 2.1, 3000.0, 41), 0.3, 7, "chung-lu-30k p=0.3"),
        (inputs.er_2000(), 1.0, 0, "er(2000,0.005) p=1 (smaller)"),
        (_hub_graph(), 0.5, 11, "two hubs p=0.5 (split class)"),
        (inputs.rmat(13, 16, 0.57, 0.19, 0.19, 9), 1.0, 0, "rmat-13 p=1 (larger)"),
        (inputs.from_edges(6, [(0, 1), (1, 2)]), 1.0, 0, "tiny"),
    ]
    free0 = None
    for g, p, seed, what in cases:
        assert g.m <= MAX_EDGES, what
        _say("%s: n=%d m=%d" % (what, g.n, g.m))
        h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
        try:
            want_lib = lge.lge_estimate(ctx, h, p, seed)
            free_before = _free_bytes()
            got = lge.lge_estimate_noalloc(ctx, h, p, seed)
            again = lge.lge_estimate_noalloc(ctx, h, p, seed)
            free_after = _free_bytes()
        finally:
            lge.lge_graph_destroy(h)
        assert free_after == free_before, (what, free_before, free_after)  # nothing allocated
        _same(got, want_lib, what)
        _same(again, want_lib, what + " (again)")
        _parity(got, oracle.estimate(g.row_ptr, g.col, p, seed), what)
        if free0 is None:
            free0 = free_before


def test_noalloc_rejects_beyond_its_limit(ctx):
    g = inputs.chung_lu(60000, 10.0, 2.1, 3000.0, 5)  # m > 2^18
    assert g.m > MAX_EDGES
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    try:
        with pytest.raises(lge.LgeError) as ei:
            lge.lge_estimate_noalloc(ctx, h, 0.5, 1)
        assert ei.value.code == lge.LGE_ERANGE
        # the context and the graph stay usable on both paths
        base = lge.lge_estimate(ctx, h, 0.01, 2)
        _parity(base, oracle.estimate(g.row_ptr, g.col, 0.01, 2), "after rejection")
    finally:
        lge.lge_graph_destroy(h)
    g2 = inputs.er_2000()
    h2 = lge.lge_graph_create_host(ctx, g2.row_ptr, g2.col)
    try:
        _same(lge.lge_estimate_noalloc(ctx, h2, 0.7, 4), lge.lge_estimate(ctx, h2, 0.7, 4), "after rejection")
    finally:
        lge.lge_graph_destroy(h2)


def test_noalloc_rejects_split_work_beyond_its_layout(ctx):
    # complete bipartite 200 x 1300: every edge has an endpoint of degree
    # 1300 > 1024, so all 260,000 edges are split-class work items, more than
    # the layout's 16,384; the call fails cleanly and lge_estimate still serves
    na, nb = 200, 1300
    e = [(a, na + b) for a in range(na) for b in range(nb)]
    g = inputs.from_edges(na + nb, np.array(e, dtype=np.int32))
    assert g.m <= MAX_EDGES
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    try:
        with pytest.raises(lge.LgeError) as ei:
            lge.lge_estimate_noalloc(ctx, h, 1.0, 0)
        assert ei.value.code == lge.LGE_ERANGE
        r = lge.lge_estimate(ctx, h, 1.0, 0)
        import math
        assert r["exact"][10] == math.comb(na, 2) * math.comb(nb, 2)  # 4-cycles of K_{a,b}
        assert r["exact"][3] == 0 and r["exact"][7] == 0
        small = lge.lge_estimate_noalloc(ctx, h, 0.01, 5)  # a sample that fits
        _same(small, lge.lge_estimate(ctx, h, 0.01, 5), "K_{200,1300} p=0.01")
    finally:
        lge.lge_graph_destroy(h)


def test_noalloc_bad_arguments(ctx):
    g = inputs.er_2000()
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    try:
        for p in (0.0, -1.0, 1.5):
            with pytest.raises(lge.LgeError) as ei:
                lge.lge_estimate_noalloc(ctx, h, p, 1)
            assert ei.value.code == lge.LGE_EINVAL
    finally:
        lge.lge_graph_destroy(h)
