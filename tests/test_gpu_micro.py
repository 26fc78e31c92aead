"""GPU parity of the micro-level statistics (Sec. 3, Alg. 7 with p_e = 1):
every row bit-equal to the oracle's per-edge classification, column maxima
equal to the maxima of the oracle rows, and at full size the column sums
equal to (edges of G_i) x (exact count of G_i) from the estimator at p = 1."""
import sys

import numpy as np
import pytest

import oracle
from oracle import bruteforce as bf
from paper_1701_01772_amd import inputs, lge

pytestmark = pytest.mark.gpu


def _say(msg):
    sys.stdout.write("[gpu-micro] %s\n" % msg)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = lge.lge_open(0)
    yield c
    lge.lge_close(c)


def _two_hub_graph(seed=3):
    rng = np.random.default_rng(seed)
    n = 5000
    edges = [(0, 1)]
    n0 = rng.choice(np.arange(2, n), 2600, replace=False)
    n1 = np.concatenate([n0[:1300], rng.choice(np.arange(2, n), 1400, replace=False)])
    edges += [(0, int(x)) for x in n0] + [(1, int(x)) for x in n1]
    cl = rng.choice(np.arange(2, n), 40, replace=False)
    edges += [(int(a), int(b)) for i, a in enumerate(cl) for b in cl[i + 1:]]
    a = rng.integers(2, n, 12000)
    b = rng.integers(2, n, 12000)
    edges += [(int(x), int(y)) for x, y in zip(a, b)]
    return inputs.from_edges(n, edges)


def check_rows(ctx, g, e0=0, e1=None, what=""):
    e1 = g.m if e1 is None else e1
    _say("%s n=%d m=%d rows [%d, %d)" % (what, g.n, g.m, e0, e1))
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    try:
        rows, cm = lge.lge_micro(ctx, h, e0, e1)
        got = rows.cpu().numpy()
    finally:
        lge.lge_graph_destroy(h)
    want = oracle.micro(g.row_ptr, g.col, np.arange(e0, e1))
    assert got.shape == want.shape
    bad = np.argwhere(got != want)
    assert bad.size == 0, (what, bad[:5].tolist(), got[bad[0][0]].tolist(), want[bad[0][0]].tolist())
    wmax = want.max(axis=0).tolist() if want.shape[0] else [0] * 17
    assert cm == [0] + wmax
    return got


@pytest.mark.parametrize("maker,name", [
    (lambda: inputs.er_2000(), "er-2000"),
    (lambda: inputs.chung_lu(8000, 10.0, 2.1, 1500.0, 17), "chung-lu-8k"),
    (lambda: _two_hub_graph(), "two-hub"),
    (lambda: inputs.rmat(11, 16, 0.57, 0.19, 0.19, 3), "rmat-11"),
])
def test_rows_equal_oracle(ctx, maker, name):
    check_rows(ctx, maker(), what=name)


def test_ranges_and_degenerate(ctx):
    g = inputs.chung_lu(6000, 8.0, 2.1, 1200.0, 5)
    for e0, e1 in [(0, 0), (5, 6), (123, 4567), (g.m - 1, g.m)]:
        check_rows(ctx, g, e0, e1, "range")
    check_rows(ctx, inputs.from_edges(2, [(0, 1)]), what="one edge")
    check_rows(ctx, inputs.from_edges(9, [(0, i) for i in range(1, 9)]), what="star")
    check_rows(ctx, inputs.from_edges(7, [(a, b) for a in range(7) for b in range(a + 1, 7)]), what="K7")
    empty = inputs.from_edges(4, [])
    h = lge.lge_graph_create_host(ctx, empty.row_ptr, empty.col)
    try:
        rows, cm = lge.lge_micro(ctx, h)
        assert tuple(rows.shape) == (0, 17) and cm == [0] * 18
        with pytest.raises(lge.LgeError) as ei:
            lge.lge_micro(ctx, h, 0, 1)
        assert ei.value.code == lge.LGE_EINVAL
    finally:
        lge.lge_graph_destroy(h)


def test_tiny_graphs_equal_bruteforce(ctx, table1):
    for seed in range(6):
        g = inputs.erdos_renyi(10, 0.5, 100 + seed)
        got = check_rows(ctx, g, what="tiny")
        us, vs = oracle.canonical_edges(g.row_ptr, g.col)
        el = list(zip(us.tolist(), vs.tolist()))
        for k, (u, v) in enumerate(el):
            assert got[k].tolist() == bf.micro_census(g.n, el, table1, u, v)[1:]


def test_repeat_calls_and_estimates_between(ctx):
    g = inputs.chung_lu(6000, 8.0, 2.1, 1200.0, 8)
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    try:
        a, ca = lge.lge_micro(ctx, h)
        lge.lge_estimate(ctx, h, 0.3, 1)
        b, cb = lge.lge_micro(ctx, h, 10, g.m - 10)
        assert (a[10:g.m - 10] == b).all().item()
        assert all(x >= y for x, y in zip(ca, cb))
    finally:
        lge.lge_graph_destroy(h)


def test_full_size_chung_lu(ctx, table1):
    import torch
    g = inputs.chung_lu_1m()
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    try:
        _say("full-size micro n=%d m=%d" % (g.n, g.m))
        rows, cm = lge.lge_micro(ctx, h)
        sums = rows.sum(dim=0).cpu().tolist()
        maxes = rows.max(dim=0).values.cpu().tolist()
        idx = np.random.default_rng(7).choice(g.m, 500, replace=False)
        idx.sort()
        sample = rows[torch.from_numpy(idx).to(rows.device)].cpu().numpy()
        del rows
        exact = lge.lge_estimate(ctx, h, 1.0, 0)["exact"]
    finally:
        lge.lge_graph_destroy(h)
    assert cm == [0] + maxes
    ne = {r["id"]: r["edges"] for r in table1}
    for i in range(3, 17):
        assert sums[i - 1] == ne[i] * exact[i], i
    _say("oracle on %d sampled rows" % len(idx))
    assert (sample == oracle.micro(g.row_ptr, g.col, idx)).all()
