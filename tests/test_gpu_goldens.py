"""Whole-graph parity at full size: the HIP path (through the C ABI, default
launch configuration, as the benchmark runs it) against stored oracle
goldens of the full-size workloads.

The goldens (tests/golden/*.json) were written by
tests/golden/make_goldens.py, which calls only the oracle (split over host
threads, whose exact integer sums add up to one call's) and the seeded input
generators.  Each holds the generated graph's SHA-256 fingerprint, checked
first.  Bar: the sampled-edge count, the 13 C, 15 Z and 15 Q sums and (at
p = 1) the 17 exact counts bit-equal; every FP64 output within a relative
1e-12.  Each run must also give every edge class (wavefront, workgroup,
split global) at least 1,000 sampled edges, so the kernels that dominate the
workload are the ones compared; the test logs the per-class counts.
"""
import os
import sys

import pytest

from paper_1701_01772_amd import inputs, lge

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_goldens  # noqa: E402

REL = 1e-12
CLASS_NAMES = ("wavefront", "workgroup", "split")


def _say(msg):
    sys.stdout.write("[gpu-golden] %s\n" % msg)
    sys.stdout.flush()


def _close(a, b):
    return a == b or abs(a - b) <= REL * max(abs(a), abs(b))


_graphs = {}


@pytest.fixture(scope="module")
def ctx():
    c = lge.lge_open(0)
    yield c
    for k in list(_graphs):  # graphs first: a graph must not outlive its context
        lge.lge_graph_destroy(_graphs.pop(k)[1])
    lge.lge_close(c)


def _resident(ctx, maker):
    if maker not in _graphs:
        for k in list(_graphs):  # one full-size graph resident at a time
            lge.lge_graph_destroy(_graphs.pop(k)[1])
        _say("generating %s" % maker)
        g = getattr(inputs, maker)()
        _graphs[maker] = (g, lge.lge_graph_create_host(ctx, g.row_ptr, g.col))
    return _graphs[maker]


@pytest.mark.parametrize("name", ["chung_lu_1m_p0.01", "chung_lu_1m_p0.1", "chung_lu_1m_p1", "rmat_s22_p0.01"])
def test_whole_graph_equals_golden(ctx, name):
    if not os.path.exists(make_goldens.path_of(name)):
        pytest.skip("golden %s not written" % name)
    want = make_goldens.load(name)
    g, h = _resident(ctx, want["maker"])
    assert make_goldens.graph_fingerprint(g) == want["graph_sha256"], "generator output changed"
    assert (g.n, g.m) == (want["n"], want["m"])
    _say("%s: n=%d m=%d p=%g seed=%d" % (name, g.n, g.m, want["p"], want["seed"]))
    got = lge.lge_estimate(ctx, h, want["p"], want["seed"])
    cls = lge.lge_last_timing(ctx)["class_edges"]
    _say("%s: sampled %d, per class %s" % (
        name, got["sampled"], ", ".join("%s %d" % (c, k) for c, k in zip(CLASS_NAMES, cls))))
    assert got["sampled"] == want["sampled"]
    assert sum(cls) == want["sampled"]
    assert all(k >= 1000 for k in cls), cls
    for key in ("csum", "zsum", "qsum"):
        for i in range(3, 18):
            assert got[key][i] == want[key][i], (name, key, i, got[key][i], want[key][i])
    if want["p"] == 1.0:
        assert got["exact"][1:] == want["exact"][1:], name
    for key in ("estimate", "variance", "lower95", "upper95"):
        for i in range(1, 18):
            assert _close(got[key][i], want[key][i]), (name, key, i, got[key][i], want[key][i])


@pytest.mark.parametrize("n", [100_000, 1_000_000])
@pytest.mark.parametrize("p", [1.0, 0.5])
def test_constants_above_2_53(ctx, n, p):
    # an empty graph's X6 = C(n,3) and X17 = C(n,4) exercise the library's
    # correctly rounded int128 -> double conversion above 2^53
    import math
    g = inputs.from_edges(n, [])
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    try:
        r = lge.lge_estimate(ctx, h, p, 3)
    finally:
        lge.lge_graph_destroy(h)
    assert r["estimate"][17] == float(math.comb(n, 4))
    assert r["estimate"][6] == float(math.comb(n, 3))
    assert r["exact"][17] == math.comb(n, 4)
