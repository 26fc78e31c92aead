"""GPU parity of the other sampling designs: k-core numbers, weighted
(degree / k-core) Horvitz-Thompson sampling and fixed-size samples with the
ratio estimator, against the oracle.  Integers bit-equal; class
probabilities equal; FP64 within a relative 1e-12 of the larger magnitude.
Both sides combine the exact per-class sums in class order with the same
IEEE operations, so the weighted estimate is held to the same bar even when
its class terms cancel."""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import designs as D
from paper_1701_01772_amd import inputs, lge

pytestmark = pytest.mark.gpu
REL = 1e-12


def _say(msg):
    sys.stdout.write("[gpu-designs] %s\n" % msg)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = lge.lge_open(0)
    yield c
    lge.lge_close(c)


def _close(a, b):
    if a == b or (math.isnan(a) and math.isnan(b)):
        return True
    return abs(a - b) <= REL * max(abs(a), abs(b))


GRAPHS = [
    (lambda: inputs.er_2000(), "er-2000"),
    (lambda: inputs.chung_lu(20000, 10.0, 2.1, 3000.0, 41), "chung-lu-20k"),
    (lambda: inputs.rmat(12, 16, 0.57, 0.19, 0.19, 5), "rmat-12"),
    (lambda: inputs.from_edges(9, [(a, b) for a in range(6) for b in range(a + 1, 6)] + [(6, 7)]), "K6+edge+isolated"),
]


@pytest.mark.parametrize("maker,name", GRAPHS)
def test_core_numbers(ctx, maker, name):
    g = maker()
    _say("cores %s n=%d m=%d" % (name, g.n, g.m))
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    try:
        core, mc = lge.lge_core_numbers(ctx, h)
        got = core.cpu().numpy()
    finally:
        lge.lge_graph_destroy(h)
    want = D.core_numbers(g.row_ptr, g.col)
    assert (got == want).all()
    assert mc == int(want.max())


def _weighted_check(ctx, g, mode, p_mean, seed, what):
    _say("weighted %s mode=%d p=%g" % (what, mode, p_mean))
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    try:
        got, info = lge.lge_estimate_weighted(ctx, h, mode, p_mean, seed)
    finally:
        lge.lge_graph_destroy(h)
    want = D.estimate_weighted(g.row_ptr, g.col, mode, p_mean, seed)
    for l in range(16):
        assert info["p_level"][l] == want["p_level"][l], (l, info["p_level"][l], want["p_level"][l])
    assert info["edges"] == want["hist"]
    assert info["sampled"] == want["sampled_level"]
    assert got["sampled"] == want["sampled"]
    for key in ("csum", "zsum", "qsum"):
        for i in range(3, 18):
            assert got[key][i] == want[key][i], (key, i)
    for i in range(1, 18):
        assert _close(got["estimate"][i], want["estimate"][i]), (i, got["estimate"][i], want["estimate"][i])
        assert _close(got["variance"][i], want["variance"][i]), (i, got["variance"][i], want["variance"][i])
    return got, info


@pytest.mark.parametrize("mode", [lge.LGE_WEIGHT_DEGREE, lge.LGE_WEIGHT_KCORE])
@pytest.mark.parametrize("p_mean", [0.05, 0.3, 1.0])
def test_weighted_equals_oracle(ctx, mode, p_mean):
    g = inputs.chung_lu(20000, 10.0, 2.1, 3000.0, 41)
    _weighted_check(ctx, g, mode, p_mean, 17, "chung-lu-20k")


def test_weighted_other_graphs(ctx):
    _weighted_check(ctx, inputs.er_2000(), lge.LGE_WEIGHT_KCORE, 0.5, 3, "er-2000")
    _weighted_check(ctx, inputs.rmat(12, 16, 0.57, 0.19, 0.19, 5), lge.LGE_WEIGHT_DEGREE, 0.1, 4, "rmat-12")


def test_weighted_bad_args(ctx):
    g = inputs.er_2000()
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    try:
        for mode, p in ((0, 0.5), (3, 0.5), (1, 0.0), (2, 1.5)):
            with pytest.raises(lge.LgeError) as ei:
                lge.lge_estimate_weighted(ctx, h, mode, p, 1)
            assert ei.value.code == lge.LGE_EINVAL
        for k in (0, g.m + 1):
            with pytest.raises(lge.LgeError) as ei:
                lge.lge_estimate_fixed_k(ctx, h, k, 1)
            assert ei.value.code == lge.LGE_EINVAL
    finally:
        lge.lge_graph_destroy(h)


@pytest.mark.parametrize("maker,name", GRAPHS[:3])
def test_fixed_k_equals_oracle(ctx, maker, name):
    g = maker()
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    try:
        for k in (1, 2, 1000, g.m // 3, g.m):
            _say("fixed-K %s K=%d m=%d" % (name, k, g.m))
            got = lge.lge_estimate_fixed_k(ctx, h, k, 11)
            want = D.estimate_fixed_k(g.row_ptr, g.col, k, 11)
            assert got["sampled"] == k
            for key in ("csum", "zsum", "qsum"):
                for i in range(3, 18):
                    assert got[key][i] == want[key][i], (key, i)
            for i in range(1, 18):
                assert _close(got["estimate"][i], want["estimate"][i]), (i, got["estimate"][i], want["estimate"][i])
                assert _close(got["variance"][i], want["variance"][i]), (i, got["variance"][i], want["variance"][i])
    finally:
        lge.lge_graph_destroy(h)


def test_full_size_cores_and_classes(ctx):
    g = inputs.chung_lu_1m()
    h = lge.lge_graph_create_host(ctx, g.row_ptr, g.col)
    try:
        _say("full-size cores and k-core classes n=%d m=%d" % (g.n, g.m))
        core, mc = lge.lge_core_numbers(ctx, h)
        got_core = core.cpu().numpy()
        r, info = lge.lge_estimate_weighted(ctx, h, lge.LGE_WEIGHT_KCORE, 0.1, 2024)
        k = 200000
        fk = lge.lge_estimate_fixed_k(ctx, h, k, 2024)
    finally:
        lge.lge_graph_destroy(h)
    want_core = D.core_numbers(g.row_ptr, g.col)
    assert (got_core == want_core).all() and mc == int(want_core.max())
    lv = D.levels_of(D.edge_weights(g.row_ptr, g.col, D.WEIGHT_KCORE))
    hist = [int((lv == l).sum()) for l in range(16)]
    assert info["edges"] == hist
    pl = D.plan(hist, 0.1, g.m)
    for l in range(16):
        assert _close(info["p_level"][l], pl[l])
        mask = oracle.sample_mask(2024, pl[l], g.m) & (lv == l)
        assert info["sampled"][l] == int(mask.sum()), l
    assert fk["sampled"] == k
    # the fixed-size sample is the K smallest keys
    keys = oracle.philox_keys(2024, g.m)
    kth = np.sort(keys)[k - 1]
    assert int((keys <= kth).sum()) == k
