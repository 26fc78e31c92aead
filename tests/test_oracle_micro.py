"""Pins of the micro-level oracle (Sec. 3, Alg. 7 with p_e = 1): per-edge
rows against a brute-force enumeration of the subsets holding both ends of
the edge, column sums against (edges of G_i) x (count of G_i), and closed
forms on complete, bipartite, cycle and star graphs."""
import math

import numpy as np
import pytest

import oracle
from oracle import bruteforce as bf
from paper_1701_01772_amd import inputs


def _edges_per_graphlet(table):
    return {r["id"]: r["edges"] for r in table}


@pytest.mark.parametrize("n,dens,seed", [(9, 0.3, 1), (10, 0.5, 2), (11, 0.7, 3), (12, 0.4, 4), (8, 0.9, 5)])
def test_rows_equal_bruteforce(table1, n, dens, seed):
    g = inputs.erdos_renyi(n, dens, seed)
    us, vs = oracle.canonical_edges(g.row_ptr, g.col)
    rows = oracle.micro(g.row_ptr, g.col)
    assert rows.shape == (g.m, 17)
    edges = list(zip(us.tolist(), vs.tolist()))
    for k, (u, v) in enumerate(edges):
        want = bf.micro_census(n, edges, table1, u, v)[1:]
        assert rows[k].tolist() == want, (u, v)


def test_rows_equal_bruteforce_structured(table1):
    # a hub, a clique, pendant paths: every role of every graphlet shows up
    edges = [(0, i) for i in range(1, 9)] + [(1, 2), (2, 3), (1, 3), (3, 4), (5, 6), (6, 10), (10, 11),
                                            (7, 12), (12, 13), (9, 13), (4, 5)]
    g = inputs.from_edges(14, edges)
    us, vs = oracle.canonical_edges(g.row_ptr, g.col)
    rows = oracle.micro(g.row_ptr, g.col)
    el = list(zip(us.tolist(), vs.tolist()))
    for k, (u, v) in enumerate(el):
        assert rows[k].tolist() == bf.micro_census(14, el, table1, u, v)[1:], (u, v)


@pytest.mark.parametrize("maker", [
    lambda: inputs.erdos_renyi(400, 0.04, 11),
    lambda: inputs.chung_lu(1500, 8.0, 2.1, 300.0, 12),
    lambda: inputs.rmat(9, 8, 0.57, 0.19, 0.19, 13),
])
def test_column_sums_are_edge_weighted_counts(table1, maker):
    # every induced copy of G_i is counted once per edge it has
    g = maker()
    rows = oracle.micro(g.row_ptr, g.col)
    exact = oracle.estimate(g.row_ptr, g.col, 1.0, 0)["exact"]
    ne = _edges_per_graphlet(table1)
    sums = rows.sum(axis=0, dtype=object)
    for i in range(1, 18):
        assert sums[i - 1] == ne[i] * exact[i], i


def test_eid_subset_matches_full():
    g = inputs.chung_lu(800, 6.0, 2.2, 120.0, 3)
    full = oracle.micro(g.row_ptr, g.col)
    idx = np.array([0, g.m - 1, 17, 5, 5, 300])
    assert (oracle.micro(g.row_ptr, g.col, idx) == full[idx]).all()


def test_closed_forms():
    C = math.comb
    # K_n: every edge has T = the other n-2 vertices
    n = 9
    g = inputs.from_edges(n, [(a, b) for a in range(n) for b in range(a + 1, n)])
    row = oracle.micro(g.row_ptr, g.col)[0]
    want = [0] * 17
    want[0], want[2], want[6] = 1, n - 2, C(n - 2, 2)
    assert row.tolist() == want
    # K_{a,b}: T empty, S_u = b-1, S_v = a-1 (u on the a side), 4-cycles (a-1)(b-1)
    a, b = 4, 6
    g = inputs.from_edges(a + b, [(x, a + y) for x in range(a) for y in range(b)])
    row = oracle.micro(g.row_ptr, g.col)[0]
    su, sv = b - 1, a - 1
    want = [0] * 17
    want[0], want[3], want[9] = 1, su + sv, su * sv
    want[10] = C(su, 2) + C(sv, 2)
    assert row.tolist() == want
    # C_n (n >= 6): two 2-stars, two 4-paths with e in the middle... and ends
    n = 10
    g = inputs.from_edges(n, [(i, (i + 1) % n) for i in range(n)])
    rows = oracle.micro(g.row_ptr, g.col)
    r = n - 4
    for row in rows:
        assert row[3] == 2 and row[4] == r and row[11] == 3
        assert row[13] == 2 * r - 2 and row[14] == r - 1 and row[15] == C(r, 2) - (r - 1)
    # star K_{1,k}: each edge is in C(k-1,2) 3-stars and k-1 2-stars
    k = 7
    g = inputs.from_edges(k + 1, [(0, i) for i in range(1, k + 1)])
    for row in oracle.micro(g.row_ptr, g.col):
        assert row[3] == k - 1 and row[10] == C(k - 1, 2) and row[4] == 0 and row[15] == 0
