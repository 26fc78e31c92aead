"""Pins of the CPU oracle against facts that do not come from the oracle.

* Table 1 fixture: its properties separate the 17 graphlets, and every
  labelled 3-/4-vertex graph falls into a class whose printed triangle
  count, mean degree and chromatic number it has.
* Brute-force census of every 3-/4-subset (classes from Table 1).
* Closed forms on complete, complete bipartite, star, cycle, empty graphs.
* Textbook counting identities at sizes brute force cannot reach (traces of
  A^3, common-neighbour counts, degree sums, triangle extension).
"""
import itertools
import math
import random

import numpy as np
import pytest

import oracle
from oracle import bruteforce as bf
from paper_1701_01772_amd import inputs


def _graph(n, edges):
    return inputs.from_edges(n, edges)


def _exact(g):
    r = oracle.estimate(g.row_ptr, g.col, 1.0, 0)
    assert r["sampled"] == g.m
    return r["exact"]


# --------------------------------------------------------------------------
# Table 1 fixture
# --------------------------------------------------------------------------

def _chromatic(k, edges):
    for c in range(1, k + 1):
        for col in itertools.product(range(c), repeat=k):
            if all(col[a] != col[b] for a, b in edges):
                return c
    return k


def test_table1_separates_all_graphlets(table1):
    cls = bf.classifier(table1)
    assert sorted(cls.values()) == list(range(1, 18))
    for r in table1:
        assert abs(r["meandeg"] - 2 * r["edges"] / r["k"]) < 0.01


@pytest.mark.parametrize("k", [2, 3, 4])
def test_every_labelled_graph_matches_table1(table1, k):
    cls = bf.classifier(table1)
    rows = {r["id"]: r for r in table1}
    pairs = list(itertools.combinations(range(k), 2))
    seen = set()
    for mask in range(1 << len(pairs)):
        es = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        adj = [set() for _ in range(k)]
        for a, b in es:
            adj[a].add(b)
            adj[b].add(a)
        gid = cls[bf.signature(tuple(range(k)), adj)]
        seen.add(gid)
        row = rows[gid]
        tri = sum(1 for a, b, c in itertools.combinations(range(k), 3)
                  if b in adj[a] and c in adj[a] and c in adj[b])
        assert tri == row["triangles"]
        assert _chromatic(k, es) == row["chromatic"]
    expect = {2: {1, 2}, 3: {3, 4, 5, 6}, 4: set(range(7, 18))}[k]
    assert seen == expect


# --------------------------------------------------------------------------
# Brute force
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(40))
def test_oracle_matches_bruteforce(table1, seed):
    rng = random.Random(seed)
    n = rng.randint(4, 13)
    q = rng.choice([0.1, 0.25, 0.4, 0.6, 0.8, 0.95])
    g = inputs.erdos_renyi(n, q, 1000 + seed)
    assert _exact(g)[1:] == bf.census_csr(g.row_ptr, g.col, table1)[1:]


def test_oracle_matches_bruteforce_powerlaw(table1):
    g = inputs.chung_lu(22, 5.0, 2.1, 21.0, 7)
    assert _exact(g)[1:] == bf.census_csr(g.row_ptr, g.col, table1)[1:]


def test_isolated_vertices_count(table1):
    # vertices with no edges still belong to every disconnected graphlet
    g = _graph(9, [(0, 1), (1, 2), (2, 0), (3, 4)])
    assert _exact(g)[1:] == bf.census_csr(g.row_ptr, g.col, table1)[1:]


# --------------------------------------------------------------------------
# Closed forms
# --------------------------------------------------------------------------

def _vec(**kw):
    v = [0] * 18
    for k, x in kw.items():
        v[int(k[1:])] = x
    return v


def test_complete_graph():
    for n in (4, 5, 9):
        g = _graph(n, itertools.combinations(range(n), 2))
        assert _exact(g) == _vec(G1=math.comb(n, 2), G3=math.comb(n, 3), G7=math.comb(n, 4))


def test_complete_bipartite():
    for a, b in ((2, 3), (3, 4), (4, 6)):
        es = [(i, a + j) for i in range(a) for j in range(b)]
        g = _graph(a + b, es)
        n = a + b
        want = _vec(G1=a * b, G2=math.comb(a, 2) + math.comb(b, 2),
                    G4=a * math.comb(b, 2) + b * math.comb(a, 2),
                    G6=math.comb(a, 3) + math.comb(b, 3),
                    G10=math.comb(a, 2) * math.comb(b, 2),
                    G11=a * math.comb(b, 3) + b * math.comb(a, 3),
                    G17=math.comb(a, 4) + math.comb(b, 4))
        # 3-node-1-edge: an edge plus a vertex of the same side as one endpoint
        want[5] = a * b * (n - 2) - 2 * want[4]
        # every vertex is adjacent to the whole other side, so no induced
        # subgraph has an isolated vertex next to an edge: G13..G16 vanish
        got = _exact(g)
        assert got == want


def test_star():
    for k in (3, 5, 8):
        g = _graph(k + 1, [(0, i) for i in range(1, k + 1)])
        n = k + 1
        want = _vec(G1=k, G2=math.comb(k, 2), G4=math.comb(k, 2), G5=0, G6=math.comb(k, 3),
                    G11=math.comb(k, 3), G17=math.comb(k, 4))
        want[14] = 0
        got = _exact(g)
        assert got == want


def test_cycle():
    for n in (5, 6, 9):
        g = _graph(n, [(i, (i + 1) % n) for i in range(n)])
        got = _exact(g)
        assert got[3] == 0 and got[10] == 0
        assert got[4] == n and got[12] == n
        assert got[1] == n
        assert sum(got[3:7]) == math.comb(n, 3)
        assert sum(got[7:18]) == math.comb(n, 4)


def test_four_cycle_exactly():
    g = _graph(4, [(0, 1), (1, 2), (2, 3), (3, 0)])
    assert _exact(g) == _vec(G1=4, G2=2, G4=4, G10=1)


def test_empty_graph():
    for n in (1, 4, 7):
        g = _graph(n, [])
        r = oracle.estimate(g.row_ptr, g.col, 1.0, 0)
        assert r["sampled"] == 0
        assert r["exact"] == _vec(G2=math.comb(n, 2), G6=math.comb(n, 3), G17=math.comb(n, 4))


# --------------------------------------------------------------------------
# Counting identities at moderate n
# --------------------------------------------------------------------------

def _identity_census(g):
    """Exact G1..G17 from degree sums, A^2/A^3 and an independent 4-clique
    enumeration (triangle extension over bitsets); no per-edge local search."""
    n, m = g.n, g.m
    A = np.zeros((n, n), dtype=np.int64)
    src = np.repeat(np.arange(n), g.degrees())
    A[src, g.col] = 1
    d = A.sum(1)
    A2 = A @ A
    A3d = np.einsum("ij,ji->i", A2, A)  # diag of A^3
    tri = int(A3d.sum() // 6)
    tv = A3d // 2  # triangles at each vertex
    wedges = int((d * (d - 1) // 2).sum())
    # 4-cliques: extend each triangle i<j<k by l>k adjacent to all three
    nb = [set(np.nonzero(A[i])[0].tolist()) for i in range(n)]
    k4 = 0
    for i in range(n):
        for j in (x for x in nb[i] if x > i):
            cij = nb[i] & nb[j]
            for k in (x for x in cij if x > j):
                k4 += sum(1 for l in (cij & nb[k]) if l > k)
    iu = np.triu_indices(n, 1)
    cod = A2[iu]
    adj = A[iu] == 1
    c2 = cod * (cod - 1) // 2
    s_adj = int(c2[adj].sum())  # = 6 G7 + G8
    s_non = int(c2[~adj].sum())  # = G8 + 2 G10
    G = [0] * 18
    G[1] = m
    G[2] = math.comb(n, 2) - m
    G[3] = tri
    G[4] = wedges - 3 * tri
    G[5] = m * (n - 2) - 3 * G[3] - 2 * G[4]
    G[6] = math.comb(n, 3) - G[3] - G[4] - G[5]
    G[7] = k4
    G[8] = s_adj - 6 * k4
    G[10] = (s_non - G[8]) // 2
    G[9] = int((tv * (d - 2)).sum()) - 4 * G[8] - 12 * G[7]
    G[11] = int((d * (d - 1) * (d - 2) // 6).sum()) - G[9] - 2 * G[8] - 4 * G[7]
    eu, ev = np.nonzero(np.triu(A, 1))
    p4 = int(((d[eu] - 1) * (d[ev] - 1)).sum()) - 3 * tri
    G[12] = p4 - 4 * G[10] - 2 * G[9] - 6 * G[8] - 12 * G[7]
    G[13] = tri * (n - 3) - G[9] - 2 * G[8] - 4 * G[7]
    G[14] = (wedges * (n - 3) - 12 * G[7] - 8 * G[8] - 5 * G[9] - 4 * G[10] - 3 * G[11]
             - 2 * G[12] - 3 * G[13])
    disjoint = math.comb(m, 2) - wedges
    G[15] = disjoint - G[12] - 2 * G[10] - G[9] - 2 * G[8] - 3 * G[7]
    e4 = [0, 0, 0, 0, 0, 0, 0, 6, 5, 4, 4, 3, 3, 3, 2, 2, 1, 0]
    G[16] = m * math.comb(n - 2, 2) - sum(e4[i] * G[i] for i in range(7, 16))
    G[17] = math.comb(n, 4) - sum(G[7:17])
    # the closed-4-walk identity is a further check of G7, G8, G10
    tr4 = int((A2 * A2).sum())
    assert (tr4 - 2 * int((d * d).sum()) + 2 * m) // 8 == G[10] + G[8] + 3 * G[7]
    return G


@pytest.mark.parametrize("maker", [
    lambda: inputs.erdos_renyi(300, 0.08, 11),
    lambda: inputs.erdos_renyi(120, 0.5, 12),
    lambda: inputs.chung_lu(800, 12.0, 2.1, 200.0, 13),
    lambda: inputs.rmat(9, 8, 0.57, 0.19, 0.19, 14),
])
def test_counting_identities(maker):
    g = maker()
    assert _exact(g) == _identity_census(g)


def test_identity_census_agrees_with_bruteforce(table1):
    # the identity census itself is pinned to the enumeration
    for s in range(6):
        g = inputs.erdos_renyi(11, 0.45, 500 + s)
        assert _identity_census(g)[1:] == bf.census_csr(g.row_ptr, g.col, table1)[1:]


def test_sum_invariants_bruteforce(table1):
    g = inputs.erdos_renyi(12, 0.5, 3)
    c = bf.census_csr(g.row_ptr, g.col, table1)
    assert sum(c[1:3]) == math.comb(12, 2)
    assert sum(c[3:7]) == math.comb(12, 3)
    assert sum(c[7:18]) == math.comb(12, 4)
