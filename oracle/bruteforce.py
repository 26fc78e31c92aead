"""ORACLE (test infrastructure only): brute-force graphlet census.

Enumerates every 2-, 3- and 4-vertex subset of a tiny graph, takes the
induced subgraph (Sec. 2.1: a k-graphlet is an induced k-vertex subgraph)
and identifies its class from the properties listed in Table 1
(table:graphlet_notation): number of vertices k, number of edges
(density * C(k,2)), maximum degree and number of connected components.
Those four properties single out each of G1..G17, so the census needs no
hand-written pattern matching.  Pure Python: meant for n up to ~25.
"""
from __future__ import annotations

import itertools
import math


def load_table(path: str):
    """Rows of the Table 1 fixture: dicts with id, k, edges, maxdeg,
    meandeg, triangles, components, name."""
    rows = []
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            f = line.split()
            k = int(f[1])
            density = float(f[2])
            rows.append({
                "id": int(f[0]), "k": k, "density": density,
                "edges": int(round(density * math.comb(k, 2))),
                "maxdeg": int(f[3]), "meandeg": float(f[4]), "triangles": int(f[5]),
                "kcore": int(f[6]), "chromatic": int(f[7]), "components": int(f[8]), "name": f[9],
            })
    return rows


def _components(vs, adj):
    seen, comps = set(), 0
    for s in vs:
        if s in seen:
            continue
        comps += 1
        stack = [s]
        seen.add(s)
        while stack:
            x = stack.pop()
            for y in vs:
                if y not in seen and y in adj[x]:
                    seen.add(y)
                    stack.append(y)
    return comps


def signature(vs, adj):
    """(k, edges, maxdeg, components) of the subgraph induced by vs."""
    deg = {x: sum(1 for y in vs if y != x and y in adj[x]) for x in vs}
    edges = sum(deg.values()) // 2
    return len(vs), edges, max(deg.values()) if deg else 0, _components(vs, adj)


def classifier(table):
    """Map signature -> graphlet id, asserting that Table 1 makes it unique."""
    out = {}
    for r in table:
        key = (r["k"], r["edges"], r["maxdeg"], r["components"])
        if key in out:
            raise ValueError("Table 1 properties do not separate G%d and G%d" % (out[key], r["id"]))
        out[key] = r["id"]
    return out


def census(n: int, edges, table):
    """Exact counts of G1..G17 (list indexed 0..17, slot 0 unused)."""
    adj = [set() for _ in range(n)]
    for a, b in edges:
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    cls = classifier(table)
    counts = [0] * 18
    for k in (2, 3, 4):
        for vs in itertools.combinations(range(n), k):
            counts[cls[signature(vs, adj)]] += 1
    return counts


def census_csr(row_ptr, col, table):
    n = len(row_ptr) - 1
    edges = [(a, int(col[j])) for a in range(n) for j in range(row_ptr[a], row_ptr[a + 1]) if a < col[j]]
    return census(n, edges, table)


def micro_census(n: int, edges, table, u: int, v: int):
    """Per-edge census: counts of G1..G17 over the 2-, 3- and 4-vertex
    subsets that contain both u and v (list indexed 0..17, slot 0 unused)."""
    adj = [set() for _ in range(n)]
    for a, b in edges:
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    cls = classifier(table)
    counts = [0] * 18
    rest = [x for x in range(n) if x != u and x != v]
    for extra in (0, 1, 2):
        for more in itertools.combinations(rest, extra):
            counts[cls[signature((u, v) + more, adj)]] += 1
    return counts
