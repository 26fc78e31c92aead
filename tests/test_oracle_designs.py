"""Pins of the weighted and fixed-size sampling designs (Alg. 1 with a
weighted F or a sample size K; Sec. 2.2, 2.3, 2.4, 5): k-core numbers against
a brute-force subgraph search and closed forms, the class plan's expected
sample size, and exact unbiasedness of X and of the variance estimate by
enumerating every sample outcome."""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import designs as D
from paper_1701_01772_amd import inputs


def _core_brute(n, edges):
    adj = [set() for _ in range(n)]
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    best = [0] * n
    for mask in range(1, 1 << n):
        S = [v for v in range(n) if mask >> v & 1]
        k = min(len(adj[v] & set(S)) for v in S)
        for v in S:
            best[v] = max(best[v], k)
    return best


@pytest.mark.parametrize("seed,dens", [(1, 0.3), (2, 0.5), (3, 0.7), (4, 0.2)])
def test_core_numbers_bruteforce(seed, dens):
    g = inputs.erdos_renyi(11, dens, seed)
    us, vs = oracle.canonical_edges(g.row_ptr, g.col)
    assert D.core_numbers(g.row_ptr, g.col).tolist() == _core_brute(g.n, list(zip(us.tolist(), vs.tolist())))


def test_core_numbers_closed_forms():
    n = 8
    kn = inputs.from_edges(n, [(a, b) for a in range(n) for b in range(a + 1, n)])
    assert D.core_numbers(kn.row_ptr, kn.col).tolist() == [n - 1] * n
    cyc = inputs.from_edges(9, [(i, (i + 1) % 9) for i in range(9)])
    assert D.core_numbers(cyc.row_ptr, cyc.col).tolist() == [2] * 9
    path = inputs.from_edges(6, [(i, i + 1) for i in range(4)])  # vertex 5 isolated
    assert D.core_numbers(path.row_ptr, path.col).tolist() == [1] * 5 + [0]
    kab = inputs.from_edges(9, [(x, 4 + y) for x in range(4) for y in range(5)])
    assert D.core_numbers(kab.row_ptr, kab.col).tolist() == [4] * 9


def test_levels_and_weights():
    assert D.levels_of([0, 1, 2, 3, 4, 7, 8, 1 << 15, (1 << 20)]).tolist() == [0, 0, 1, 1, 2, 2, 3, 15, 15]
    g = inputs.from_edges(5, [(0, 1), (1, 2), (2, 3), (1, 3)])
    # canonical order (0,1), (1,2), (1,3), (2,3); degrees 1, 3, 2, 2
    assert D.edge_weights(g.row_ptr, g.col, D.WEIGHT_DEGREE).tolist() == [2, 3, 3, 2]
    assert D.edge_weights(g.row_ptr, g.col, D.WEIGHT_KCORE).tolist() == [1, 2, 2, 2]


@pytest.mark.parametrize("p_mean", [0.01, 0.1, 0.37, 0.9, 1.0])
def test_plan_expected_size(p_mean):
    hist = [0, 500, 1200, 0, 300, 40, 9, 0, 1, 0, 0, 0, 0, 0, 0, 3]
    m = sum(hist)
    pl = D.plan(hist, p_mean, m)
    assert all(0.0 < p <= 1.0 for p in pl)
    assert abs(sum(h * p for h, p in zip(hist, pl)) - p_mean * m) <= 1e-9 * m
    for l in range(15):
        if pl[l + 1] < 1.0:
            assert pl[l + 1] == 2.0 * pl[l]  # proportional to the class weight 2^l
        assert pl[l + 1] >= pl[l]


def _tiny():
    return inputs.from_edges(7, [(0, 1), (0, 2), (1, 2), (2, 3), (3, 4), (1, 3), (4, 5), (5, 6), (0, 6), (2, 5)])


def _enum_weighted(mod):
    """Largest relative bias of X and of V over every Bernoulli outcome."""
    g = _tiny()
    m = g.m
    lv = mod.levels_of(mod.edge_weights(g.row_ptr, g.col, mod.WEIGHT_DEGREE))
    pl = [min(1.0, 0.3 * (l + 1) / 4) for l in range(16)]
    pe = [pl[l] for l in lv]
    exact = oracle.estimate(g.row_ptr, g.col, 1.0, 0)["exact"]
    ex, ex2, ev = [0.0] * 18, [0.0] * 18, [0.0] * 18
    for bits in range(1 << m):
        mask = np.array([(bits >> e) & 1 for e in range(m)], dtype=np.uint8)
        w = math.prod(pe[e] if mask[e] else 1.0 - pe[e] for e in range(m))
        if w == 0.0:
            continue
        r = mod.weighted_from_mask(g.row_ptr, g.col, lv, pl, mask)
        for i in range(3, 18):
            ex[i] += w * r["estimate"][i]
            ex2[i] += w * r["estimate"][i] ** 2
            ev[i] += w * r["variance"][i]
    return _errors(ex, ex2, ev, exact)


def _enum_fixed(mod, k):
    g = _tiny()
    m = g.m
    exact = oracle.estimate(g.row_ptr, g.col, 1.0, 0)["exact"]
    subsets = list(itertools.combinations(range(m), k))
    ex, ex2, ev = [0.0] * 18, [0.0] * 18, [0.0] * 18
    for sub in subsets:
        mask = np.zeros(m, dtype=np.uint8)
        mask[list(sub)] = 1
        r = mod.estimate_fixed_k(g.row_ptr, g.col, k, 0, mask=mask)
        for i in range(3, 18):
            ex[i] += r["estimate"][i] / len(subsets)
            ex2[i] += r["estimate"][i] ** 2 / len(subsets)
            ev[i] += r["variance"][i] / len(subsets)
    return _errors(ex, ex2, ev, exact)


def _errors(ex, ex2, ev, exact):
    bias_x = max(abs(ex[i] - exact[i]) / max(1.0, abs(exact[i])) for i in range(3, 18))
    bias_v = max(abs(ev[i] - (ex2[i] - ex[i] ** 2)) / max(1.0, ex2[i]) for i in range(3, 18))
    return bias_x, bias_v


def test_weighted_unbiased_by_enumeration():
    bx, bv = _enum_weighted(D)
    assert bx <= 1e-9 and bv <= 1e-9, (bx, bv)


@pytest.mark.parametrize("k", [2, 3, 6])
def test_fixed_k_unbiased_by_enumeration(k):
    bx, bv = _enum_fixed(D, k)
    assert bx <= 1e-9 and bv <= 1e-9, (bx, bv)


@pytest.mark.parametrize("old,new,which", [
    ("float(m) * float(m - k) / (float(k) * float(k) * float(k - 1))",
     "float(m) * float(m) / (float(k) * float(k) * float(k - 1))", "fixed"),   # no finite-population term
    ("sigma = float(m) / float(k)", "sigma = float(m) / float(k + 1)", "fixed"),  # off-by-one ratio
    ("(1.0 - pl[l]) / (pl[l] * pl[l])", "(1.0 - pl[l]) / pl[l]", "weighted"),    # variance factor
    ("(per[l][\"zsum\"][i], 1.0 / pl[l])", "(per[l][\"zsum\"][i], 1.0 / pl[0])", "weighted"),  # one class p
])
def test_planted_design_mistakes_are_caught(old, new, which):
    import importlib.util
    import types
    src = open(D.__file__).read()
    assert old in src
    mod = types.ModuleType("oracle._planted_designs")
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new), "planted", "exec"), mod.__dict__)
    bx, bv = _enum_fixed(mod, 3) if which == "fixed" else _enum_weighted(mod)
    assert bx > 1e-6 or bv > 1e-6


def test_fixed_k_selection_and_full():
    g = inputs.chung_lu(500, 6.0, 2.2, 80.0, 9)
    seed = 77
    # the K smallest (key, id) pairs, keys from single Philox calls
    keys = []
    for e in range(g.m):
        x = oracle.philox4x32_10([e & 0xFFFFFFFF, e >> 32, 0, 0], [seed & 0xFFFFFFFF, seed >> 32])
        keys.append(((x[1] << 32) | x[0], e))
    for k in (1, 37, g.m // 2):
        want = sorted(keys)[:k]
        mask = D.fixed_k_mask(seed, g.m, k)
        assert mask.sum() == k
        assert sorted(np.nonzero(mask)[0].tolist()) == sorted(e for _, e in want)
    full = D.estimate_fixed_k(g.row_ptr, g.col, g.m, seed)
    ex = oracle.estimate(g.row_ptr, g.col, 1.0, 0)["exact"]
    assert [full["estimate"][i] for i in range(1, 18)] == [float(x) for x in ex[1:]]
    assert all(v == 0.0 for v in full["variance"][3:])


def test_weighted_full_probability_is_exact():
    g = inputs.chung_lu(800, 6.0, 2.2, 100.0, 4)
    r = D.estimate_weighted(g.row_ptr, g.col, D.WEIGHT_KCORE, 1.0, 5)
    ex = oracle.estimate(g.row_ptr, g.col, 1.0, 0)["exact"]
    assert r["sampled"] == g.m
    assert [r["estimate"][i] for i in range(1, 18)] == [float(x) for x in ex[1:]]
