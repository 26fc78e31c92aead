"""ORACLE (test infrastructure only): other sampling designs of Alg. 1.

Weighted edge sampling (Sec. 2.2: the edge neighbourhoods may be drawn from a
weighted distribution F, e.g. by k-core numbers or degrees; Sec. 5 uses
k-core weights for the extremal problem).  Each edge e gets its own
inclusion probability p_e and the estimate is the Horvitz-Thompson sum
X_i = K_i + sum_{e in J} Y_i(e) / p_e with the variance estimate
V_i = sum_{e in J} (1 - p_e) / p_e^2 Y_i(e)^2 (the Sec. 2.4 argument with a
per-edge probability).  The weights are quantised to 16 classes,
class(e) = min(15, floor(log2 max(1, w_e))), and p_e = min(1, c 2^class(e))
with c chosen so that the expected sample size is p_mean * M; the sums are
then exact integers per class.  Edge weights: "degree" w_e = d_u + d_v - 2
(the edges sharing an end with e), "kcore" w_e = min(core(u), core(v)).

Fixed-size sampling (Alg. 1 with a sample size K): the K edges with the
smallest 64-bit Philox keys (ties by edge id), a uniformly random K-subset;
the ratio estimator sigma = M / K (the printed p_i = |J| / |E|), i.e.
X_i = K_i + (M / K) sum_{e in J} Y_i(e), and the unbiased variance estimate
of simple random sampling without replacement,
V_i = M (M - K) s_i^2 / K with s_i^2 the sample variance of Y_i(e).
"""
from __future__ import annotations

import math

import numpy as np

from . import canonical_edges, estimate, philox_keys, sample_mask

LEVELS = 16
WEIGHT_DEGREE = 1
WEIGHT_KCORE = 2


def core_numbers(row_ptr, col) -> np.ndarray:
    """k-core numbers by the definition: the k-core is what is left after
    repeatedly deleting vertices of degree < k; core(v) is the largest k whose
    k-core holds v."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    cl = np.asarray(col, dtype=np.int64)[:rp[-1]]
    n = rp.shape[0] - 1
    src = np.repeat(np.arange(n), np.diff(rp))
    alive = np.ones(n, dtype=bool)
    deg = np.diff(rp).copy()
    core = np.zeros(n, dtype=np.int64)
    k = 1
    while alive.any():
        drop = alive & (deg < k)
        if not drop.any():
            k += 1
            continue
        core[drop] = k - 1
        alive[drop] = False
        # the dropped vertices no longer count in their neighbours' degrees
        hit = drop[src]
        deg -= np.bincount(cl[hit], minlength=n)
    return core


def edge_weights(row_ptr, col, mode: int) -> np.ndarray:
    rp = np.asarray(row_ptr, dtype=np.int64)
    us, vs = canonical_edges(row_ptr, col)
    deg = np.diff(rp)
    if mode == WEIGHT_DEGREE:
        return deg[us] + deg[vs] - 2
    if mode == WEIGHT_KCORE:
        core = core_numbers(row_ptr, col)
        return np.minimum(core[us], core[vs])
    raise ValueError("unknown weight mode")


def levels_of(weights) -> np.ndarray:
    w = np.maximum(np.asarray(weights, dtype=np.int64), 1)
    lv = np.zeros(w.shape, dtype=np.int64)
    for b in range(1, LEVELS):
        lv[w >= (1 << b)] = b
    return lv


def plan(hist, p_mean: float, m: int) -> list:
    """Class probabilities p_l = min(1, c 2^l) with sum_l hist[l] p_l =
    p_mean * m.  The levels from j up are saturated (p = 1) for the first j,
    counting down from 16, whose c leaves every non-empty lower class below 1
    and every non-empty saturated class at or above 1."""
    if p_mean >= 1.0:
        return [1.0] * LEVELS
    target = p_mean * m
    for j in range(LEVELS, 0, -1):
        s = sum(int(hist[l]) for l in range(j, LEVELS))
        w = sum(int(hist[l]) << l for l in range(j))
        if w == 0:
            continue
        c = (target - float(s)) / float(w)
        if c <= 0.0:
            continue
        if any(hist[l] and c * 2.0 ** l >= 1.0 for l in range(j)):
            continue
        if any(hist[l] and c * 2.0 ** l < 1.0 for l in range(j, LEVELS)):
            continue
        return [min(1.0, c * 2.0 ** l) for l in range(LEVELS)]
    raise ValueError("no class plan (empty graph?)")


def _finish(n, m, z_terms, q_terms, exact_if_full, full):
    """z_terms[i] / q_terms[i]: lists of (integer sum, factor) pairs in class
    order; X_i = K_i + sum (Z * f) / 12, V_i = sum (Q * g) / 144."""
    K = [0] * 18
    K[6] = math.comb(n, 3)
    K[17] = math.comb(n, 4)
    est, var = [0.0] * 18, [0.0] * 18
    est[1], est[2] = float(m), float(math.comb(n, 2) - m)
    for i in range(3, 18):
        if full:
            est[i] = float(exact_if_full[i])
            continue
        x = float(K[i])
        for zz, f in z_terms[i]:
            x += (float(zz) * f) / 12.0
        v = 0.0
        for qq, gfac in q_terms[i]:
            v += (float(qq) * gfac) / 144.0
        est[i], var[i] = x, v
    lo = [est[i] - 1.96 * math.sqrt(var[i]) for i in range(18)]
    hi = [est[i] + 1.96 * math.sqrt(var[i]) for i in range(18)]
    return est, var, lo, hi


def weighted_from_mask(row_ptr, col, lv, pl, mask) -> dict:
    """The weighted estimate for a given sample (mask) with edge classes lv
    and class probabilities pl: exact class sums from the plain oracle, then
    the Horvitz-Thompson combination in class order."""
    rp = np.asarray(row_ptr)
    n, m = rp.shape[0] - 1, int(rp[-1]) // 2
    mask = np.asarray(mask, dtype=np.uint8)
    per = [estimate(row_ptr, col, 1.0, 0, mask=(mask & (lv == l)).astype(np.uint8)) for l in range(LEVELS)]
    hist = [int((lv == l).sum()) for l in range(LEVELS)]
    tot = {k: [sum(r[k][i] for r in per) for i in range(18)] for k in ("csum", "zsum", "qsum")}
    full = all(p == 1.0 for p, h in zip(pl, hist) if h)
    exact = estimate(row_ptr, col, 1.0, 0)["exact"] if full else None
    z_terms = [[(per[l]["zsum"][i], 1.0 / pl[l]) for l in range(LEVELS)] for i in range(18)]
    q_terms = [[(per[l]["qsum"][i], (1.0 - pl[l]) / (pl[l] * pl[l])) for l in range(LEVELS)] for i in range(18)]
    est, var, lo, hi = _finish(n, m, z_terms, q_terms, exact, full)
    return {"p_level": list(pl), "hist": hist, "sampled_level": [r["sampled"] for r in per],
            "sampled": sum(r["sampled"] for r in per), "zsum_level": [r["zsum"] for r in per],
            "qsum_level": [r["qsum"] for r in per], **tot,
            "estimate": est, "variance": var, "lower95": lo, "upper95": hi}


def estimate_weighted(row_ptr, col, mode: int, p_mean: float, seed: int) -> dict:
    """Weighted Bernoulli sample: edge e is kept iff its Philox uniform is
    below the probability of its class."""
    rp = np.asarray(row_ptr)
    m = int(rp[-1]) // 2
    lv = levels_of(edge_weights(row_ptr, col, mode))
    hist = [int((lv == l).sum()) for l in range(LEVELS)]
    pl = plan(hist, p_mean, m)
    mask = np.zeros(m, dtype=np.uint8)
    for l in range(LEVELS):
        mask |= (sample_mask(seed, pl[l], m) & (lv == l)).astype(np.uint8)
    return weighted_from_mask(row_ptr, col, lv, pl, mask)


def fixed_k_mask(seed: int, m: int, k: int) -> np.ndarray:
    keys = philox_keys(seed, m)
    order = np.lexsort((np.arange(m), keys))
    mask = np.zeros(m, dtype=np.uint8)
    mask[order[:k]] = 1
    return mask


def estimate_fixed_k(row_ptr, col, k: int, seed: int, mask=None) -> dict:
    rp = np.asarray(row_ptr)
    n, m = rp.shape[0] - 1, int(rp[-1]) // 2
    if mask is None:
        mask = fixed_k_mask(seed, m, k)
    r = estimate(row_ptr, col, 1.0, seed, mask=mask)
    assert r["sampled"] == k
    full = k == m
    exact = estimate(row_ptr, col, 1.0, seed)["exact"] if full else None
    sigma = float(m) / float(k)
    z_terms = [[(r["zsum"][i], sigma)] for i in range(18)]
    # V = M (M - K) (K Q - Z^2) / (144 K^2 (K - 1)), the integer part exact
    q_terms = []
    for i in range(18):
        if k < 2:
            q_terms.append([(0, float("nan"))])
            continue
        num = k * r["qsum"][i] - r["zsum"][i] ** 2
        q_terms.append([(num, float(m) * float(m - k) / (float(k) * float(k) * float(k - 1)))])
    est, var, lo, hi = _finish(n, m, z_terms, q_terms, exact, full)
    return {**r, "estimate": est, "variance": var, "lower95": lo, "upper95": hi, "k": k}
