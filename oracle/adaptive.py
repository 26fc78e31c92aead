"""ORACLE (test infrastructure only): adaptive graphlet estimation.

Sec. 4, Alg. 8 under the Bernoulli sampling design: the sample starts empty;
each round adds a fraction phi of the edges not yet sampled (the expected
K_t = phi (m - |J|) of the algorithm), i.e. the sampling probability grows to
p_t = p_{t-1} + phi (1 - p_{t-1}); the round's estimate X^(t) is computed from
the whole sample; the loss is the maximum relative change of the 4-vertex
graphlet estimates (eq. est-obj-max-rel-error, the previous round playing the
role of the best solution so far); phi is halved; the loop ends when the loss
is <= beta or after t_max rounds.  phi0 = 0 takes 1/sqrt(m), the value of the
algorithm's default with the initial error 1.

Each round's sample is "uniform < p_t" for the same Philox uniforms, so the
samples are nested and every round is a plain oracle estimate at p_t.
"""
import math

from . import estimate


def relative_change(prev, cur):
    """Largest relative change of the G7..G17 estimates (a zero previous value
    with a non-zero new one counts as 1)."""
    d = 0.0
    for i in range(7, 18):
        x0, x1 = prev["estimate"][i], cur["estimate"][i]
        if x0 != 0.0:
            d = max(d, abs(x1 - x0) / abs(x0))
        elif x1 != 0.0:
            d = max(d, 1.0)
    return d


def adaptive(row_ptr, col, seed, beta=0.01, t_max=20, phi0=0.0):
    m = len(col) // 2
    phi = phi0 if phi0 > 0 else (1.0 / math.sqrt(m) if m > 0 else 1.0)
    phi = min(phi, 1.0)
    p = 0.0
    prev = None
    trace = {"p": [], "delta": [], "sampled": []}
    est = None
    for _ in range(t_max):
        p_new = p + phi * (1.0 - p)
        est = estimate(row_ptr, col, p_new, seed)
        delta = -1.0 if prev is None else relative_change(prev, est)
        trace["p"].append(p_new)
        trace["delta"].append(delta)
        trace["sampled"].append(est["sampled"])
        prev = est
        p = p_new
        phi = phi * 0.5
        if 0.0 <= delta <= beta:
            break
    trace["rounds"] = len(trace["p"])
    return est, trace
