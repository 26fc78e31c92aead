"""Pins of the adaptive oracle (Sec. 4, Alg. 8)."""
import math

import oracle
from oracle import adaptive, bruteforce as bf
from paper_1701_01772_amd import inputs


def test_schedule_closed_form():
    g = inputs.erdos_renyi(200, 0.05, 4)
    est, tr = adaptive.adaptive(g.row_ptr, g.col, 9, beta=0.0, t_max=12, phi0=0.2)
    assert tr["rounds"] == 12  # beta = 0 and changes > 0 at these sizes: every round runs
    for t, p in enumerate(tr["p"]):
        want = 1.0 - math.prod(1.0 - 0.2 / 2 ** k for k in range(t + 1))
        assert abs(p - want) <= 1e-14
    assert tr["sampled"] == sorted(tr["sampled"])  # nested samples grow


def test_full_sample_reaches_exact_counts(table1):
    g = inputs.erdos_renyi(11, 0.4, 7)
    est, tr = adaptive.adaptive(g.row_ptr, g.col, 3, beta=0.01, t_max=5, phi0=1.0)
    # phi0 = 1 samples every edge in round 1; round 2 changes nothing and stops
    assert tr["rounds"] == 2 and tr["p"] == [1.0, 1.0] and tr["delta"][1] == 0.0
    assert est["exact"][1:] == bf.census_csr(g.row_ptr, g.col, table1)[1:]
    assert [est["estimate"][i] for i in range(1, 18)] == [float(x) for x in est["exact"][1:]]


def test_default_phi_and_stopping():
    g = inputs.chung_lu(3000, 10.0, 2.2, 400.0, 5)
    est, tr = adaptive.adaptive(g.row_ptr, g.col, 21, beta=0.05, t_max=20)
    assert abs(tr["p"][0] - 1.0 / math.sqrt(g.m)) <= 1e-15
    k = tr["rounds"]
    # stops at the first round whose change is within beta, else at t_max
    firsts = [t for t in range(1, k) if tr["delta"][t] <= 0.05]
    assert (firsts and firsts[0] == k - 1) or (not firsts and k == 20)
    # the returned estimate is the plain estimate at the final probability
    plain = oracle.estimate(g.row_ptr, g.col, tr["p"][-1], 21)
    assert plain["qsum"] == est["qsum"] and plain["sampled"] == est["sampled"]
