"""Pin of the oracle's int128 -> double conversion (the one rounding step of
the finalisation, applied to every exact sum before the 1/p scaling).

Values above 2^53 must round to nearest with ties to even.  The expected
values come from exact integer arithmetic (ties built as mantissa * 2^s plus
half a unit, whose correct result is written down directly) and from
Python's ``float(int)``, which rounds correctly.  The case set is checked to
separate the plausible wrong rules (truncation, ties away from zero, ties
toward zero, an off-by-one shift), so each of them would fail a case.
Full-size estimates go through this branch: C(10^6, 4) ~ 4.2e22 > 2^53.
"""
import math
import random

import pytest

import oracle
from paper_1701_01772_amd import inputs


def _tie_cases():
    """(x, exact expected double as an int) for exact ties at many shifts."""
    rng = random.Random(128)
    out = []
    for sh in list(range(1, 12)) + [20, 31, 32, 33, 52, 63, 64, 65, 73, 74]:
        for want_odd in (False, True):
            mant = rng.randrange(1 << 52, 1 << 53)
            if (mant & 1) != want_odd:
                mant ^= 1
            x = (mant << sh) + (1 << (sh - 1))
            up = mant + 1 if mant & 1 else mant  # ties to even
            out.append((x, up << sh))
            out.append((x - 1, mant << sh))          # just below the tie: down
            out.append((x + 1, (mant + 1) << sh))    # just above the tie: up
    return out


def _random_cases(count=4000):
    rng = random.Random(53)
    out = []
    for _ in range(count):
        bits = rng.randrange(1, 128)
        x = rng.getrandbits(bits) | (1 << (bits - 1))
        if x >= 1 << 127:
            x = (1 << 127) - 1
        out.append(x if rng.random() < 0.5 else -x)
    return out


EDGE_VALUES = [0, 1, -1, (1 << 53) - 1, 1 << 53, (1 << 53) + 1, (1 << 53) + 2, (1 << 53) + 3,
               (1 << 54) + 2, (1 << 64) - 1, 1 << 64, (1 << 64) + 1, (1 << 127) - 1, -(1 << 127),
               -((1 << 53) + 1), -((1 << 53) + 3), -((1 << 127) - 1)]


def test_ties_round_to_even():
    for x, want in _tie_cases():
        assert oracle.i128_to_double(x) == float(want), (x, want)
        assert oracle.i128_to_double(-x) == -float(want), (-x, want)


def test_random_and_edge_values_match_correct_rounding():
    for x in _random_cases() + EDGE_VALUES:
        assert oracle.i128_to_double(x) == float(x), x


def _round(x, rule):
    """Alternative (wrong) conversions of a non-negative x, for the case-set check."""
    if x < (1 << 53):
        return float(x)
    sh = x.bit_length() - 53
    mant, rem, half = x >> sh, x & ((1 << sh) - 1), 1 << (sh - 1)
    if rule == "truncate":
        pass
    elif rule == "ties_away":
        mant += 1 if rem >= half else 0
    elif rule == "ties_down":
        mant += 1 if rem > half else 0
    elif rule == "shift_off_by_one":
        sh += 1
        mant, rem, half = x >> sh, x & ((1 << sh) - 1), 1 << (sh - 1)
        mant += 1 if rem > half or (rem == half and mant & 1) else 0
    return float(mant << sh)


@pytest.mark.parametrize("rule", ["truncate", "ties_away", "ties_down", "shift_off_by_one"])
def test_case_set_separates_wrong_rules(rule):
    xs = [x for x, _ in _tie_cases()] + [x for x in _random_cases() if x > 0]
    assert any(_round(x, rule) != float(x) for x in xs), rule


@pytest.mark.parametrize("n", [100_000, 1_000_000])
@pytest.mark.parametrize("p", [1.0, 0.5])
def test_empty_graph_constants_above_2_53(n, p):
    # no edges: X6 = C(n,3) and X17 = C(n,4), each one conversion of an exact
    # integer that has more than 53 significant bits
    g = inputs.from_edges(n, [])
    r = oracle.estimate(g.row_ptr, g.col, p, 7)
    c3, c4 = math.comb(n, 3), math.comb(n, 4)
    assert c4 > 1 << 53 and int(float(c4)) != c4  # the rounding branch is taken
    assert r["estimate"][17] == float(c4)
    assert r["estimate"][6] == float(c3)
    assert r["exact"][17] == c4 and r["exact"][6] == c3
