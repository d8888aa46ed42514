"""Pins for the move set S_1(0) \\ {0} (Sec. II-C, Eq. (2)-(3); Table II).

* the count equals the closed form for the number of minimum-weight
  codewords of RM(r, m) (the number of (m-r)-flats of EG(m, 2));
* every move is a codeword of weight 2^(m-r), all are distinct, and they are
  in canonical order (ascending sorted support, lexicographic);
* brute force: the weight-2^(m-r) words among ALL 2^K codewords (generated
  from the monomial definition of RM, not from the oracle) are exactly the
  oracle's moves;
* Table II's printed value for RM(128,29) is kept as a golden fixture with
  its reading.
"""
import json
import os

import numpy as np
import pytest

import oracle
from test_oracle_code import monomial_generator

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2_sphere_cardinality.json")


def closed_form_min_weight_count(r, m):
    num, den = 1, 1
    for i in range(m - r):
        num *= (1 << (m - i)) - 1
        den *= (1 << (m - r - i)) - 1
    assert num % den == 0
    return (1 << r) * num // den


@pytest.mark.parametrize("r,m,P", [(1, 5, 62), (2, 5, 620), (2, 6, 2604), (1, 7, 254), (2, 7, 10668), (3, 7, 94488)])
def test_count_matches_closed_form(r, m, P):
    supp, w = oracle.moves(r, m)
    assert closed_form_min_weight_count(r, m) == P
    assert supp.shape == (P, 1 << (m - r)) and w == 1 << (m - r)


@pytest.mark.slow
def test_count_rm38():
    supp, w = oracle.moves(3, 8)
    assert supp.shape == (777240, 32) == (closed_form_min_weight_count(3, 8), w)


@pytest.mark.parametrize("r,m", [(1, 5), (2, 6), (2, 7), (3, 7)])
def test_moves_are_distinct_sorted_codewords(r, m):
    supp, w = oracle.moves(r, m)
    n = 1 << m
    # supports sorted within each move and moves in lexicographic order
    assert np.all(np.diff(supp.astype(np.int64), axis=1) > 0)
    keys = [tuple(row) for row in supp.tolist()]
    assert keys == sorted(keys)
    assert len(set(keys)) == len(keys)
    # membership: u = c F^{(x)m} (an involution) must vanish off the info set
    frozen = oracle.frozen_mask(r, m).astype(bool)
    rng = np.random.default_rng(0)
    for p in rng.choice(len(supp), size=min(400, len(supp)), replace=False):
        c = np.zeros(n, np.uint8)
        c[supp[p]] = 1
        assert not oracle.encode(m, c)[frozen].any()


def all_codewords_bits(r, m):
    """Every codeword of RM(r, m) as a uint64 pair (low, high) bitmask."""
    G = monomial_generator(r, m)
    n = 1 << m
    lo = np.array([int(sum(int(b) << j for j, b in enumerate(row[:64]))) for row in G], np.uint64)
    hi = np.array([int(sum(int(b) << j for j, b in enumerate(row[64:n]))) for row in G], np.uint64)
    words_lo = np.zeros(1, np.uint64)
    words_hi = np.zeros(1, np.uint64)
    for a, b in zip(lo, hi):
        words_lo = np.concatenate([words_lo, words_lo ^ a])
        words_hi = np.concatenate([words_hi, words_hi ^ b])
    return words_lo, words_hi


def popcount64(x):
    return np.bitwise_count(x).astype(np.int64)


@pytest.mark.parametrize("r,m", [(1, 5), (2, 5), (2, 6), (1, 7)])
def test_bruteforce_weight_enumeration(r, m):
    lo, hi = all_codewords_bits(r, m)
    wt = popcount64(lo) + popcount64(hi)
    dmin = 1 << (m - r)
    assert wt[1:].min() == dmin
    sel = np.nonzero(wt == dmin)[0]
    brute = set(zip(lo[sel].tolist(), hi[sel].tolist()))
    supp, w = oracle.moves(r, m)
    mine = set()
    for row in supp.tolist():
        a = b = 0
        for j in row:
            if j < 64:
                a |= 1 << j
            else:
                b |= 1 << (j - 64)
        mine.add((a, b))
    assert mine == brute


def test_packing_lsb_first():
    supp, w = oracle.moves(2, 6)
    rows = oracle.pack_supports(6, supp)
    assert rows.shape == (2604, 8)
    bits = np.unpackbits(rows, axis=1, bitorder="little")
    for p in (0, 1, 1000, 2603):
        assert np.array_equal(np.nonzero(bits[p])[0], supp[p])


def test_table2_rm_row_reading():
    g = json.load(open(GOLDEN))
    row = g["rows"][0]
    r, m = row["r_m"]
    P = oracle.moves(r, m)[0].shape[0]
    assert P == 10668
    # the printed value differs from the closed form in one digit (8 for 6)
    assert row["paper_value"] == 10688
    diff = [a != b for a, b in zip(str(P), str(row["paper_value"]))]
    assert sum(diff) == 1
