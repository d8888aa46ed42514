"""Pins for spheres of radius >= 2 (Eq. (1)-(2)): the oracle's exhaustive
weight distribution and its S_rho(0) tables.

* RM(2, m): the weight distribution of second-order Reed-Muller codes in
  closed form (Sloane and Berlekamp, IEEE Trans. IT 16, 1970): the weight
  2^(m-1) -+ 2^(m-1-h) occurs
      2^(h(h+1)) prod_{i=m-2h+1}^{m} (2^i - 1) / prod_{i=1}^{h} (4^i - 1)
  times, for 1 <= h <= floor(m/2);
* RM(1, m): 2^(m+1) - 2 words of weight 2^(m-1) and the all-one word;
* MacWilliams: the transform of RM(2,6)'s distribution is that of its dual
  RM(3,6): B_1..B_7 = 0 and B_8 = the number of 3-flats of EG(6,2); RM(2,5)
  is self-dual, so the transform is the identity;
* radius 1 equals the flat enumeration of ``oracle.moves`` row for row;
* every row of S_2(0) is a codeword (monomial generator, not the oracle's
  encoder), of the right weight, all distinct, in (weight, support) order;
* with the sphere taken as the whole code, one stage-2 step from any anchor
  lands on a maximum-likelihood codeword (brute force).
"""
import math

import numpy as np
import pytest

import oracle
from test_oracle_code import monomial_generator


def rm2_distribution(m):
    n = 1 << m
    K = 1 + m + m * (m - 1) // 2
    A = {0: 1, n: 1}
    for h in range(1, m // 2 + 1):
        num = 1
        for i in range(m - 2 * h + 1, m + 1):
            num *= (1 << i) - 1
        den = 1
        for i in range(1, h + 1):
            den *= (1 << (2 * i)) - 1
        assert (num << (h * (h + 1))) % den == 0
        a = (num << (h * (h + 1))) // den
        for w in (n // 2 - (n >> (h + 1)), n // 2 + (n >> (h + 1))):
            A[w] = A.get(w, 0) + a
    A[n // 2] = (1 << K) - sum(A.values())
    return A


def dense(A, n):
    out = np.zeros(n + 1, np.int64)
    for w, a in A.items():
        out[w] = a
    return out


def macwilliams(A, n, K):
    """B_j = 2^-K sum_i A_i K_j(i), Krawtchouk K_j(i) = sum_s (-1)^s C(i,s) C(n-i,j-s)."""
    B = []
    for j in range(n + 1):
        tot = 0
        for i in range(n + 1):
            if A[i]:
                kj = sum((-1) ** s * math.comb(i, s) * math.comb(n - i, j - s) for s in range(0, min(i, j) + 1))
                tot += int(A[i]) * kj
        assert tot % (1 << K) == 0
        B.append(tot >> K)
    return B


def flats(m, k):
    """Number of k-dimensional flats of EG(m, 2)."""
    num, den = 1, 1
    for i in range(k):
        num *= (1 << (m - i)) - 1
        den *= (1 << (k - i)) - 1
    return (num // den) << (m - k)


@pytest.mark.parametrize("m", [3, 4, 5, 6])
def test_rm2_distribution_closed_form(m):
    n = 1 << m
    assert np.array_equal(oracle.weight_distribution(2, m), dense(rm2_distribution(m), n))


@pytest.mark.parametrize("m", [2, 3, 4, 5, 6, 7])
def test_rm1_distribution(m):
    n = 1 << m
    A = oracle.weight_distribution(1, m)
    assert np.array_equal(A, dense({0: 1, n // 2: 2 * n - 2, n: 1}, n))


def test_macwilliams_rm26_dual_is_rm36():
    A = oracle.weight_distribution(2, 6)
    B = macwilliams(A, 64, 22)
    assert B[0] == 1 and all(b == 0 for b in B[1:8])
    assert B[8] == flats(6, 3) == 11160
    assert all(b >= 0 for b in B) and sum(B) == 1 << 42
    assert all(B[j] == 0 for j in range(65) if j % 2)  # RM(3,6) is even


def test_macwilliams_rm25_self_dual():
    A = oracle.weight_distribution(2, 5)
    assert macwilliams(A, 32, 16) == A.tolist()


@pytest.mark.parametrize("r,m", [(1, 4), (1, 5), (1, 6), (2, 5), (2, 6)])
def test_radius1_equals_flats(r, m):
    s1, st = oracle.sphere(r, m, 1)
    mv, w = oracle.moves(r, m)
    assert st == w
    assert np.array_equal(s1, mv)


def check_table(r, m, radius):
    supp, stride = oracle.sphere(r, m, radius)
    n = 1 << m
    A = oracle.weight_distribution(r, m)
    weights = [w for w in range(1, n + 1) if A[w]][:radius]
    assert stride == weights[-1]
    assert len(supp) == sum(int(A[w]) for w in weights)
    wt = (supp != oracle.SUPP_END).sum(1)
    # padding only at the end of each row, positions ascending
    for row, w in zip(supp, wt):
        assert np.all(row[w:] == oracle.SUPP_END)
    rows = [tuple(row[:w]) for row, w in zip(supp.tolist(), wt.tolist())]
    assert all(np.all(np.diff(r_) > 0) for r_ in rows[:2000])
    keys = list(zip(wt.tolist(), rows))
    assert keys == sorted(keys) and len(set(rows)) == len(rows)
    assert set(wt.tolist()) == set(weights)
    # membership through the monomial generator: c in the row space of G
    basis = gf2_basis(monomial_generator(r, m))
    rng = np.random.default_rng(5)
    for p in rng.choice(len(supp), size=min(300, len(supp)), replace=False):
        c = np.zeros(n, np.uint8)
        c[list(rows[p])] = 1
        assert in_span(basis, c)
    return supp, wt


def gf2_basis(G):
    """Reduced rows of G over GF(2), as (pivot, row) pairs."""
    rows = [g.astype(np.uint8) % 2 for g in G]
    basis = []
    for v in rows:
        v = v.copy()
        for p, b in basis:
            if v[p]:
                v ^= b
        nz = np.flatnonzero(v)
        if len(nz):
            p = nz[0]
            basis = [(q, b ^ v if b[p] else b) for q, b in basis]
            basis.append((p, v))
    return basis


def in_span(basis, c):
    v = c.copy()
    for p, b in basis:
        if v[p]:
            v ^= b
    return not v.any()


@pytest.mark.parametrize("r,m,radius", [(2, 5, 2), (2, 5, 3), (2, 6, 2), (1, 5, 2)])
def test_sphere_tables(r, m, radius):
    check_table(r, m, radius)


def test_sphere_rm26_r2_cardinality():
    supp, stride = oracle.sphere(2, 6, 2)
    assert supp.shape == (2604 + 291648, 24) and stride == 24


def test_too_few_weights():
    with pytest.raises(ValueError):
        oracle.sphere(1, 4, 3)   # RM(1,4) has the nonzero weights 8 and 16 only


@pytest.mark.parametrize("r,m", [(1, 4), (2, 5)])
def test_whole_code_sphere_reaches_ml_in_one_step(r, m):
    n = 1 << m
    A = oracle.weight_distribution(r, m)
    radius = int((A[1:] > 0).sum())
    supp, stride = oracle.sphere(r, m, radius)
    assert len(supp) == (1 << oracle.rm_dims(r, m)[1]) - 1
    G = monomial_generator(r, m)
    rng = np.random.default_rng(11 + m)
    for trial in range(6):
        msg = rng.integers(0, 2, len(G))
        c = (msg @ G % 2).astype(np.uint8)
        y = 1 - 2.0 * c + rng.standard_normal(n) * 1.0
        q = np.clip(np.rint(y * 8), -127, 127)
        a_msg = rng.integers(0, 2, len(G))
        anchor = (a_msg @ G % 2).astype(np.uint8)
        for mode, obs in ((oracle.INT, q), (oracle.F64, y)):
            e_ml, _ = oracle.ml(r, m, mode, obs)
            paths, logs, met, kb = oracle.stage2_frame(mode, supp, obs, anchor[None], 2)
            assert met[0] == pytest.approx(e_ml, abs=1e-9)
            # after the first step nothing improves: the second entry is -1
            assert logs[0, 1] == -1


def test_eq5_identity_mixed_weights():
    r, m = 2, 6
    supp, stride = oracle.sphere(r, m, 2)
    n = 1 << m
    rng = np.random.default_rng(3)
    G = monomial_generator(r, m)
    for trial in range(20):
        c = (rng.integers(0, 2, len(G)) @ G % 2).astype(np.uint8)
        y = rng.standard_normal(n)
        p = int(rng.integers(2604, len(supp)))   # a weight-24 move
        s = supp[p][supp[p] != oracle.SUPP_END]
        assert len(s) == 24
        cw = c.copy()
        cw[s] ^= 1
        ed = lambda v: float(((y - (1 - 2.0 * v)) ** 2).sum())
        assert ed(cw) - ed(c) == pytest.approx(4 * float((y * (1 - 2.0 * c))[s].sum()), abs=1e-9)
        # the oracle's one-step search from c scores this move exactly so:
        # forcing T=1 with a table holding only this move
        one = supp[p:p + 1]
        path, log = oracle.stage2_path(oracle.F64, one, y, c, 1)
        z = (y * (1 - 2.0 * c))[s].sum()
        assert (log[0] == 0) == (z < 0)
        assert np.array_equal(path, cw if z < 0 else c)
