"""Pins for the oracle's code construction (Sec. II-B: c = mG).

The generator is the Reed-Muller code RM(r, m) written in the Kronecker form
F^{(x)m}; the pins below reach the same objects by routes that share nothing
with the oracle: numpy's Kronecker product and the textbook definition of
RM(r, m) as the evaluations of all monomials of degree <= r.
"""
import itertools

import numpy as np
import pytest

import oracle


def gf2_rank(M: np.ndarray) -> int:
    M = (np.array(M, np.uint8) & 1).copy()
    rank, rows, cols = 0, M.shape[0], M.shape[1]
    for c in range(cols):
        piv = np.nonzero(M[rank:, c])[0]
        if len(piv) == 0:
            continue
        p = rank + piv[0]
        M[[rank, p]] = M[[p, rank]]
        others = np.nonzero(M[:, c])[0]
        others = others[others != rank]
        M[others] ^= M[rank]
        rank += 1
        if rank == rows:
            break
    return rank


def kron_power(m):
    F = np.array([[1, 0], [1, 1]], np.int64)
    G = np.ones((1, 1), np.int64)
    for _ in range(m):
        G = np.kron(G, F)
    return (G % 2).astype(np.uint8)


def monomial_generator(r, m):
    """Rows: evaluations of x_S = prod_{b in S} x_b, |S| <= r, at all points."""
    pts = np.arange(1 << m)
    rows = []
    for d in range(r + 1):
        for S in itertools.combinations(range(m), d):
            row = np.ones(1 << m, np.uint8)
            for b in S:
                row &= ((pts >> b) & 1).astype(np.uint8)
            rows.append(row)
    return np.array(rows, np.uint8)


@pytest.mark.parametrize("r,m,K", [(1, 3, 4), (1, 5, 6), (2, 6, 22), (2, 7, 29), (3, 7, 64), (3, 8, 93)])
def test_dimensions(r, m, K):
    assert oracle.rm_dims(r, m) == (1 << m, K)
    assert len(oracle.rm_info_set(r, m)) == K


@pytest.mark.parametrize("m", [1, 2, 3, 5, 6])
def test_encode_def_is_kronecker_product(m):
    G = kron_power(m)
    rng = np.random.default_rng(m)
    for _ in range(8):
        u = rng.integers(0, 2, 1 << m).astype(np.uint8)
        assert np.array_equal(oracle.encode_def(m, u), (u.astype(np.int64) @ G) % 2)


@pytest.mark.parametrize("m", [3, 6, 7, 8])
def test_butterfly_equals_definition_and_is_involution(m):
    rng = np.random.default_rng(10 + m)
    for _ in range(6):
        u = rng.integers(0, 2, 1 << m).astype(np.uint8)
        c = oracle.encode(m, u)
        assert np.array_equal(c, oracle.encode_def(m, u))
        assert np.array_equal(oracle.encode(m, c), u)


@pytest.mark.parametrize("r,m", [(1, 4), (2, 5), (2, 6), (3, 7)])
def test_info_rows_span_reed_muller(r, m):
    G = kron_power(m)[oracle.rm_info_set(r, m)]
    Mono = monomial_generator(r, m)
    K = oracle.rm_dims(r, m)[1]
    assert gf2_rank(G) == K
    assert gf2_rank(Mono) == K
    assert gf2_rank(np.vstack([G, Mono])) == K
