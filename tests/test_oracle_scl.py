"""Pins for stage 1, min-sum SC-list decoding (Sec. III-A).

* Path-metric identity: with the min-sum check-node rule, the metric of any
  complete path equals the correlation discrepancy of its codeword,
      PM(c) = sum_{j : c_j != HD(y_j)} |y_j|,
  an affine, increasing function of the squared distance ||y - x(c)||^2.
  Any slip in f, g, the partial sums, the tree order or the metric update
  breaks it.  Exact in integer mode.
* With L = 2^K no path is ever dropped: the list is the whole code, and its
  first entry is a maximum-likelihood codeword (brute force over 2^K words).
* L = 1 on a noiseless observation returns the transmitted codeword.
* Scale invariance: q and 2q (integer mode) give identical lists.
"""
import numpy as np
import pytest

import oracle


def discrepancy(y, c):
    hd = (np.asarray(y) < 0).astype(np.uint8)
    return float(np.abs(np.asarray(y, np.float64))[hd != c].sum())


def random_codeword(r, m, rng):
    u = np.zeros(1 << m, np.uint8)
    A = oracle.rm_info_set(r, m)
    u[A] = rng.integers(0, 2, len(A))
    return oracle.encode(m, u)


@pytest.mark.parametrize("r,m,L", [(1, 4, 4), (2, 5, 8), (2, 6, 4), (3, 7, 8)])
def test_path_metric_is_discrepancy(r, m, L):
    rng = np.random.default_rng(100 + m)
    fr = oracle.frozen_mask(r, m)
    for trial in range(6 if m < 7 else 2):
        c0 = random_codeword(r, m, rng)
        q = np.clip(np.rint((1 - 2.0 * c0 + rng.standard_normal(1 << m) * 0.9) * 12), -127, 127)
        u, c, pm = oracle.scl(m, L, oracle.INT, q, fr)
        assert len(pm) == L
        assert np.all(np.diff(pm) >= 0)
        for l in range(L):
            assert pm[l] == discrepancy(q, c[l])
            assert np.array_equal(oracle.encode(m, u[l]), c[l])
            assert not u[l][fr.astype(bool)].any()


@pytest.mark.parametrize("r,m", [(1, 3), (1, 4), (2, 4)])
def test_full_list_is_whole_code_and_ml_first(r, m):
    K = oracle.rm_dims(r, m)[1]
    fr = oracle.frozen_mask(r, m)
    rng = np.random.default_rng(7)
    for trial in range(3):
        y = 1 - 2.0 * random_codeword(r, m, rng) + rng.standard_normal(1 << m)
        u, c, pm = oracle.scl(m, 1 << K, oracle.F64, y, fr)
        assert len(set(map(bytes, c))) == 1 << K
        e_ml, c_ml = oracle.ml(r, m, oracle.F64, y)
        assert oracle.metric(oracle.F64, y, c[0]) == pytest.approx(e_ml, rel=1e-12)


@pytest.mark.parametrize("r,m,L", [(2, 6, 1), (3, 7, 1), (3, 7, 8)])
def test_noiseless_recovery(r, m, L):
    rng = np.random.default_rng(9)
    fr = oracle.frozen_mask(r, m)
    c0 = random_codeword(r, m, rng)
    u, c, pm = oracle.scl(m, L, oracle.INT, 20.0 * (1 - 2.0 * c0), fr)
    assert np.array_equal(c[0], c0) and pm[0] == 0


def test_scale_invariance_integer_mode():
    rng = np.random.default_rng(11)
    fr = oracle.frozen_mask(3, 7)
    for _ in range(2):
        q = np.clip(np.rint(rng.standard_normal(128) * 30), -63, 63)
        a = oracle.scl(7, 8, oracle.INT, q, fr)
        b = oracle.scl(7, 8, oracle.INT, 2 * q, fr)
        assert np.array_equal(a[1], b[1]) and np.array_equal(2 * a[2], b[2])
