"""Pins for stage 2, MP-WSD (Sec. III-B, Eq. (4)-(5), Alg. 1, Remark 1).

* Eq. (5) identity: for a centre c and move w, the change of the squared
  distance ||y - x(c xor w)||^2 - ||y - x(c)||^2 equals 4 S(w) with
  S(w) = sum_{j in supp w} y_j x_j(c) = -G(w)/2, recomputed from scratch.
* Brute-force ML on RM(1, m): every codeword other than the centre and its
  complement is one minimum-weight move away, and if the complement is better
  some move already improves, so T = 2 iterations from any anchor reach a
  maximum-likelihood codeword (the metric equals the exhaustive minimum).
* Remark 1: the metric strictly decreases at every accepted move and the
  final decision is no worse than the best anchor.
* Eq. (3) equivariance: decoding y' = y * x(c0) from anchors a_k xor c0 gives
  identical move logs and the decision xor c0.
* A path that stops is a local optimum: every move has S >= 0.
* Noiseless single-move recovery: y = Q x(c), anchor c xor w_p0 gives p0 as
  the unique first move and c as the decision (pins the move indexing).
* Filter equivalence: Alg. 1 as printed (top-m filter by G, exact-distance
  search, early break) gives the same paths as the full argmin, for m = 1,
  10 and the paper's rule max(10, ceil(0.02 |S|)).
"""
import math

import numpy as np
import pytest

import oracle
from test_oracle_scl import random_codeword


def ed(y, c):
    return float(((np.asarray(y, np.float64) - (1 - 2.0 * np.asarray(c))) ** 2).sum())


def test_eq5_identity():
    rng = np.random.default_rng(21)
    supp, w = oracle.moves(2, 6)
    for _ in range(20):
        y = rng.standard_normal(64) * 1.3
        c = random_codeword(2, 6, rng)
        p = rng.integers(len(supp))
        cw = c.copy()
        cw[supp[p]] ^= 1
        z = y * (1 - 2.0 * c)
        S = z[supp[p]].sum()
        G = (-2 * y * (1 - 2.0 * c))[supp[p]].sum()
        assert ed(y, cw) - ed(y, c) == pytest.approx(4 * S, abs=1e-9)
        assert S == pytest.approx(-G / 2, abs=1e-12)


@pytest.mark.parametrize("m", [5, 7])
def test_rm1_reaches_ml(m):
    rng = np.random.default_rng(30 + m)
    supp, w = oracle.moves(1, m)
    n = 1 << m
    for trial in range(12):
        y = 1 - 2.0 * random_codeword(1, m, rng) + rng.standard_normal(n) * 1.2
        q = np.clip(np.rint(y * 8), -127, 127)
        anchors = np.array([random_codeword(1, m, rng) for _ in range(3)])
        for mode, obs in ((oracle.INT, q), (oracle.F64, y)):
            paths, logs, met, kb = oracle.stage2_frame(mode, supp, obs, anchors, 2)
            e_ml, _ = oracle.ml(1, m, mode, obs)
            assert met[kb] == pytest.approx(e_ml, abs=1e-9)
            # every path alone reaches ML as well
            for k in range(3):
                assert met[k] == pytest.approx(e_ml, abs=1e-9)


@pytest.mark.parametrize("r,m,T", [(2, 6, 6), (3, 7, 8)])
def test_monotone_and_no_worse_than_anchor(r, m, T):
    rng = np.random.default_rng(40 + m)
    supp, w = oracle.moves(r, m)
    n = 1 << m
    for trial in range(3):
        y = 1 - 2.0 * random_codeword(r, m, rng) + rng.standard_normal(n) * 1.0
        q = np.clip(np.rint(y * 10), -127, 127)
        anchors = np.array([random_codeword(r, m, rng) for _ in range(4)])
        paths, logs, met, kb = oracle.stage2_frame(oracle.INT, supp, q, anchors, T)
        for k in range(4):
            c = anchors[k].copy()
            prev = oracle.metric(oracle.INT, q, c)
            stopped = False
            for t in range(T):
                p = logs[k, t]
                if p < 0:
                    stopped = True
                    continue
                assert not stopped
                c[supp[p]] ^= 1
                cur = oracle.metric(oracle.INT, q, c)
                assert cur < prev
                prev = cur
            assert np.array_equal(c, paths[k]) and met[k] == prev
        assert met[kb] <= min(oracle.metric(oracle.INT, q, a) for a in anchors)
        assert kb == int(np.argmin(met))


def test_equivariance():
    rng = np.random.default_rng(50)
    supp, w = oracle.moves(2, 6)
    for _ in range(5):
        q = np.clip(np.rint(rng.standard_normal(64) * 15), -127, 127)
        anchors = np.array([random_codeword(2, 6, rng) for _ in range(4)])
        c0 = random_codeword(2, 6, rng)
        a = oracle.stage2_frame(oracle.INT, supp, q, anchors, 5)
        b = oracle.stage2_frame(oracle.INT, supp, q * (1 - 2.0 * c0), anchors ^ c0, 5)
        assert np.array_equal(a[1], b[1])
        assert np.array_equal(a[0] ^ c0, b[0])
        assert a[3] == b[3]


def test_stopped_paths_are_local_optima():
    rng = np.random.default_rng(60)
    supp, w = oracle.moves(2, 6)
    for _ in range(5):
        q = np.clip(np.rint(rng.standard_normal(64) * 15), -127, 127)
        c = random_codeword(2, 6, rng)
        cf, log = oracle.stage2_path(oracle.INT, supp, q, c, 30)
        assert log[-1] == -1
        z = q * (1 - 2.0 * cf)
        assert (z[supp].sum(1) >= 0).all()


@pytest.mark.parametrize("r,m", [(2, 6), (2, 7), (3, 7)])
def test_single_move_recovery(r, m):
    rng = np.random.default_rng(70 + m)
    supp, w = oracle.moves(r, m)
    for p0 in rng.choice(len(supp), 5, replace=False):
        c = random_codeword(r, m, rng)
        a = c.copy()
        a[supp[p0]] ^= 1
        q = 9.0 * (1 - 2.0 * c)
        cf, log = oracle.stage2_path(oracle.INT, supp, q, a, 3)
        assert log.tolist() == [p0, -1, -1]
        assert np.array_equal(cf, c)


@pytest.mark.parametrize("r,m", [(2, 6), (1, 7)])
def test_paper_filter_gives_full_argmin(r, m):
    rng = np.random.default_rng(80 + m)
    supp, w = oracle.moves(r, m)
    n = 1 << m
    rule = max(10, math.ceil(0.02 * len(supp)))
    for trial in range(4):
        y = 1 - 2.0 * random_codeword(r, m, rng) + rng.standard_normal(n) * 1.1
        anchors = np.array([random_codeword(r, m, rng) for _ in range(4)])
        ref_paths, ref_logs, met, kb = oracle.stage2_frame(oracle.F64, supp, y, anchors, 4)
        for mf in (1, 10, rule):
            paths, logs, kb2 = oracle.stage2_alg1(supp, y, anchors, 4, mf)
            assert np.array_equal(paths, ref_paths)
            assert np.array_equal(logs, ref_logs)
            assert kb2 == kb
