"""Pins for the oracle's ordered-statistics decoder (OSD(k) stage 1).

* order K lists the whole code: with L = 2^K the list is every codeword once
  and its first entry attains the brute-force ML metric;
* the most reliable basis is what it claims: K positions in reliability
  order whose columns of the monomial generator (not the oracle's) are
  independent, each skipped position being dependent on the basis
  positions ranked before it;
* every candidate is a codeword that differs from the hard decisions on the
  MRB in at most k positions, the count is sum_{s<=k} C(K, s), all distinct;
* the sent codeword is in the list exactly when it has at most k hard
  decision errors on the MRB;
* with all-zero LLRs every metric ties and the list is the candidate
  numbering itself: the zero word, then the K unit patterns in MRB order,
  then the pairs in lexicographic order.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2602_08501_amd import synth
from test_oracle_code import monomial_generator
from test_oracle_sphere import gf2_basis, in_span


def gf2_rank(cols):
    return len(gf2_basis(np.array(cols, np.uint8)))


def codeword_set(r, m):
    G = monomial_generator(r, m)
    K = len(G)
    msgs = ((np.arange(1 << K)[:, None] >> np.arange(K)) & 1).astype(np.int64)
    return {tuple(x) for x in (msgs @ G % 2).astype(np.uint8)}


@pytest.mark.parametrize("r,m", [(1, 5), (2, 5)])
def test_order_K_lists_whole_code_and_ml_first(r, m):
    N, K = oracle.rm_dims(r, m)
    code = codeword_set(r, m)
    rng = np.random.default_rng(1 + m)
    for trial in range(3):
        y = 1 - 2.0 * rng.integers(0, 2, N) + rng.standard_normal(N)
        q = np.clip(np.rint(y * 6), -127, 127)
        for mode, obs in ((oracle.INT, q), (oracle.F64, y)):
            a, met, mrb = oracle.osd(r, m, K, 1 << K, mode, obs)
            assert len(a) == 1 << K
            assert {tuple(x) for x in a} == code
            e_ml, _ = oracle.ml(r, m, mode, obs)
            assert met[0] == pytest.approx(e_ml, abs=1e-9)
            assert np.all(np.diff(met) >= 0)


@pytest.mark.parametrize("r,m,k", [(2, 6, 2), (2, 7, 1), (1, 5, 3), (3, 6, 1)])
def test_mrb_and_candidates(r, m, k):
    N, K = oracle.rm_dims(r, m)
    G = monomial_generator(r, m)
    rng = np.random.default_rng(10 + r + m)
    C = sum(math.comb(K, s) for s in range(k + 1))
    for trial in range(4):
        y = 1 - 2.0 * rng.integers(0, 2, N) + rng.standard_normal(N) * 0.9
        q = np.clip(np.rint(y * 7), -127, 127)
        a, met, mrb = oracle.osd(r, m, k, C + 5, oracle.INT, q)
        # reliability order, ties to the smaller position
        order = sorted(range(N), key=lambda j: (-abs(q[j]), j))
        rank = {j: i for i, j in enumerate(order)}
        assert [rank[j] for j in mrb] == sorted(rank[j] for j in mrb)
        assert gf2_rank(G[:, mrb].T) == K
        basis_cols = []
        for j in order[:rank[mrb[-1]] + 1]:
            col = G[:, j].copy()
            if j in set(mrb.tolist()):
                basis_cols.append(col)
            else:
                assert basis_cols and in_span(gf2_basis(np.array(basis_cols)), col), j
        # candidates
        assert len(a) == C and len({tuple(x) for x in a}) == C
        hd = (q < 0).astype(np.uint8)
        basis = gf2_basis(G)
        for x in a:
            assert in_span(basis, x)
            assert int((x[mrb] != hd[mrb]).sum()) <= k
        assert np.all(np.diff(met) >= 0)
        for x, mt in zip(a[:20], met[:20]):
            assert mt == q[x == 1].sum()


@pytest.mark.parametrize("k", [1, 2])
def test_sent_word_listed_iff_few_mrb_errors(k):
    wl = synth.Workload(r=2, m=6, k_pay=22, crc_len=0, ebn0_db=1.0, wid=21)
    pay, c, y = synth.generate(wl, 0, 0, 60)
    q = oracle.quantize(y, wl.llr_scale).astype(np.float64)
    N, K = oracle.rm_dims(2, 6)
    C = sum(math.comb(K, s) for s in range(k + 1))
    seen = {True: 0, False: 0}
    for f in range(len(q)):
        a, met, mrb = oracle.osd(2, 6, k, C, oracle.INT, q[f])
        errs = int(((q[f][mrb] < 0).astype(np.uint8) != c[f][mrb]).sum())
        listed = any(np.array_equal(x, c[f]) for x in a)
        assert listed == (errs <= k), (f, errs)
        seen[listed] += 1
    assert seen[True] > 0 and seen[False] > 0


def test_numbering_when_all_metrics_tie():
    r, m, k = 2, 6, 2
    N, K = oracle.rm_dims(r, m)
    C = sum(math.comb(K, s) for s in range(k + 1))
    a, met, mrb = oracle.osd(r, m, k, C, oracle.INT, np.zeros(N))
    assert np.all(met == 0)
    # all reliabilities tie: the MRB is the first K independent positions by index
    G = monomial_generator(r, m)
    kept = []
    for j in range(N):
        if gf2_rank(G[:, kept + [j]].T) == len(kept) + 1:
            kept.append(j)
        if len(kept) == K:
            break
    assert mrb.tolist() == kept
    assert not a[0].any()                        # candidate 0: the zero word (HD of 0 is 0)
    unit = np.eye(K, dtype=np.uint8)
    for i in range(K):                           # candidates 1..K: e = {i}
        assert np.array_equal(a[1 + i][mrb], unit[i])
    pairs = [(i, j) for i in range(K) for j in range(i + 1, K)]
    for t, (i, j) in enumerate(pairs):           # then the pairs in lexicographic order
        assert np.array_equal(a[1 + K + t][mrb], unit[i] ^ unit[j])
