"""The paired-half int8 search (tables of mpwsd_group_moves) on the device,
with the moves it keeps apart searched with plain rows (RM(2,7)).

Bit-exact against the oracle on inputs built to make many moves tie at the
minimum (small integer LLRs), so that the smallest-index rule is exercised
inside a chunk, between the two halves of a row and across chunks; and
bit-identical to the plain N-long search for every tile variant, on batches
spanning several column tiles with a ragged last tile, for RM(3,7) and
RM(3,8)."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2602_08501_amd import decoder as D
from paper_2602_08501_amd import synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
_codes = {}


def code(r, m, grouped):
    key = (r, m, grouped)
    if key not in _codes:
        _codes[key] = D.Code(r, m, DEV, grouped=grouped)
    return _codes[key]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def random_codewords(rng, r, m, n):
    A = oracle.rm_info_set(r, m)
    out = np.zeros((n, 1 << m), np.uint8)
    for i in range(n):
        u = np.zeros(1 << m, np.uint8)
        u[A] = rng.integers(0, 2, len(A))
        out[i] = oracle.encode(m, u)
    return out


def decode(cd, q, anchors, L, T, variant=-1, bpc=0):
    st = D.Stage2([(cd, q.shape[0])], L, T, "i8", DEV)
    llr = torch.from_numpy(q).to(DEV)
    anc = torch.from_numpy(np.packbits(anchors, axis=-1, bitorder="little")).to(DEV)
    o = st.run([llr], [anc], [None], variant=variant, blocks_per_cu=bpc)[0]
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in o.items()}, st.stats.cpu().numpy()


@pytest.mark.parametrize("r,m,F,L,T", [(3, 7, 48, 4, 4), (3, 8, 6, 4, 3), (2, 7, 64, 4, 4)])
def test_ties_follow_smallest_index(r, m, F, L, T):
    say("case: grouped ties", r, m, F, L, T)
    cd = code(r, m, True)
    assert cd.grouped is not None
    rng = np.random.default_rng(70 + m)
    n = 1 << m
    # LLRs in {-2 .. 2}: many moves share the minimum S
    q = rng.integers(-2, 3, (F, n)).astype(np.int8)
    anchors = random_codewords(rng, r, m, F * L).reshape(F, L, n)
    out, _ = decode(cd, q, anchors, L, T)
    supp, _ = oracle.moves(r, m)
    for f in range(F):
        paths, logs, met, kb = oracle.stage2_frame(oracle.INT, supp, q[f].astype(np.float64), anchors[f], T)
        assert np.array_equal(out["moves"][f], logs), f
        assert out["k"][f] == kb and out["metric"][f] == int(met[kb]), f
        assert np.array_equal(np.unpackbits(out["cw"][f], bitorder="little"), paths[kb]), f


@pytest.mark.parametrize("wl,L,T,F", [(synth.RM37, 8, 8, 3000), (synth.RM38, 16, 4, 400), (synth.RM27, 8, 8, 3000)],
                         ids=["rm37", "rm38", "rm27"])
def test_grouped_equals_plain_every_variant(wl, L, T, F):
    say("case: grouped vs plain", wl.r, wl.m, F)
    rng = np.random.default_rng(wl.m)
    c = random_codewords(rng, wl.r, wl.m, F)
    n = 1 << wl.m
    # noisy received words around the codewords; anchors: each codeword with
    # a few flipped bits, so that the searches run several iterations
    y = (1 - 2.0 * c) + rng.standard_normal((F, n)) * 0.9
    q = np.clip(np.rint(y * 10), -127, 127).astype(np.int8)
    anchors = np.repeat(c[:, None, :], L, 1)
    flips = rng.random((F, L, n)) < 0.04
    anchors = anchors ^ flips.astype(np.uint8)
    ref, st_ref = decode(code(wl.r, wl.m, False), q, anchors, L, T)
    assert st_ref[1] == F * L and st_ref[2] > 0  # every path searched, some still moving
    cd = code(wl.r, wl.m, True)
    for variant in range(len(D._lib.mpwsd_search_variants())):
        for bpc in (0, 1):
            got, st = decode(cd, q, anchors, L, T, variant, bpc)
            for key in ref:
                assert np.array_equal(got[key], ref[key]), (variant, bpc, key)
            assert np.array_equal(st, st_ref), (variant, bpc)


def _noisy_case(rng, r, m, F, L):
    c = random_codewords(rng, r, m, F)
    n = 1 << m
    y = (1 - 2.0 * c) + rng.standard_normal((F, n)) * 0.9
    q = np.clip(np.rint(y * 10), -127, 127).astype(np.int8)
    anchors = np.repeat(c[:, None, :], L, 1) ^ (rng.random((F, L, n)) < 0.04).astype(np.uint8)
    return q, anchors


def _decode_segments(codes, cases, L, T):
    st = D.Stage2([(cd, q.shape[0]) for cd, (q, _) in zip(codes, cases)], L, T, "i8", DEV)
    llrs = [torch.from_numpy(q).to(DEV) for q, _ in cases]
    ancs = [torch.from_numpy(np.packbits(a, axis=-1, bitorder="little")).to(DEV) for _, a in cases]
    outs = st.run(llrs, ancs, [None] * len(cases))
    torch.cuda.synchronize()
    return [{k: v.cpu().numpy() for k, v in o.items()} for o in outs], st.stats.cpu().numpy()


@pytest.mark.parametrize("mix", [[(2, 7), (3, 7), (2, 6)], [(2, 7), (3, 7), (2, 6), (2, 7)]],
                         ids=["extras_in_the_launch", "extras_launched_apart"])
def test_moves_kept_apart_in_a_mixed_launch(mix):
    """RM(2,7) with its layout (4096 moves kept apart) beside other codes in
    one search launch per iteration: the kept-apart moves are entries of the
    same launch while there is room (at most 4), else launches of their own;
    every output equals the plain tables'."""
    say("case: kept-apart moves in a mixed launch", mix)
    rng = np.random.default_rng(90 + len(mix))
    L, T = 8, 6
    cases = [_noisy_case(rng, r, m, 700, L) for r, m in mix]
    ref, st_ref = _decode_segments([code(r, m, False) for r, m in mix], cases, L, T)
    grouped = [code(r, m, True) for r, m in mix]
    assert grouped[0].grouped is not None and grouped[0].grouped_extras == 4096
    got, st = _decode_segments(grouped, cases, L, T)
    for i in range(len(mix)):
        for key in ref[i]:
            assert np.array_equal(got[i][key], ref[i][key]), (mix[i], key)
    assert np.array_equal(st, st_ref)
