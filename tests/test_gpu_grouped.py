"""The paired-half int8 search (tables of mpwsd_group_moves) on the device.

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


@pytest.mark.parametrize("r,m,F,L,T", [(3, 7, 48, 4, 4), (3, 8, 6, 4, 3)])
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


@pytest.mark.parametrize("wl,L,T,F", [(synth.RM37, 8, 8, 3000), (synth.RM38, 16, 4, 400)],
                         ids=["rm37", "rm38"])
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
