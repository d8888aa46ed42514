"""Merging of equal centres in stage 2 (on by default), on inputs built to
make paths of a frame meet: anchors that repeat, and anchors made of the
frame's codeword plus zero to three of four nearby moves, so that paths reach
common centres after different numbers of moves (a leader may later follow
another path: chains).  Every frame goes to stage 2 (no CRC).  Checked
bit-exactly against the oracle, which searches every path, with and without
merging, for list sizes that leave idle lanes in a frame's lane group (L = 3,
5), fill half a wave (L = 32) or give one lane per frame (L = 1), in the int8
and binary32 forms; the searched counts must equal the merging rule replayed
over the oracle's logs."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2602_08501_amd import decoder as D

from merge_rule import replay, searched_counts

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
_codes = {}


def code(r, m):
    if (r, m) not in _codes:
        _codes[(r, m)] = D.Code(r, m, DEV)
    return _codes[(r, m)]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def make_case(r, m, F, L, seed):
    rng = np.random.default_rng(seed)
    n = 1 << m
    A = oracle.rm_info_set(r, m)
    supp, _ = oracle.moves(r, m)
    c = np.zeros((F, n), np.uint8)
    for f in range(F):
        u = np.zeros(n, np.uint8)
        u[A] = rng.integers(0, 2, len(A))
        c[f] = oracle.encode(m, u)
    y = (1 - 2.0 * c) + rng.standard_normal((F, n)) * 0.8
    q = np.clip(np.rint(y * 12), -127, 127).astype(np.int8)
    anchors = np.zeros((F, L, n), np.uint8)
    for f in range(F):
        near = rng.choice(len(supp), 4, replace=False)
        for k in range(L):
            kind = rng.integers(0, 5) if k > 0 else 1
            a = c[f].copy()
            if kind == 4:
                a = anchors[f, k - 1].copy()           # repeat the previous anchor
            else:
                # the codeword plus 0 .. 3 of the frame's four nearby moves:
                # paths reach common centres after different numbers of moves
                for p in rng.choice(near, kind, replace=False):
                    a[supp[p]] ^= 1
            anchors[f, k] = a
    return q, y.astype(np.float32), anchors, supp


def run(cd, obs, anchors, L, T, dtype, merge):
    F = obs.shape[0]
    st = D.Stage2([(cd, F)], L, T, dtype, DEV)
    anc = torch.from_numpy(np.packbits(anchors, axis=-1, bitorder="little")).to(DEV)
    o = st.run([torch.from_numpy(obs).to(DEV)], [anc], [None], merge=merge)[0]
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in o.items()}, st.stats.cpu().numpy()


CASES = [
    ("rm26_L3", 2, 6, 300, 3, 6),
    ("rm26_L5", 2, 6, 300, 5, 6),
    ("rm26_L1", 2, 6, 200, 1, 4),
    ("rm37_L5", 3, 7, 120, 5, 5),
    ("rm37_L32", 3, 7, 40, 32, 4),
]


@pytest.mark.parametrize("name,r,m,F,L,T", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("dtype", ["i8", "f32"])
def test_merge_edges(name, r, m, F, L, T, dtype):
    say("case: merge edges", name, dtype)
    q, y, anchors, supp = make_case(r, m, F, L, 80 + L + m)
    obs = q if dtype == "i8" else y
    mode = oracle.INT if dtype == "i8" else oracle.F32
    cd = code(r, m)
    got, st = run(cd, obs, anchors, L, T, dtype, True)
    raw, st_raw = run(cd, obs, anchors, L, T, dtype, False)
    for key in got:
        assert np.array_equal(got[key], raw[key]), key
    logs = np.zeros((F, L, T), np.int32)
    follows = stops = chains = 0
    for f in range(F):
        paths, lg, met, kb = oracle.stage2_frame(mode, supp, obs[f].astype(np.float64), anchors[f], T)
        logs[f] = lg
        assert np.array_equal(got["moves"][f], lg), f
        assert got["k"][f] == kb, f
        assert np.array_equal(np.unpackbits(got["cw"][f], bitorder="little"), paths[kb]), f
        if dtype == "i8":
            assert got["metric"][f] == int(met[kb]), f
        else:
            assert got["metric"][f:f + 1].view(np.float32)[0] == np.float32(met[kb]), f
        ev = replay(anchors[f], lg, supp)[1]
        follows += sum(1 for e in ev if e[2] == "follow")
        stops += sum(1 for e in ev if e[2] == "stop")
        followers = {e[1] for e in ev if e[2] == "follow"}
        chains += sum(1 for e in ev if e[2] == "follow" and e[3] in followers)
    assert np.array_equal(st[1:1 + T], searched_counts(anchors, logs, supp))
    moved = [F * L] + [int((logs[:, :, t - 1] >= 0).sum()) for t in range(1, T)]
    assert np.array_equal(st_raw[1:1 + T], moved)
    say("  searched", st[1:1 + T].tolist(), "without merging", moved, "follow", follows, "stop", stops,
        "chains", chains)
    if L > 1:
        assert follows > 0 and stops > 0
    if L == 32:
        assert chains > 0


@pytest.mark.parametrize("L", [3, 5, 32])
def test_multi_code_resolve_odd_lists(L):
    """One resolve launch for several codes (a multi-code call), with list
    sizes that leave lanes idle in a frame's group (3, 5) or put two frames on
    a wave (32): every output and the searched counts equal each code decoded
    alone."""
    say("case: multi-code merge, L", L)
    T = 5
    parts = [(2, 6, 150), (3, 7, 60), (2, 7, 90)]
    cases = []
    for i, (r, m, F) in enumerate(parts):
        q, y, anchors, supp = make_case(r, m, F, L, 300 + 10 * L + i)
        cases.append((code(r, m), q, anchors))
    st = D.Stage2([(cd, q.shape[0]) for cd, q, a in cases], L, T, "i8", DEV)
    ancs = [torch.from_numpy(np.packbits(a, axis=-1, bitorder="little")).to(DEV) for cd, q, a in cases]
    outs = st.run([torch.from_numpy(q).to(DEV) for cd, q, a in cases], ancs, [None] * len(cases))
    torch.cuda.synchronize()
    outs = [{k: v.cpu().numpy() for k, v in o.items()} for o in outs]
    tot = np.zeros(2 + T, np.int64)
    for (cd, q, anchors), o in zip(cases, outs):
        ref, stats = run(cd, q, anchors, L, T, "i8", True)
        tot += stats
        for k in ref:
            assert np.array_equal(o[k], ref[k]), k
    assert np.array_equal(st.stats.cpu().numpy(), tot)
