"""int8 LLRs of -128 at the boundary: every call reads them as -127.

The int8 form works in the symmetric range [-127, 127], where the negation
z = q (1 - 2c) of Eq. (5) is exact in int8 and every stage-1 value stays
within 127 N.  A caller may still pass -128; the library reads it as -127.
So decoding q with -128 entries must equal, bit for bit, the oracle's decode
of q clipped to [-127, 127], and the library's own decode of the clipped q.
Frames of RM(3,8) made entirely of +-127 / -128 drive every stage-1 level to
its bound (127 * 256 = 32512 at the root).
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2602_08501_amd import decoder as D
from paper_2602_08501_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def unpack(t):
    return np.unpackbits(t.cpu().numpy(), axis=-1, bitorder="little")


def with_m128(wl, F, seed):
    """Seeded frames of the workload with -128 planted: 2% of the entries of
    every frame, plus two frames of full-scale values (+127 / -128)."""
    pay, c, y = synth.generate(wl, seed, 0, F)
    q = oracle.quantize(y, wl.llr_scale)
    rng = np.random.default_rng(seed)
    q[rng.random(q.shape) < 0.02] = -128
    N = q.shape[1]
    for f in (1, F - 1):
        q[f] = np.where(rng.random(N) < 0.5, 127, -128).astype(np.int8)
    assert (q == -128).any()
    return q


CASES = [("rm37", synth.RM37, 8, 8, 48), ("rm38", synth.RM38, 4, 3, 12)]


@pytest.mark.parametrize("name,wl,L,T,F", CASES, ids=[c[0] for c in CASES])
def test_minus128_reads_as_minus127(name, wl, L, T, F):
    say("case: int8 -128", name, "L", L, "T", T, "F", F)
    q = with_m128(wl, F, 11)
    qc = np.clip(q, -127, 127)
    cd = D.Code(wl.r, wl.m, DEV)
    outs = []
    for arr in (q, qc):
        qd = torch.from_numpy(arr).to(DEV)
        s1 = D.stage1(cd, L, qd, wl.crc_len, wl.crc_poly, want_pm=True)
        st = D.Stage2([(cd, F)], L, T, "i8", DEV)
        o = st.run([qd], [s1["anchors"]], [s1["crc_ok"]])[0]
        torch.cuda.synchronize()
        res = {k: v.cpu().numpy() for k, v in o.items()}
        res.update({"anchors": s1["anchors"].cpu().numpy(), "crc_ok": s1["crc_ok"].cpu().numpy(),
                    "pm": s1["pm"].cpu().numpy(), "stats": st.stats.cpu().numpy()})
        outs.append(res)
    for k in outs[1]:
        assert np.array_equal(outs[0][k], outs[1][k]), k
    got = outs[0]
    assert got["stats"][-1] == 0
    ref = oracle.decode_batch(wl.r, wl.m, wl.crc_len, wl.crc_poly, L, T, oracle.INT,
                              qc.astype(np.float64), threads=8)
    assert np.array_equal(got["crc_ok"], ref["crc_ok"])
    assert np.array_equal(np.unpackbits(got["anchors"], axis=-1, bitorder="little"), ref["anchors"])
    assert np.array_equal(np.unpackbits(got["cw"], axis=-1, bitorder="little"), ref["c"])
    assert np.array_equal(got["k"], ref["k"])
    assert np.array_equal(got["metric"], ref["metric"].astype(np.int32))
    assert np.array_equal(got["moves"], ref["logs"])
    # the full-scale frames' path metrics against the oracle's list
    fr = oracle.frozen_mask(wl.r, wl.m)
    for f in (1, F - 1):
        u, c, pm = oracle.scl(wl.m, L, oracle.INT, qc[f].astype(np.float64), fr)
        assert np.array_equal(got["pm"][f], pm.astype(np.int32)), f


def test_minus128_osd():
    say("case: int8 -128, OSD(2) RM(2,7)")
    wl = synth.Workload(r=2, m=7, k_pay=29, crc_len=0, ebn0_db=2.0, wid=37)
    F, L, T = 40, 8, 3
    q = with_m128(wl, F, 12)
    qc = np.clip(q, -127, 127)
    cd = D.Code(2, 7, DEV)
    outs = []
    for arr in (q, qc):
        qd = torch.from_numpy(arr).to(DEV)
        s1 = D.stage1_osd(cd, 2, L, qd, want_metric=True)
        st = D.Stage2([(cd, F)], L, T, "i8", DEV)
        o = st.run([qd], [s1["anchors"]], [None])[0]
        torch.cuda.synchronize()
        res = {k: v.cpu().numpy() for k, v in o.items()}
        res.update({"anchors": s1["anchors"].cpu().numpy(), "anchor_metric": s1["metric"].cpu().numpy()})
        outs.append(res)
    for k in outs[1]:
        assert np.array_equal(outs[0][k], outs[1][k]), k
    ref = oracle.decode_osd_batch(2, 7, 2, L, T, oracle.INT, qc.astype(np.float64), threads=8)
    got = outs[0]
    assert np.array_equal(np.unpackbits(got["anchors"], axis=-1, bitorder="little"), ref["anchors"])
    assert np.array_equal(got["anchor_metric"], ref["anchor_metric"].astype(np.int32))
    assert np.array_equal(np.unpackbits(got["cw"], axis=-1, bitorder="little"), ref["c"])
    assert np.array_equal(got["moves"], ref["logs"])
    assert np.array_equal(got["metric"], ref["metric"].astype(np.int32))
