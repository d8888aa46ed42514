"""mpwsd_decode_batch_noalloc: the same results as mpwsd_decode_batch, from
the library's fixed per-GPU scratch array instead of a caller workspace.

Calls go through the C-ABI (ctypes binding) one after another on one stream,
the later ones with smaller inputs, so every call must rebuild its state in
the shared array instead of reading what the previous call left there.  Each
result is compared bit for bit with mpwsd_decode_batch on the same inputs
(decisions, chosen paths, metrics, move logs and statistics).  A batch whose
workspace exceeds the array is refused on the host with MPWSD_ERR_SIZE.
"""
import dataclasses
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2602_08501_amd import _lib
from paper_2602_08501_amd import decoder as D
from paper_2602_08501_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def stage1_inputs(wl, F, L, dtype, seed):
    pay, c, y = synth.generate(wl, seed, 0, F)
    code = D.Code(wl.r, wl.m, DEV)
    if dtype == "i8":
        llr = torch.from_numpy(oracle.quantize(y, wl.llr_scale)).to(DEV)
    else:
        llr = torch.from_numpy(y).to(DEV)
    s1 = D.stage1(code, L, llr, wl.crc_len, wl.crc_poly)
    return code, llr, s1


def run_both(parts, L, T, dtype):
    """parts: [(code, llr, s1)]; returns (noalloc outputs, workspace outputs)."""
    res = []
    for mode in ("noalloc", "ws"):
        st = D.Stage2([(code, llr.shape[0]) for code, llr, s1 in parts], L, T, dtype, DEV)
        segs = st._segs([p[1] for p in parts], [p[2]["anchors"] for p in parts], [p[2]["crc_ok"] for p in parts])
        stream = torch.cuda.current_stream().cuda_stream
        if mode == "noalloc":
            rc = _lib.mpwsd_decode_batch_noalloc(segs, L, T, st.stats.data_ptr(), stream)
        else:
            rc = _lib.mpwsd_decode_batch(segs, L, T, st.ws_ptr, st.ws_bytes, st.stats.data_ptr(), stream)
        _lib.check(rc)
        torch.cuda.synchronize()
        res.append(([{k: v.cpu().numpy() for k, v in o.items()} for o in st.outs], st.stats.cpu().numpy()))
    return res


def assert_same(a, b):
    (oa, sa), (ob, sb) = a, b
    assert np.array_equal(sa, sb)
    assert sa[-1] == 0
    for x, y in zip(oa, ob):
        for k in y:
            assert np.array_equal(x[k], y[k]), k


RM26_25 = dataclasses.replace(synth.RM26, ebn0_db=2.5)


def test_noalloc_equals_workspace_calls_in_a_row():
    say("case: noalloc call 1: RM(3,7) 6000 frames L=8 T=8 int8")
    a = stage1_inputs(synth.RM37, 6000, 8, "i8", 3)
    r1 = run_both([a], 8, 8, "i8")
    assert r1[0][1][0] > 100  # frames that reached stage 2
    assert_same(*r1)
    say("case: noalloc call 2 (smaller): RM(2,6) 500 frames L=4 T=4 int8")
    b = stage1_inputs(RM26_25, 500, 4, "i8", 4)
    r2 = run_both([b], 4, 4, "i8")
    assert_same(*r2)
    say("case: noalloc call 3 (smaller): RM(3,7) 700 frames L=8 T=8 int8")
    c = stage1_inputs(synth.RM37, 700, 8, "i8", 5)
    r3 = run_both([c], 8, 8, "i8")
    assert_same(*r3)


def test_noalloc_mixed_and_float():
    say("case: noalloc mixed RM(2,6) + RM(3,7), then binary32 RM(2,6)")
    p = [stage1_inputs(RM26_25, 900, 8, "i8", 6), stage1_inputs(synth.RM37, 1200, 8, "i8", 7)]
    assert_same(*run_both(p, 8, 6, "i8"))
    f = stage1_inputs(RM26_25, 300, 4, "f32", 8)
    assert_same(*run_both([f], 4, 4, "f32"))


def test_noalloc_refuses_oversized_batch():
    say("case: noalloc size limit (host check, nothing enqueued)")
    code = D.Code(3, 7, DEV)
    F, L, T = 60000, 8, 8
    seg = _lib.Segment(3, 7, code.moves.data_ptr(), code.P, None, _lib.MPWSD_I8, F, None, None, None, None, None,
                       None, None, 0, 0)
    assert _lib.mpwsd_workspace_bytes([seg], L, T) > _lib.MPWSD_NOALLOC_SCRATCH_BYTES
    q = torch.zeros((F, 128), dtype=torch.int8, device=DEV)
    anc = torch.zeros((F, L, 16), dtype=torch.uint8, device=DEV)
    out = torch.zeros((F, 16), dtype=torch.uint8, device=DEV)
    seg = _lib.Segment(3, 7, code.moves.data_ptr(), code.P, q.data_ptr(), _lib.MPWSD_I8, F, anc.data_ptr(), None,
                       out.data_ptr(), None, None, None, None, 0, 0)
    rc = _lib.mpwsd_decode_batch_noalloc([seg], L, T, None, torch.cuda.current_stream().cuda_stream)
    assert rc == _lib.MPWSD_ERR_SIZE
    assert "noalloc" in _lib.last_error()
    torch.cuda.synchronize()
    assert not out.any()
