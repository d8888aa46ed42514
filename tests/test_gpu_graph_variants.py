"""Search tile variants give bit-identical results, and a recorded HIP graph
of the whole decoder replays to the eager result every time (replays are
interleaved with other eager work and synchronisations)."""
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


@pytest.mark.parametrize("wl,L,T,F", [(dataclasses.replace(synth.RM37, ebn0_db=2.0), 8, 8, 700),
                                      (synth.RM26, 4, 4, 500),
                                      (dataclasses.replace(synth.RM27, ebn0_db=2.0), 8, 6, 300)])
def test_variants_bit_identical(wl, L, T, F):
    say("case: variants", wl.r, wl.m, L, T, F)
    pay, c, y = synth.generate(wl, 11, 0, F)
    q = torch.from_numpy(oracle.quantize(y, wl.llr_scale)).to(DEV)
    code = D.Code(wl.r, wl.m, DEV)
    s1 = D.stage1(code, L, q, wl.crc_len, wl.crc_poly)
    st = D.Stage2([(code, F)], L, T, "i8", DEV)
    st.run([q], [s1["anchors"]], [s1["crc_ok"]])
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in st.outs[0].items()}
    nv = len(_lib.mpwsd_search_variants())
    for var in range(nv):
        for bpc in (0, 1, 3):
            st.run([q], [s1["anchors"]], [s1["crc_ok"]], variant=var, blocks_per_cu=bpc)
            torch.cuda.synchronize()
            for k in ref:
                assert torch.equal(ref[k], st.outs[0][k]), (var, bpc, k)
    # a different tile variant and grid for every iteration
    iv = [t % nv for t in range(T)]
    ib = [(0, 1, 2, 3)[t % 4] for t in range(T)]
    st.run([q], [s1["anchors"]], [s1["crc_ok"]], variant=iv, blocks_per_cu=ib)
    torch.cuda.synchronize()
    for k in ref:
        assert torch.equal(ref[k], st.outs[0][k]), ("per iteration", k)


def test_graph_replay_matches_eager():
    wl = dataclasses.replace(synth.RM37, ebn0_db=2.0)
    F, L, T = 1024, 8, 8
    say("case: graph replay", F)
    pay, c, y = synth.generate(wl, 12, 0, F)
    y_d = torch.from_numpy(y).to(DEV)
    code = D.Code(wl.r, wl.m, DEV)
    q = torch.empty(y.shape, dtype=torch.int8, device=DEV)
    s1 = {"anchors": torch.empty((F, L, 16), dtype=torch.uint8, device=DEV),
          "crc_ok": torch.empty(F, dtype=torch.uint8, device=DEV)}
    st = D.Stage2([(code, F)], L, T, "i8", DEV)
    scale = float(wl.llr_scale)

    D.quantize(y_d, scale, out=q)
    D.stage1(code, L, q, wl.crc_len, wl.crc_poly, out=s1)
    st.run([q], [s1["anchors"]], [s1["crc_ok"]])
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in st.outs[0].items()}
    ref_stats = st.stats.clone()

    def record(raw):
        D.quantize(y_d, scale, out=q, raw_stream=raw)
        D.stage1(code, L, q, wl.crc_len, wl.crc_poly, out=s1, raw_stream=raw)
        st.run([q], [s1["anchors"]], [s1["crc_ok"]], raw_stream=raw)

    g = D.Graph(record)
    for rep in range(4):
        for v in st.outs[0].values():
            v.fill_(-7)            # eager work between replays
        s1["anchors"].zero_()
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(ref[k], st.outs[0][k]), (rep, k)
        assert torch.equal(ref_stats, st.stats)
    del g
