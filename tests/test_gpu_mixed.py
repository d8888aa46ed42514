"""Mixed-code batches: several codes' failing frames searched in ONE launch
per iteration.  Results equal the per-code decodes bit for bit and the oracle
on samples, at small and at full size (262144 frames, 1:1:1)."""
import dataclasses
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2602_08501_amd import autotune
from paper_2602_08501_amd import decoder as D
from paper_2602_08501_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def prepare(wls, Fs, L, seed):
    segs = []
    for wl, F in zip(wls, Fs):
        pay, c, y = synth.generate(wl, seed, 0, F)
        code = D.Code(wl.r, wl.m, DEV)
        q = D.quantize(torch.from_numpy(y).to(DEV), wl.llr_scale)
        s1 = D.stage1(code, L, q, wl.crc_len, wl.crc_poly)
        segs.append((wl, code, q, s1, c))
    torch.cuda.synchronize()
    return segs


def run_mixed(segs, L, T, variant=-1):
    st = D.Stage2([(code, q.shape[0]) for wl, code, q, s1, c in segs], L, T, "i8", DEV)
    st.run([seg[2] for seg in segs], [seg[3]["anchors"] for seg in segs], [seg[3]["crc_ok"] for seg in segs],
           variant=variant)
    torch.cuda.synchronize()
    return [{k: v.cpu().numpy() for k, v in o.items()} for o in st.outs], st.stats.cpu().numpy()


def run_single(seg, L, T):
    wl, code, q, s1, c = seg
    st = D.Stage2([(code, q.shape[0])], L, T, "i8", DEV)
    st.run([q], [s1["anchors"]], [s1["crc_ok"]])
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in st.outs[0].items()}, st.stats.cpu().numpy()


MIX = [dataclasses.replace(synth.RM26, ebn0_db=2.5), dataclasses.replace(synth.RM27, ebn0_db=2.0),
       dataclasses.replace(synth.RM37, ebn0_db=2.0)]


@pytest.mark.parametrize("variant", [-1, 0, 1, 2])
def test_mixed_equals_single(variant):
    say("case: mixed small, variant", variant)
    L, T = 8, 8
    segs = prepare(MIX, [300, 200, 400], L, 21)
    outs, stats = run_mixed(segs, L, T, variant)
    tot = np.zeros_like(stats)
    for seg, o in zip(segs, outs):
        ref, st1 = run_single(seg, L, T)
        tot += st1
        for k in ref:
            assert np.array_equal(ref[k], o[k]), k
    assert np.array_equal(tot, stats)


def test_mixed_with_rm38_and_oracle():
    say("case: mixed incl. RM(3,8)")
    L, T = 8, 6
    wls = [dataclasses.replace(synth.RM37, ebn0_db=2.0), dataclasses.replace(synth.RM38, ebn0_db=1.75)]
    segs = prepare(wls, [200, 60], L, 22)
    outs, stats = run_mixed(segs, L, T)
    for (wl, code, q, s1, c), o in zip(segs, outs):
        qq = q.cpu().numpy()
        ok = s1["crc_ok"].cpu().numpy()
        rows = np.concatenate([np.nonzero(ok == 0)[0][:10], np.nonzero(ok)[0][:3]])
        ref = oracle.decode_batch(wl.r, wl.m, wl.crc_len, wl.crc_poly, L, T, oracle.INT,
                                  qq[rows].astype(np.float64), threads=8)
        assert np.array_equal(np.unpackbits(o["cw"][rows], axis=-1, bitorder="little"), ref["c"])
        assert np.array_equal(o["moves"][rows], ref["logs"])
        assert np.array_equal(o["metric"][rows], ref["metric"].astype(np.int32))


def test_mixed_full_size_config():
    """262144 frames, RM(2,6) / RM(2,7) / RM(3,7) in equal shares at 2.5 dB."""
    say("case: mixed full size")
    L, T = 8, 8
    wls = [dataclasses.replace(w, ebn0_db=2.5) for w in (synth.RM26, synth.RM27, synth.RM37)]
    Fs = [87382, 87381, 87381]
    segs = prepare(wls, Fs, L, 0)
    outs, stats = run_mixed(segs, L, T)
    say("  stats", stats.tolist())
    rng = np.random.default_rng(5)
    for (wl, code, q, s1, c), o in zip(segs, outs):
        ok = s1["crc_ok"].cpu().numpy()
        fail = np.nonzero(ok == 0)[0]
        rows = np.sort(np.concatenate([rng.choice(fail, min(40, len(fail)), replace=False),
                                       rng.choice(np.nonzero(ok)[0], 20, replace=False)]))
        qq = q.cpu().numpy()[rows].astype(np.float64)
        ref = oracle.decode_batch(wl.r, wl.m, wl.crc_len, wl.crc_poly, L, T, oracle.INT, qq, threads=8)
        assert np.array_equal(np.unpackbits(o["cw"][rows], axis=-1, bitorder="little"), ref["c"])
        assert np.array_equal(o["moves"][rows], ref["logs"])
        assert np.array_equal(o["k"][rows], ref["k"])
        assert np.array_equal(o["metric"][rows], ref["metric"].astype(np.int32))
    # the configuration bench.py --workload mixed times: quantize, stage 1 and
    # one stage-2 call over the three codes recorded as a HIP graph, autotuned
    # per-iteration tiles, no move logs; replayed twice
    say("case: mixed full size, bench configuration (graph, autotuned tiles, no move logs)")
    ys = [torch.from_numpy(synth.generate(wl, 0, 0, F)[2]).to(DEV) for wl, F in zip(wls, Fs)]
    qs = [torch.empty(y.shape, dtype=torch.int8, device=DEV) for y in ys]
    s1s = [{"anchors": torch.empty((F, L, code.N // 8), dtype=torch.uint8, device=DEV),
            "crc_ok": torch.empty(F, dtype=torch.uint8, device=DEV)} for (wl, code, q, s1, c), F in zip(segs, Fs)]
    st = D.Stage2([(seg[1], F) for seg, F in zip(segs, Fs)], L, T, "i8", DEV, want_moves=False)

    def stage1_all(raw=None):
        for (wl, code, q, s1, c), y, qq, ss in zip(segs, ys, qs, s1s):
            kw = {} if raw is None else {"raw_stream": raw}
            D.stage1_quantized(code, L, y, float(wl.llr_scale), wl.crc_len, wl.crc_poly, q=qq, out=ss, **kw)

    stage1_all()
    torch.cuda.synchronize()
    variant, bpc = autotune.tune(st, qs, [x["anchors"] for x in s1s], [x["crc_ok"] for x in s1s], reps=1,
                                 use_cache=False)
    say("  tiles", variant, bpc)

    def record(raw):
        stage1_all(raw)
        st.run(qs, [x["anchors"] for x in s1s], [x["crc_ok"] for x in s1s], variant=variant, blocks_per_cu=bpc,
               raw_stream=raw)

    g = D.Graph(record)
    g.launch()
    g.launch()
    torch.cuda.synchronize()
    assert np.array_equal(st.stats.cpu().numpy(), stats)
    for i, ((wl, code, q, s1, c), o) in enumerate(zip(segs, outs)):
        assert np.array_equal(qs[i].cpu().numpy(), q.cpu().numpy())
        assert np.array_equal(s1s[i]["anchors"].cpu().numpy(), s1["anchors"].cpu().numpy())
        b = {k: v.cpu().numpy() for k, v in st.outs[i].items()}
        assert "moves" not in b
        for k in ("cw", "k", "metric"):
            assert np.array_equal(b[k], o[k]), (i, k)
    del g
