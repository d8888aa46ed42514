"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (whole step recorded as a HIP graph, autotuned search tiles, and
also without move logs, as bench.py runs it), checked
against the oracle on sampled frames (every frame is decoded independently,
so the oracle decodes the sampled rows alone)."""
import dataclasses
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2602_08501_amd import autotune
from paper_2602_08501_amd import decoder as D
from paper_2602_08501_amd import synth

from merge_rule import searched_counts

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run_pipeline(wl, F, L, T, seed, want_moves=True, tiles=None):
    """The step bench.py times: quantizer + stage 1 (one launch) and stage 2
    recorded as one HIP graph with autotuned per-iteration tiles (or the given
    ones), replayed twice.  bench.py itself runs it with want_moves=False (no
    move logs)."""
    pay, c, y = synth.generate(wl, seed, 0, F)
    code = D.Code(wl.r, wl.m, DEV)
    y_d = torch.from_numpy(y).to(DEV)
    q = torch.empty(y.shape, dtype=torch.int8, device=DEV)
    s1 = {"anchors": torch.empty((F, L, code.N // 8), dtype=torch.uint8, device=DEV),
          "crc_ok": torch.empty(F, dtype=torch.uint8, device=DEV)}
    st = D.Stage2([(code, F)], L, T, "i8", DEV, want_moves=want_moves)
    scale = float(wl.llr_scale)
    D.stage1_quantized(code, L, y_d, scale, wl.crc_len, wl.crc_poly, q=q, out=s1)
    torch.cuda.synchronize()
    if tiles is None:
        variant, bpc = autotune.tune(st, [q], [s1["anchors"]], [s1["crc_ok"]], reps=1, use_cache=False)
    else:
        variant, bpc = tiles

    def record(raw):
        D.stage1_quantized(code, L, y_d, scale, wl.crc_len, wl.crc_poly, q=q, out=s1, raw_stream=raw)
        st.run([q], [s1["anchors"]], [s1["crc_ok"]], variant=variant, blocks_per_cu=bpc, raw_stream=raw)

    g = D.Graph(record)
    g.launch()
    g.launch()
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in st.outs[0].items()}
    out["crc_ok"] = s1["crc_ok"].cpu().numpy()
    out["anchors"] = s1["anchors"].cpu().numpy()
    out["q"] = q.cpu().numpy()
    stats = st.stats.cpu().numpy()
    del g
    return c, y, out, stats, (variant, bpc)


def check_sample(wl, L, T, out, rows):
    q = out["q"][rows].astype(np.float64)
    ref = oracle.decode_batch(wl.r, wl.m, wl.crc_len, wl.crc_poly, L, T, oracle.INT, q, threads=8)
    cw = np.unpackbits(out["cw"][rows], axis=-1, bitorder="little")
    anc = np.unpackbits(out["anchors"][rows], axis=-1, bitorder="little")
    assert np.array_equal(out["crc_ok"][rows], ref["crc_ok"])
    assert np.array_equal(anc, ref["anchors"])
    if "moves" in out:
        assert np.array_equal(out["moves"][rows], ref["logs"])
    assert np.array_equal(cw, ref["c"])
    assert np.array_equal(out["k"][rows], ref["k"])
    assert np.array_equal(out["metric"][rows], ref["metric"].astype(np.int32))


def test_rm37_bench_size():
    wl = synth.RM37
    F, L, T = 65536, 8, 8
    say("case: RM(3,7) 65536 frames, graph + autotuned tiles")
    c, y, out, stats, tiles = run_pipeline(wl, F, L, T, 0)
    say("  tiles", tiles, "stats", stats.tolist())
    fail = np.nonzero(out["crc_ok"] == 0)[0]
    assert stats[0] == len(fail) and stats[1] == len(fail) * L and stats[-1] == 0
    # the searched paths per iteration replay from the logged moves (one path
    # per distinct centre of a frame)
    anc = np.unpackbits(out["anchors"][fail], axis=-1, bitorder="little")
    supp = oracle.moves(wl.r, wl.m)[0]
    assert np.array_equal(stats[1:1 + T], searched_counts(anc, out["moves"][fail], supp))
    rng = np.random.default_rng(0)
    rows = np.sort(np.concatenate([rng.choice(fail, 160, replace=False),
                                   rng.choice(np.nonzero(out["crc_ok"])[0], 64, replace=False),
                                   [0, F - 1]]))
    check_sample(wl, L, T, out, rows)
    # exactly what bench.py times: the same graph without move logs
    say("case: RM(3,7) 65536 frames, bench configuration (no move logs)")
    c2, y2, out2, stats2, _ = run_pipeline(wl, F, L, T, 0, want_moves=False, tiles=tiles)
    assert "moves" not in out2
    for k in ("cw", "k", "metric", "crc_ok", "anchors", "q"):
        assert np.array_equal(out2[k], out[k]), k
    assert np.array_equal(stats2, stats)
    check_sample(wl, L, T, out2, rows)


def test_rm38_config_size():
    wl = synth.RM38
    F, L, T = 32768, 16, 12
    say("case: RM(3,8) 32768 frames, graph + autotuned tiles")
    c, y, out, stats, tiles = run_pipeline(wl, F, L, T, 0)
    say("  tiles", tiles, "stats", stats.tolist())
    fail = np.nonzero(out["crc_ok"] == 0)[0]
    assert stats[0] == len(fail) and stats[-1] == 0
    rng = np.random.default_rng(1)
    rows = np.sort(np.concatenate([rng.choice(fail, 6, replace=False),
                                   rng.choice(np.nonzero(out["crc_ok"])[0], 10, replace=False)]))
    check_sample(wl, L, T, out, rows)
    # as bench.py --workload rm38 times it: the same graph without move logs
    say("case: RM(3,8) 32768 frames, bench configuration (no move logs)")
    c2, y2, out2, stats2, _ = run_pipeline(wl, F, L, T, 0, want_moves=False, tiles=tiles)
    for k in ("cw", "k", "metric", "crc_ok", "anchors", "q"):
        assert np.array_equal(out2[k], out[k]), k
    assert np.array_equal(stats2, stats)
