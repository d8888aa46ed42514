"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (whole step recorded as a HIP graph, autotuned search tiles, without
move logs, several batches in flight on their own streams), checked
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


class Batch:
    """The buffers of one batch: int8 LLRs, stage-1 outputs, stage-2 outputs
    and workspace; the input y is shared."""

    def __init__(self, wl, code, y_d, L, T, want_moves):
        F = y_d.shape[0]
        self.wl, self.code, self.y_d, self.L = wl, code, y_d, L
        self.q = torch.empty(y_d.shape, dtype=torch.int8, device=DEV)
        self.s1 = {"anchors": torch.empty((F, L, code.N // 8), dtype=torch.uint8, device=DEV),
                   "crc_ok": torch.empty(F, dtype=torch.uint8, device=DEV)}
        self.st = D.Stage2([(code, F)], L, T, "i8", DEV, want_moves=want_moves)

    def stage1(self, raw=None):
        wl = self.wl
        D.stage1_quantized(self.code, self.L, self.y_d, float(wl.llr_scale), wl.crc_len, wl.crc_poly,
                           q=self.q, out=self.s1, raw_stream=raw)

    def record(self, tiles):
        def rec(raw):
            self.stage1(raw)
            self.st.run([self.q], [self.s1["anchors"]], [self.s1["crc_ok"]], variant=tiles[0],
                        blocks_per_cu=tiles[1], raw_stream=raw)
        return rec

    def result(self):
        out = {k: v.cpu().numpy() for k, v in self.st.outs[0].items()}
        out["crc_ok"] = self.s1["crc_ok"].cpu().numpy()
        out["anchors"] = self.s1["anchors"].cpu().numpy()
        out["q"] = self.q.cpu().numpy()
        return out


def run_pipeline(wl, F, L, T, seed, want_moves=True, tiles=None, in_flight=1, replays=2):
    """The step bench.py times: quantizer + stage 1 (one launch) and stage 2
    recorded as one HIP graph with autotuned per-iteration tiles (or the given
    ones).  With in_flight = B, B such graphs with their own buffers are
    replayed round-robin on B streams (replays per batch), so B batches run at
    once; bench.py times the step that way, with want_moves=False (no move
    logs).  Returns the outputs of every batch."""
    pay, c, y = synth.generate(wl, seed, 0, F)
    code = D.Code(wl.r, wl.m, DEV)
    y_d = torch.from_numpy(y).to(DEV)
    batches = [Batch(wl, code, y_d, L, T, want_moves) for _ in range(in_flight)]
    b0 = batches[0]
    b0.stage1()
    torch.cuda.synchronize()
    if tiles is None:
        tiles = autotune.tune(b0.st, [b0.q], [b0.s1["anchors"]], [b0.s1["crc_ok"]], reps=1, use_cache=False)
    graphs = [D.Graph(b.record(tiles)) for b in batches]
    streams = [torch.cuda.Stream() for _ in batches]
    torch.cuda.synchronize()
    for k in range(replays * in_flight):
        graphs[k % in_flight].launch(streams[k % in_flight])
    torch.cuda.synchronize()
    outs = [b.result() for b in batches]
    stats = [b.st.stats.cpu().numpy() for b in batches]
    del graphs
    if in_flight == 1:
        return c, y, outs[0], stats[0], tuple(tiles)
    return c, y, outs, stats, tuple(tiles)


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


def test_rm37_batches_in_flight():
    """bench.py's timed loop: three batches in flight, each step's graph on its
    own stream, replayed round-robin.  Every batch must hold exactly the
    outputs of one batch decoded alone (and of the oracle on a sample)."""
    wl = synth.RM37
    F, L, T = 65536, 8, 8
    say("case: RM(3,7) 65536 frames, one batch, bench configuration")
    c, y, ref, stats, tiles = run_pipeline(wl, F, L, T, 0, want_moves=False)
    say("case: RM(3,7) 65536 frames, 3 batches in flight, 3 replays each")
    c3, y3, outs, stats3, _ = run_pipeline(wl, F, L, T, 0, want_moves=False, tiles=tiles, in_flight=3, replays=3)
    for b, (out, sb) in enumerate(zip(outs, stats3)):
        for k in ("cw", "k", "metric", "crc_ok", "anchors", "q"):
            assert np.array_equal(out[k], ref[k]), (b, k)
        assert np.array_equal(sb, stats), b
    fail = np.nonzero(ref["crc_ok"] == 0)[0]
    rng = np.random.default_rng(2)
    rows = np.sort(np.concatenate([rng.choice(fail, 48, replace=False), [0, F - 1]]))
    check_sample(wl, L, T, outs[-1], rows)
