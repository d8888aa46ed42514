"""Serving with continuous batching: every frame's result is the same alone
and in the mix (bit-exact), equals the batch decoder's result for that frame,
and (on a sample) the oracle's."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2602_08501_amd import decoder as D
from paper_2602_08501_amd import serve, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
ROWS = 384


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def setup():
    codes = [D.Code(wl.r, wl.m, DEV) for wl, L, T in serve.MIX]
    pools, scales, truth = serve.build_pools(ROWS, lo=1.5, hi=2.5)
    return codes, pools, scales, truth


def batch_reference(codes, pools, scales):
    """mpwsd_decode_batch on each code's whole pool."""
    refs = []
    for ci, (wl, L, T) in enumerate(serve.MIX):
        y = torch.from_numpy(pools[ci]).to(DEV)
        sc = torch.from_numpy(scales[ci]).to(DEV)
        q = torch.empty(y.shape, dtype=torch.int8, device=DEV)
        for f in range(ROWS):  # per-frame scales
            D.quantize(y[f], float(scales[ci][f]), out=q[f])
        s1 = D.stage1(codes[ci], L, q, wl.crc_len, wl.crc_poly)
        st = D.Stage2([(codes[ci], ROWS)], L, T, "i8", DEV)
        o = st.run([q], [s1["anchors"]], [s1["crc_ok"]])[0]
        torch.cuda.synchronize()
        refs.append({"cw": o["cw"].cpu().numpy(), "k": o["k"].cpu().numpy(), "metric": o["metric"].cpu().numpy(),
                     "stage": 2 - s1["crc_ok"].cpu().numpy().astype(np.int32), "q": q.cpu().numpy()})
    return refs


def test_alone_vs_mix_vs_batch(setup):
    codes, pools, scales, truth = setup
    specs = [dict(L=L, T=T, capacity=256) for wl, L, T in serve.MIX]
    refs = batch_reference(codes, pools, scales)
    # the mix: every frame of every pool, Poisson arrivals, capacity 256 per code
    rng = np.random.default_rng(3)
    code = np.repeat(np.arange(3, dtype=np.int32), ROWS)
    row = np.tile(np.arange(ROWS, dtype=np.int64), 3)
    perm = rng.permutation(len(code))
    code, row = code[perm], row[perm]
    arrival = np.cumsum(rng.exponential(1.0 / 2e5, len(code)))
    scale = np.array([scales[c][r] for c, r in zip(code, row)], np.float32)
    say("case: serving mix of", len(code), "frames")
    srv = serve.Server(codes, specs)
    mix = serve.results_table(srv.serve_trace(code, row, scale, arrival, pools))
    srv.close()
    assert (mix["tag"] == np.arange(len(code))).all()
    N = [1 << wl.m for wl, L, T in serve.MIX]
    for i, (c, r) in enumerate(zip(code, row)):
        ref = refs[c]
        nb = N[c] // 8
        assert mix["stage"][i] == ref["stage"][r], (c, r)
        assert np.array_equal(mix["cw"][i][:nb], ref["cw"][r]), (c, r)
        assert mix["k"][i] == ref["k"][r] and mix["metric"][i] == ref["metric"][r], (c, r)
    say("  stage-2 frames in the mix:", int((mix["stage"] == 2).sum()))
    # alone: a fresh server per frame for a sample including stage-2 frames
    pick = []
    for c in range(3):
        s2 = np.nonzero(refs[c]["stage"] == 2)[0][:6]
        s1 = np.nonzero(refs[c]["stage"] == 1)[0][:2]
        pick += [(c, int(r)) for r in np.concatenate([s2, s1])]
    for c, r in pick:
        srv = serve.Server(codes, specs)
        srv.submit(c, pools[c][r:r + 1], scales[c][r:r + 1], np.array([7], np.uint64))
        res = serve.results_table((serve.Result * 1)(*srv.drain()))
        srv.close()
        i = int(np.nonzero((code == c) & (row == r))[0][0])
        assert res["tag"][0] == 7
        for key in ("stage", "k", "metric"):
            assert res[key][0] == mix[key][i], (c, r, key)
        assert np.array_equal(res["cw"][0], mix["cw"][i]), (c, r)  # bytes past N/8 are zero in both
    # oracle on a few stage-2 frames of RM(3,7)
    wl, L, T = serve.MIX[1]
    rows = np.nonzero(refs[1]["stage"] == 2)[0][:8]
    ref = oracle.decode_batch(wl.r, wl.m, wl.crc_len, wl.crc_poly, L, T, oracle.INT,
                              refs[1]["q"][rows].astype(np.float64), threads=8)
    assert np.array_equal(np.unpackbits(refs[1]["cw"][rows], axis=-1, bitorder="little"), ref["c"])
    assert np.array_equal(refs[1]["metric"][rows], ref["metric"].astype(np.int32))


def test_memory_gate_small_capacity(setup):
    """More frames than slots: admission waits for slots and still completes."""
    codes, pools, scales, truth = setup
    specs = [dict(L=L, T=T, capacity=8) for wl, L, T in serve.MIX]
    srv = serve.Server(codes, specs)
    n = 120
    code = np.arange(n, dtype=np.int32) % 3
    row = np.arange(n, dtype=np.int64) % ROWS
    scale = np.array([scales[c][r] for c, r in zip(code, row)], np.float32)
    res = serve.results_table(srv.serve_trace(code, row, scale, np.zeros(n), pools))
    srv.close()
    assert (res["tag"] == np.arange(n)).all()
    assert set(np.unique(res["stage"])) <= {1, 2}


def test_trace_rejects_bad_arrivals(setup):
    """A trace whose arrival times cannot all come (NaN, negative) is refused
    before anything runs; the server stays usable."""
    say("case: serving trace with bad arrivals")
    codes, pools, scales, truth = setup
    specs = [dict(L=L, T=T, capacity=64) for wl, L, T in serve.MIX]
    srv = serve.Server(codes, specs)
    n = 9
    code = np.arange(n, dtype=np.int32) % 3
    row = np.arange(n, dtype=np.int64)
    scale = np.array([scales[c][r] for c, r in zip(code, row)], np.float32)
    for bad in (np.nan, -1.0):
        arr = np.zeros(n)
        arr[4] = bad
        with pytest.raises(Exception, match="bad trace entry 4"):
            srv.serve_trace(code, row, scale, arr, pools)
    res = serve.results_table(srv.serve_trace(code, row, scale, np.zeros(n), pools))
    srv.close()
    assert (res["tag"] == np.arange(n)).all()


def test_submit_from_other_threads(setup):
    """Two threads submit frames while this thread ticks and polls (the
    header lets submission run on other threads): every frame comes back
    once, and equal to mpwsd_decode_batch's result for it."""
    import threading
    import time
    say("case: serving with two submitting threads")
    codes, pools, scales, truth = setup
    refs = batch_reference(codes, pools, scales)
    specs = [dict(L=L, T=T, capacity=64) for wl, L, T in serve.MIX]
    srv = serve.Server(codes, specs)
    jobs = [[(c, r) for c in range(3) for r in range(ROWS) if (c + r) % 2 == t] for t in range(2)]

    def producer(t):
        for c, r in jobs[t]:
            srv.submit(c, pools[c][r:r + 1], scales[c][r:r + 1], np.array([c * ROWS + r], np.uint64))

    threads = [threading.Thread(target=producer, args=(t,)) for t in range(2)]
    for th in threads:
        th.start()
    got = []
    deadline = time.time() + 120
    while len(got) < 3 * ROWS and time.time() < deadline:
        srv.tick()
        got += srv.poll()
    for th in threads:
        th.join()
    srv.close()
    res = serve.results_table((serve.Result * len(got))(*got))
    assert np.array_equal(np.sort(res["tag"]), np.arange(3 * ROWS))
    N = [1 << wl.m for wl, L, T in serve.MIX]
    for i in range(len(res)):
        c, r = divmod(int(res["tag"][i]), ROWS)
        ref = refs[c]
        assert res["stage"][i] == ref["stage"][r] and res["k"][i] == ref["k"][r], (c, r)
        assert res["metric"][i] == ref["metric"][r], (c, r)
        assert np.array_equal(res["cw"][i][:N[c] // 8], ref["cw"][r]), (c, r)
