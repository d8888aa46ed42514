"""The premise of merging equal centres in stage 2 (Sec. III-B, Alg. 1),
checked on the oracle, which searches every path of every frame: two paths
of one frame at the same centre after an iteration make the same moves from
then on, and a path that reaches the centre of a path that stopped makes no
further move.  The GPU decoder searches one path per distinct centre and
copies the leader's moves to its followers; these pins show that this gives
the logs of searching every path."""
import dataclasses

import numpy as np

import oracle
from paper_2602_08501_amd import synth

from merge_rule import replay, searched_counts


def _failing(wl, L, T, F, seed):
    pay, c, y = synth.generate(wl, seed, 0, F)
    q = oracle.quantize(y, wl.llr_scale).astype(np.float64)
    ref = oracle.decode_batch(wl.r, wl.m, wl.crc_len, wl.crc_poly, L, T, oracle.INT, q, threads=8)
    fail = ref["crc_ok"] == 0
    return ref["anchors"][fail], ref["logs"][fail]


def _check(wl, L, T, F, seed):
    anchors, logs = _failing(wl, L, T, F, seed)
    supp, _ = oracle.moves(wl.r, wl.m)
    kinds = {"stop": 0, "follow": 0}
    for f in range(logs.shape[0]):
        searched, events = replay(anchors[f], logs[f], supp)
        for t1, k, kind, lead in events:
            kinds[kind] += 1
            if kind == "stop":
                assert (logs[f, k, t1:] < 0).all(), (f, k, t1)
            else:
                assert lead < k
                assert np.array_equal(logs[f, k, t1:], logs[f, lead, t1:]), (f, k, t1, lead)
    merged = searched_counts(anchors, logs, supp)
    raw = np.array([logs.shape[0] * L] + [int((logs[:, :, t - 1] >= 0).sum()) for t in range(1, T)])
    assert merged[0] == raw[0] and (merged <= raw).all()
    return kinds, merged, raw


def test_equal_centres_share_their_future_rm26():
    wl = dataclasses.replace(synth.RM26, ebn0_db=1.0)
    kinds, merged, raw = _check(wl, 8, 6, 600, 5)
    assert kinds["follow"] > 0 and kinds["stop"] > 0, kinds
    assert merged.sum() < raw.sum()


def test_equal_centres_share_their_future_rm37():
    wl = dataclasses.replace(synth.RM37, ebn0_db=2.0)
    kinds, merged, raw = _check(wl, 8, 8, 400, 6)
    assert kinds["follow"] > 0, kinds
    assert merged.sum() < raw.sum()


def test_replay_on_a_hand_made_frame():
    # n = 8 positions, moves = single positions {0}, {1}, {2}, {3}
    supp = np.array([[0], [1], [2], [3]], np.uint16)
    anchors = np.zeros((4, 8), np.uint8)
    anchors[1, 0] = 1                  # path 1 starts at {0}
    anchors[2, 1] = 1                  # path 2 starts at {1}
    anchors[3, 0] = anchors[3, 1] = 1  # path 3 starts at {0, 1}
    logs = np.full((4, 3), -1, np.int32)
    logs[0, 0] = 0                     # path 0: {} -> {0}, then stops
    logs[1, 0] = 1                     # path 1: {0} -> {0, 1} -> {0, 1, 2}
    logs[1, 1] = 2
    logs[2, 0] = 0                     # path 2: {1} -> {0, 1}: follows path 1
    logs[2, 1] = 2
    # path 3 stays at {0, 1} in iteration 0 (did not move), so paths 1 and 2
    # moved onto a stopped centre: both stop
    searched, events = replay(anchors, logs, supp)
    assert searched.tolist() == [4, 1, 0]
    assert (1, 1, "stop", -1) in events and (1, 2, "stop", -1) in events
    assert (1, 0, "stop", -1) not in events
    # without path 3, path 2 follows path 1
    logs3 = logs[:3]
    searched, events = replay(anchors[:3], logs3, supp)
    assert searched.tolist() == [3, 2, 1]
    assert events == [(1, 2, "follow", 1)]
