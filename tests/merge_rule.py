"""Searched-path counts of stage 2 when paths of one frame that reach the
same centre are merged, replayed from a decoder's anchors and move logs.

What a path does in an iteration (the move it picks, or stopping) depends on
its centre alone, so the decoder searches a centre once per frame and
iteration.  After iteration t:
  * a path that moved onto the centre of a path that did not move (and is
    not a follower) stops: it would find no improving move there;
  * a path that moved onto the centre of a moved path of smaller index
    follows that path (the leader) and is not searched again;
  * every other path that moved is searched in iteration t + 1.
This module holds no arithmetic of the method: it only replays logged moves.
"""
import numpy as np


def _apply(c, row):
    c[row[row < c.shape[0]]] ^= 1


def replay(anchors, logs, supp):
    """One frame.  anchors: [L][n] 0/1, logs: [L][T] move index or -1,
    supp: [P][w] move supports (padded with values >= n).

    Returns (searched[T], events): events lists (t + 1, k, kind, leader)
    for every path k merged after iteration t, kind "stop" or "follow"."""
    L, T = logs.shape
    cen = np.array(anchors, dtype=np.uint8, copy=True)
    follower = np.zeros(L, bool)
    active = list(range(L))
    searched = np.zeros(T, np.int64)
    events = []
    for t in range(T):
        searched[t] = len(active)
        moved = []
        for k in active:
            p = logs[k, t]
            if p >= 0:
                _apply(cen[k], supp[p])
                moved.append(k)
        if t + 1 == T:
            break
        mset = set(moved)
        still = [j for j in range(L) if not follower[j] and j not in mset]
        nxt = []
        for k in moved:
            if any(np.array_equal(cen[j], cen[k]) for j in still):
                events.append((t + 1, k, "stop", -1))
                continue
            leads = [j for j in moved if j < k and np.array_equal(cen[j], cen[k])]
            if leads:
                follower[k] = True
                events.append((t + 1, k, "follow", leads[0]))
                continue
            nxt.append(k)
        active = nxt
    return searched, events


def searched_counts(anchors, logs, supp):
    """anchors [F][L][n], logs [F][L][T] of the frames sent to stage 2:
    the searched paths per iteration, summed over the frames."""
    tot = np.zeros(logs.shape[2], np.int64)
    for f in range(logs.shape[0]):
        tot += replay(anchors[f], logs[f], supp)[0]
    return tot
