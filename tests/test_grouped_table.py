"""The paired-half move layout (mpwsd_group_moves) against the oracle's move
table: every row, read back through the documented position order, must be
exactly the oracle's move for its recorded index on half 0 and that move's
translate by e_i on half 1; the moves kept apart are exactly those whose
direction space has no normal below N/4, stored as the oracle's rows; every
move appears once; rows are in canonical order within each chunk for both
halves.  Host-only (no GPU)."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2602_08501_amd import _lib

ROWS = 128


def _group(m, moves):
    rc, chunks, extras, nbytes = _lib.mpwsd_group_moves(m, moves.ctypes.data, moves.shape[0], None, 0)
    if rc != 0:
        return rc, None, chunks, extras
    buf = np.zeros(nbytes, np.uint8)
    rc, chunks2, extras2, nbytes2 = _lib.mpwsd_group_moves(m, moves.ctypes.data, moves.shape[0], buf.ctypes.data,
                                                           buf.nbytes)
    assert rc == 0 and (chunks2, extras2, nbytes2) == (chunks, extras, nbytes)
    return rc, buf, chunks, extras


def _al(x):
    return (x + 255) // 256 * 256


def _ins(e, i, v):
    return ((e >> i) << (i + 1)) | (v << i) | (e & ((1 << i) - 1))


def _parity(x):
    return bin(int(x)).count("1") & 1


def _positions(m, u):
    """x of position k of half h: [2][N/2] (the order stated in group.h)."""
    N = 1 << m
    LB, KW = N // 4, N // 2
    ulo, uhi = u & (LB - 1), u // LB
    i = (ulo & -ulo).bit_length() - 1
    pos = np.zeros((2, KW), np.int64)
    for k in range(KW):
        lg, e = divmod(k, KW // 4)
        b = _parity(ulo & _ins(e, i, 0)) ^ _parity(uhi & lg)
        for h in range(2):
            pos[h, k] = lg * LB + _ins(e, i, b ^ h)
    return pos, i


def _check(r, m):
    N = 1 << m
    supp, _ = oracle.moves(r, m)
    table = oracle.pack_supports(m, supp)
    P = table.shape[0]
    rc, buf, chunks, E = _group(m, table)
    assert rc == 0, _lib.last_error()
    hdr = np.frombuffer(buf[:48].tobytes(), dtype=np.dtype([("magic", "<u4"), ("version", "<i4"), ("m", "<i4"),
                                                             ("N", "<i4"), ("P", "<i8"), ("chunks", "<i8"),
                                                             ("KW", "<i4"), ("res", "<i4"), ("extras", "<i8")]))[0]
    assert hdr["magic"] == 0x4757504D and hdr["version"] == 4 and hdr["m"] == m and hdr["N"] == N
    assert hdr["P"] == P and hdr["chunks"] == chunks and hdr["KW"] == N // 2 and hdr["extras"] == E
    KW = N // 2
    u_off = 256
    rows_off = u_off + ((4 * chunks + 255) // 256) * 256
    canon_off = rows_off + chunks * ROWS * KW
    u = np.frombuffer(buf[u_off:u_off + 4 * chunks].tobytes(), np.int32)
    raw = buf[rows_off:canon_off].reshape(chunks, ROWS, KW)
    assert np.isin(raw, [0, 0x80]).all()
    # undo the 16-byte segment swizzle: segment s of row r sits at s ^ swz(r)
    nseg = KW // 16
    swz = (np.arange(ROWS) // (256 // KW)) % nseg
    seg = np.arange(nseg)[None, :] ^ swz[:, None]                       # [row][s] -> stored segment
    idx = (16 * seg[:, :, None] + np.arange(16)[None, None, :]).reshape(ROWS, KW)
    bits = (np.take_along_axis(raw, np.broadcast_to(idx, raw.shape), axis=2) == 0x80).astype(np.uint8)
    sel_off = canon_off + chunks * 2 * ROWS * 4
    canon = np.frombuffer(buf[canon_off:sel_off].tobytes(), np.int32).reshape(chunks, 2, ROWS)
    LB = N // 4
    xrows_off = sel_off + _al(LB * LB * 4)
    xcanon_off = xrows_off + _al(E * N // 8)
    assert buf.nbytes == xcanon_off + _al(E * 4)
    seltab = np.frombuffer(buf[sel_off:sel_off + LB * LB * 4].tobytes(), np.uint32).reshape(LB, LB)
    xrows = buf[xrows_off:xrows_off + E * N // 8].reshape(E, N // 8)
    xcanon = np.frombuffer(buf[xcanon_off:xcanon_off + 4 * E].tobytes(), np.int32)
    # the moves kept apart: the oracle's rows, ascending index, and exactly the
    # moves for which no normal 0 < u < N/4 keeps u.x constant on the support
    assert np.array_equal(xrows, table[xcanon]) and (np.diff(xcanon) > 0).all()
    dense_all = np.unpackbits(table, axis=-1, bitorder="little").astype(bool)
    xs = np.arange(N)
    us = list(range(1, LB))
    par = np.array([[_parity(un & x) for x in xs] for un in us], bool)   # [u][x]
    kept = set(xcanon.tolist())
    for p in range(P):
        sup = dense_all[p]
        has_normal = bool((par[:, sup].all(1) | (~par[:, sup]).all(1)).any())
        assert has_normal == (p not in kept), p
    assert ((u > 0) & (u < LB)).all()   # normals inside the lane groups
    real = canon[:, 0, :] < P
    assert np.array_equal(real, canon[:, 1, :] < P)
    assert (canon[:, 0, :][~real] == P).all() and (canon[:, 1, :][~real] == P).all() and not bits[~real].any()
    # every move exactly once, over both halves and the moves kept apart
    seen = np.sort(np.concatenate([canon[:, 0, :][real], canon[:, 1, :][real], xcanon]))
    assert np.array_equal(seen, np.arange(P))
    # canonical order inside each chunk, both halves
    assert (real[:, :-1] >= real[:, 1:]).all()  # padding rows at the end of a chunk
    for h in range(2):
        d = np.diff(canon[:, h, :].astype(np.int64), axis=1)
        assert (d[real[:, 1:]] > 0).all()
    # each row read back through the position order of its normal
    dense = np.unpackbits(table, axis=-1, bitorder="little").astype(bool)
    for un in np.unique(u):
        pos, i = _positions(m, int(un))
        sel = np.nonzero(u == un)[0]
        for h in range(2):
            got = np.zeros((len(sel), ROWS, N), bool)
            b = bits[sel].astype(bool)
            got[:, :, pos[h]] = b
            want = dense[np.minimum(canon[sel, h, :], P - 1)]
            ok = real[sel]
            assert np.array_equal(got[ok], want[ok]), (int(un), h)
        # half 1 is half 0 translated by e_i
        a = canon[sel, 0, :][real[sel]]
        b1 = canon[sel, 1, :][real[sel]]
        assert np.array_equal(dense[b1], dense[a][:, np.arange(N) ^ (1 << i)])
    # the byte selectors of every normal gather exactly the two halves of a
    # lane group's bytes in the stated order, and scatter them back
    rng = np.random.default_rng(m)
    zb = rng.integers(0, 256, LB).astype(np.uint64)
    zd = [int(sum(int(zb[4 * d + j]) << (8 * j) for j in range(4))) for d in range(LB // 4)]
    W = LB // 8
    for un in range(1, LB):
        pos, i = _positions(m, un)
        S = int(seltab[un, 0])
        assert S == max(i - 2, 0)
        halves = []
        for h in range(2):
            out = []
            for k in range(W):
                lo = ((k >> S) << (S + 1)) | (k & ((1 << S) - 1))
                out.append(_perm(zd[lo + (1 << S)], zd[lo], int(seltab[un, 1 + h * W + k])))
            halves.append(out)
            got = [(out[e // 4] >> (8 * (e % 4))) & 0xFF for e in range(LB // 2)]
            # lane group 0: positions k < N/8 of half h are x = ins(e, i, b ^ h)
            assert got == [int(zb[pos[h, e]]) for e in range(LB // 2)], (un, h)
        back = [0] * (LB // 4)
        for k in range(W):
            lo = ((k >> S) << (S + 1)) | (k & ((1 << S) - 1))
            for d in (lo, lo + (1 << S)):
                back[d] = _perm(halves[1][k], halves[0][k], int(seltab[un, 1 + 2 * W + d]))
        assert back == zd, un
    return chunks, P, E


def _perm(a, b, s):
    """v_perm_b32: byte j of the result is byte (s >> 8j) & 0xFF of a:b (b low)."""
    comb = (a << 32) | b
    out = 0
    for j in range(4):
        q = (s >> (8 * j)) & 0xFF
        assert q < 8
        out |= ((comb >> (8 * q)) & 0xFF) << (8 * j)
    return out


def test_rm37_layout():
    chunks, P, E = _check(3, 7)
    assert E == 0 and chunks * ROWS <= 1.02 * P / 2      # at most 2% padding


def test_rm27_layout_keeps_codimension_2_apart():
    chunks, P, E = _check(2, 7)
    assert P == 10668 and E == 4096 and chunks * ROWS <= 1.25 * (P - E) / 2


def test_rm17_layout():
    chunks, P, E = _check(1, 7)
    assert 0 < E < P


@pytest.mark.slow
def test_rm38_layout():
    chunks, P, E = _check(3, 8)
    assert E == 0 and chunks * ROWS <= 1.02 * P / 2


def test_tables_without_layout_and_errors():
    supp, _ = oracle.moves(2, 6)
    t = oracle.pack_supports(6, supp)
    assert _lib.mpwsd_group_moves(6, t.ctypes.data, t.shape[0], None, 0)[0] == _lib.MPWSD_ERR_UNSUPPORTED
    supp, _ = oracle.moves(3, 7)
    t = oracle.pack_supports(7, supp)
    rc, chunks, extras, nbytes = _lib.mpwsd_group_moves(7, t.ctypes.data, t.shape[0], None, 0)
    assert rc == 0 and nbytes > 0 and extras == 0
    small = np.zeros(nbytes - 1, np.uint8)
    rc, c2, e2, n2 = _lib.mpwsd_group_moves(7, t.ctypes.data, t.shape[0], small.ctypes.data, small.nbytes)
    assert rc == _lib.MPWSD_ERR_SIZE and (c2, e2, n2) == (chunks, extras, nbytes)
    # a table whose moves lack their translates
    rc, *_ = _lib.mpwsd_group_moves(7, t.ctypes.data, 1000, None, 0)
    assert rc == _lib.MPWSD_ERR_UNSUPPORTED
    assert _lib.mpwsd_group_moves(7, None, 10, None, 0)[0] == _lib.MPWSD_ERR_ARG
