"""The C-ABI library on the CPU: it loads, exports every declared call, its
host-side move table is byte-identical to the oracle's, and argument errors
are reported before anything is enqueued (none of these touch a GPU)."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2602_08501_amd import _lib
from paper_2602_08501_amd._lib import Segment


def test_library_exports_every_declared_call():
    lib = _lib.load()
    names = _lib.header_functions()
    assert set(names) == {"mpwsd_last_error", "mpwsd_build_moves", "mpwsd_build_sphere", "mpwsd_group_moves",
                          "mpwsd_quantize_llr",
                          "mpwsd_stage1_osd",
                          "mpwsd_stage1_scl", "mpwsd_stage1_scl_quantized", "mpwsd_workspace_bytes",
                          "mpwsd_decode_batch",
                          "mpwsd_decode_batch_noalloc",
                          "mpwsd_decode_batch_ex", "mpwsd_search_variants", "mpwsd_graph_begin",
                          "mpwsd_graph_end", "mpwsd_graph_launch", "mpwsd_graph_destroy",
                          "mpwsd_server_arena_bytes", "mpwsd_server_create", "mpwsd_server_submit",
                          "mpwsd_server_tick", "mpwsd_server_poll", "mpwsd_server_destroy", "mpwsd_serve_trace"}
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.parametrize("r,m", [(1, 5), (2, 6), (1, 7), (2, 7), (3, 7), (4, 7), (1, 6)])
def test_move_table_matches_oracle(r, m):
    rc, P, N, w = _lib.mpwsd_build_moves(r, m, None, 0)
    assert rc == 0 and N == 1 << m and w == 1 << (m - r)
    buf = np.zeros((P, N // 8), np.uint8)
    rc, *_ = _lib.mpwsd_build_moves(r, m, buf.ctypes.data, buf.nbytes)
    assert rc == 0
    supp, w2 = oracle.moves(r, m)
    assert np.array_equal(buf, oracle.pack_supports(m, supp))


@pytest.mark.slow
def test_move_table_matches_oracle_rm38():
    rc, P, N, w = _lib.mpwsd_build_moves(3, 8, None, 0)
    assert P == 777240
    buf = np.zeros((P, N // 8), np.uint8)
    assert _lib.mpwsd_build_moves(3, 8, buf.ctypes.data, buf.nbytes)[0] == 0
    supp, _ = oracle.moves(3, 8)
    assert np.array_equal(buf, oracle.pack_supports(8, supp))


def test_build_moves_errors():
    rc, *_ = _lib.mpwsd_build_moves(0, 6, None, 0)
    assert rc == _lib.MPWSD_ERR_UNSUPPORTED and "r" in _lib.last_error()
    rc, *_ = _lib.mpwsd_build_moves(6, 6, None, 0)
    assert rc == _lib.MPWSD_ERR_UNSUPPORTED
    buf = np.zeros(10, np.uint8)
    rc, P, N, w = _lib.mpwsd_build_moves(2, 6, buf.ctypes.data, buf.nbytes)
    assert rc == _lib.MPWSD_ERR_SIZE and P == 2604
    assert "need" in _lib.last_error()


@pytest.mark.parametrize("r,m,radius", [(2, 6, 2), (2, 5, 2), (2, 5, 3), (1, 5, 2), (1, 6, 1), (2, 6, 1)])
def test_sphere_table_matches_oracle(r, m, radius):
    rc, P, N, wmax = _lib.mpwsd_build_sphere(r, m, radius, None, 0)
    assert rc == 0, _lib.last_error()
    supp, stride = oracle.sphere(r, m, radius)
    assert (P, N, wmax) == (len(supp), 1 << m, stride)
    buf = np.zeros((P, N // 8), np.uint8)
    rc, *_ = _lib.mpwsd_build_sphere(r, m, radius, buf.ctypes.data, buf.nbytes)
    assert rc == 0
    assert np.array_equal(buf, oracle.pack_supports(m, supp))


def test_build_sphere_errors():
    rc, *_ = _lib.mpwsd_build_sphere(3, 7, 2, None, 0)      # K = 64: no exhaustive walk
    assert rc == _lib.MPWSD_ERR_UNSUPPORTED and "K" in _lib.last_error()
    rc, *_ = _lib.mpwsd_build_sphere(1, 4, 3, None, 0)      # RM(1,4): weights 8 and 16 only
    assert rc == _lib.MPWSD_ERR_ARG
    rc, *_ = _lib.mpwsd_build_sphere(2, 6, 0, None, 0)
    assert rc == _lib.MPWSD_ERR_UNSUPPORTED
    rc, P, *_ = _lib.mpwsd_build_sphere(2, 6, 2, np.zeros(8, np.uint8).ctypes.data, 8)
    assert rc == _lib.MPWSD_ERR_SIZE and P == 294252


def _seg(**kw):
    d = dict(r=3, m=7, moves=0x1000, P=94488, llr=0x2000, dtype=0, F=16, anchors=0x3000,
             crc_ok=None, out_cw=0x4000, out_k=None, out_metric=None, out_moves=None)
    d.update(kw)
    return Segment(**d)


def test_decode_batch_validates_before_enqueue():
    ok = _lib.mpwsd_workspace_bytes([_seg()], 8, 8)
    assert ok > 0
    cases = [
        ([_seg(P=8128)], 8, 8, _lib.MPWSD_ERR_ARG),          # not the RM(3,7) move count
        ([_seg(m=9, r=3)], 8, 8, _lib.MPWSD_ERR_UNSUPPORTED),
        ([_seg()], 0, 8, _lib.MPWSD_ERR_UNSUPPORTED),
        ([_seg()], 33, 8, _lib.MPWSD_ERR_UNSUPPORTED),
        ([_seg()], 8, 0, _lib.MPWSD_ERR_UNSUPPORTED),
        ([_seg()], 8, 65, _lib.MPWSD_ERR_UNSUPPORTED),
        ([_seg(dtype=7)], 8, 8, _lib.MPWSD_ERR_ARG),
        ([_seg(), _seg(dtype=1)], 8, 8, _lib.MPWSD_ERR_ARG),
        ([_seg(F=-1)], 8, 8, _lib.MPWSD_ERR_ARG),
        ([_seg(llr=None)], 8, 8, _lib.MPWSD_ERR_ARG),
        ([_seg(moves=0x1001)], 8, 8, _lib.MPWSD_ERR_ARG),
        ([_seg(r=2, m=6, P=2604 + 291647)], 8, 8, _lib.MPWSD_ERR_ARG),   # not a sphere size of RM(2,6)
        # paired-half layouts: only for m >= 7, with a chunk count that fits P, 256-byte aligned
        ([_seg(r=2, m=6, P=2604, grouped=0x100000, grouped_chunks=11)], 8, 8, _lib.MPWSD_ERR_ARG),
        ([_seg(grouped=0x100000, grouped_chunks=368)], 8, 8, _lib.MPWSD_ERR_ARG),
        ([_seg(grouped=0x100000, grouped_chunks=370 + 128 + 1)], 8, 8, _lib.MPWSD_ERR_ARG),
        ([_seg(grouped=0x100080, grouped_chunks=373)], 8, 8, _lib.MPWSD_ERR_ARG),
        # moves kept apart: a count in [0, P], and the chunks must hold the rest
        ([_seg(grouped=0x100000, grouped_chunks=373, grouped_extras=-1)], 8, 8, _lib.MPWSD_ERR_ARG),
        ([_seg(grouped=0x100000, grouped_chunks=373, grouped_extras=94489)], 8, 8, _lib.MPWSD_ERR_ARG),
        ([_seg(r=2, m=7, P=10668, grouped=0x100000, grouped_chunks=25, grouped_extras=4096)], 8, 8,
         _lib.MPWSD_ERR_ARG),
    ]
    for segs, L, T, code in cases:
        if segs[-1].llr and segs[-1].moves % 4 == 0:  # size query ignores pointers
            assert _lib.mpwsd_workspace_bytes(segs, L, T) == 0
        assert _lib.mpwsd_decode_batch(segs, L, T, 0x10000, 1 << 40, None, None) == code, _lib.last_error()
    # every sphere size of RM(2,6) is accepted: S_1, S_2 and S_3 without the zero word
    for P in (2604, 2604 + 291648, 2604 + 291648 + 888832):
        assert _lib.mpwsd_workspace_bytes([_seg(r=2, m=6, P=P)], 8, 8) > 0, _lib.last_error()
    assert _lib.mpwsd_workspace_bytes([_seg(grouped=0x100000, grouped_chunks=373)], 8, 8) == ok
    assert _lib.mpwsd_workspace_bytes([_seg(r=2, m=7, P=10668, grouped=0x100000, grouped_chunks=26,
                                            grouped_extras=4096)], 8, 8) > 0, _lib.last_error()
    # workspace too small / missing / misaligned
    assert _lib.mpwsd_decode_batch([_seg()], 8, 8, 0x10000, ok - 1, None, None) == _lib.MPWSD_ERR_SIZE
    assert _lib.mpwsd_decode_batch([_seg()], 8, 8, None, ok, None, None) == _lib.MPWSD_ERR_SIZE
    assert _lib.mpwsd_decode_batch([_seg()], 8, 8, 0x10010, ok, None, None) == _lib.MPWSD_ERR_ARG
    # pointer alignment (int8 q: 16 bytes, float y: 4, anchors and decisions: 4); the size query
    # does not look at pointers
    for seg in (_seg(llr=0x2008), _seg(llr=0x2002, dtype=1), _seg(anchors=0x3002), _seg(out_cw=0x4002)):
        assert _lib.mpwsd_workspace_bytes([seg], 8, 8) > 0
        assert _lib.mpwsd_decode_batch([seg], 8, 8, 0x10000, 1 << 40, None, None) == _lib.MPWSD_ERR_ARG
        assert "aligned" in _lib.last_error()
    for seg in (_seg(llr=0x2010), _seg(llr=0x2004, dtype=1)):
        assert _lib.mpwsd_workspace_bytes([seg], 8, 8) > 0


def test_stage1_validates_before_enqueue():
    A = 0x1000
    cases = [
        (dict(r=3, m=9), _lib.MPWSD_ERR_UNSUPPORTED),
        (dict(L=6), _lib.MPWSD_ERR_UNSUPPORTED),
        (dict(L=64), _lib.MPWSD_ERR_UNSUPPORTED),
        (dict(r=1, m=5, L=128), _lib.MPWSD_ERR_UNSUPPORTED),
        (dict(crc_len=17), _lib.MPWSD_ERR_UNSUPPORTED),
        (dict(crc_poly=0x03), _lib.MPWSD_ERR_ARG),
        (dict(dtype=5), _lib.MPWSD_ERR_ARG),
        (dict(F=-2), _lib.MPWSD_ERR_ARG),
        (dict(anchors=None), _lib.MPWSD_ERR_ARG),
        (dict(anchors=A + 2), _lib.MPWSD_ERR_ARG),
    ]
    for kw, code in cases:
        a = dict(r=3, m=7, crc_len=6, crc_poly=0x43, L=8, llr=A, dtype=0, F=4, anchors=A, crc_ok=A, pm=None,
                 stream=None)
        a.update(kw)
        rc = _lib.mpwsd_stage1_scl(a["r"], a["m"], a["crc_len"], a["crc_poly"], a["L"], a["llr"], a["dtype"],
                                   a["F"], a["anchors"], a["crc_ok"], a["pm"], a["stream"])
        assert rc == code, (kw, _lib.last_error())
        assert _lib.last_error()
    # nothing to do is not an error
    assert _lib.mpwsd_stage1_scl(3, 7, 6, 0x43, 8, None, 0, 0, None, None, None, None) == 0
    assert _lib.mpwsd_quantize_llr(None, 0, 1.0, None, None, None) == 0
    assert _lib.mpwsd_quantize_llr(None, 5, 1.0, None, None, None) == _lib.MPWSD_ERR_ARG
    assert _lib.mpwsd_quantize_llr(A, 5, float("inf"), A, None, None) == _lib.MPWSD_ERR_ARG


def test_stage1_quantized_validates_before_enqueue():
    A = 0x1000
    cases = [
        (dict(r=3, m=9), _lib.MPWSD_ERR_UNSUPPORTED),
        (dict(L=6), _lib.MPWSD_ERR_UNSUPPORTED),
        (dict(crc_len=17), _lib.MPWSD_ERR_UNSUPPORTED),
        (dict(crc_poly=0x03), _lib.MPWSD_ERR_ARG),
        (dict(scale=float("nan")), _lib.MPWSD_ERR_ARG),
        (dict(F=-2), _lib.MPWSD_ERR_ARG),
        (dict(y=None), _lib.MPWSD_ERR_ARG),
        (dict(q=None), _lib.MPWSD_ERR_ARG),
        (dict(anchors=None), _lib.MPWSD_ERR_ARG),
        (dict(anchors=A + 2), _lib.MPWSD_ERR_ARG),
    ]
    for kw, code in cases:
        a = dict(r=3, m=7, crc_len=6, crc_poly=0x43, L=8, y=A, scale=12.9, F=4, q=A, bad=None, anchors=A, crc_ok=A,
                 pm=None, stream=None)
        a.update(kw)
        rc = _lib.mpwsd_stage1_scl_quantized(a["r"], a["m"], a["crc_len"], a["crc_poly"], a["L"], a["y"],
                                             a["scale"], a["F"], a["q"], a["bad"], a["anchors"], a["crc_ok"],
                                             a["pm"], a["stream"])
        assert rc == code, (kw, _lib.last_error())
        assert "quantized" in _lib.last_error()
    assert _lib.mpwsd_stage1_scl_quantized(3, 7, 6, 0x43, 8, None, 1.0, 0, None, None, None, None, None,
                                           None) == 0


def test_search_variants_and_option_errors():
    vs = _lib.mpwsd_search_variants()
    assert len(vs) >= 2
    for v in vs:
        assert v["columns"] == 16 * v["col_blocks"] * v["waves"]
    ok = _lib.mpwsd_workspace_bytes([_seg()], 8, 8)
    assert _lib.mpwsd_decode_batch_ex([_seg()], 8, 8, 0x10000, ok, None, variant=len(vs)) == _lib.MPWSD_ERR_ARG
    assert _lib.mpwsd_decode_batch_ex([_seg()], 8, 8, 0x10000, ok, None, variant=-2) == _lib.MPWSD_ERR_ARG
    assert _lib.mpwsd_decode_batch_ex([_seg()], 8, 8, 0x10000, ok, None, blocks_per_cu=-1) == _lib.MPWSD_ERR_ARG
    # per-iteration tiles: every entry is checked
    assert _lib.mpwsd_decode_batch_ex([_seg()], 8, 8, 0x10000, ok, None,
                                      variant=[0, 1, 2, 0, 1, 2, 0, len(vs)]) == _lib.MPWSD_ERR_ARG
    assert "iteration 7" in _lib.last_error()
    assert _lib.mpwsd_decode_batch_ex([_seg()], 8, 8, 0x10000, ok, None,
                                      blocks_per_cu=[1, 2, 3, 4, 17, 1, 1, 1]) == _lib.MPWSD_ERR_ARG
    assert _lib.load().mpwsd_graph_launch(None, None) == _lib.MPWSD_ERR_ARG
    assert _lib.load().mpwsd_graph_destroy(None) == 0


def test_server_argument_errors():
    from paper_2602_08501_amd._lib import ServerCode
    import ctypes
    lib = _lib.load()
    good = ServerCode(3, 7, 0x1000, 94488, 8, 8, 6, 0x43, 64)
    arr = (ServerCode * 1)(good)
    assert lib.mpwsd_server_arena_bytes(arr, 1) > 0
    kept = (ServerCode * 1)(ServerCode(2, 7, 0x1000, 10668, 8, 8, 6, 0x43, 64, 0x100000, 26, 4096))
    assert lib.mpwsd_server_arena_bytes(kept, 1) > 0, _lib.last_error()
    for bad in (ServerCode(3, 7, 0x1000, 8128, 8, 8, 6, 0x43, 64), ServerCode(3, 9, 0x1000, 94488, 8, 8, 6, 0x43, 64),
                ServerCode(3, 7, 0x1000, 94488, 6, 8, 6, 0x43, 64), ServerCode(3, 7, 0x1000, 94488, 8, 8, 6, 0x43, 0),
                ServerCode(3, 7, None, 94488, 8, 8, 6, 0x43, 64),
                # paired-half layout: kept-apart count out of range, chunks too few for the rest
                ServerCode(3, 7, 0x1000, 94488, 8, 8, 6, 0x43, 64, 0x100000, 373, -1),
                ServerCode(2, 7, 0x1000, 10668, 8, 8, 6, 0x43, 64, 0x100000, 25, 4096)):
        a = (ServerCode * 1)(bad)
        assert lib.mpwsd_server_arena_bytes(a, 1) == 0
        h = ctypes.c_void_p()
        assert lib.mpwsd_server_create(a, 1, 0x10000, 1 << 40, ctypes.byref(h)) < 0
    h = ctypes.c_void_p()
    need = lib.mpwsd_server_arena_bytes(arr, 1)
    assert lib.mpwsd_server_create(arr, 1, 0x10000, need - 1, ctypes.byref(h)) == _lib.MPWSD_ERR_SIZE
    assert lib.mpwsd_server_create(arr, 1, 0x10010, need, ctypes.byref(h)) == _lib.MPWSD_ERR_ARG
    assert lib.mpwsd_server_tick(None, None) == _lib.MPWSD_ERR_ARG
    assert lib.mpwsd_server_destroy(None) == 0


def test_stage1_osd_validates_before_enqueue():
    A = 0x1000
    base = dict(r=2, m=7, order=2, L=8, llr=A, dtype=0, F=4, anchors=A, metric=None)
    cases = [
        (dict(m=9), _lib.MPWSD_ERR_UNSUPPORTED),
        (dict(r=4, m=8), _lib.MPWSD_ERR_UNSUPPORTED),      # K = 163 > 64
        (dict(order=5), _lib.MPWSD_ERR_UNSUPPORTED),
        (dict(order=-1), _lib.MPWSD_ERR_UNSUPPORTED),
        (dict(L=33), _lib.MPWSD_ERR_UNSUPPORTED),
        (dict(L=0), _lib.MPWSD_ERR_UNSUPPORTED),
        (dict(order=0, L=2), _lib.MPWSD_ERR_ARG),          # one candidate only
        (dict(dtype=3), _lib.MPWSD_ERR_ARG),
        (dict(F=-1), _lib.MPWSD_ERR_ARG),
        (dict(llr=None), _lib.MPWSD_ERR_ARG),
        (dict(anchors=None), _lib.MPWSD_ERR_ARG),
    ]
    for kw, code in cases:
        a = dict(base, **kw)
        rc = _lib.mpwsd_stage1_osd(a["r"], a["m"], a["order"], a["L"], a["llr"], a["dtype"], a["F"],
                                   a["anchors"], a["metric"], None)
        assert rc == code, (kw, rc, _lib.last_error())
    # F = 0 is a no-op that needs no pointers
    assert _lib.mpwsd_stage1_osd(2, 7, 2, 8, None, 0, 0, None, None, None) == 0
