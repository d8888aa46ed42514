"""ctypes binding of libmpwsd.so: the C-ABI declared in include/mpwsd.h.

Argument marshalling only.  Every step of the decoder runs in the library's
HIP kernels; there is no fallback: if the library is missing this module
raises on first use.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpwsd.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mpwsd.h")

MPWSD_OK, MPWSD_ERR_ARG, MPWSD_ERR_SIZE, MPWSD_ERR_DEVICE, MPWSD_ERR_UNSUPPORTED = 0, -1, -2, -3, -4
MPWSD_I8, MPWSD_F32 = 0, 1
MPWSD_NOALLOC_SCRATCH_BYTES = 64 << 20

_p, _i, _i64, _u32, _f, _sz = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint32,
                               ctypes.c_float, ctypes.c_size_t)


class Segment(ctypes.Structure):
    """struct mpwsd_segment."""
    _fields_ = [("r", _i), ("m", _i), ("moves", _p), ("P", _i64), ("llr", _p), ("dtype", _i),
                ("F", _i64), ("anchors", _p), ("crc_ok", _p), ("out_cw", _p), ("out_k", _p),
                ("out_metric", _p), ("out_moves", _p), ("grouped", _p), ("grouped_chunks", _i64),
                ("grouped_extras", _i64)]


class VariantInfo(ctypes.Structure):
    """struct mpwsd_variant_info."""
    _fields_ = [("col_blocks", _i), ("waves", _i), ("columns", _i), ("blocks_per_cu", _i)]


class Options(ctypes.Structure):
    """struct mpwsd_options."""
    _fields_ = [("search_variant", _i), ("blocks_per_cu", _i), ("events", ctypes.POINTER(_p)),
                ("iter_variant", ctypes.POINTER(_i)), ("iter_blocks_per_cu", ctypes.POINTER(_i)),
                ("no_merge", _i)]


class ServerCode(ctypes.Structure):
    """struct mpwsd_server_code."""
    _fields_ = [("r", _i), ("m", _i), ("moves", _p), ("P", _i64), ("L", _i), ("T", _i), ("crc_len", _i),
                ("crc_poly", _u32), ("capacity", _i), ("grouped", _p), ("grouped_chunks", _i64),
                ("grouped_extras", _i64)]


class Result(ctypes.Structure):
    """struct mpwsd_result."""
    _fields_ = [("tag", ctypes.c_uint64), ("code", ctypes.c_int32), ("stage", ctypes.c_int32),
                ("k", ctypes.c_int32), ("metric", ctypes.c_int32), ("cw", ctypes.c_uint8 * 32),
                ("t_submit", ctypes.c_double), ("t_done", ctypes.c_double)]


class MpwsdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (code %d)" % (msg, code))
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmpwsd.so is not built (run __graft_entry__.build() or "
                              "python paper_2602_08501_amd/build.py): " + LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        lib.mpwsd_last_error.restype = ctypes.c_char_p
        lib.mpwsd_last_error.argtypes = []
        lib.mpwsd_build_moves.argtypes = [_i, _i, _p, _sz, _p, _p, _p]
        lib.mpwsd_build_sphere.argtypes = [_i, _i, _i, _p, _sz, _p, _p, _p]
        lib.mpwsd_group_moves.argtypes = [_i, _p, _i64, _p, _sz, _p, _p, _p]
        lib.mpwsd_quantize_llr.argtypes = [_p, _i64, _f, _p, _p, _p]
        lib.mpwsd_stage1_scl.argtypes = [_i, _i, _i, _u32, _i, _p, _i, _i64, _p, _p, _p, _p]
        lib.mpwsd_stage1_osd.argtypes = [_i, _i, _i, _i, _p, _i, _i64, _p, _p, _p]
        lib.mpwsd_stage1_scl_quantized.argtypes = [_i, _i, _i, _u32, _i, _p, _f, _i64, _p, _p, _p, _p, _p, _p]
        lib.mpwsd_workspace_bytes.argtypes = [ctypes.POINTER(Segment), _i, _i, _i]
        lib.mpwsd_workspace_bytes.restype = _sz
        lib.mpwsd_decode_batch.argtypes = [ctypes.POINTER(Segment), _i, _i, _i, _p, _sz, _p, _p]
        lib.mpwsd_decode_batch_noalloc.argtypes = [ctypes.POINTER(Segment), _i, _i, _i, _p, _p]
        lib.mpwsd_decode_batch_ex.argtypes = [ctypes.POINTER(Segment), _i, _i, _i, _p, _sz, _p,
                                              ctypes.POINTER(Options), _p]
        lib.mpwsd_search_variants.argtypes = [ctypes.POINTER(VariantInfo), _i]
        lib.mpwsd_graph_begin.argtypes = [ctypes.POINTER(_p)]
        lib.mpwsd_graph_end.argtypes = [_p, ctypes.POINTER(_p)]
        lib.mpwsd_graph_launch.argtypes = [_p, _p]
        lib.mpwsd_graph_destroy.argtypes = [_p]
        lib.mpwsd_server_arena_bytes.argtypes = [ctypes.POINTER(ServerCode), _i]
        lib.mpwsd_server_arena_bytes.restype = _sz
        lib.mpwsd_server_create.argtypes = [ctypes.POINTER(ServerCode), _i, _p, _sz, ctypes.POINTER(_p)]
        lib.mpwsd_server_submit.argtypes = [_p, _i, _i, _p, _p, _p]
        lib.mpwsd_server_tick.argtypes = [_p, ctypes.POINTER(ctypes.c_int64)]
        lib.mpwsd_server_poll.argtypes = [_p, ctypes.POINTER(Result), _i]
        lib.mpwsd_server_destroy.argtypes = [_p]
        lib.mpwsd_serve_trace.argtypes = [_p, _i64, _p, _p, _p, _p, ctypes.POINTER(_p), ctypes.POINTER(Result)]
        for name in ("mpwsd_build_moves", "mpwsd_build_sphere", "mpwsd_group_moves", "mpwsd_quantize_llr",
                     "mpwsd_stage1_scl", "mpwsd_stage1_scl_quantized", "mpwsd_stage1_osd", "mpwsd_decode_batch",
                     "mpwsd_decode_batch_noalloc", "mpwsd_decode_batch_ex", "mpwsd_search_variants", "mpwsd_graph_begin", "mpwsd_graph_end",
                     "mpwsd_graph_launch", "mpwsd_graph_destroy", "mpwsd_server_create", "mpwsd_server_submit",
                     "mpwsd_server_tick", "mpwsd_server_poll", "mpwsd_server_destroy", "mpwsd_serve_trace"):
            getattr(lib, name).restype = _i
        _lib = lib
    return _lib


def header_functions() -> list[str]:
    """Names of the functions include/mpwsd.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(mpwsd_\w+)\s*\(", text, re.M)))


def last_error() -> str:
    return load().mpwsd_last_error().decode()


def check(rc: int) -> int:
    if rc != MPWSD_OK:
        raise MpwsdError(rc, last_error())
    return rc


# ------------------------------------------------------------------ the C calls
def mpwsd_build_moves(r: int, m: int, moves_ptr, cap_bytes: int):
    """Returns (rc, P, N, w); moves_ptr may be None for a size query."""
    P, N, w = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int()
    rc = load().mpwsd_build_moves(r, m, moves_ptr, cap_bytes, ctypes.byref(P), ctypes.byref(N),
                                  ctypes.byref(w))
    return rc, P.value, N.value, w.value


def mpwsd_build_sphere(r: int, m: int, radius: int, moves_ptr, cap_bytes: int):
    """Returns (rc, P, N, w_max); moves_ptr may be None for a size query."""
    P, N, w = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int()
    rc = load().mpwsd_build_sphere(r, m, radius, moves_ptr, cap_bytes, ctypes.byref(P), ctypes.byref(N),
                                   ctypes.byref(w))
    return rc, P.value, N.value, w.value


def mpwsd_group_moves(m: int, moves_ptr, P: int, out_ptr, cap_bytes: int):
    """Returns (rc, chunks, extras, bytes); out_ptr may be None for a query."""
    chunks, extras, nbytes = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
    rc = load().mpwsd_group_moves(m, moves_ptr, P, out_ptr, cap_bytes, ctypes.byref(chunks), ctypes.byref(extras),
                                  ctypes.byref(nbytes))
    return rc, chunks.value, extras.value, nbytes.value


def mpwsd_quantize_llr(y_ptr, n: int, scale: float, q_ptr, bad_ptr, stream: int) -> int:
    return load().mpwsd_quantize_llr(y_ptr, n, scale, q_ptr, bad_ptr, stream)


def mpwsd_stage1_scl(r, m, crc_len, crc_poly, L, llr_ptr, dtype, F, anchors_ptr, crc_ok_ptr,
                     pm_ptr, stream) -> int:
    return load().mpwsd_stage1_scl(r, m, crc_len, crc_poly, L, llr_ptr, dtype, F, anchors_ptr,
                                   crc_ok_ptr, pm_ptr, stream)


def mpwsd_stage1_scl_quantized(r, m, crc_len, crc_poly, L, y_ptr, scale, F, q_ptr, bad_ptr, anchors_ptr,
                               crc_ok_ptr, pm_ptr, stream) -> int:
    return load().mpwsd_stage1_scl_quantized(r, m, crc_len, crc_poly, L, y_ptr, scale, F, q_ptr, bad_ptr,
                                             anchors_ptr, crc_ok_ptr, pm_ptr, stream)


def mpwsd_stage1_osd(r, m, order, L, llr_ptr, dtype, F, anchors_ptr, metric_ptr, stream) -> int:
    return load().mpwsd_stage1_osd(r, m, order, L, llr_ptr, dtype, F, anchors_ptr, metric_ptr, stream)


def segments_array(segs):
    arr = (Segment * len(segs))(*segs)
    return arr


def mpwsd_workspace_bytes(segs, L: int, T: int) -> int:
    arr = segments_array(segs)
    return load().mpwsd_workspace_bytes(arr, len(segs), L, T)


def mpwsd_decode_batch(segs, L: int, T: int, ws_ptr, ws_bytes: int, stats_ptr, stream) -> int:
    arr = segments_array(segs)
    return load().mpwsd_decode_batch(arr, len(segs), L, T, ws_ptr, ws_bytes, stats_ptr, stream)


def mpwsd_decode_batch_noalloc(segs, L: int, T: int, stats_ptr, stream) -> int:
    arr = segments_array(segs)
    return load().mpwsd_decode_batch_noalloc(arr, len(segs), L, T, stats_ptr, stream)


def mpwsd_decode_batch_ex(segs, L: int, T: int, ws_ptr, ws_bytes: int, stats_ptr, variant=-1,
                          blocks_per_cu=0, event_handles=None, stream=None, merge=True) -> int:
    """variant / blocks_per_cu: one value, or a list of T values (one per iteration).
    merge=False searches every active path (sets mpwsd_options.no_merge)."""
    arr = segments_array(segs)
    opt = Options(-1, 0, None, None, None, 0 if merge else 1)
    if isinstance(variant, (list, tuple)):
        iv = (_i * len(variant))(*variant)
        opt.iter_variant = ctypes.cast(iv, ctypes.POINTER(_i))
    else:
        opt.search_variant = variant
    if isinstance(blocks_per_cu, (list, tuple)):
        ib = (_i * len(blocks_per_cu))(*blocks_per_cu)
        opt.iter_blocks_per_cu = ctypes.cast(ib, ctypes.POINTER(_i))
    else:
        opt.blocks_per_cu = blocks_per_cu
    if event_handles is not None:
        evs = (_p * len(event_handles))(*event_handles)
        opt.events = ctypes.cast(evs, ctypes.POINTER(_p))
    return load().mpwsd_decode_batch_ex(arr, len(segs), L, T, ws_ptr, ws_bytes, stats_ptr, ctypes.byref(opt), stream)


def mpwsd_search_variants() -> list:
    n = load().mpwsd_search_variants(None, 0)
    buf = (VariantInfo * n)()
    load().mpwsd_search_variants(buf, n)
    return [dict(col_blocks=v.col_blocks, waves=v.waves, columns=v.columns, blocks_per_cu=v.blocks_per_cu)
            for v in buf]


def mpwsd_graph_begin() -> int:
    s = _p()
    check(load().mpwsd_graph_begin(ctypes.byref(s)))
    return s.value


def mpwsd_graph_end(record_stream) -> int:
    g = _p()
    check(load().mpwsd_graph_end(record_stream, ctypes.byref(g)))
    return g.value


def mpwsd_graph_launch(graph, stream) -> int:
    return load().mpwsd_graph_launch(graph, stream)


def mpwsd_graph_destroy(graph) -> int:
    return load().mpwsd_graph_destroy(graph)
