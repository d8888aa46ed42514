"""Thin torch-backed driver over the C-ABI: owns device buffers, calls the
library.  PyTorch is used for device memory and streams only."""
from __future__ import annotations

import math

import numpy as np
import torch

from . import _lib
from ._lib import MPWSD_F32, MPWSD_I8, Segment, check


_POPCOUNT8 = np.array([bin(i).count("1") for i in range(256)], np.uint8)


def build_moves_host(r: int, m: int, radius: int = 1) -> np.ndarray:
    """Move table S_radius(0) \\ {0} of RM(r, m), [P][N/8] uint8 (host, via the library)."""
    rc, P, N, w = _lib.mpwsd_build_sphere(r, m, radius, None, 0)
    check(rc)
    buf = np.zeros((P, N // 8), np.uint8)
    rc, P, N, w = _lib.mpwsd_build_sphere(r, m, radius, buf.ctypes.data, buf.nbytes)
    check(rc)
    return buf


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def group_moves_host(m: int, moves: np.ndarray):
    """Paired-half layout of a move table (mpwsd_group_moves), as (bytes, chunks,
    extras), or None when the table does not group (then the plain table is
    searched)."""
    P = moves.shape[0]
    if m not in (7, 8):
        return None
    rc, chunks, extras, nbytes = _lib.mpwsd_group_moves(m, moves.ctypes.data, P, None, 0)
    if rc == _lib.MPWSD_ERR_UNSUPPORTED:
        return None
    check(rc)
    buf = np.zeros(nbytes, np.uint8)
    rc, chunks, extras, nbytes = _lib.mpwsd_group_moves(m, moves.ctypes.data, P, buf.ctypes.data, buf.nbytes)
    check(rc)
    return buf, chunks, extras


class Code:
    """Device-resident move table of RM(r, m): the sphere S_radius(0), and its
    paired-half layout for the int8 search.  grouped="auto" takes the layout
    only when it keeps no move apart (RM(3,7), RM(3,8)): where moves are kept
    apart (RM(2,7)) the layout's normals carry about one chunk each and the
    plain table is faster; True takes any layout that exists; False keeps the
    plain table only."""

    def __init__(self, r: int, m: int, device="cuda:0", radius: int = 1, grouped="auto"):
        self.r, self.m, self.N, self.radius = r, m, 1 << m, radius
        host = build_moves_host(r, m, radius)
        self.P = host.shape[0]
        wts = _POPCOUNT8[host].sum(1, dtype=np.int64)
        self.w_max = int(wts.max())
        self.w = float(wts.mean())  # mean move weight (2^(m-r) for radius 1)
        self.moves = torch.from_numpy(host).to(device)
        self.K = sum(math.comb(m, d) for d in range(r + 1))
        self.grouped, self.grouped_chunks, self.grouped_extras = None, 0, 0
        g = group_moves_host(m, host) if grouped else None
        if g is not None and grouped == "auto" and g[2] > 0:
            g = None
        if g is not None:
            buf, self.grouped_chunks, self.grouped_extras = g
            self._grouped_store = torch.empty(buf.nbytes + 256, dtype=torch.uint8, device=device)
            off = (-self._grouped_store.data_ptr()) % 256
            self.grouped = self._grouped_store[off:off + buf.nbytes]
            self.grouped.copy_(torch.from_numpy(buf))

    def grouped_ptr(self):
        return None if self.grouped is None else self.grouped.data_ptr()


def quantize(y: torch.Tensor, scale: float, bad: torch.Tensor | None = None, stream=None,
             out: torch.Tensor | None = None, raw_stream=None) -> torch.Tensor:
    q = out if out is not None else torch.empty(y.shape, dtype=torch.int8, device=y.device)
    check(_lib.mpwsd_quantize_llr(y.data_ptr(), y.numel(), float(np.float32(scale)), q.data_ptr(),
                                  _ptr(bad), raw_stream if raw_stream is not None else _stream(stream)))
    return q


class Graph:
    """A recorded sequence of library calls (HIP graph), replayed with launch()."""

    def __init__(self, record):
        """record(raw_stream) enqueues the calls to record on raw_stream."""
        s = _lib.mpwsd_graph_begin()
        try:
            record(s)
        finally:
            self.handle = _lib.mpwsd_graph_end(s)

    def launch(self, stream=None):
        check(_lib.mpwsd_graph_launch(self.handle, _stream(stream)))

    def __del__(self):
        h = getattr(self, "handle", None)
        if not h:
            return
        self.handle = None
        try:
            _lib.mpwsd_graph_destroy(h)
        except (AttributeError, TypeError, OSError):
            pass  # interpreter teardown: the module or the library is already gone


def stage1(code: Code, L: int, llr: torch.Tensor, crc_len: int = 6, crc_poly: int = 0x43,
           out=None, stream=None, want_pm: bool = False, raw_stream=None):
    F = llr.shape[0]
    dev = llr.device
    if out is None:
        out = {"anchors": torch.empty((F, L, code.N // 8), dtype=torch.uint8, device=dev),
               "crc_ok": torch.empty(F, dtype=torch.uint8, device=dev)}
        if want_pm:
            out["pm"] = torch.empty((F, L), dtype=torch.int32, device=dev)
    dtype = MPWSD_I8 if llr.dtype == torch.int8 else MPWSD_F32
    check(_lib.mpwsd_stage1_scl(code.r, code.m, crc_len, crc_poly, L, llr.data_ptr(), dtype, F,
                                out["anchors"].data_ptr(), out["crc_ok"].data_ptr(),
                                _ptr(out.get("pm")), raw_stream if raw_stream is not None else _stream(stream)))
    return out


def stage1_quantized(code: Code, L: int, y: torch.Tensor, scale: float, crc_len: int = 6, crc_poly: int = 0x43,
                     q: torch.Tensor | None = None, bad: torch.Tensor | None = None, out=None, stream=None,
                     want_pm: bool = False, raw_stream=None):
    """quantize() then stage1() on the int8 values, in one launch: returns
    the stage-1 outputs with the quantized values under "q"."""
    F = y.shape[0]
    dev = y.device
    if out is None:
        out = {"anchors": torch.empty((F, L, code.N // 8), dtype=torch.uint8, device=dev),
               "crc_ok": torch.empty(F, dtype=torch.uint8, device=dev)}
        if want_pm:
            out["pm"] = torch.empty((F, L), dtype=torch.int32, device=dev)
    if q is None:
        q = torch.empty(y.shape, dtype=torch.int8, device=dev)
    out["q"] = q
    check(_lib.mpwsd_stage1_scl_quantized(code.r, code.m, crc_len, crc_poly, L, y.data_ptr(),
                                          float(np.float32(scale)), F, q.data_ptr(), _ptr(bad),
                                          out["anchors"].data_ptr(), out["crc_ok"].data_ptr(), _ptr(out.get("pm")),
                                          raw_stream if raw_stream is not None else _stream(stream)))
    return out


def stage1_osd(code: Code, order: int, L: int, llr: torch.Tensor, out=None, stream=None, want_metric: bool = False,
               raw_stream=None):
    """OSD(order) anchors of every frame, smallest metric first (no CRC: run
    stage 2 with crc_ok None, the always-on mode)."""
    F = llr.shape[0]
    dev = llr.device
    if out is None:
        out = {"anchors": torch.empty((F, L, code.N // 8), dtype=torch.uint8, device=dev)}
        if want_metric:
            out["metric"] = torch.empty((F, L), dtype=torch.int32, device=dev)
    dtype = MPWSD_I8 if llr.dtype == torch.int8 else MPWSD_F32
    check(_lib.mpwsd_stage1_osd(code.r, code.m, order, L, llr.data_ptr(), dtype, F, out["anchors"].data_ptr(),
                                _ptr(out.get("metric")), raw_stream if raw_stream is not None else _stream(stream)))
    return out


class Stage2:
    """Buffers and one call of mpwsd_decode_batch for a fixed batch shape."""

    def __init__(self, codes_F, L: int, T: int, dtype: str, device="cuda:0", want_moves=True):
        """codes_F: list of (Code, F) per segment."""
        self.L, self.T, self.device = L, T, device
        self.dt = MPWSD_I8 if dtype == "i8" else MPWSD_F32
        self.codes_F = codes_F
        self.outs = []
        for code, F in codes_F:
            o = {"cw": torch.empty((F, code.N // 8), dtype=torch.uint8, device=device),
                 "k": torch.empty(F, dtype=torch.int32, device=device),
                 "metric": torch.empty(F, dtype=torch.int32, device=device)}
            if want_moves:
                o["moves"] = torch.empty((F, L, T), dtype=torch.int32, device=device)
            self.outs.append(o)
        self.stats = torch.zeros(2 + T, dtype=torch.int32, device=device)
        need = _lib.mpwsd_workspace_bytes(self._segs([None] * len(codes_F), [None] * len(codes_F),
                                                     [None] * len(codes_F)), L, T)
        if need == 0:
            raise _lib.MpwsdError(-1, _lib.last_error())
        self.ws = torch.empty(need + 256, dtype=torch.uint8, device=device)
        off = (-self.ws.data_ptr()) % 256
        self.ws_ptr, self.ws_bytes = self.ws.data_ptr() + off, need

    def _segs(self, llrs, anchors, crc_oks):
        segs = []
        for (code, F), llr, anc, ok, o in zip(self.codes_F, llrs, anchors, crc_oks,
                                              self.outs or [None] * len(self.codes_F)):
            segs.append(Segment(code.r, code.m, code.moves.data_ptr(), code.P, _ptr(llr), self.dt, F,
                                _ptr(anc), _ptr(ok), _ptr(o["cw"]) if o else None,
                                _ptr(o["k"]) if o else None, _ptr(o["metric"]) if o else None,
                                _ptr(o.get("moves")) if o else None, code.grouped_ptr(), code.grouped_chunks,
                                code.grouped_extras))
        return segs

    def run(self, llrs, anchors, crc_oks, stream=None, events=None, variant=-1, blocks_per_cu=0,
            raw_stream=None, merge=True):
        """events: optional list of 2 * T * nseg recorded torch.cuda.Event
        (enable_timing=True); re-recorded around every search launch.
        variant / blocks_per_cu: one value, or T values (per iteration).
        raw_stream: a hipStream_t handle (int) to enqueue on instead of a
        torch stream (used while recording a graph).
        merge=False searches every active path, also paths of a frame that
        reached the same centre (same outputs, more searched paths)."""
        segs = self._segs(llrs, anchors, crc_oks)
        st = raw_stream if raw_stream is not None else _stream(stream)
        per_iter = isinstance(variant, (list, tuple)) or isinstance(blocks_per_cu, (list, tuple))
        if events is None and not per_iter and variant < 0 and blocks_per_cu == 0 and merge:
            check(_lib.mpwsd_decode_batch(segs, self.L, self.T, self.ws_ptr, self.ws_bytes,
                                          self.stats.data_ptr(), st))
        else:
            check(_lib.mpwsd_decode_batch_ex(segs, self.L, self.T, self.ws_ptr, self.ws_bytes,
                                             self.stats.data_ptr(), variant, blocks_per_cu,
                                             None if events is None else [e.cuda_event for e in events], st,
                                             merge=merge))
        return self.outs
