"""Reference oracle for MP-WSD — TEST INFRASTRUCTURE ONLY.

A plain, slow CPU implementation (``mpwsd_oracle.c``) of what the decoder
computes, written from the paper's definitions, with a ctypes binding.  Only
the test suite, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the HIP library and never calls
it.

Arithmetic modes: ``INT`` (quantized LLRs, exact integer arithmetic),
``F32`` (every sum rounded to binary32) and ``F64``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

INT, F32, F64 = 0, 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mpwsd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
            "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, u32, f32 = ctypes.c_int, ctypes.c_int64, ctypes.c_uint32, ctypes.c_float
        lib.orc_rm_dims.argtypes = [i32, i32, P, P]
        lib.orc_rm_info_set.argtypes = [i32, i32, P]
        lib.orc_encode_def.argtypes = [i32, P, P]
        lib.orc_encode.argtypes = [i32, P, P]
        lib.orc_moves.argtypes = [i32, i32, P, i64, P]
        lib.orc_moves.restype = i64
        lib.orc_pack_supports.argtypes = [i32, i64, i32, P, P]
        lib.orc_weight_distribution.argtypes = [i32, i32, P]
        lib.orc_sphere.argtypes = [i32, i32, i32, P, i64, P]
        lib.orc_sphere.restype = i64
        lib.orc_crc.argtypes = [P, i32, i32, u32, P]
        lib.orc_crc_ok.argtypes = [P, i32, i32, u32]
        lib.orc_quantize.argtypes = [P, i64, f32, P]
        lib.orc_scl.argtypes = [i32, i32, i32, P, P, P, P, P]
        lib.orc_metric.argtypes = [i32, i32, P, P]
        lib.orc_metric.restype = ctypes.c_double
        lib.orc_stage2_path.argtypes = [i32, i32, i64, i32, P, P, P, i32, P]
        lib.orc_stage2_frame.argtypes = [i32, i32, i64, i32, P, P, i32, P, i32, P, P, P]
        lib.orc_stage2_alg1.argtypes = [i32, i64, i32, P, P, i32, P, i32, i64, P, P]
        lib.orc_osd.argtypes = [i32, i32, i32, i32, i32, P, P, P, P]
        lib.orc_ml.argtypes = [i32, i32, i32, P, P]
        lib.orc_ml.restype = ctypes.c_double
        lib.orc_decode_batch.argtypes = [i32, i32, i32, u32, i32, i32, i32, i64, i32, P,
                                         P, i64, i64, P, P, P, P, P, P]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


# ---------------------------------------------------------------- code (Sec. II-B)
def rm_dims(r: int, m: int):
    N, K = ctypes.c_int(), ctypes.c_int()
    if _L().orc_rm_dims(r, m, ctypes.byref(N), ctypes.byref(K)) != 0:
        raise ValueError("bad RM parameters")
    return N.value, K.value


def rm_info_set(r: int, m: int) -> np.ndarray:
    A = np.zeros(1 << m, np.int32)
    k = _L().orc_rm_info_set(r, m, _p(A))
    return A[:k].copy()


def frozen_mask(r: int, m: int) -> np.ndarray:
    fr = np.ones(1 << m, np.uint8)
    fr[rm_info_set(r, m)] = 0
    return fr


def encode_def(m: int, u) -> np.ndarray:
    u = np.ascontiguousarray(u, np.uint8)
    c = np.zeros(1 << m, np.uint8)
    _L().orc_encode_def(m, _p(u), _p(c))
    return c


def encode(m: int, u) -> np.ndarray:
    u = np.ascontiguousarray(u, np.uint8)
    c = np.zeros(1 << m, np.uint8)
    _L().orc_encode(m, _p(u), _p(c))
    return c


# ---------------------------------------------------------------- moves (Sec. II-C)
_moves_cache: dict = {}


def moves(r: int, m: int):
    """(supp[P][w] uint16 in canonical order, w)."""
    key = (r, m)
    if key not in _moves_cache:
        w = ctypes.c_int()
        P = _L().orc_moves(r, m, None, 0, ctypes.byref(w))
        if P < 0:
            raise ValueError("bad RM parameters")
        supp = np.zeros((P, w.value), np.uint16)
        P2 = _L().orc_moves(r, m, _p(supp), P, ctypes.byref(w))
        assert P2 == P
        _moves_cache[key] = (supp, w.value)
    return _moves_cache[key]


SUPP_END = 0xFFFF  # pads support rows of moves lighter than the row stride


def weight_distribution(r: int, m: int) -> np.ndarray:
    """A[0..N]: codewords of RM(r, m) per weight, by visiting all 2^K (K <= 30)."""
    A = np.zeros((1 << m) + 1, np.int64)
    if _L().orc_weight_distribution(r, m, _p(A)) != 0:
        raise ValueError("bad RM parameters or K too large")
    return A


_sphere_cache: dict = {}


def sphere(r: int, m: int, radius: int):
    """(supp[P][stride] uint16, stride): the nonzero words of S_radius(0) by
    weight, then canonical order; rows padded with SUPP_END.  radius 1 gives
    the table of ``moves`` (via a different enumeration)."""
    key = (r, m, radius)
    if key not in _sphere_cache:
        st = ctypes.c_int()
        P = _L().orc_sphere(r, m, radius, None, 0, ctypes.byref(st))
        if P < 0:
            raise ValueError("bad RM parameters, K too large, or too few weights")
        supp = np.zeros((P, st.value), np.uint16)
        P2 = _L().orc_sphere(r, m, radius, _p(supp), P, ctypes.byref(st))
        assert P2 == P
        _sphere_cache[key] = (supp, st.value)
    return _sphere_cache[key]


def pack_supports(m: int, supp: np.ndarray) -> np.ndarray:
    supp = np.ascontiguousarray(supp, np.uint16)
    P, w = supp.shape
    rows = np.zeros((P, (1 << m) // 8), np.uint8)
    _L().orc_pack_supports(m, P, w, _p(supp), _p(rows))
    return rows


# ---------------------------------------------------------------- CRC (Sec. II-B)
def crc(bits, L: int, poly: int) -> np.ndarray:
    b = np.ascontiguousarray(bits, np.uint8)
    out = np.zeros(L, np.uint8)
    _L().orc_crc(_p(b), len(b), L, poly, _p(out))
    return out


def crc_ok(v, L: int, poly: int) -> bool:
    v = np.ascontiguousarray(v, np.uint8)
    return bool(_L().orc_crc_ok(_p(v), len(v), L, poly))


# ---------------------------------------------------------------- quantizer
def quantize(y, s: float) -> np.ndarray:
    y = np.ascontiguousarray(y, np.float32)
    q = np.zeros(y.shape, np.int8)
    _L().orc_quantize(_p(y), y.size, float(np.float32(s)), _p(q))
    return q


# ---------------------------------------------------------------- stage 1 (Sec. III-A)
def scl(m: int, L: int, mode: int, llr, frozen):
    n = 1 << m
    llr = np.ascontiguousarray(llr, np.float64)
    frozen = np.ascontiguousarray(frozen, np.uint8)
    u = np.zeros((L, n), np.uint8)
    c = np.zeros((L, n), np.uint8)
    pm = np.zeros(L, np.float64)
    np_ = _L().orc_scl(m, L, mode, _p(llr), _p(frozen), _p(u), _p(c), _p(pm))
    return u[:np_], c[:np_], pm[:np_]


# ---------------------------------------------------------------- stage 2 (Sec. III-B)
def metric(mode: int, y, c) -> float:
    y = np.ascontiguousarray(y, np.float64)
    c = np.ascontiguousarray(c, np.uint8)
    return _L().orc_metric(mode, len(y), _p(y), _p(c))


def stage2_path(mode: int, supp: np.ndarray, y, c, T: int):
    y = np.ascontiguousarray(y, np.float64)
    c = np.array(c, np.uint8, copy=True)
    log = np.zeros(T, np.int32)
    P, w = supp.shape
    _L().orc_stage2_path(mode, len(y), P, w, _p(supp), _p(y), _p(c), T, _p(log))
    return c, log


def stage2_frame(mode: int, supp: np.ndarray, y, anchors, T: int):
    y = np.ascontiguousarray(y, np.float64)
    anchors = np.ascontiguousarray(anchors, np.uint8)
    L, n = anchors.shape
    paths = np.zeros((L, n), np.uint8)
    logs = np.zeros((L, T), np.int32)
    met = np.zeros(L, np.float64)
    P, w = supp.shape
    kb = _L().orc_stage2_frame(mode, n, P, w, _p(supp), _p(y), L, _p(anchors), T,
                               _p(paths), _p(logs), _p(met))
    return paths, logs, met, kb


def stage2_alg1(supp: np.ndarray, y, anchors, J: int, mfilt: int):
    y = np.ascontiguousarray(y, np.float64)
    anchors = np.ascontiguousarray(anchors, np.uint8)
    L, n = anchors.shape
    paths = np.zeros((L, n), np.uint8)
    logs = np.zeros((L, J), np.int32)
    P, w = supp.shape
    kb = _L().orc_stage2_alg1(n, P, w, _p(supp), _p(y), L, _p(anchors), J, mfilt,
                              _p(paths), _p(logs))
    return paths, logs, kb


def osd(r: int, m: int, order: int, L: int, mode: int, llr):
    """OSD(order) list of one frame: (anchors[n][N], metric[n], mrb[K]),
    n = min(L, number of candidates), smallest metric first."""
    llr = np.ascontiguousarray(llr, np.float64)
    N, K = rm_dims(r, m)
    anchors = np.zeros((L, N), np.uint8)
    met = np.zeros(L, np.float64)
    mrb = np.zeros(K, np.int32)
    nl = _L().orc_osd(r, m, order, L, mode, _p(llr), _p(anchors), _p(met), _p(mrb))
    if nl < 0:
        raise ValueError("bad OSD parameters")
    return anchors[:nl], met[:nl], mrb


def ml(r: int, m: int, mode: int, y):
    y = np.ascontiguousarray(y, np.float64)
    c = np.zeros(1 << m, np.uint8)
    e = _L().orc_ml(r, m, mode, _p(y), _p(c))
    return e, c


# ---------------------------------------------------------------- two-stage decoder
def decode_batch(r: int, m: int, crc_len: int, crc_poly: int, L: int, T: int, mode: int,
                 llr, threads: int = 1, frames=None, radius: int = 1):
    """Decode llr[F][N] (Sec. III).  Returns a dict of per-frame outputs.

    ``frames`` optionally restricts the work to a sub-range (f0, f1); the
    outputs still have F rows (untouched rows are zero / -1).  ``radius``
    selects the sphere S_radius(0) searched by stage 2.
    """
    llr = np.ascontiguousarray(llr, np.float64)
    F, n = llr.shape
    assert n == 1 << m
    supp, w = moves(r, m) if radius == 1 else sphere(r, m, radius)
    P = supp.shape[0]
    out = {
        "c": np.zeros((F, n), np.uint8),
        "anchors": np.zeros((F, L, n), np.uint8),
        "crc_ok": np.zeros(F, np.uint8),
        "k": np.zeros(F, np.int32),
        "metric": np.zeros(F, np.float64),
        "logs": np.full((F, L, T), -1, np.int32),
    }
    f0, f1 = frames if frames is not None else (0, F)
    lib = _L()

    def run(a, b):
        lib.orc_decode_batch(r, m, crc_len, crc_poly, L, T, mode, P, w, _p(supp), _p(llr),
                             a, b, _p(out["c"]), _p(out["anchors"]), _p(out["crc_ok"]),
                             _p(out["k"]), _p(out["metric"]), _p(out["logs"]))

    if threads <= 1 or f1 - f0 <= 1:
        run(f0, f1)
    else:
        # one frame per task keeps the threads busy when stage 2 is uneven
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(lambda f: run(f, f + 1), range(f0, f1)))
    return out


def decode_osd_batch(r: int, m: int, order: int, L: int, T: int, mode: int, llr, threads: int = 1,
                     radius: int = 1):
    """OSD(order) stage 1 and stage 2 on every frame (always-on mode, Sec.
    III-C: no CRC, P_act = 1).  Returns anchors, metric of the anchors, the
    decision, the chosen path, its metric and the move logs per frame."""
    llr = np.ascontiguousarray(llr, np.float64)
    F, n = llr.shape
    supp, w = moves(r, m) if radius == 1 else sphere(r, m, radius)
    out = {
        "anchors": np.zeros((F, L, n), np.uint8),
        "anchor_metric": np.zeros((F, L), np.float64),
        "c": np.zeros((F, n), np.uint8),
        "k": np.zeros(F, np.int32),
        "metric": np.zeros(F, np.float64),
        "logs": np.full((F, L, T), -1, np.int32),
    }

    def run(f):
        a, met, _ = osd(r, m, order, L, mode, llr[f])
        out["anchors"][f] = a
        out["anchor_metric"][f] = met
        paths, logs, pm, kb = stage2_frame(mode, supp, llr[f], a, T)
        out["c"][f] = paths[kb]
        out["k"][f] = kb
        out["metric"][f] = pm[kb]
        out["logs"][f] = logs

    if threads <= 1:
        for f in range(F):
            run(f)
    else:
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(run, range(F)))
    return out
