"""Serving: a continuous-batching server over the C-ABI and a trace-driven
load test (Poisson arrivals of frames of several codes).

    python -m paper_2602_08501_amd.serve --rate 1e5 3e5 1e6 --seconds 10

Codes RM(2,7) / RM(3,7) / RM(3,8) in equal shares, Eb/N0 uniform in
[1.5, 3.5] dB per frame, int8 LLRs, up to 8192 frames of each code in flight
(the memory gate).  One JSON line per rate: offered and served frames/s,
p50 / p99 latency (submission to the host seeing the result), the fraction
of frames decided in stage 2.
"""
from __future__ import annotations

import argparse
import ctypes
import dataclasses
import json
import sys

import numpy as np
import torch

from . import _lib
from . import decoder as D
from . import synth
from ._lib import Result, ServerCode, check


class Server:
    def __init__(self, codes, specs, device="cuda:0"):
        """codes: list of decoder.Code; specs: list of dicts with L, T,
        crc_len, crc_poly, capacity."""
        self.codes = codes
        arr = (ServerCode * len(codes))()
        for i, (c, sp) in enumerate(zip(codes, specs)):
            arr[i] = ServerCode(c.r, c.m, c.moves.data_ptr(), c.P, sp["L"], sp["T"], sp.get("crc_len", 6),
                                sp.get("crc_poly", synth.CRC6_POLY), sp["capacity"], c.grouped_ptr(), c.grouped_chunks,
                                c.grouped_extras)
        self._arr = arr
        need = _lib.load().mpwsd_server_arena_bytes(arr, len(codes))
        if need == 0:
            raise _lib.MpwsdError(-1, _lib.last_error())
        self.arena = torch.empty(need + 256, dtype=torch.uint8, device=device)
        off = (-self.arena.data_ptr()) % 256
        h = ctypes.c_void_p()
        check(_lib.load().mpwsd_server_create(arr, len(codes), self.arena.data_ptr() + off, need, ctypes.byref(h)))
        self.h = h.value
        torch.cuda.synchronize()

    def submit(self, code: int, y: np.ndarray, scale: np.ndarray, tags: np.ndarray):
        y = np.ascontiguousarray(y, np.float32)
        scale = np.ascontiguousarray(scale, np.float32)
        tags = np.ascontiguousarray(tags, np.uint64)
        check(_lib.load().mpwsd_server_submit(self.h, code, len(tags), y.ctypes.data, scale.ctypes.data,
                                              tags.ctypes.data))

    def tick(self) -> int:
        n = ctypes.c_int64()
        check(_lib.load().mpwsd_server_tick(self.h, ctypes.byref(n)))
        return n.value

    def poll(self, cap: int = 4096):
        buf = (Result * cap)()
        k = _lib.load().mpwsd_server_poll(self.h, buf, cap)
        if k < 0:
            raise _lib.MpwsdError(k, _lib.last_error())
        return list(buf[:k])

    def drain(self):
        out = []
        while True:
            left = self.tick()
            out += self.poll()
            if left == 0:
                return out

    def serve_trace(self, code, row, scale, arrival, pools):
        n = len(code)
        code = np.ascontiguousarray(code, np.int32)
        row = np.ascontiguousarray(row, np.int64)
        scale = np.ascontiguousarray(scale, np.float32)
        arrival = np.ascontiguousarray(arrival, np.float64)
        pools = [np.ascontiguousarray(p, np.float32) for p in pools]
        parr = (ctypes.c_void_p * len(pools))(*[p.ctypes.data for p in pools])
        out = (Result * n)()
        check(_lib.load().mpwsd_serve_trace(self.h, n, code.ctypes.data, row.ctypes.data, scale.ctypes.data,
                                            arrival.ctypes.data, parr, out))
        return out

    def close(self):
        if getattr(self, "h", None):
            _lib.load().mpwsd_server_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


def results_table(res):
    """numpy views of a Result array: tag, stage, k, metric, cw bytes, latency."""
    n = len(res)
    a = np.ctypeslib.as_array((ctypes.c_uint8 * (ctypes.sizeof(Result) * n)).from_address(ctypes.addressof(res)))
    dt = np.dtype([("tag", "<u8"), ("code", "<i4"), ("stage", "<i4"), ("k", "<i4"), ("metric", "<i4"),
                   ("cw", "u1", 32), ("t_submit", "<f8"), ("t_done", "<f8")])
    assert dt.itemsize == ctypes.sizeof(Result)
    return a.view(dt).copy()  # owns its memory: the ctypes array may be freed


MIX = [(synth.RM27, 8, 8), (synth.RM37, 8, 8), (synth.RM38, 16, 12)]


def build_pools(rows: int, seed: int = 5, lo: float = 1.5, hi: float = 3.5):
    pools, scales, truth = [], [], []
    for wl, L, T in MIX:
        pay, c, y, eb, sc = synth.generate_snr_mix(wl, seed, 0, rows, lo, hi)
        pools.append(y)
        scales.append(sc)
        truth.append(c)
    return pools, scales, truth


def make_trace(rate: float, seconds: float, rows: int, seed: int = 9):
    rng = np.random.default_rng(seed)
    n = int(rate * seconds)
    arrival = np.cumsum(rng.exponential(1.0 / rate, n))
    code = rng.integers(0, len(MIX), n).astype(np.int32)
    row = rng.integers(0, rows, n).astype(np.int64)
    return code, row, arrival


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rate", type=float, nargs="+", default=[1e5, 3e5, 1e6])
    ap.add_argument("--seconds", type=float, default=10.0)
    ap.add_argument("--rows", type=int, default=16384, help="distinct frames per code in the pool")
    ap.add_argument("--capacity", type=int, default=8192)
    args = ap.parse_args()
    codes = [D.Code(wl.r, wl.m, "cuda:0") for wl, L, T in MIX]
    specs = [dict(L=L, T=T, capacity=args.capacity) for wl, L, T in MIX]
    pools, scales, truth = build_pools(args.rows)
    for rate in args.rate:
        srv = Server(codes, specs)
        code, row, arrival = make_trace(rate, args.seconds, args.rows)
        scale = np.stack(scales).astype(np.float32)[code, row]
        res = srv.serve_trace(code, row, scale, arrival, pools)
        srv.close()
        t = results_table(res)
        lat = (t["t_done"] - t["t_submit"]) * 1e3
        span = t["t_done"].max() - t["t_submit"].min()
        # frame errors per code, all frames of a code at once (compared as packed bytes)
        err = np.zeros(len(code), bool)
        for ci, (wl, L, T) in enumerate(MIX):
            sel = np.nonzero(code == ci)[0]
            nb = (1 << wl.m) // 8
            ref = np.packbits(truth[ci], axis=-1, bitorder="little")
            err[sel] = (t["cw"][sel, :nb] != ref[row[sel]]).any(1)
        print(json.dumps({
            "offered_frames_per_s": rate, "frames": len(code), "served_frames_per_s": len(code) / span,
            "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
            "latency_ms_max": float(lat.max()), "stage2_fraction": float((t["stage"] == 2).mean()),
            "fer": float(err.mean()), "capacity_per_code": args.capacity,
            "codes": ["RM(%d,%d) L=%d T=%d" % (wl.r, wl.m, L, T) for wl, L, T in MIX]}), flush=True)


if __name__ == "__main__":
    sys.exit(main())
