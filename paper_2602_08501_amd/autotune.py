"""Autotuner for the stage-2 move search.

Times every search tile variant (column blocks per wave x waves per
workgroup) and persistent-grid size on the caller's own batch, checks that
all of them produce bit-identical decisions and move logs, and keeps the
fastest for every iteration separately (the active columns shrink from
iteration to iteration, and small searches prefer small tiles).  Choices are cached per device, code, list size, iteration count and
batch size in a JSON file (MPWSD_TUNE_CACHE, default
~/.cache/mpwsd/tune.json).
"""
from __future__ import annotations

import json
import os

import torch

from . import _lib

CACHE = os.environ.get("MPWSD_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "mpwsd", "tune.json"))


def _key(stage2) -> str:
    name = torch.cuda.get_device_name(torch.device(stage2.device))
    segs = "+".join("RM(%d,%d)P%dxF%d" % (code.r, code.m, code.P, F) for code, F in stage2.codes_F)
    return "%s|%s|L%d|T%d|%s" % (name, segs, stage2.L, stage2.T, "i8" if stage2.dt == _lib.MPWSD_I8 else "f32")


def _load() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(d: dict) -> None:
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def candidates(N: int, multi: bool = False, grouped: bool = False):
    """(variant, workgroups per CU) pairs to time; a batch of several codes
    is searched by one launch that exists for the first three variants.  The
    workgroups per CU go up to what the 160 KB of LDS of a CU holds: the
    plain search stages two 128-row chunks of N + 16 bytes per row, the
    paired-half search three chunks of N/2-byte rows and eight chunks'
    indices."""
    vs = _lib.mpwsd_search_variants()
    if multi:
        vs = vs[:3]
    kp = max(N, 64)
    lds = 3 * 128 * (N // 2) + 8 * 2 * 128 * 4 if grouped and not multi else 2 * 128 * (kp + 16)
    lds_fit = (160 * 1024) // lds
    out = []
    for i, v in enumerate(vs):
        for bpc in sorted({v["blocks_per_cu"], 1, 2, 3, 4, 5, 6}):
            if 1 <= bpc <= lds_fit:
                out.append((i, bpc))
    return out


def tune(stage2, llrs, anchors, crc_oks, reps: int = 3, stream=None, use_cache: bool = True, verbose=False):
    """Returns ([variant] * T, [blocks_per_cu] * T) for this Stage2 and its inputs."""
    key = _key(stage2)
    cache = _load() if use_cache else {}
    if key in cache and isinstance(cache[key].get("choice", [None])[0], list):
        v, b = cache[key]["choice"]
        return list(v), list(b)
    stream = stream or torch.cuda.current_stream()
    T = stage2.T
    nseg = len(stage2.codes_F)
    multi = nseg > 1 and stage2.dt == _lib.MPWSD_I8
    events = [torch.cuda.Event(enable_timing=True) for _ in range(2 * T * nseg)]
    for e in events:
        e.record(stream)
    ref = None
    results = []  # (variant, bpc, [ms per iteration])
    grouped = all(c.grouped is not None for c, _ in stage2.codes_F)
    for var, bpc in candidates(max(c.N for c, _ in stage2.codes_F), multi, grouped):
        per_iter = None
        for r in range(reps + 1):
            stage2.run(llrs, anchors, crc_oks, stream=stream, events=events, variant=var, blocks_per_cu=bpc)
            stream.synchronize()
            if r == 0:
                out = [{k: v.clone() for k, v in o.items()} for o in stage2.outs]
                if ref is None:
                    ref = out
                else:
                    for k in ref[0]:
                        if not all(torch.equal(a[k], b[k]) for a, b in zip(ref, out)):
                            raise RuntimeError("search variant %d / %d differs from variant %d in %s"
                                               % (var, bpc, results[0][0], k))
                continue
            # per iteration: the launches of every segment (one launch when several codes share it)
            ms = [sum(events[2 * (s * T + t)].elapsed_time(events[2 * (s * T + t) + 1])
                      for s in range(1 if multi else nseg)) for t in range(T)]
            per_iter = ms if per_iter is None else [min(a, b) for a, b in zip(per_iter, ms)]
        results.append((var, bpc, per_iter))
        if verbose:
            print("variant %d blocks/CU %d: %s ms" % (var, bpc, " ".join("%.3f" % x for x in per_iter)))
    best_v, best_b, best_ms = [], [], []
    for t in range(T):
        v, b, ms = min(results, key=lambda x: x[2][t])
        best_v.append(v)
        best_b.append(b)
        best_ms.append(ms[t])
    cache[key] = {"choice": [best_v, best_b], "search_ms": sum(best_ms),
                  "all": [[v, b, ms] for v, b, ms in results]}
    if use_cache:
        _save(cache)
    return best_v, best_b
