"""Frame-error-rate comparison of the int8 and binary32 forms of the decoder
on the same received values, with the binary64 oracle on a subset.  Test
infrastructure (it may call the oracle), run as a script from the repository
root:

    python -u tests/fer_compare.py --code rm37 --ebn0 2.0 2.5 3.0 3.5 4.0 --frames 262144

Prints one JSON line per Eb/N0 point and a final summary line with the
Eb/N0 at which each form reaches FER 1e-3 (log-linear interpolation) and the
gap between the two forms in dB.  The oracle subset is decoded only when
--oracle-frames > 0.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2602_08501_amd import decoder as D  # noqa: E402
from paper_2602_08501_amd import synth  # noqa: E402


def decode_gpu(code, wl, L, T, y, dtype, chunk=65536):
    F = y.shape[0]
    out = np.zeros((F, code.N // 8), np.uint8)
    n2 = 0
    for f0 in range(0, F, chunk):
        yy = torch.from_numpy(y[f0:f0 + chunk]).to("cuda:0")
        n = yy.shape[0]
        llr = D.quantize(yy, float(wl.llr_scale)) if dtype == "i8" else yy
        s1 = D.stage1(code, L, llr, wl.crc_len, wl.crc_poly)
        st = D.Stage2([(code, n)], L, T, dtype, "cuda:0", want_moves=False)
        o = st.run([llr], [s1["anchors"]], [s1["crc_ok"]])[0]
        torch.cuda.synchronize()
        out[f0:f0 + n] = o["cw"].cpu().numpy()
        n2 += int(st.stats[0].item())
    return np.unpackbits(out, axis=-1, bitorder="little"), n2


def ebn0_at(points, key, target=1e-3):
    pts = sorted((p["ebn0"], p[key]) for p in points if p[key] > 0)
    for (e0, f0), (e1, f1) in zip(pts, pts[1:]):
        if f0 >= target >= f1:
            a = (math.log10(target) - math.log10(f0)) / (math.log10(f1) - math.log10(f0))
            return e0 + a * (e1 - e0)
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--code", default="rm37", choices=["rm26", "rm37", "rm27", "rm38"])
    ap.add_argument("--ebn0", type=float, nargs="+", default=[2.0, 2.5, 3.0, 3.5, 4.0])
    ap.add_argument("--frames", type=int, default=262144)
    ap.add_argument("--L", type=int, default=8)
    ap.add_argument("--T", type=int, default=8)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--oracle-frames", type=int, default=0)
    ap.add_argument("--oracle-threads", type=int, default=16)
    args = ap.parse_args()
    base = {"rm26": synth.RM26, "rm37": synth.RM37, "rm27": synth.RM27, "rm38": synth.RM38}[args.code]
    code = D.Code(base.r, base.m, "cuda:0")
    points = []
    for si, e in enumerate(args.ebn0):
        wl = dataclasses.replace(base, ebn0_db=e, snr_index=si)
        t0 = time.time()
        pay, c, y = synth.generate(wl, args.seed, 0, args.frames)
        res = {"code": args.code, "ebn0": e, "frames": args.frames, "L": args.L, "T": args.T}
        for dt in ("i8", "f32"):
            cw, n2 = decode_gpu(code, wl, args.L, args.T, y, dt)
            err = (cw != c).any(1)
            res["fer_" + dt] = float(err.mean())
            res["errors_" + dt] = int(err.sum())
            res["stage2_frames_" + dt] = n2
            res["_err_" + dt] = err
        res["disagree_i8_f32"] = int((res["_err_i8"] != res["_err_f32"]).sum())
        if args.oracle_frames > 0:
            import oracle  # the binary64 reference decoder
            n = min(args.oracle_frames, args.frames)
            ref = oracle.decode_batch(wl.r, wl.m, wl.crc_len, wl.crc_poly, args.L, args.T, oracle.F64,
                                      y[:n].astype(np.float64), threads=args.oracle_threads)
            err64 = (ref["c"] != c[:n]).any(1)
            res["oracle_f64_frames"] = n
            res["oracle_f64_errors"] = int(err64.sum())
            res["f32_vs_f64_decision_mismatch"] = int((ref["c"] != decode_gpu(
                code, wl, args.L, args.T, y[:n], "f32")[0]).any(1).sum())
        res["seconds"] = time.time() - t0
        for k in [k for k in res if k.startswith("_")]:
            del res[k]
        points.append(res)
        print(json.dumps(res), flush=True)
    summ = {"summary": True, "code": args.code,
            "ebn0_at_fer1e-3_i8": ebn0_at(points, "fer_i8"),
            "ebn0_at_fer1e-3_f32": ebn0_at(points, "fer_f32")}
    if summ["ebn0_at_fer1e-3_i8"] is not None and summ["ebn0_at_fer1e-3_f32"] is not None:
        summ["gap_db"] = summ["ebn0_at_fer1e-3_i8"] - summ["ebn0_at_fer1e-3_f32"]
    print(json.dumps(summ), flush=True)


if __name__ == "__main__":
    sys.exit(main())
