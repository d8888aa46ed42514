"""Benchmark: decoded frames/s of the two-stage MP-WSD decoder on one GPU.

One step = the whole decoder over one batch resident in HBM: int8 LLR
quantization and stage-1 SC-list decoding with the CRC test (one launch;
quantization on its own before OSD), compaction of the
failing frames, T iterations of the stage-2 move search / apply, and the
final choice.  The step is recorded once as a HIP graph and replayed.  By
default three batches are in flight: each has its own buffers and its own
graph on its own stream, and the steps are replayed round-robin, so that the
GPU fills one batch's idle time (the small, latency-bound late stage-2
launches) with another's work; the default 48 steps give every stream the
same number of replays.  ms_per_step is the timed span over the K steps divided by K;
ms_per_step_one_in_flight is the same with one batch at a time (one step's
latency).  Afterwards every batch's outputs must equal the first batch's.

Default workload (the metric's): RM(3,7) (N=128, K=64 = 58 payload + CRC-6),
BPSK over AWGN at Eb/N0 = 2.5 dB, 65536 frames, int8 LLRs (scale 8/sigma^2),
L = 8 anchors, T = 8 iterations, 94488 moves (seeded synthetic data).
Other workloads: --workload rm38 (RM(3,8), 32768 frames at 2.0 dB, L=16,
T=12, 777240 moves), --workload mixed (262144 frames, RM(2,6) / RM(2,7)
/ RM(3,7) in equal shares at 2.5 dB, L=8, T=8, all codes' failing frames in
one search launch per iteration), --workload rm26 (65536 RM(2,6) frames at
3.0 dB, L=8, T=8, 2604 moves), --workload rm26s2 (the same frames with the
sphere of radius 2: 2604 + 291648 moves) and --workload rm27osd (65536
RM(2,7) frames at 2.5 dB without CRC, OSD(k) stage 1 with L=8 anchors, stage
2 on every frame, T=4, 10668 moves).

Prints one JSON line.  The roofline entry is for the stage-2 move-search
kernel: the method's own work per searched path and iteration, P w adds and
P compares (w the mean move weight), over that kernel's launch durations
measured with HIP events on the stream it runs on, against the int8 matrix
core peak that carries it.  Two more counts sit beside it: "executed", the
int8 MFMA operations the kernel issues (rows of N/2 against both halves for
the paired-half tables of RM(3,7) and RM(3,8), rows of N otherwise), and
"dense_equivalent", 2 P N per path, the dense product W Z.  The CPU
baseline is the test oracle on bounded samples of the same frames, on one
core and on all the cores it may use.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MI355X_INT8_DENSE_TOPS = 5000.0  # AMD published dense int8 MFMA peak (TOP/s)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=48)
    ap.add_argument("--warmup", type=int, default=6)
    ap.add_argument("--workload", default="rm37", choices=["rm37", "rm38", "mixed", "rm26", "rm26s2", "rm27osd"])
    ap.add_argument("--osd-order", type=int, default=2, help="OSD order k of the rm27osd workload")
    ap.add_argument("--frames", type=int, default=0, help="override the workload's frame count")
    ap.add_argument("--ebn0", type=float, default=None, help="override the workload's Eb/N0")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-frames", type=int, default=-1,
                    help="oracle sample size in frames on all cores, one eighth of it on one core (0 = skip; "
                         "default: up to 32768, 2048 for rm38)")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--in-flight", type=int, default=3,
                    help="batches decoded at once, each step's graph on its own stream (1 = one after another)")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="first run one device-to-device copy of this many MiB (a reference dispatch of "
                         "known traffic for hardware counters)")
    return ap.parse_args()


def workload(args, synth):
    """[(Workload, frames)], L, T, sphere radius of the move tables, OSD order
    of stage 1 (None: SCL with the CRC)."""
    if args.workload == "rm27osd":
        wl = synth.Workload(r=2, m=7, k_pay=29, crc_len=0, ebn0_db=2.5, wid=4)
        segs, L, T = [(wl, 65536)], 8, 4
    elif args.workload == "rm37":
        segs, L, T = [(synth.RM37, 65536)], 8, 8
    elif args.workload == "rm38":
        segs, L, T = [(synth.RM38, 32768)], 16, 12
    elif args.workload in ("rm26", "rm26s2"):
        segs, L, T = [(synth.RM26, 65536)], 8, 8
    else:
        segs = [(dataclasses.replace(w, ebn0_db=2.5), f)
                for w, f in ((synth.RM26, 87382), (synth.RM27, 87381), (synth.RM37, 87381))]
        L, T = 8, 8
    if args.ebn0 is not None:
        segs = [(dataclasses.replace(w, ebn0_db=args.ebn0), f) for w, f in segs]
    if args.frames:
        segs = [(w, max(1, args.frames // len(segs))) for w, f in segs]
    radius = 2 if args.workload == "rm26s2" else 1
    osd = args.osd_order if args.workload == "rm27osd" else None
    return segs, L, T, radius, osd


def recorded_traffic(args):
    """HBM bytes per search launch from the committed counter summary, or None
    when the kernel source changed since the counters were taken, or there is
    no summary for this workload (the counters were taken on the default
    RM(3,7) batch: no other workload, frame count or Eb/N0)."""
    import hashlib
    import re
    if args.workload != "rm37" or args.frames or args.ebn0 is not None:
        return None
    path = os.path.join(ROOT, "profiles", "search_pw_rm37_65536f_hbm_traffic.txt")
    try:
        m = re.search(r"bench-traffic: source=(\S+) sha256=(\w+) hbm_bytes_per_launch=(\d+)", open(path).read())
        src = open(os.path.join(ROOT, m.group(1)), "rb").read()
    except (OSError, AttributeError):
        return None
    if hashlib.sha256(src).hexdigest() != m.group(2):
        return None
    return int(m.group(3))


def cpu_baseline(segs, ys, L, T, nframes, threads, radius=1, osd=None):
    """The oracle on the first frames of every code's batch (the sample split
    evenly over the codes), int8 arithmetic, whole two-stage decode, with
    `threads` threads (one frame per task)."""
    import oracle
    qs, parts = [], []
    for (wl, F), y in zip(segs, ys):
        n = min(max(1, nframes // len(segs)), len(y))
        qs.append(oracle.quantize(y[:n], wl.llr_scale).astype(np.float64))
        oracle.moves(wl.r, wl.m) if radius == 1 else oracle.sphere(wl.r, wl.m, radius)  # built outside the timing
        parts.append("%d RM(%d,%d)" % (n, wl.r, wl.m))
    t0 = time.perf_counter()
    for (wl, F), q in zip(segs, qs):
        if osd is None:
            oracle.decode_batch(wl.r, wl.m, wl.crc_len, wl.crc_poly, L, T, oracle.INT, q, threads=threads,
                                radius=radius)
        else:
            oracle.decode_osd_batch(wl.r, wl.m, osd, L, T, oracle.INT, q, threads=threads, radius=radius)
    dt = time.perf_counter() - t0
    n = sum(len(q) for q in qs)
    return {"value": n / dt, "unit": "decoded frames/s", "cores": threads, "kind": "oracle",
            "sample": "first %s frames of the batch (int8 LLRs, full two-stage decode), %.1f s wall"
                      % (" + ".join(parts), dt)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: measures one GPU only (--gpus %d requested); "
              "the decoder shards by frame with no communication between GPUs" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2602_08501_amd import _lib, autotune, complexity
    from paper_2602_08501_amd import decoder as D
    from paper_2602_08501_amd import synth

    segs, L, T, radius, osd = workload(args, synth)
    dev = "cuda:0"
    stream = torch.cuda.Stream()
    if args.calib_copy > 0:
        src = torch.ones(args.calib_copy << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    codes, ys, txs, y_d = [], [], [], []
    for wl, F in segs:
        pay, c_tx, y = synth.generate(wl, args.seed, 0, F)
        code = D.Code(wl.r, wl.m, dev, radius=radius)
        codes.append(code)
        ys.append(y)
        txs.append(c_tx)
        y_d.append(torch.from_numpy(y).to(dev))
    F_total = sum(F for _, F in segs)
    nseg = len(segs)
    B = args.in_flight
    if B < 1:
        sys.exit("bench.py: --in-flight must be at least 1")

    class Batch:
        """The buffers of one batch in flight: int8 LLRs, stage-1 outputs and
        the stage-2 outputs and workspace (the input y is shared, read-only)."""

        def __init__(self):
            self.q = [torch.empty(y.shape, dtype=torch.int8, device=dev) for y in ys]
            self.s1 = [{"anchors": torch.empty((F, L, c.N // 8), dtype=torch.uint8, device=dev),
                        "crc_ok": torch.empty(F, dtype=torch.uint8, device=dev)} for c, (_, F) in zip(codes, segs)]
            self.st = D.Stage2([(c, F) for c, (_, F) in zip(codes, segs)], L, T, "i8", dev, want_moves=False)
            # OSD has no CRC: stage 2 runs on every frame (always-on mode)
            self.crc_oks = [None if osd is not None else s["crc_ok"] for s in self.s1]
            self.anchors = [s["anchors"] for s in self.s1]

        def stage1(self, raw=None):
            for i, (wl, F) in enumerate(segs):
                kw = {"stream": stream} if raw is None else {"raw_stream": raw}
                if osd is None:
                    # quantizer and SCL in one launch (the int8 values also go to q for stage 2)
                    D.stage1_quantized(codes[i], L, y_d[i], float(wl.llr_scale), wl.crc_len, wl.crc_poly,
                                       q=self.q[i], out=self.s1[i], **kw)
                else:
                    D.quantize(y_d[i], float(wl.llr_scale), out=self.q[i], **kw)
                    D.stage1_osd(codes[i], osd, L, self.q[i], out=self.s1[i], **kw)

        def stage2(self, events=None, variant=-1, bpc=0, raw=None):
            self.st.run(self.q, self.anchors, self.crc_oks, stream=None if raw else stream,
                        events=events, variant=variant, blocks_per_cu=bpc, raw_stream=raw)

    batches = [Batch() for _ in range(B)]
    b0 = batches[0]
    st, q_d, s1, crc_oks = b0.st, b0.q, b0.s1, b0.crc_oks

    with torch.cuda.stream(stream):
        b0.stage1()
        b0.stage2()
        torch.cuda.synchronize()
        variant, bpc = autotune.tune(st, q_d, b0.anchors, crc_oks, stream=stream, use_cache=False)

        # the whole step recorded once per batch in flight as a HIP graph; the
        # steps are replayed round-robin on one stream per batch, so that up
        # to B batches are decoded at once (the GPU fills the idle time of one
        # batch's small late launches and launch gaps with another's work)
        def record(b, raw):
            b.stage1(raw)
            b.stage2(variant=variant, bpc=bpc, raw=raw)

        graphs = [D.Graph(lambda raw, b=b: record(b, raw)) for b in batches]
        streams = [stream] + [torch.cuda.Stream() for _ in range(B - 1)]
        ran = set()  # batches whose graph has run (fewer than B when W + K < B)

        def timed(nb, steps):
            """steps replays round-robin over the first nb batches; returns
            ms per step between events that bracket every stream."""
            torch.cuda.synchronize()
            t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0.record(streams[0])
            for s in streams[1:nb]:
                s.wait_event(t0)
            for k in range(steps):
                graphs[k % nb].launch(streams[k % nb])
                ran.add(k % nb)
            for s in streams[1:nb]:
                e = torch.cuda.Event()
                e.record(s)
                streams[0].wait_event(e)
            t1.record(streams[0])
            torch.cuda.synchronize()
            return t0.elapsed_time(t1) / steps

        for k in range(args.warmup):
            graphs[k % B].launch(streams[k % B])
            ran.add(k % B)
        torch.cuda.synchronize()
        wall0 = time.perf_counter()
        ms = timed(B, args.steps)
        wall = time.perf_counter() - wall0
        # one batch at a time (the latency of one step)
        ms_serial = timed(1, args.steps) if B > 1 else ms
        # every batch in flight decoded the same frames: the same outputs
        # (batch 0 also ran eagerly before the graphs were recorded)
        for b in (batches[i] for i in sorted(ran) if i > 0):
            for x, y in zip(b.st.outs, st.outs):
                for k in x:
                    assert torch.equal(x[k], y[k]), k
            for x, y in zip(b.s1, s1):
                for k in x:
                    assert torch.equal(x[k], y[k]), k

        # the same steps launched one by one with HIP events around every
        # search launch (its durations for the roofline entry)
        nev = 2 * T * nseg
        evs = []
        for _ in range(args.steps):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(nev)]
            for x in e:
                x.record(stream)
            evs.append(e)
        torch.cuda.synchronize()
        e_start, e_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e_start.record(stream)
        for k in range(args.steps):
            b0.stage1()
            b0.stage2(evs[k], variant, bpc)
        e_end.record(stream)
        torch.cuda.synchronize()
        ms_eager = e_start.elapsed_time(e_end) / args.steps

    # searched paths per iteration and segment (deterministic per segment)
    per_seg_stats = []
    for i, (wl, F) in enumerate(segs if nseg > 1 else []):
        one = D.Stage2([(codes[i], F)], L, T, "i8", dev, want_moves=False)
        one.run([q_d[i]], [s1[i]["anchors"]], [crc_oks[i]])
        torch.cuda.synchronize()
        per_seg_stats.append(one.stats.cpu().numpy().astype(np.int64))
    stats = st.stats.cpu().numpy()
    if nseg == 1:
        per_seg_stats = [stats.astype(np.int64)]
    per_seg_cols = [x[1:1 + T] for x in per_seg_stats]
    ed_units = [complexity.report(c.N, c.K, c.P, c.w, L, T, F, int(x[0]), x[1:1 + T].tolist(),
                                  ms if nseg == 1 else None,
                                  c_init=None if osd is None else float(complexity.c_osd(c.K, osd)))
                for c, (_, F), x in zip(codes, segs, per_seg_stats)]
    launches = np.array([[evs[k][2 * t].elapsed_time(evs[k][2 * t + 1]) for t in range(T)]
                         for k in range(args.steps)]).mean(0)
    secs = launches.sum() * 1e-3
    # the method's work per searched path and iteration: P w adds + P compares
    alg_per_path = [c.P * (c.w + 1.0) for c in codes]
    alg_ops = sum(a * cols for a, cols in zip(alg_per_path, per_seg_cols))  # per launch
    achieved = float(alg_ops.sum() / secs / 1e12)
    dense_per_path = [2.0 * c.P * c.N for c in codes]
    dense_ops = sum(d * cols for d, cols in zip(dense_per_path, per_seg_cols))
    dense = float(dense_ops.sum() / secs / 1e12)
    # int8 MFMA work the kernels execute: a paired-half table runs rows of N/2
    # against both halves (chunks * 128 rows * 2 * N/2 MACs per path), the
    # plain table N-long rows padded to 128-move chunks
    exec_per_path = [(2.0 * c.grouped_chunks * 128 * 2 * (c.N // 2)) if c.grouped is not None
                     else (2.0 * -(-c.P // 128) * 128 * max(c.N, 64)) for c in codes]
    exec_ops = sum(e * cols for e, cols in zip(exec_per_path, per_seg_cols))
    executed = float(exec_ops.sum() / secs / 1e12)
    fer, fer1 = [], []
    for i in range(nseg):
        cw = np.unpackbits(st.outs[i]["cw"].cpu().numpy(), axis=-1, bitorder="little")
        fer.append(float((cw != txs[i]).any(1).mean()))
        a0 = np.unpackbits(s1[i]["anchors"][:, 0].cpu().numpy(), axis=-1, bitorder="little")
        fer1.append(float((a0 != txs[i]).any(1).mean()))
    move_evals = float(sum(c.P * cols.sum() for c, cols in zip(codes, per_seg_cols)))
    names = ["RM(%d,%d) N=%d P=%d%s Eb/N0 %.2f dB %d frames"
             % (w.r, w.m, c.N, c.P, " (sphere S_%d)" % radius if radius > 1 else "", w.ebn0_db, F)
             for (w, F), c in zip(segs, codes)]
    res = {
        "metric": "decoded frames/sec at FER parity; stage-2 move-evals/sec (% int8 MFMA peak)",
        "value": F_total / (ms * 1e-3),
        "unit": "decoded frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "batches_in_flight": B,
        "ms_per_step_one_in_flight": ms_serial,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",
        "data": "synthetic (seeded BPSK/AWGN frames, random payloads)",
        "config": {"workload": "; ".join(names) + "; int8 LLRs, %s, T=%d"
                               % ("SCL L=%d with CRC-6" % L if osd is None
                                  else "OSD(%d) L=%d, no CRC, stage 2 always on" % (osd, L), T),
                   "frames": F_total, "stage2_frames": int(stats[0]), "p_act": int(stats[0]) / F_total,
                   "paths_searched_per_iteration": stats[1:1 + T].tolist(), "fer": fer,
                   "fer_stage1_first_anchor": fer1},
        "stage2_move_evals_per_s": move_evals / (launches.sum() * 1e-3),
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": MI355X_INT8_DENSE_TOPS, "unit": "TOP/s",
                     "frac": achieved / MI355X_INT8_DENSE_TOPS, "traffic": recorded_traffic(args),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0 KiB)",
                     "kernel": ("search_i8_multi_kernel" if nseg > 1 else
                                "search_pw_kernel" if codes[0].grouped is not None else "search_i8_kernel"),
                     "launch_ms": launches.tolist(),
                     "searched_paths_per_launch": [int(x) for x in sum(per_seg_cols)],
                     "work_per_launch": "P*w adds + P compares per searched path (the method's count)",
                     "ops_per_path": alg_per_path,
                     "executed": {"achieved": executed, "frac": executed / MI355X_INT8_DENSE_TOPS,
                                  "ops_per_path": exec_per_path,
                                  "note": "int8 MFMA ops the kernel issues (2 per MAC)"},
                     "dense_equivalent": {"achieved": dense, "frac": dense / MI355X_INT8_DENSE_TOPS,
                                          "ops_per_path": dense_per_path,
                                          "note": "2*P*N per path: the dense product W Z"}},
        "complexity_ed_units": ed_units if nseg > 1 else ed_units[0],
        "wall_s": wall,
        "ms_per_step_eager": ms_eager,
        "search_tiles": [{"iteration": t, "variant": v, "blocks_per_cu": b,
                          **{k: x for k, x in _lib.mpwsd_search_variants()[v].items() if k != "blocks_per_cu"}}
                         for t, (v, b) in enumerate(zip(variant, bpc))],
    }
    if args.cpu_frames < 0:
        args.cpu_frames = {"rm38": 2048, "rm26s2": 4096, "rm27osd": 8192}.get(args.workload, min(F_total, 32768))
    if args.cpu_frames > 0:
        # all the cores this process may use (at most 16 threads: the host CPU
        # share of one GPU), and one core on a smaller sample
        avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        thr = args.cpu_threads or min(16, avail)
        cb = cpu_baseline(segs, ys, L, T, args.cpu_frames, thr, radius, osd)
        one = cpu_baseline(segs, ys, L, T, max(1, args.cpu_frames // 8), 1, radius, osd)
        cb.update({"host_cpus": os.cpu_count(), "affinity_cpus": avail,
                   "single_core": {"value": one["value"], "unit": one["unit"], "cores": 1, "sample": one["sample"]}})
        res["cpu_baseline"] = cb
    print(json.dumps(res))


if __name__ == "__main__":
    main()
