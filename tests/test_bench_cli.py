"""bench.py without a GPU: the one-GPU rule, the workload table, and the
machine-readable traffic line of the committed counter summary."""
import argparse
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2602_08501_amd import synth  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _args(**kw):
    d = dict(workload="rm37", osd_order=2, frames=0, ebn0=None)
    d.update(kw)
    return argparse.Namespace(**d)


@pytest.mark.parametrize("name,codes,frames,L,T,radius,osd", [
    ("rm37", [(3, 7)], [65536], 8, 8, 1, None),
    ("rm38", [(3, 8)], [32768], 16, 12, 1, None),
    ("mixed", [(2, 6), (2, 7), (3, 7)], [87382, 87381, 87381], 8, 8, 1, None),
    ("rm26", [(2, 6)], [65536], 8, 8, 1, None),
    ("rm26s2", [(2, 6)], [65536], 8, 8, 2, None),
    ("rm27osd", [(2, 7)], [65536], 8, 4, 1, 2),
])
def test_workloads(name, codes, frames, L, T, radius, osd):
    segs, l, t, rad, o = bench.workload(_args(workload=name), synth)
    assert [(w.r, w.m) for w, _ in segs] == codes
    assert [f for _, f in segs] == frames
    assert (l, t, rad, o) == (L, T, radius, osd)
    if name == "mixed":
        assert all(w.ebn0_db == 2.5 for w, _ in segs)
    if name == "rm27osd":
        assert segs[0][0].crc_len == 0


def test_frames_and_ebn0_overrides():
    segs, *_ = bench.workload(_args(workload="mixed", frames=3000, ebn0=3.0), synth)
    assert [f for _, f in segs] == [1000, 1000, 1000]
    assert all(w.ebn0_db == 3.0 for w, _ in segs)


def test_traffic_line_parses():
    text = open(os.path.join(ROOT, "profiles", "search_pw_rm37_65536f_hbm_traffic.txt")).read()
    m = re.search(r"bench-traffic: source=(\S+) sha256=([0-9a-f]{64}) hbm_bytes_per_launch=(\d+)", text)
    assert m and os.path.exists(os.path.join(ROOT, m.group(1)))
    assert 1e6 < int(m.group(3)) < 1e9
    # only the batch the counters were taken on
    assert bench.recorded_traffic(_args(workload="rm38")) is None
    assert bench.recorded_traffic(_args(frames=8192)) is None
    assert bench.recorded_traffic(_args(ebn0=3.0)) is None
