"""GPU parity: the HIP path through the C-ABI against the oracle, element by
element on the same seeded inputs.

Integer (int8 LLR) work is compared bit-exactly: stage-1 lists, CRC flags
and path metrics; stage-2 decisions, chosen paths, metrics and every logged
move index.  The float form is compared bit-exactly against the oracle's
binary32 mode (same summation order), and its metric within 1e-5 relative
of the double-precision distance.
"""
import dataclasses
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2602_08501_amd import decoder as D
from paper_2602_08501_amd import synth

from merge_rule import searched_counts

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
_codes = {}


def code(r, m):
    if (r, m) not in _codes:
        _codes[(r, m)] = D.Code(r, m, DEV)
    return _codes[(r, m)]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def unpack(t):
    return np.unpackbits(t.cpu().numpy(), axis=-1, bitorder="little")


def workload(wl, seed, F, f0=0):
    pay, c, y = synth.generate(wl, seed, f0, f0 + F)
    q = oracle.quantize(y, wl.llr_scale)
    return c, y, q


def run_gpu(wl, L, T, obs, dtype, crc=True, anchors=None, crc_ok=None, merge=True):
    cd = code(wl.r, wl.m)
    llr = torch.from_numpy(obs).to(DEV)
    if anchors is None:
        s1 = D.stage1(cd, L, llr, wl.crc_len if crc else 0, wl.crc_poly, want_pm=True)
        anchors, crc_ok = s1["anchors"], s1["crc_ok"]
    else:
        s1 = None
    st = D.Stage2([(cd, obs.shape[0])], L, T, dtype, DEV)
    out = st.run([llr], [anchors], [crc_ok], merge=merge)[0]
    torch.cuda.synchronize()
    return s1, out, st.stats.cpu().numpy()


# ---------------------------------------------------------------- quantizer
def test_quantizer_parity_and_nonfinite():
    say("case: quantizer")
    rng = np.random.default_rng(0)
    y = (rng.standard_normal(100003) * 4).astype(np.float32)
    y[:5] = [0.5 / 3.0, 1e30, -1e30, 63.5 / 3.0, -63.5 / 3.0]
    s = np.float32(3.0)
    bad = torch.zeros(1, dtype=torch.int32, device=DEV)
    q = D.quantize(torch.from_numpy(y).to(DEV), s, bad).cpu().numpy()
    assert np.array_equal(q, oracle.quantize(y, s))
    assert bad.item() == 0
    y2 = y.copy()
    y2[[7, 11, 13]] = [np.nan, np.inf, -np.inf]
    q2 = D.quantize(torch.from_numpy(y2).to(DEV), s, bad).cpu().numpy()
    assert bad.item() == 3 and q2[7] == q2[11] == q2[13] == 0
    # unaligned input and output (one value in): the same values element by element
    yd = torch.from_numpy(y2).to(DEV)
    bad.zero_()
    q3 = D.quantize(yd[1:], s, bad).cpu().numpy()
    assert np.array_equal(q3, q2[1:]) and bad.item() == 3
    out = torch.zeros(len(y2) + 1, dtype=torch.int8, device=DEV)
    D.quantize(yd, s, bad, out=out[1:])
    assert np.array_equal(out[1:].cpu().numpy(), q2)


# ---------------------------------------------------------------- stage 1
@pytest.mark.parametrize("wl,L,F", [(synth.RM37, 8, 640), (synth.RM38, 16, 40), (synth.RM26, 4, 333),
                                    (synth.RM27, 32, 24)])
@pytest.mark.parametrize("offset", [0, 1])
def test_stage1_quantized_equals_quantize_then_scl(wl, L, F, offset):
    """mpwsd_stage1_scl_quantized against mpwsd_quantize_llr + mpwsd_stage1_scl
    (int8): the fused launch for aligned buffers, the two-launch form for y and
    q one element off alignment; non-finite values included."""
    say("case: stage1 quantized", wl, L, F, "offset", offset)
    c, y, q_ref = workload(wl, 3, F)
    y = y.copy()
    y[1, [3, 77 % y.shape[1]]] = [np.nan, np.inf]
    y[F - 1, 5] = -np.inf
    n = y.size
    ybuf = torch.zeros(n + 8, dtype=torch.float32, device=DEV)
    ybuf[offset:offset + n] = torch.from_numpy(y.ravel()).to(DEV)
    yd = ybuf[offset:offset + n].view(y.shape)
    qbuf = torch.full((n + 8,), 99, dtype=torch.int8, device=DEV)
    qd = qbuf[offset:offset + n].view(y.shape)
    cd = code(wl.r, wl.m)
    bad = torch.zeros(1, dtype=torch.int32, device=DEV)
    got = D.stage1_quantized(cd, L, yd, wl.llr_scale, wl.crc_len, wl.crc_poly, q=qd, bad=bad, want_pm=True)
    bad2 = torch.zeros(1, dtype=torch.int32, device=DEV)
    q2 = D.quantize(yd.contiguous(), wl.llr_scale, bad2)
    ref = D.stage1(cd, L, q2, wl.crc_len, wl.crc_poly, want_pm=True)
    torch.cuda.synchronize()
    # non-finite values quantize to 0 (and are counted)
    assert np.array_equal(qd.cpu().numpy(), oracle.quantize(np.where(np.isfinite(y), y, 0.0), wl.llr_scale))
    assert np.array_equal(qd.cpu().numpy(), q2.cpu().numpy())
    assert bad.item() == bad2.item() == 3
    assert (qbuf[:offset] == 99).all() and (qbuf[offset + n:] == 99).all()
    for k in ("anchors", "crc_ok", "pm"):
        assert np.array_equal(got[k].cpu().numpy(), ref[k].cpu().numpy()), k


# the last two: a 16-bit CRC (x^16 + x^12 + x^5 + 1) and an 11-bit one (x^11 + x^10 + x^9 + x^5 + 1)
# whose test rows span every word of the decided bits
CRC16_RM37 = dataclasses.replace(synth.RM37, k_pay=48, crc_len=16, crc_poly=0x11021)
CRC11_RM38 = dataclasses.replace(synth.RM38, k_pay=82, crc_len=11, crc_poly=0xE21)


@pytest.mark.parametrize("wl,L,F", [(synth.RM26, 4, 300), (synth.RM37, 8, 256), (synth.RM27, 8, 128),
                                    (synth.RM38, 16, 24), (synth.RM37, 1, 64), (synth.RM37, 32, 16),
                                    (CRC16_RM37, 8, 256), (CRC11_RM38, 8, 48)])
@pytest.mark.parametrize("dtype", ["i8", "f32"])
def test_stage1_parity(wl, L, F, dtype):
    say("case: stage1", wl, L, F, dtype)
    c, y, q = workload(wl, 1, F)
    obs = q if dtype == "i8" else y
    cd = code(wl.r, wl.m)
    s1 = D.stage1(cd, L, torch.from_numpy(obs).to(DEV), wl.crc_len, wl.crc_poly, want_pm=True)
    torch.cuda.synchronize()
    anc = unpack(s1["anchors"])
    ok = s1["crc_ok"].cpu().numpy()
    pm = s1["pm"].cpu().numpy()
    fr = oracle.frozen_mask(wl.r, wl.m)
    A = oracle.rm_info_set(wl.r, wl.m)
    mode = oracle.INT if dtype == "i8" else oracle.F32
    for f in range(F):
        u, cc, opm = oracle.scl(wl.m, L, mode, obs[f].astype(np.float64), fr)
        assert np.array_equal(anc[f], cc), f
        if dtype == "i8":
            assert np.array_equal(pm[f], opm.astype(np.int32)), f
        else:
            assert np.array_equal(pm[f].view(np.float32), opm.astype(np.float32)), f
        assert ok[f] == oracle.crc_ok(u[0][A], wl.crc_len, wl.crc_poly), f



def test_stage1_unaligned_llr():
    # int8 q one byte off a 4-byte boundary takes the byte-wise channel staging;
    # the lists must be those of the aligned copy
    say("case: stage1 unaligned q")
    wl, L, F = synth.RM37, 8, 96
    c, y, q = workload(wl, 5, F)
    cd = code(wl.r, wl.m)
    qd = torch.from_numpy(q).to(DEV)
    buf = torch.zeros(F * wl.N + 1, dtype=torch.int8, device=DEV)
    buf[1:].copy_(qd.reshape(-1))
    q1 = buf[1:].view(F, wl.N)
    assert q1.data_ptr() % 4 == 1
    a = D.stage1(cd, L, qd, wl.crc_len, wl.crc_poly, want_pm=True)
    b = D.stage1(cd, L, q1, wl.crc_len, wl.crc_poly, want_pm=True)
    torch.cuda.synchronize()
    for key in ("anchors", "crc_ok", "pm"):
        assert torch.equal(a[key], b[key]), key


# ---------------------------------------------------------------- stage 2 (end to end)
E2E = [
    ("rm26_cfg", synth.RM26, 4, 4, 500),
    ("rm37_2dB", dataclasses.replace(synth.RM37, ebn0_db=2.0), 8, 8, 384),
    ("rm27", dataclasses.replace(synth.RM27, ebn0_db=2.0), 8, 8, 192),
    ("rm37_T1_L2", dataclasses.replace(synth.RM37, ebn0_db=1.5), 2, 1, 128),
    # the largest list and iteration count the library takes (L = 32, T = 64)
    ("rm26_L32_T64", dataclasses.replace(synth.RM26, ebn0_db=1.0), 32, 64, 80),
]


@pytest.mark.parametrize("name,wl,L,T,F", E2E, ids=[e[0] for e in E2E])
@pytest.mark.parametrize("dtype", ["i8", "f32"])
@pytest.mark.parametrize("merge", [True, False], ids=["merge", "nomerge"])
def test_decode_parity(name, wl, L, T, F, dtype, merge):
    say("case: decode", name, dtype, "merge" if merge else "no merge")
    c, y, q = workload(wl, 2, F)
    obs = q if dtype == "i8" else y
    s1, out, stats = run_gpu(wl, L, T, obs, dtype, merge=merge)
    mode = oracle.INT if dtype == "i8" else oracle.F32
    ref = oracle.decode_batch(wl.r, wl.m, wl.crc_len, wl.crc_poly, L, T, mode, obs.astype(np.float64), threads=8)
    assert np.array_equal(s1["crc_ok"].cpu().numpy(), ref["crc_ok"])
    assert np.array_equal(unpack(s1["anchors"]), ref["anchors"])
    nfail = int((ref["crc_ok"] == 0).sum())
    assert stats[0] == nfail and stats[-1] == 0
    assert stats[1] == nfail * L
    assert np.array_equal(out["moves"].cpu().numpy(), ref["logs"])
    assert np.array_equal(unpack(out["cw"]), ref["c"])
    assert np.array_equal(out["k"].cpu().numpy(), ref["k"])
    met = out["metric"].cpu().numpy()
    if dtype == "i8":
        assert np.array_equal(met, ref["metric"].astype(np.int32))
    else:
        assert np.array_equal(met.view(np.float32), ref["metric"].astype(np.float32))
        ed64 = np.array([oracle.metric(oracle.F64, y[f].astype(np.float64), ref["c"][f]) for f in range(F)])
        assert np.allclose(met.view(np.float32).astype(np.float64), ed64, rtol=1e-5, atol=0)
    # searched paths per iteration: the oracle's moved paths without merging,
    # one path per distinct centre of a frame with it
    fail = ref["crc_ok"] == 0
    logs = ref["logs"][fail]
    if merge:
        supp = oracle.moves(wl.r, wl.m)[0]
        assert np.array_equal(stats[1:1 + T], searched_counts(ref["anchors"][fail], logs, supp))
    else:
        for t in range(1, T):
            assert stats[1 + t] == int((logs[:, :, t - 1] >= 0).sum())
    say("  failing frames", nfail, "searched per iteration", stats[1:1 + T].tolist())


def test_always_on_no_crc():
    wl = dataclasses.replace(synth.RM26, crc_len=6)
    c, y, q = workload(wl, 3, 64)
    s1, out, stats = run_gpu(wl, 4, 3, q, "i8", crc=False)
    ref = oracle.decode_batch(wl.r, wl.m, 0, wl.crc_poly, 4, 3, oracle.INT, q.astype(np.float64))
    assert stats[0] == 64 and (s1["crc_ok"].cpu().numpy() == 0).all()
    assert np.array_equal(out["moves"].cpu().numpy(), ref["logs"])
    assert np.array_equal(unpack(out["cw"]), ref["c"])


def test_all_frames_decided_by_stage1():
    wl = dataclasses.replace(synth.RM37, ebn0_db=8.0)
    c, y, q = workload(wl, 4, 200)
    s1, out, stats = run_gpu(wl, 8, 4, q, "i8")
    assert stats[0] == 0 and (s1["crc_ok"].cpu().numpy() == 1).all()
    assert np.array_equal(unpack(out["cw"]), c)
    assert (out["k"].cpu().numpy() == 0).all() and (out["moves"].cpu().numpy() == -1).all()


def test_empty_batch():
    cd = code(3, 7)
    st = D.Stage2([(cd, 0)], 8, 8, "i8", DEV)
    llr = torch.zeros((0, 128), dtype=torch.int8, device=DEV)
    anc = torch.zeros((0, 8, 16), dtype=torch.uint8, device=DEV)
    st.run([llr], [anc], [None])
    torch.cuda.synchronize()


# ---------------------------------------------------------------- pins on the device
@pytest.mark.parametrize("m", [5, 7, 8])
def test_rm1_reaches_ml(m):
    """Sphere of RM(1, m) covers the code within two moves: T = 2 reaches ML."""
    say("case: rm1 ML", m)
    rng = np.random.default_rng(40 + m)
    n, F, L = 1 << m, 48, 3
    K = m + 1
    A = oracle.rm_info_set(1, m)
    ys, anchors = [], []
    for f in range(F):
        u = np.zeros(n, np.uint8)
        u[A] = rng.integers(0, 2, K)
        ys.append(1 - 2.0 * oracle.encode(m, u) + rng.standard_normal(n) * 1.3)
        for k in range(L):
            u = np.zeros(n, np.uint8)
            u[A] = rng.integers(0, 2, K)
            anchors.append(oracle.encode(m, u))
    q = np.clip(np.rint(np.array(ys) * 9), -127, 127).astype(np.int8)
    anc = torch.from_numpy(np.packbits(np.array(anchors).reshape(F, L, n), axis=-1, bitorder="little")).to(DEV)
    wl = synth.Workload(r=1, m=m, k_pay=K)
    _, out, stats = run_gpu(wl, L, 2, q, "i8", anchors=anc, crc_ok=None)
    met = out["metric"].cpu().numpy()
    for f in range(F):
        e_ml, _ = oracle.ml(1, m, oracle.INT, q[f].astype(np.float64))
        assert met[f] == e_ml


def test_single_move_recovery_pins_indices():
    say("case: single move recovery")
    rng = np.random.default_rng(5)
    cd = code(3, 7)
    supp, w = oracle.moves(3, 7)
    A = oracle.rm_info_set(3, 7)
    F, n = 96, 128
    p0 = rng.choice(cd.P, F, replace=False)
    p0[:3] = [0, cd.P - 1, cd.P - 25]  # first, last and the ragged tail chunk
    cs, anchors = [], []
    for f in range(F):
        u = np.zeros(n, np.uint8)
        u[A] = rng.integers(0, 2, len(A))
        c0 = oracle.encode(7, u)
        a = c0.copy()
        a[supp[p0[f]]] ^= 1
        cs.append(c0)
        anchors.append(a)
    q = (20 * (1 - 2.0 * np.array(cs))).astype(np.int8)
    anc = torch.from_numpy(np.packbits(np.array(anchors)[:, None, :], axis=-1, bitorder="little")).to(DEV)
    _, out, _ = run_gpu(synth.RM37, 1, 3, q, "i8", anchors=anc, crc_ok=None)
    mv = out["moves"].cpu().numpy()
    assert np.array_equal(mv[:, 0, 0], p0)
    assert (mv[:, 0, 1:] == -1).all()
    assert np.array_equal(unpack(out["cw"]), np.array(cs))


def test_repeat_runs_identical():
    wl = dataclasses.replace(synth.RM37, ebn0_db=2.0)
    c, y, q = workload(wl, 6, 512)
    a = run_gpu(wl, 8, 8, q, "i8")[1]
    b = run_gpu(wl, 8, 8, q, "i8")[1]
    for key in a:
        assert torch.equal(a[key], b[key])
