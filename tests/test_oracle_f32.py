"""Pins for the oracle's binary32 mode.

The float form of the decoder (Sec. III-A SCL, Sec. III-B Eq. (4)-(5) and
Alg. 1, and the OSD list of Sec. III-A / IV-A) is specified bit for bit in
IEEE single precision: every sum, difference and square is rounded to
binary32, and sums run in ascending position order.  The oracle evaluates it
by holding values in doubles and rounding after every operation.  Here the
same quantities are computed a second, independent way, with numpy float32
scalars and arrays, whose every +, - and * is itself a single-precision
operation, written from the definitions:

* metric:  ED(c) = sum_j (y_j - x_j(c))^2, each difference, square and
  partial sum in float32, ascending j (small channel values make the
  rounding of the difference itself matter);
* stage 2: z = y x(c); S_p = float32 sum of z over supp(w_p), ascending
  positions; p* = the first index attaining the minimum; the move is taken
  iff S_p* < 0; a path that finds none stops;
* SCL:     f = sgn(a) sgn(b) min(|a|, |b|) (exact), g = b + (1 - 2v) a in
  float32, PM += |l| in float32 on disagreement, children ranked by
  (PM, parent slot, bit), computed top-down over the halves of the
  Kronecker generator;
* OSD of order K: the list is the L codewords of smallest float32 metric.

The inputs put channel magnitudes near 2^23, where float32 values are spaced
one apart and sums of a few of them round, and the stage-2 inputs add one
entry of 2^21.  Each test asserts that binary32 and binary64 then reach
different decisions or values on part of the sample, so a rounding the
oracle dropped, added or moved, or a sum taken in another order, changes its
output and fails the comparison.
"""
import numpy as np
import pytest

import oracle


def _f32(x):
    return np.asarray(x, np.float64).astype(np.float32)


def near_2p23(rng, n):
    """float32 channel values of magnitude 2^23 + [0, 16), random signs."""
    mag = (2 ** 23 + rng.integers(0, 16, n)).astype(np.float64)
    return _f32(rng.choice([-1.0, 1.0], n) * mag)


def generator(m):
    """F^{(x)m}, F = [[1,0],[1,1]], built with np.kron (natural order)."""
    G = np.ones((1, 1), np.int64)
    for _ in range(m):
        G = np.kron(G, np.array([[1, 0], [1, 1]], np.int64))
    return G


def info_positions(r, m):
    return np.array([i for i in range(1 << m) if bin(i).count("1") >= m - r])


def codeword(r, m, rng):
    u = np.zeros(1 << m, np.int64)
    u[info_positions(r, m)] = rng.integers(0, 2, len(info_positions(r, m)))
    return (u @ generator(m) % 2).astype(np.uint8)


# ---------------------------------------------------------------- numpy forms
def np_metric(y, c, dt):
    y = np.asarray(y, dt)
    x = np.where(np.asarray(c) == 1, dt(-1), dt(1))
    d = y - x
    sq = d * d
    e = dt(0)
    for v in sq:
        e = dt(e + v)
    return e


def np_stage2_path(supp, y, c, T, dt):
    """One MP-WSD path in dtype dt (Sec. III-B, Eq. (5))."""
    y = np.asarray(y, dt)
    c = np.array(c, np.uint8)
    valid = supp != oracle.SUPP_END
    idx = np.where(valid, supp, 0).astype(np.int64)
    log = []
    active = True
    for _ in range(T):
        if not active:
            log.append(-1)
            continue
        z = np.where(c == 1, -y, y)
        s = np.zeros(len(supp), dt)
        for i in range(supp.shape[1]):
            s = s + np.where(valid[:, i], z[idx[:, i]], dt(0))
        p = int(np.argmin(s))
        if s[p] < 0:
            c[idx[p][valid[p]]] ^= 1
            log.append(p)
        else:
            log.append(-1)
            active = False
    return c, np.array(log, np.int32)


def np_stage2_frame(supp, y, anchors, T, dt):
    paths, logs, met = [], [], []
    for a in anchors:
        c, lg = np_stage2_path(supp, y, a, T, dt)
        paths.append(c)
        logs.append(lg)
        met.append(np_metric(y, c, dt))
    met = np.array(met, dt)
    return np.array(paths), np.array(logs), met, int(np.argmin(met))


def np_scl(m, L, y, frozen, dt):
    """Min-sum SCL(L) in dtype dt; returns (u, c, pm) in (PM, slot) order."""
    n = 1 << m
    y = np.asarray(y, dt)
    G = generator(m)

    def leaf(u, i):
        l, uu, k, size = y, u, i, n
        while size > 1:
            h = size // 2
            a, b = l[:h], l[h:]
            if k < h:
                sgn = np.where(a < 0, dt(-1), dt(1)) * np.where(b < 0, dt(-1), dt(1))
                l = sgn * np.minimum(np.abs(a), np.abs(b))
                uu = uu[:h]
            else:
                lev = h.bit_length() - 1
                v = (uu[:h].astype(np.int64) @ generator(lev) % 2).astype(bool)
                l = np.where(v, b - a, b + a)
                uu = uu[h:]
                k -= h
            size = h
        return l[0]

    paths = [(np.zeros(n, np.uint8), dt(0))]
    for i in range(n):
        lam = [leaf(u, i) for u, _ in paths]
        if frozen[i]:
            paths = [(u, dt(pm + abs(lm)) if lm < 0 else pm) for (u, pm), lm in zip(paths, lam)]
            continue
        kids = []
        for s, ((u, pm), lm) in enumerate(zip(paths, lam)):
            hd = 1 if lm < 0 else 0
            for b in (0, 1):
                kids.append((pm if b == hd else dt(pm + abs(lm)), s, b))
        kids.sort(key=lambda t: (t[0], t[1], t[2]))
        nxt = []
        for pm, s, b in kids[:L]:
            u = paths[s][0].copy()
            u[i] = b
            nxt.append((u, pm))
        paths = nxt
    order = sorted(range(len(paths)), key=lambda s: (paths[s][1], s))
    u = np.array([paths[s][0] for s in order])
    c = (u.astype(np.int64) @ G % 2).astype(np.uint8)
    pm = np.array([paths[s][1] for s in order], np.float64)
    return u, c, pm


# ---------------------------------------------------------------- tests
def test_metric_binary32():
    rng = np.random.default_rng(3)
    n_diff = 0
    n_d = 0
    for trial in range(40):
        n = 128
        lo, hi = (-3, 12) if trial % 2 else (-14, 0)
        y = _f32(rng.standard_normal(n) * 2.0 ** rng.uniform(lo, hi, n))
        c = rng.integers(0, 2, n).astype(np.uint8)
        got = oracle.metric(oracle.F32, y.astype(np.float64), c)
        ref = np_metric(y, c, np.float32)
        assert got == float(ref)
        assert np_metric(y, c, np.float64) == oracle.metric(oracle.F64, y.astype(np.float64), c)
        n_diff += got != oracle.metric(oracle.F64, y.astype(np.float64), c)
        # a variant that keeps each difference y_j - x_j unrounded
        x = np.where(c == 1, -1.0, 1.0)
        d64 = y.astype(np.float64) - x
        e = np.float32(0)
        for v in d64 * d64:
            e = np.float32(e + np.float32(v))
        n_d += e != ref
    assert n_diff >= 30
    assert n_d >= 3


@pytest.mark.parametrize("r,m,radius", [(2, 6, 1), (1, 5, 2), (2, 5, 1)])
def test_stage2_binary32(r, m, radius):
    rng = np.random.default_rng(10 + m + radius)
    supp, w = oracle.moves(r, m) if radius == 1 else oracle.sphere(r, m, radius)
    n = 1 << m
    n_diff = 0
    for trial in range(24):
        anchors = np.array([codeword(r, m, rng) for _ in range(3)])
        if trial % 2:
            y = near_2p23(rng, n)
        else:
            y = _f32((1 - 2.0 * anchors[0]) * rng.standard_normal(n) * 3)
            j0 = supp[rng.integers(len(supp)), 0]
            y[j0] = _f32(-(1 - 2.0 * anchors[0][j0]) * 2.0 ** 21)
        yd = y.astype(np.float64)
        paths, logs, met, kb = oracle.stage2_frame(oracle.F32, supp, yd, anchors, 4)
        rp, rl, rm, rk = np_stage2_frame(supp, y, anchors, 4, np.float32)
        assert np.array_equal(logs, rl)
        assert np.array_equal(paths, rp)
        assert np.array_equal(met, rm.astype(np.float64))
        assert kb == rk
        p64, l64, m64, k64 = oracle.stage2_frame(oracle.F64, supp, yd, anchors, 4)
        n_diff += not np.array_equal(l64, logs)
    assert n_diff >= 3


@pytest.mark.parametrize("r,m,L", [(1, 3, 2), (1, 4, 4), (2, 4, 4), (2, 5, 8), (2, 6, 4)])
def test_scl_binary32(r, m, L):
    rng = np.random.default_rng(20 + r + m)
    n = 1 << m
    frozen = np.ones(n, np.uint8)
    frozen[info_positions(r, m)] = 0
    n_list = n_pm = 0
    trials = 16 if m <= 5 else 6
    for trial in range(trials):
        y = near_2p23(rng, n) if trial % 4 else _f32(rng.standard_normal(n) * 2.0 ** rng.uniform(-3, 12, n))
        yd = y.astype(np.float64)
        u, c, pm = oracle.scl(m, L, oracle.F32, yd, frozen)
        ru, rc, rpm = np_scl(m, L, y, frozen, np.float32)
        assert np.array_equal(u, ru)
        assert np.array_equal(c, rc)
        assert np.array_equal(pm, rpm)
        u64, c64, pm64 = oracle.scl(m, L, oracle.F64, yd, frozen)
        n_list += not np.array_equal(u64, u)
        n_pm += not np.array_equal(pm64, pm)
    assert n_pm >= trials // 2
    if m >= 4:
        assert n_list >= 1


def test_scl_binary64_matches_numpy_double():
    """The same numpy form in float64 reproduces the oracle's binary64 mode,
    so the comparison above tests the rounding and nothing else."""
    rng = np.random.default_rng(29)
    r, m, L = 2, 5, 8
    frozen = np.ones(32, np.uint8)
    frozen[info_positions(r, m)] = 0
    for _ in range(6):
        y = rng.standard_normal(32) * 1.7 + 0.3
        u, c, pm = oracle.scl(m, L, oracle.F64, y, frozen)
        ru, rc, rpm = np_scl(m, L, y, frozen, np.float64)
        assert np.array_equal(u, ru) and np.array_equal(pm, rpm)


@pytest.mark.parametrize("r,m,L", [(1, 4, 8), (2, 4, 16)])
def test_osd_binary32_full_order(r, m, L):
    """Order K enumerates the whole code, so the list is the L codewords of
    smallest binary32 metric."""
    N, K = oracle.rm_dims(r, m)
    G = generator(m)[info_positions(r, m)]
    msgs = ((np.arange(1 << K)[:, None] >> np.arange(K)) & 1).astype(np.int64)
    code = (msgs @ G % 2).astype(np.uint8)
    rng = np.random.default_rng(40 + m)
    n_diff = 0
    for trial in range(8):
        y = near_2p23(rng, N)
        yd = y.astype(np.float64)
        a, met, _ = oracle.osd(r, m, K, L, oracle.F32, yd)
        allm = np.array([np_metric(y, c, np.float32) for c in code], np.float64)
        assert np.array_equal(met, np.sort(allm)[:L])
        for c, e in zip(a, met):
            assert float(np_metric(y, c, np.float32)) == e
            assert any(np.array_equal(c, x) for x in code)
        assert len({bytes(c) for c in a}) == L
        _, m64, _ = oracle.osd(r, m, K, L, oracle.F64, yd)
        n_diff += not np.array_equal(m64, met)
    assert n_diff >= 4


def crc_remainder(bits, L, poly):
    """Long division of bits(x) * x^L by g(x) over GF(2), first bit highest."""
    reg = list(bits) + [0] * L
    g = [(poly >> (L - i)) & 1 for i in range(L + 1)]
    for i in range(len(bits)):
        if reg[i]:
            for t in range(L + 1):
                reg[i + t] ^= g[t]
    return reg[-L:]


def test_two_stage_binary32():
    """The whole two-stage decoder (Sec. III) in binary32 on RM(2,6) with
    CRC-6: numpy SCL, the CRC of the best entry, numpy stage 2 and choice."""
    r, m, L, T, crc_len, poly = 2, 6, 4, 4, 6, 0x43
    n = 64
    A = info_positions(r, m)
    frozen = np.ones(n, np.uint8)
    frozen[A] = 0
    supp, _ = oracle.moves(r, m)
    rng = np.random.default_rng(51)
    F = 8
    y = np.stack([near_2p23(rng, n) if f % 2 else
                  _f32((1 - 2.0 * codeword(r, m, rng)) + rng.standard_normal(n) * 0.9)
                  for f in range(F)])
    out = oracle.decode_batch(r, m, crc_len, poly, L, T, oracle.F32, y.astype(np.float64))
    for f in range(F):
        u, c, pm = np_scl(m, L, y[f], frozen, np.float32)
        v = u[0][A]
        ok = not any(crc_remainder(v, crc_len, poly))
        assert out["crc_ok"][f] == ok
        assert np.array_equal(out["anchors"][f], c)
        if ok:
            assert np.array_equal(out["c"][f], c[0])
            continue
        rp, rl, rm, rk = np_stage2_frame(supp, y[f], c, T, np.float32)
        assert np.array_equal(out["logs"][f], rl)
        assert out["k"][f] == rk
        assert np.array_equal(out["c"][f], rp[rk])
        assert out["metric"][f] == float(rm[rk])
