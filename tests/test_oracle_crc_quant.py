"""Pins for the CRC precoder (Sec. II-B) and the LLR quantizer.

CRC: the remainder of p(x) x^6 modulo g(x) = x^6 + x + 1 is computed here by
plain polynomial long division on Python integers (first payload bit = highest
degree), and the oracle's shift register must agree; the residue of v =
payload || crc is zero; the code is linear; every single-bit error and every
burst of length <= 6 is detected (g has degree 6 and a nonzero constant term).

Quantizer: q = clamp(round-half-even(fl32(y s)), -127, 127), checked against
numpy's float32 product and rint on random and hand-picked values.
"""
import numpy as np
import pytest

import oracle

POLY = 0x43


def long_division_crc(bits, L=6, poly=POLY):
    val = 0
    for b in bits:
        val = (val << 1) | int(b)
    val <<= L
    deg = val.bit_length() - 1
    while deg >= L:
        val ^= poly << (deg - L)
        deg = val.bit_length() - 1
    return [(val >> (L - 1 - i)) & 1 for i in range(L)]


def test_crc_equals_long_division():
    rng = np.random.default_rng(1)
    for n in (1, 5, 16, 23, 58, 87):
        for _ in range(20):
            p = rng.integers(0, 2, n).astype(np.uint8)
            assert oracle.crc(p, 6, POLY).tolist() == long_division_crc(p)


def test_crc_residue_and_linearity():
    rng = np.random.default_rng(2)
    for _ in range(50):
        a = rng.integers(0, 2, 58).astype(np.uint8)
        b = rng.integers(0, 2, 58).astype(np.uint8)
        va = np.concatenate([a, oracle.crc(a, 6, POLY)])
        assert oracle.crc_ok(va, 6, POLY)
        assert np.array_equal(oracle.crc(a ^ b, 6, POLY), oracle.crc(a, 6, POLY) ^ oracle.crc(b, 6, POLY))


def test_crc_detects_single_errors_and_short_bursts():
    rng = np.random.default_rng(3)
    a = rng.integers(0, 2, 58).astype(np.uint8)
    v = np.concatenate([a, oracle.crc(a, 6, POLY)])
    n = len(v)
    for i in range(n):
        e = v.copy()
        e[i] ^= 1
        assert not oracle.crc_ok(e, 6, POLY)
    for length in range(2, 7):
        for start in range(n - length + 1):
            for inner in range(1 << max(0, length - 2)):
                e = v.copy()
                e[start] ^= 1
                e[start + length - 1] ^= 1
                for t in range(length - 2):
                    if inner >> t & 1:
                        e[start + 1 + t] ^= 1
                assert not oracle.crc_ok(e, 6, POLY)


def test_quantizer_matches_float32_rint():
    rng = np.random.default_rng(4)
    y = (rng.standard_normal(20000) * 3).astype(np.float32)
    for s in (np.float32(7.981), np.float32(12.89), np.float32(0.5)):
        ref = np.clip(np.rint(y * s), -127, 127).astype(np.int8)
        assert np.array_equal(oracle.quantize(y, s), ref)


def test_quantizer_ties_clamp_and_symmetry():
    s = np.float32(2.0)
    y = np.array([0.25, 0.75, 1.25, -0.25, -0.75, 100.0, -100.0, 63.49, 0.0], np.float32)
    assert oracle.quantize(y, s).tolist() == [0, 2, 2, 0, -2, 127, -127, 127, 0]
    rng = np.random.default_rng(5)
    z = (rng.standard_normal(5000) * 20).astype(np.float32)
    assert np.array_equal(oracle.quantize(-z, np.float32(3.3)), -oracle.quantize(z, np.float32(3.3)))
