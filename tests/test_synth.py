"""The seeded workload generator against the oracle and against statistics.

The generator is the transmitter and channel of Sec. II-B; these checks tie
it to the oracle (every transmitted word is a codeword whose information bits
pass the oracle's CRC) and to the channel model (noise variance sigma^2).
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2602_08501_amd import synth


@pytest.mark.parametrize("wl", [synth.RM26, synth.RM37, synth.RM27, synth.RM38])
def test_transmitted_words_are_crc_codewords(wl):
    pay, c, y = synth.generate(wl, 0, 0, 40)
    A = oracle.rm_info_set(wl.r, wl.m)
    fr = oracle.frozen_mask(wl.r, wl.m).astype(bool)
    for f in range(len(c)):
        u = oracle.encode(wl.m, c[f])
        assert not u[fr].any()
        v = u[A]
        assert np.array_equal(v[: wl.k_pay], pay[f])
        assert oracle.crc_ok(v, wl.crc_len, wl.crc_poly)
    assert y.dtype == np.float32 and y.shape == (40, wl.N)


def test_frames_do_not_depend_on_batch():
    a = synth.generate(synth.RM37, 3, 0, 100)
    b = synth.generate(synth.RM37, 3, 37, 61)
    for x, z in zip(a, b):
        assert np.array_equal(x[37:61], z)
    c = synth.generate(synth.RM37, 4, 37, 61)
    assert not np.array_equal(c[2], b[2])


def test_noise_variance_and_sigma_table():
    wl = dataclasses.replace(synth.RM37, ebn0_db=2.0)
    assert wl.sigma2 == pytest.approx(0.69623, abs=1e-5)
    pay, c, y = synth.generate(wl, 0, 0, 4000)
    n = y.astype(np.float64) - (1 - 2.0 * c)
    assert n.mean() == pytest.approx(0.0, abs=0.01)
    assert n.var() == pytest.approx(wl.sigma2, rel=0.01)
    assert synth.RM26.sigma2 == pytest.approx(1.00237, abs=1e-5)
    assert synth.RM38.sigma2 == pytest.approx(0.92831, abs=1e-5)


def test_splitmix_reference_values():
    # SplitMix64 seeded with 0: first outputs of the published generator
    out = synth.stream(np.array([0], np.uint64), 3)[0]
    assert [int(v) for v in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
