"""The autotuner's candidate tiles (host logic, no GPU): every tile variant
the library reports, at one workgroup per CU up to what a CU's 160 KB of LDS
holds for the table's staging buffers; multi-code launches only for the
variants the multi-code kernel is built for."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2602_08501_amd import _lib, autotune  # noqa: E402

LDS = 160 * 1024


def test_variants_reported():
    vs = _lib.mpwsd_search_variants()
    assert [(v["col_blocks"], v["waves"]) for v in vs] == [(8, 4), (4, 4), (4, 8), (8, 2), (2, 4), (3, 4)]
    for v in vs:
        assert v["columns"] == 16 * v["col_blocks"] * v["waves"] and v["blocks_per_cu"] >= 1


def _bpc(cands):
    out = {}
    for v, b in cands:
        out.setdefault(v, []).append(b)
    return out


def test_paired_half_lds_fit():
    # three chunks of 128 rows of N/2 bytes plus eight chunks' canonical indices
    for N, fit in ((128, 5), (256, 2)):
        assert (LDS // (3 * 128 * (N // 2) + 8 * 2 * 128 * 4)) == fit
        b = _bpc(autotune.candidates(N, grouped=True))
        assert sorted(b) == list(range(6))
        assert all(x == list(range(1, fit + 1)) for x in b.values())


def test_plain_lds_fit():
    # two chunks of 128 rows of max(N, 64) + 16 bytes
    for N, fit in ((64, 8), (128, 4), (256, 2)):
        assert LDS // (2 * 128 * (max(N, 64) + 16)) == fit
        b = _bpc(autotune.candidates(N))
        assert sorted(b) == list(range(6))
        assert all(x == list(range(1, min(fit, 6) + 1)) for x in b.values())


def test_multi_code_variants():
    b = _bpc(autotune.candidates(128, multi=True))
    assert sorted(b) == [0, 1, 2]
    # the multi-code kernel's LDS is the plain staging of the largest N, which
    # also holds the paired-half staging (3 * 128 * N/2 + 8 KB)
    for N in (128, 256):
        assert 3 * 128 * (N // 2) + 8 * 2 * 128 * 4 <= 2 * 128 * (N + 16)
    b = _bpc(autotune.candidates(256, multi=True, grouped=True))
    assert sorted(b) == [0, 1, 2] and all(x == [1, 2] for x in b.values())
