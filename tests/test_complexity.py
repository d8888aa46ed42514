"""ED-unit complexity models of Sec. III-C / Table I / Eq. (6)-(7), checked
on values worked out by hand and on the structural properties the formulas
must have."""
import math

import pytest

from paper_2602_08501_amd import complexity as C


def test_filter_size_rule():
    # m = max(10, ceil(0.02 |S|)): RM(2,7) has 10668 moves -> ceil(213.36) = 214
    assert C.filter_size(10668) == 214
    assert C.filter_size(2604) == 53        # ceil(52.08)
    assert C.filter_size(94488) == 1890     # ceil(1889.76)
    assert C.filter_size(500) == 10         # exactly 10.0 -> 10
    assert C.filter_size(501) == 11         # 10.02 -> 11
    assert C.filter_size(100) == 10         # floor of the rule
    assert C.filter_size(0) == 10


def test_scl_osd_mld_models():
    # (4/3) L log2 N: L=8, N=128 -> 4/3 * 8 * 7
    assert C.c_scl(8, 128) == pytest.approx(224.0 / 3.0)
    assert C.c_scl(1, 2) == pytest.approx(4.0 / 3.0)
    # OSD(k) on K=29: 1, 1+29, 1+29+406, 1+29+406+3654, +23751
    assert [C.c_osd(29, k) for k in range(5)] == [1, 30, 436, 4090, 27841]
    assert C.c_osd(5, 5) == 32 == C.c_mld(5)
    assert C.c_mld(29) == 536870912


def test_wsd_eq6_worked_value():
    # RM(2,7), J = 4, r = 1: |S| = 10668, w = 32, m = 214, N = 128
    per_iter = 214 * (1 + 1 / 384) + 10668 * (32 + math.log2(214)) / 384
    assert C.c_wsd_iteration(10668, 32, 128) == pytest.approx(per_iter, rel=1e-15)
    assert C.c_wsd(4, 10668, 32, 128) == pytest.approx(4 * per_iter, rel=1e-15)
    # the filtering term dominates: |S| (w + log2 m) / 3N is ~1100 of ~1320 units
    assert 1300 < per_iter < 1330


def test_wsd_eq6_structure():
    # linear in J; with |S| = 0 only the exact-ED term m (1 + 1/3N) is left
    assert C.c_wsd(0, 1000, 16, 64) == 0
    assert C.c_wsd(3, 1000, 16, 64) == pytest.approx(3 * C.c_wsd(1, 1000, 16, 64))
    assert C.c_wsd_iteration(0, 16, 64, m=10) == pytest.approx(10 * (1 + 1 / 192))
    # each extra move costs (w + log2 m) / 3N units
    d = C.c_wsd_iteration(1001, 16, 64, m=16) - C.c_wsd_iteration(1000, 16, 64, m=16)
    assert d == pytest.approx((16 + 4) / 192)


def test_mp_wsd_eq7():
    assert C.c_mp_wsd(10.0, 0.0, 8, 1e6) == 10.0          # CRC always passes: stage 1 only
    assert C.c_mp_wsd(10.0, 1.0, 8, 5.0) == 50.0          # always-on mode
    assert C.c_mp_wsd(2.0, 0.25, 4, 3.0) == pytest.approx(5.0)


def test_report_consistency():
    r = C.report(N=128, K=64, S=94488, w_bar=16, L=8, J=8, frames=1000, stage2_frames=50,
                 paths_per_iteration=[400, 300, 100, 0, 0, 0, 0, 0], ms_per_step=0.5)
    assert r["p_act"] == 0.05
    it = C.c_wsd_iteration(94488, 16, 128)
    assert r["c_init"] == C.c_scl(8, 128)
    assert r["c_mp_wsd_eq7"] == pytest.approx(C.c_scl(8, 128) + 0.05 * 8 * 8 * it)
    # measured activity (800 path-iterations) is below the worst case (50 * 8 * 8 = 3200)
    assert r["c_mp_wsd_measured_activity"] == pytest.approx(C.c_scl(8, 128) + 0.8 * it)
    assert r["c_mp_wsd_measured_activity"] < r["c_mp_wsd_eq7"]
    assert r["dense_search_ed_units_per_path_iteration"] == pytest.approx(2 * 94488 / 3)
    assert r["ns_per_frame"] == pytest.approx(500.0)


def test_report_osd_always_on():
    # OSD(2) on RM(2,7): C_osd = 1 + 29 + 406 = 436; always on: P_act = 1
    r = C.report(N=128, K=29, S=10668, w_bar=32, L=8, J=4, frames=10, stage2_frames=10,
                 paths_per_iteration=[80, 20, 5, 0], c_init=float(C.c_osd(29, 2)))
    assert r["c_init"] == 436 and r["p_act"] == 1.0
    assert r["c_mp_wsd_eq7"] == pytest.approx(436 + 8 * C.c_wsd(4, 10668, 32, 128))
