"""Complexity accounting in ED units (Sec. III-C, Table I, Eq. (6), Eq. (7)).

One ED unit is the cost of one squared Euclidean distance over a length-N
vector, taken as 3N floating-point operations.  The paper's models:

    SC list decoding        C_scl  = (4/3) L log2 N
    OSD of order k          C_osd  = sum_{i=0}^{k} binom(K, i)
    brute-force ML          C_mld  = 2^K
    one WSD trajectory      C_wsd  = J (m (1 + 1/(3N)) + |S| (w_bar + log2 m) / (3N))     (Eq. 6)
    whole decoder           C_mp   = C_init + P_act L_init C_wsd                          (Eq. 7)

with m the size of the correlation filter, m = max(10, ceil(0.02 |S|))
(Sec. IV-A), |S| the number of nonzero moves and w_bar their mean weight.

Eq. (6) is a worst case (every path runs all J iterations).  ``report``
puts it beside the activity the decoder actually had (the paths still
searching at each iteration, read back from the device) and beside the
dense work the matrix-core search spends: 2 P N integer operations per
searched path, i.e. 2P/3 ED units.
"""
from __future__ import annotations

import math


def ed_unit_flops(N: int) -> int:
    """Floating-point operations in one ED unit (Sec. III-C)."""
    return 3 * N


def c_scl(L: int, N: int) -> float:
    """SC list decoding with L paths, Table I."""
    return 4.0 / 3.0 * L * math.log2(N)


def c_osd(K: int, k: int) -> int:
    """Order-k OSD reprocessing, Table I."""
    return sum(math.comb(K, i) for i in range(k + 1))


def c_mld(K: int) -> int:
    """Brute-force maximum likelihood over 2^K codewords, Table I."""
    return 1 << K


def filter_size(S: int) -> int:
    """m = max(10, ceil(0.02 |S|)) of Sec. IV-A, in exact integer arithmetic."""
    return max(10, (2 * S + 99) // 100)


def c_wsd_iteration(S: int, w_bar: float, N: int, m: int | None = None) -> float:
    """One iteration of one trajectory: exact ED and min over the m filtered
    candidates plus filtering and sorting of all |S| moves (the bracket of
    Eq. (6))."""
    m = filter_size(S) if m is None else m
    return m * (1.0 + 1.0 / (3 * N)) + S * (w_bar + math.log2(m)) / (3 * N)


def c_wsd(J: int, S: int, w_bar: float, N: int, m: int | None = None) -> float:
    """Eq. (6): worst case of one trajectory, J iterations."""
    return J * c_wsd_iteration(S, w_bar, N, m)


def c_mp_wsd(c_init: float, p_act: float, L_init: int, c_wsd_value: float) -> float:
    """Eq. (7)."""
    return c_init + p_act * L_init * c_wsd_value


def report(N: int, K: int, S: int, w_bar: float, L: int, J: int, frames: int, stage2_frames: int,
           paths_per_iteration, ms_per_step: float | None = None, c_init: float | None = None) -> dict:
    """ED-unit accounting of one decoded batch.

    Stage 1 costs c_init (default: SCL(L), C_scl).  paths_per_iteration[t] is
    the number of paths still searching at iteration t over the whole batch;
    stage2_frames the frames that went to stage 2 (P_act = stage2_frames /
    frames: the CRC failures, or every frame in the always-on mode)."""
    p_act = stage2_frames / frames if frames else 0.0
    init = c_scl(L, N) if c_init is None else c_init
    it = c_wsd_iteration(S, w_bar, N)
    worst = c_mp_wsd(init, p_act, L, J * it)
    searched = sum(int(n) for n in paths_per_iteration)
    model_measured = init + searched / frames * it if frames else init
    dense_per_path = 2.0 * S * N / ed_unit_flops(N)  # = 2S/3 ED units
    out = {
        "ed_unit_flops": ed_unit_flops(N),
        "filter_m": filter_size(S),
        "c_init": init,
        "c_wsd_eq6": J * it,
        "p_act": p_act,
        "c_mp_wsd_eq7": worst,
        "searched_paths_per_frame": searched / frames if frames else 0.0,
        "c_mp_wsd_measured_activity": model_measured,
        "c_mld": float(c_mld(K)),
        "dense_search_ed_units_per_path_iteration": dense_per_path,
        "dense_search_ed_units_per_frame": searched / frames * dense_per_path if frames else 0.0,
    }
    if ms_per_step is not None and frames:
        out["ns_per_frame"] = ms_per_step * 1e6 / frames
        out["ns_per_ed_unit_eq7"] = out["ns_per_frame"] / worst
    return out
