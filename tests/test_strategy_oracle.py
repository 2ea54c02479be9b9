"""Shrink-and-expand decisions of the oracle on scripted residual histories.

Expected decision sequences are worked out by hand from Algorithms 6 and 7 and
the warm-up rule (Section 3.2), with the readings stated in ``oracle/strategy.py``.
"""
import math

import oracle as O


def run(strategy, rs, **kw):
    """Drive the controller like the solvers do; return (expand_js, shrink_js)."""
    ctl = O.SEController(O.SEParams(strategy, **kw))
    exp, shr = [], []
    for j, r in enumerate(rs, start=1):
        ctl.observe(j, r)
        if ctl.ifexpand(j):
            ctl.did_expand(j)
            exp.append(j)
        if ctl.ifshrink(j):
            ctl.did_shrink(j)
            shr.append(j)
    return exp, shr


def geometric(n, start=1.0, q=0.5):
    return [start * q ** j for j in range(1, n + 1)]


def test_none_never_acts():
    assert run("none", geometric(60)) == ([], [])


def test_fix_schedule_after_warmup():
    # r(j) = 2^-j drops below 1e-4 at j = 14 (2^-14 = 6.1e-5); j_warm = 5.
    exp, shr = run("fix", geometric(62))
    assert shr[0] == 14
    assert exp == [24, 36, 48, 60]
    assert shr == [14, 26, 38, 50, 62]


def test_fix_warmup_waits_for_min_iterations():
    rs = [1e-6] * 30  # residual condition met from the start
    exp, shr = run("fix", rs)
    assert shr[0] == 5  # j >= j_warm
    assert exp == [12, 24]
    assert shr == [5, 14, 26]


def test_slope_expands_when_rate_decays_and_shrinks_js_later():
    # fast decay (slope 1 per iteration) then slower decay (slope 0.5)
    rs, lr = [], 0.0
    for j in range(1, 31):
        lr -= 1.0 if j <= 12 else 0.5
        rs.append(10.0 ** lr)
    exp, shr = run("slope", rs)
    # warm-up: r(5) = 1e-5 <= 1e-4 -> first shrink at j = 5.
    # c(6..12) = 1 = c_max; c(13) = 0.5 and 1.1 * 0.5 < 1 -> expand at 13,
    # shrink at 13 + j_s = 15; then c stays 0.5 = c_max -> no more expansions.
    assert shr == [5, 15]
    assert exp == [13]


def test_slope_expands_on_residual_increase():
    # The text notes that slope expands whenever the residual grows (c < 0 < c_max).
    lr = [-1, -2, -3, -4, -5, -6, -7, -6.5, -7.5, -8.5, -9.5, -9.0, -10.0, -11.0]
    exp, shr = run("slope", [10.0 ** v for v in lr])
    assert shr[0] == 5
    assert 8 in exp and 12 in exp


def test_slopek_averages_over_jp():
    # oscillating residual with a steady downward trend: slope expands often,
    # slopek (j_p = 10) does not.
    lr, v = [], 0.0
    for j in range(1, 61):
        v -= 0.3
        lr.append(v + (0.25 if j % 2 else 0.0))
    rs = [10.0 ** x for x in lr]
    exp_s, _ = run("slope", rs)
    exp_k, shr_k = run("slopek", rs)
    assert len(exp_s) >= 5
    assert exp_k == []
    assert len(shr_k) == 1


def test_slopek_expands_when_average_slope_drops():
    lr, v = [], 0.0
    for j in range(1, 51):
        v -= 1.0 if j <= 25 else 0.2
        lr.append(v)
    exp, shr = run("slopek", [10.0 ** x for x in lr])
    # first shrink at j = 5 (r = 1e-5). c(j) needs r(j - 10), so it exists from j = 11; it is 1.0
    # through j = 25, then falls; 1.1 * c < 1 once c < 0.909:
    # c(26) = (9 * 1 + 0.2) / 10 = 0.92; c(27) = (8 + 0.4) / 10 = 0.84 -> expand at 27.
    assert shr[0] == 5
    assert exp[0] == 27
    assert shr[1] == 29


def test_warmup_threshold_is_inclusive_and_uses_rk():
    exp, shr = run("fix", [1e-3] * 6 + [1e-4] + [1e-5] * 5)
    assert shr == [7]
    assert math.isclose(O.SEParams().r_warm, 1e-4)
