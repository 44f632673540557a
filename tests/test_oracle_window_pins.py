"""Direct pins for the oracle's per-slope and per-pair functions.

lms_oracle_window (F at one slope), lms_oracle_eval_pairs (F at pair slopes),
lms_oracle_anchored (the anchored widths) and lms_oracle_hth_abs_residual are
checked against closed forms on sets built so that every value is exact in
binary64, and against the full search's own result. F(theta) is the narrowest
window of h consecutive intercepts z = y - theta x (Section 3.1's thinnest
slab at a fixed slope; Algorithm 1's sort and bracelet at one vertex).
"""
import numpy as np
import pytest

from workloads import gen
from workloads.gen import Stream


def test_window_on_a_line_is_slope_offset_times_x_window(orc):
    """Points on y = 3x + 5 at slope 3 + d: z = 5 - d x exactly, so F is |d|
    times the narrowest h-window of the x values, and the window sits at the
    x values that window covers."""
    x = np.array([10.0, 0.0, 30.0, 2.0, 11.0, 1.0, 12.0, 3.0])
    xy = np.stack([x, 3.0 * x + 5.0], 1)
    # sorted x: 0 1 2 3 10 11 12 30; h = 4 windows: 3, 9, 9, 9, 20
    for d in (0.5, -0.25, 2.0 ** -20):
        w, lo, hi = orc.window(xy, 3.0 + d, h=4)
        assert w == 3.0 * abs(d)
        if d > 0:  # z decreasing in x: the window is z(3) .. z(0)
            assert (lo, hi) == (5.0 - 3.0 * d, 5.0)
        else:
            assert (lo, hi) == (5.0, 5.0 - 3.0 * d)
    # h = 5: windows 10, 10, 10, 27 -> the lowest of the ties
    w, lo, hi = orc.window(xy, 3.5, h=5)
    assert w == 5.0 and (lo, hi) == (5.0 - 0.5 * 12.0, 5.0 - 0.5 * 2.0)
    assert orc.window(xy, 3.0, h=8) == (0.0, 5.0, 5.0)


def test_window_two_parallel_lines(orc):
    """m points on y = x/2, the rest on y = x/2 + 1: at slope 1/2 the width
    is 0 while h <= max(m, n - m), else exactly 1."""
    st = Stream(41, 410)
    x = st.integers(30, -50, 50).astype(np.float64)
    up = np.zeros(30, bool)
    up[:12] = True
    xy = np.stack([x, 0.5 * x + up], 1)[st.permutation(30)]
    for h in (2, 10, 18):
        assert orc.window(xy, 0.5, h=h) == (0.0, 0.0, 0.0)
    for h in (19, 25, 30):
        assert orc.window(xy, 0.5, h=h) == (1.0, 0.0, 1.0)


def test_window_default_h_and_errors(orc):
    xy = gen.planted(11, 0.3, 5)
    assert orc.window(xy, 0.3) == orc.window(xy, 0.3, h=6)
    with pytest.raises(ValueError):
        orc.window(xy, 0.3, h=12)
    bad = xy.copy()
    bad[2, 0] = np.inf
    with pytest.raises(ValueError):
        orc.window(bad, 0.3)


def test_solve_result_is_its_own_window(orc):
    """The full search's width, window and pair agree with F at its slope."""
    for xy in (gen.planted(120, 0.4, 8), gen.degenerate_int(120, 9)):
        r = orc.solve(xy)
        assert orc.window(xy, r.theta1) == (r.width, r.z_lo, r.z_hi)
        th, w, lo, hi = orc.eval_pairs(xy, [[r.pair_i, r.pair_j]])
        assert (th[0], w[0], lo[0], hi[0]) == (r.theta1, r.width, r.z_lo, r.z_hi)


def test_eval_pairs_closed_form_and_order(orc):
    """On y = 3x + 5 every pair slope is exactly 3 and every window is 0 at
    z = 5; a pair's slope is taken with the smaller index first; a vertical
    pair gives (NaN, +inf)."""
    x = np.array([1.0, 4.0, -2.0, 7.0, 4.0])
    xy = np.stack([x, 3.0 * x + 5.0], 1)
    xy[4, 1] = 0.0  # same x as point 1, off the line
    th, w, lo, hi = orc.eval_pairs(xy, [[0, 1], [3, 2], [1, 4], [2, 4]], h=3)
    assert th[0] == 3.0 and w[0] == 0.0 and lo[0] == 5.0
    assert th[1] == 3.0 and w[1] == 0.0
    assert np.isnan(th[2]) and w[2] == np.inf
    # (2, 4): slope (0 - (-1)) / (4 - (-2)) = 1/6; z = y - x/6
    assert th[3] == 1.0 / 6.0
    assert w[3] == orc.window(xy, 1.0 / 6.0, h=3)[0]
    a = orc.eval_pairs(gen.planted(50, 0.3, 3), [[7, 21]])
    b = orc.eval_pairs(gen.planted(50, 0.3, 3), [[21, 7]])
    assert all(u[0] == v[0] for u, v in zip(a, b))
    with pytest.raises(ValueError):
        orc.eval_pairs(xy, [[0, 5]])
    with pytest.raises(ValueError):
        orc.eval_pairs(xy, [[2, 2]])


def test_eval_pairs_equals_windows_at_the_pair_slopes(orc):
    """Each pair's (width, window) is F at its own slope, for many pairs."""
    xy = gen.planted(90, 0.45, 12)
    st = Stream(43, 430)
    i = st.integers(60, 0, 89)
    j = (i + 1 + st.integers(60, 0, 87)) % 90
    th, w, lo, hi = orc.eval_pairs(xy, np.stack([i, j], 1))
    for t in range(60):
        a, b = min(i[t], j[t]), max(i[t], j[t])
        slope = (xy[b, 1] - xy[a, 1]) / (xy[b, 0] - xy[a, 0])
        assert th[t] == slope
        assert (w[t], lo[t], hi[t]) == orc.window(xy, slope)


def test_anchored_closed_form(orc):
    """Anchor pair on y = 0: slope 0, c = 0, residuals d = y. Up: the h-th
    smallest of {d >= 0} (members counted as 0); down: of {-d >= 0}."""
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [2.0, 0.5], [3.0, 1.0], [4.0, -0.25],
                   [5.0, 2.0], [6.0, -3.0]])
    up, dn = orc.anchored(xy, 0, 1, h=3)
    assert (up, dn) == (0.5, 0.25)
    up, dn = orc.anchored(xy, 1, 0, h=4)
    assert (up, dn) == (1.0, 3.0)
    up, dn = orc.anchored(xy, 0, 1, h=5)
    assert (up, dn) == (2.0, np.inf)
    # a vertical pair has no slope
    v = np.array([[1.0, 0.0], [1.0, 2.0], [3.0, 1.0]])
    assert orc.anchored(v, 0, 1, h=2) == (np.inf, np.inf)


def test_hth_abs_residual_closed_form(orc):
    xy = np.array([[0.0, 1.0], [1.0, 2.5], [2.0, 2.0], [3.0, 7.0], [4.0, 4.75]])
    # line y = x + 1: residuals 0, 0.5, -1, 3, -0.25 -> |r| sorted 0 .25 .5 1 3
    assert orc.hth_abs_residual(xy, 1.0, 1.0, h=2) == 0.25
    assert orc.hth_abs_residual(xy, 1.0, 1.0, h=4) == 1.0
    assert orc.hth_abs_residual(xy, 1.0, 1.0) == 0.5  # h = 3
