"""Pins for the line-detector reference (oracle/hough.py), worked by hand:
the polar accumulator of a few pixels, its peak rule, the supporting set and
the sampling draw."""
import numpy as np

import oracle
from oracle import hough
from workloads.gen import splitmix64


def test_accumulator_by_hand():
    """Ten pixels on y = 5 in a 16 x 16 image, d_theta = 90 degrees (angle
    bins 0 and 90), d_rho = 1: rho bins are offset by width - 1 = 15.
    At 0 degrees each pixel votes in its own bin x + 15; at 90 degrees all ten
    vote in bin 5 + 15 = 20."""
    pix = np.array([[x, 5] for x in range(10)], dtype=np.int32)
    n_theta, n_rho, rho_min, c, s = hough.grid(16, 16, 1.0, 90.0)
    assert (n_theta, n_rho, rho_min) == (2, 46, -15.0)
    acc = hough.accumulator(pix, 16, 16, 1.0, 90.0)
    want = np.zeros((2, 46), dtype=np.int64)
    want[0, 15:25] = 1
    want[1, 20] = 10
    assert np.array_equal(acc, want)
    # one peak, the 90-degree cell; the 0-degree plateau of ones gives one
    # peak per run of equal cells only where the run starts (earlier cells win)
    pk = hough.peaks(acc, 2, 5)
    assert pk == [(1 * 46 + 20, 10)]
    assert hough.peaks(acc, 1, 5)[0] == (66, 10)


def test_detect_horizontal_line_by_hand():
    pix = np.array([[x, 5] for x in range(10)] + [[3, 12], [11, 1]], dtype=np.int32)
    acc, lines = hough.detect(pix, 16, 16, 1.0, 90.0, 1, 2, 4096, 0)
    L = lines[0]
    assert (L["theta_bin"], L["rho_bin"], L["votes"], L["support"]) == (1, 20, 10, 10)
    # normal at 90 degrees: the line is horizontal, fitted as y(x)
    assert L["transposed"] == 0
    r = L["result"]
    assert (r.width, r.theta1, r.theta2) == (0.0, 0.0, 5.0)


def test_steep_line_is_transposed():
    """A vertical line x = 7: its cell is at 0 degrees (rho = x), where
    |cos| > |sin|, so the set is fitted as x = 0 y + 7."""
    pix = np.array([[7, y] for y in range(12)] + [[1, 1], [13, 2]], dtype=np.int32)
    acc, lines = hough.detect(pix, 16, 16, 1.0, 90.0, 1, 2, 4096, 0)
    L = lines[0]
    assert (L["theta_bin"], L["rho_bin"], L["votes"], L["transposed"]) == (0, 22, 12, 1)
    assert np.array_equal(L["xy"][:, 0], np.arange(12.0)) and np.all(L["xy"][:, 1] == 7.0)
    r = L["result"]
    assert (r.width, r.theta1, r.theta2) == (0.0, 0.0, 7.0)


def test_sampled_support_is_the_smallest_keys():
    pix = np.array([[x, 5] for x in range(40)], dtype=np.int32)
    acc, lines = hough.detect(pix, 64, 64, 1.0, 90.0, 1, 2, 10, 99)
    L = lines[0]
    assert L["support"] == 40 and L["fitted"] == 10
    keys = splitmix64(99, 40)
    want = np.sort(np.argsort(keys, kind="stable")[:10]).astype(np.float64)
    assert np.array_equal(L["xy"][:, 0], want)
    assert L["result"].width == 0.0 and oracle.solve(L["xy"]).theta2 == 5.0
