"""The slope-bin screen's rigour, checked on the CPU against exact rationals.

The screen adds each point's window intervals to bins of a monotone map of
the slope, with two-bin margins. That is sound when every bin the kernel
computes (an interval end, or a pair's own slope, which is the same
expression) lies within one bin of the bin the exact map gives the exact
value. This emulates the kernel's FP64 arithmetic step by step in numpy
(coordinate differences, the map offset a = fma(-tc, dx, dy), the reciprocal
of dx with the hardware estimate's worst case after one Newton step, relative
2^-40 either way, the products, and the bit-pattern map fbin) and compares
with the exact map on exact rationals, on planted, integer-grid,
near-vertical and 10^+-250-scaled sets, with the map centred on, near and far
from the optimum.

The exact map: for g = |f| + 1 = 2^e (1 + m), r(g) = (2 - m) / 2^(e+1) (the
reciprocal read off the bit pattern, exact at powers of two), and the bin is
floor(R + 3 + sign(f) R (1 - r(g))), R = NB / 2.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from workloads.gen import Stream, degenerate_int, planted

RLOG = 12  # NB = 8192 bins, R = 4096
R = 1 << RLOG
KMAG = 32.0


def fbin_kernel(f: np.ndarray) -> np.ndarray:
    """fbin<RLOG> as the kernel computes it, in binary64."""
    C = float(R) + 3.0
    g = np.abs(f) + 1.0
    hiw = (g.view(np.uint64) >> np.uint64(32)).astype(np.int64)
    k = 0x7FE00000 + (RLOG << 20)
    hi = np.maximum(k - hiw, 0).astype(np.uint64)  # saturating unsigned subtraction
    v = (hi << np.uint64(32)).view(np.float64)
    return np.trunc(C + np.copysign(float(R) - v, f)).astype(np.int64)


def fbin_exact(f: Fr) -> int:
    g = abs(f) + 1
    e = g.numerator.bit_length() - g.denominator.bit_length()
    if Fr(2) ** e > g:
        e -= 1
    elif Fr(2) ** (e + 1) <= g:
        e += 1
    m = g / Fr(2) ** e - 1
    r = (2 - m) / Fr(2) ** (e + 1)
    u = 1 - r
    x = R + 3 + (u * R if f >= 0 else -u * R)
    return int(x.numerator // x.denominator) if x >= 0 else -int((-x).numerator // (-x).denominator)


def fma_exact(a: float, b: float, c: float) -> float:
    """fma(a, b, c) rounded once to binary64."""
    return float(Fr(a) * Fr(b) + Fr(c))


def recip_worst(dx: np.ndarray, sign: int) -> np.ndarray:
    """1/dx moved by 2^-40 relative, the bound after one Newton step."""
    return (1.0 / dx) * (1.0 + sign * 2.0 ** -40)


def check_set(xy, tc, W, anchors, rng_pts=400):
    xh = np.abs(xy[:, 0] - 0.5 * (xy[:, 0].min() + xy[:, 0].max())).max()
    yh = np.abs(xy[:, 1] - 0.5 * (xy[:, 1].min() + xy[:, 1].max())).max()
    sc = min(max(KMAG * xh / yh, 2.0 ** -100), 2.0 ** 100)
    tc = tc if abs(tc) * sc <= 2.0 ** 20 else 0.0
    nb = 2 * R + 256
    q = 2.0 ** -46 * nb * sc
    n = len(xy)
    st = Stream(71, 710)
    checked = 0
    for i in anchors:
        ks = st.integers(min(rng_pts, n - 1), 0, n - 2)
        ks = ks + (ks >= i)
        dx = xy[ks, 0] - xy[i, 0]
        dy = xy[ks, 1] - xy[i, 1]
        keep = (dx != 0.0) & (np.abs(dx) >= np.abs(dy) * q + 2.0 ** -900) & \
               (np.abs(dx) <= 2.0 ** 900)
        for k, ddx, ddy in zip(ks[keep], dx[keep], dy[keep]):
            a = fma_exact(-tc, ddx, ddy)
            EX = Fr(xy[k, 0]) - Fr(xy[i, 0])
            EY = Fr(xy[k, 1]) - Fr(xy[i, 1])
            for sgn in (-1, 1):
                s = sc * float(recip_worst(np.array([ddx]), sgn)[0])
                for c in (-W, 0.0, W):
                    f = (a + c) * s if c else a * s
                    got = int(fbin_kernel(np.array([f]))[0])
                    exact = (EY + Fr(c) - Fr(tc) * EX) * Fr(sc) / EX
                    want = fbin_exact(exact)
                    assert abs(got - want) <= 1, (i, int(k), c, got, want)
            checked += 1
    return checked


def test_fbin_matches_exact_map_at_known_points():
    """fbin at powers of two and at zero, worked by hand: f = 0 -> bin R + 3;
    f = 1 (g = 2, r = 1/2) -> R + 3 + R/2; f = -3 (g = 4, r = 1/4) ->
    R + 3 - 3R/4."""
    f = np.array([0.0, 1.0, -3.0, 1e300, -1e300])
    assert list(fbin_kernel(f)) == [R + 3, R + 3 + R // 2, R + 3 - 3 * R // 4, 2 * R + 3, 3]
    for v in (0.0, 1.0, -3.0):
        assert fbin_exact(Fr(v)) == int(fbin_kernel(np.array([v]))[0])


@pytest.mark.parametrize("case", ["planted", "integer", "near_vertical", "scaled_up",
                                  "scaled_down"])
def test_computed_bins_within_one_of_exact(case):
    if case == "planted":
        xy = planted(400, 0.45, 72)
    elif case == "integer":
        xy = degenerate_int(400, 73)
    elif case == "near_vertical":
        xy = planted(300, 0.4, 74)
        tw = xy[:100].copy()
        tw[:, 0] += Stream(75, 750).uniform(100, 0.5e-12, 2e-12)
        xy = np.concatenate([xy, tw])
    elif case == "scaled_up":
        xy = planted(400, 0.45, 76) * np.array([1e250, 1e249])
    else:
        xy = planted(400, 0.45, 77) * np.array([1e-250, 1e-249])
    import oracle
    o = oracle.solve(xy)
    W = o.width * (1 + 2.0 ** -50)
    anchors = list(range(0, len(xy), max(1, len(xy) // 6)))[:6]
    total = 0
    # the map centred on the optimum, near it, and far from it
    for tc in (o.theta1, o.theta1 * (1 + 1e-3) + 1e-9, -5.0 * o.theta1 - 1.0):
        total += check_set(xy, tc, W, anchors, rng_pts=120)
    assert total > 500
