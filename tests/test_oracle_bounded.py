"""Pins for the oracle's bounded search (lms_oracle_solve_bounded).

The bounded search must return exactly what the exhaustive search returns
(every field, bitwise): it evaluates F with the same code and only skips
slopes that the Lipschitz bound of F in theta proves wider than the best width
found. These tests pin it to the exhaustive search, on small sets here and on
the stored exhaustive results at 4096 points, and pin the Lipschitz bound
itself to the definition of F (Eq. (1); Section 3.1's slab at a fixed slope).
"""
import json
import os

import numpy as np
import pytest

from workloads import gen
from workloads.gen import Stream, default_h

HERE = os.path.dirname(os.path.abspath(__file__))
FIELDS = ("theta1", "theta2", "half_width", "width", "z_lo", "z_hi", "pair_i", "pair_j",
          "candidates", "vertical", "status", "h")


def same(a, b):
    return all(getattr(a, f) == getattr(b, f) for f in FIELDS)


def cases():
    st = Stream(23, 230)
    out = []
    for n in (3, 5, 17, 60, 200, 450):
        out.append((f"planted{n}", gen.planted(n, 0.45, 1000 + n), 0))
        out.append((f"int{n}", gen.degenerate_int(n, 2000 + n), 0))
    # small integer grid: many equal slopes, coincident points, exact ties
    for n, r in ((40, 3), (90, 6), (300, 20)):
        out.append((f"grid{n}", st.integers(2 * n, 0, r).reshape(n, 2).astype(np.float64), 0))
    # general h, including h = 2 and h = n (the Chebyshev fit)
    xy = gen.planted(150, 0.3, 77)
    for h in (2, 3, 40, 149, 150):
        out.append((f"h{h}", xy, h))
    # more than half the points exactly on one line: width 0
    x = st.permutation(400)[:101].astype(np.float64)
    on = np.stack([x, -2.0 * x + 5.0], 1)
    off = st.integers(2 * 99, -300, 300).reshape(99, 2).astype(np.float64)
    out.append(("collinear", np.concatenate([on, off])[st.permutation(200)], 0))
    # steep line, large offsets, tiny and huge scales
    t = gen.planted(120, 0.4, 5)
    out.append(("steep", np.stack([t[:, 0] * 1e-6, t[:, 1]], 1), 0))
    out.append(("offset", t + np.array([1e6, -1e6]), 0))
    out.append(("tiny", t * 2.0 ** -200, 0))
    out.append(("huge", t * 2.0 ** 200, 0))
    # Hough-style patches: integer pixels with many duplicates
    xy4, off4 = gen.hough_patches(6, 44)
    for b in range(6):
        out.append((f"patch{b}", xy4[off4[b]:off4[b + 1]], 0))
    return out


@pytest.mark.parametrize("name,xy,h", cases(), ids=[c[0] for c in cases()])
def test_bounded_equals_exhaustive(orc, name, xy, h):
    want = orc.solve(xy, h=h)
    got, evaluated = orc.solve_bounded(xy, h=h)
    assert same(got, want), (name, got, want)
    assert evaluated >= 1


def test_bounded_all_x_equal(orc):
    xy = np.stack([np.full(9, 2.5), Stream(3, 3).uniform(9, -1, 1)], 1)
    got, _ = orc.solve_bounded(xy)
    assert same(got, orc.solve(xy)) and got.status == 1


@pytest.mark.parametrize("key", ["c2/201", "c2/202", "c2/203", "degenerate_int_4096/302"])
def test_bounded_equals_stored_exhaustive_4096(orc, key):
    """At 4096 points the exhaustive results are stored (about ten core-hours
    each); the bounded search must reproduce every field."""
    store = json.load(open(os.path.join(HERE, "golden", "oracle_results.json")))[key]
    assert store["method"] == "exhaustive"
    name, seed = key.split("/")
    xy = gen.degenerate_int(4096, int(seed)) if name.startswith("degenerate") else \
        gen.make(name, int(seed))
    r, evaluated = orc.solve_bounded(xy)
    for f in ("width", "theta1", "theta2", "z_lo", "z_hi"):
        assert getattr(r, f) == float.fromhex(store[f]), f
    assert [r.pair_i, r.pair_j] == store["pair"]
    assert (r.candidates, r.vertical) == (store["candidates"], store["vertical"])
    # the bound leaves few slopes beyond the 4096 of the coarse pass
    assert evaluated < 4096 + 20000


def _F(orc, xy, theta, h=0):
    return orc.window(xy, theta, h)[0]


@pytest.mark.parametrize("make", [lambda: gen.planted(300, 0.45, 9),
                                  lambda: gen.degenerate_int(300, 10),
                                  lambda: gen.hough_patches(1, 3)[0]])
def test_lipschitz_bound_of_F(orc, make):
    """|F(a) - F(b)| <= (max x - min x) |a - b|, the fact the bounded search
    rests on, checked on random slope pairs near and far apart."""
    xy = make()
    L = xy[:, 0].max() - xy[:, 0].min()
    st = Stream(31, 310)
    M = np.abs(xy).max()
    for scale in (1e-6, 1e-3, 0.1, 3.0, 100.0):
        a = st.uniform(40, -2, 2)
        b = a + scale * st.uniform(40, -1, 1)
        for u, v in zip(a, b):
            Fu, Fv = _F(orc, xy, u), _F(orc, xy, v)
            slack = 1e-13 * M * (1 + abs(u) + abs(v))
            assert abs(Fu - Fv) <= L * abs(u - v) * (1 + 1e-12) + slack, (u, v, Fu, Fv)


def test_lipschitz_bound_is_attained(orc):
    """The constant cannot be lowered: with h = 2 and two points at the ends of
    the x range, F(theta) = |dy - theta dx| exactly, of slope dx = L."""
    xy = np.array([[0.0, 0.0], [8.0, 4.0]])
    for t in (0.0, 0.25, 1.0):
        assert _F(orc, xy, t, h=2) == abs(4.0 - 8.0 * t)
