"""Mutation check of the oracle's pins (CPU).

Each mutant is a copy of oracle/lms_oracle.c with one plausible mistake
planted: a window one point short, the sign of theta in the intercepts, a
skipped pair, the wrong intercept, the wrong default h, an inverted slope, a
truncated window scan, ties resolved to the highest window, the vertical test
on y. Every mutant is compiled into its own library and run through a battery
of pins that come from outside the oracle (exact h-subset minimax fits, the
Chebyshev LP for h = n, closed forms worked by hand, the optimality
certificate). The unmutated source must pass the battery and every mutant
must fail at least one pin: a pin set that a planted slip slips through would
not be worth trusting.
"""
import os

import numpy as np
import pytest

import oracle
from tests.test_oracle_pins import chebyshev_lp, lms_by_subsets
from workloads.gen import Stream, default_h, planted

pytestmark = pytest.mark.slow

SRC = os.path.join(os.path.dirname(oracle.__file__), "lms_oracle.c")

# (name, text in lms_oracle.c, replacement, occurrences to replace)
MUTANTS = [
    ("window h-1", "z[h - 1] - z[0]", "z[h - 2] - z[0]", 1),
    ("window h-1 scan", "z[s + h - 1] - z[s]", "z[s + h - 2] - z[s]", 1),
    ("sign of theta", "fma(-theta, xy[2 * k], xy[2 * k + 1]);\n  qsort",
     "fma(theta, xy[2 * k], xy[2 * k + 1]);\n  qsort", 1),
    ("skipped pairs", "for (int64_t j = i + 1; j < n; ++j) {",
     "for (int64_t j = i + 2; j < n; ++j) {", 1),
    ("intercept", "out->theta2 = 0.5 * (best.z_lo + best.z_hi);", "out->theta2 = best.z_lo;", 1),
    ("default h", "*h = n / 2 + 1;", "*h = n / 2;", 1),
    ("inverted slope", "c.theta = (xy[2 * j + 1] - xy[2 * i + 1]) / dx;",
     "c.theta = dx / (xy[2 * j + 1] - xy[2 * i + 1]);", 1),
    ("truncated scan", "for (int64_t s = 1; s + h <= n; ++s) {",
     "for (int64_t s = 1; s + h < n; ++s) {", 1),
    ("highest window on ties", "if (w < best) {", "if (w <= best) {", 1),
    ("vertical test on y", "if (xy[2 * j] == xy[2 * i]) {\n            ++vertical;",
     "if (xy[2 * j + 1] == xy[2 * i + 1]) {\n            ++vertical;", 1),
]


def battery():
    """Names of the pins the currently bound oracle library fails."""
    failed = []
    st = Stream(31, 310)
    sets = [st.integers(2 * n, 0, 6).reshape(n, 2).astype(np.float64) for n in (5, 6, 7)] + \
           [st.uniform(2 * n, -10, 10).reshape(n, 2) for n in (5, 7, 8)]
    for xy in sets:
        if len(set(xy[:, 0])) == 1:
            continue
        n = len(xy)
        for h in (0, n):
            want = float(lms_by_subsets(xy, h or default_h(n)))
            got = oracle.solve(xy, h=h)
            if not (got.status == 0 and abs(got.half_width - want) <= 1e-12 * max(want, 1e-300)
                    + (1e-12 if want == 0 else 0)):
                failed.append(f"subsets n={n} h={h}")
    xy = Stream(32, 320).uniform(24, -5, 5).reshape(12, 2)
    lp, _ = chebyshev_lp(xy)
    if not abs(oracle.solve(xy, h=12).half_width - lp) <= 1e-8 * max(1.0, lp):
        failed.append("chebyshev h=n")
    # certificate: the returned line holds h points within its half-width,
    # recomputed from the line itself
    xy = planted(60, 0.3, 33)
    r = oracle.solve(xy)
    hth = oracle.hth_abs_residual(xy, r.theta1, r.theta2)
    if not abs(hth - r.half_width) <= 1e-12 * r.half_width + 1e-14:
        failed.append("certificate")
    # all x equal, worked by hand: y = 0, 1, 2, 3, 10 with h = 2 -> width 1,
    # and the lowest of the tied windows, [0, 1]
    xe = np.array([[4.0, y] for y in (3.0, 0.0, 10.0, 2.0, 1.0)])
    r = oracle.solve(xe, h=2)
    if (r.status, r.width, r.z_lo, r.theta1) != (oracle.OK_DEGENERATE, 1.0, 0.0, 0.0):
        failed.append("all x equal")
    # a majority on y = -2x + 11 (integers): width exactly 0 on that line
    xs = np.arange(-6, 6, dtype=np.float64)
    on = np.stack([xs, -2.0 * xs + 11.0], 1)
    off = np.array([[0.5, 40.0], [3.5, -30.0], [1.5, 17.0], [-2.5, 0.0], [2.5, 9.0]])
    r = oracle.solve(np.concatenate([on, off]))
    if (r.width, r.theta1, r.theta2) != (0.0, -2.0, 11.0):
        failed.append("collinear majority")
    return failed


def _with_library(path):
    saved = oracle._lib
    oracle._lib = oracle.bind(path)
    try:
        return battery()
    finally:
        oracle._lib = saved


def test_unmutated_oracle_passes_battery(tmp_path):
    lib = oracle.build(src=SRC, out=str(tmp_path / "liblms_oracle_ref.so"))
    assert _with_library(lib) == []


@pytest.mark.parametrize("name,old,new,count", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_fails_a_pin(tmp_path, name, old, new, count):
    src = open(SRC).read()
    assert src.count(old) >= count, f"mutation site of '{name}' not found"
    mut = tmp_path / "lms_oracle_mut.c"
    mut.write_text(src.replace(old, new, count))
    # the header sits next to the original source
    lib = oracle.build(src=str(mut), out=str(tmp_path / "liblms_oracle_mut.so"))
    failed = _with_library(lib)
    print(name, "fails", failed)
    assert failed, f"mutant '{name}' passes every pin"
