"""Algorithm 1 as stated (lms_solve_bracelets) against the oracle's bracelet
search, through the C ABI.

The GPU kernels and the oracle compute the same operations (IEEE division for
the slope, fma intercepts with the pair's members set to z_i, a full sort, the
far end h - 1 ranks from the vertex rank, the canonical key), so every field
must agree bit for bit, for both rank readings. With the tied-rank reading the
minimum is also the LMS width of the exhaustive window search (to 1e-9), and
the oracle certifies the returned line.
"""
import numpy as np
import pytest
import torch

from workloads import gen
from workloads.gen import Stream, default_h, degenerate_int, planted

pytestmark = pytest.mark.gpu


def dev(xy):
    return torch.from_numpy(np.ascontiguousarray(xy)).to("cuda:0")


def fields(r):
    return (r.width, r.theta1, r.theta2, r.z_lo, r.z_hi, r.pair_i, r.pair_j, r.candidates,
            r.vertical, r.status)


@pytest.mark.parametrize("n", [2, 3, 5, 17, 64, 100, 128, 129, 255, 256, 300, 512, 777])
def test_bracelets_bitwise(gpu, orc, n):
    sets = [planted(n, 0.4, 1200 + n)]
    if 5 <= n <= 512:
        sets.append(degenerate_int(n, 1300 + n))
    for xy in sets:
        for rule in (gpu.RULE_TIED, gpu.RULE_LITERAL):
            r = gpu.solve_bracelets(dev(xy), rule=rule)
            o = orc.bracelets(xy, rule=rule)
            print(n, rule, r.width, o.width, flush=True)
            assert fields(r) == fields(o), (n, rule)
        if n <= 300:
            # the bracelet sets the pair's own two intercepts to one value,
            # the window search computes both: the widths agree to rounding
            # of the intercepts (a few ulp of the largest |z|)
            s = orc.solve(xy)
            t = gpu.solve_bracelets(dev(xy))
            ulp = 8 * 2.0 ** -53 * (np.abs(xy[:, 1]).max() + abs(t.theta1) * np.abs(xy[:, 0]).max())
            assert abs(t.width - s.width) <= 1e-9 * s.width + ulp
            assert orc.window(xy, t.theta1)[0] <= t.width + ulp


@pytest.mark.parametrize("n,h", [(64, 2), (64, 40), (64, 64), (129, 100), (256, 129)])
def test_bracelets_general_h(gpu, orc, n, h):
    xy = planted(n, 0.3, 1400 + n + h)
    for rule in (gpu.RULE_TIED, gpu.RULE_LITERAL):
        assert fields(gpu.solve_bracelets(dev(xy), h, rule)) == fields(orc.bracelets(xy, h, rule))


def test_bracelets_paper_sizes_and_stored_c1(gpu, orc):
    """The paper's set sizes (Table 1), and the stored 256-point oracle result:
    the tied-rank minimum is the LMS width."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_results.json")))
    g = gold["c1/101"]
    r = gpu.solve_bracelets(dev(gen.make("c1", 101)))
    w = float.fromhex(g["width"])
    assert abs(r.width - w) <= 1e-9 * w
    for n in (128, 512):
        xy = planted(n, 0.4, 1500 + n)
        a = gpu.solve_bracelets(dev(xy))
        b = gpu.solve(dev(xy))
        assert abs(a.width - b.width) <= 1e-9 * b.width, n


@pytest.mark.parametrize("n", [1500, 2048])
def test_bracelets_largest_sizes(gpu, orc, n):
    """Up to the largest size (the oracle's bracelet search takes minutes
    there): the tied-rank minimum is the LMS width of lms_solve, and the
    oracle certifies the returned line's window at its slope."""
    xy = planted(n, 0.45, 1600 + n)
    a = gpu.solve_bracelets(dev(xy))
    b = gpu.solve(dev(xy))
    ulp = 8 * 2.0 ** -53 * (np.abs(xy[:, 1]).max() + abs(a.theta1) * np.abs(xy[:, 0]).max())
    assert abs(a.width - b.width) <= 1e-9 * b.width + ulp
    assert orc.window(xy, a.theta1)[0] <= a.width + ulp
    assert a.candidates == n * (n - 1) // 2 - a.vertical


def test_bracelets_degenerate_inputs(gpu, orc):
    y = Stream(5, 50).uniform(40, -3, 3)
    xe = np.stack([np.full(40, 1.5), y], 1)
    r = gpu.solve_bracelets(dev(xe))
    o = orc.solve(xe)
    assert r.status == 1 and (r.width, r.z_lo, r.theta1) == (o.width, o.z_lo, 0.0)
    bad = planted(50, 0.3, 3)
    bad[7, 1] = np.nan
    assert gpu.solve_bracelets(dev(bad)).status == gpu.LMS_ERR_NONFINITE
    with pytest.raises(gpu.LmsError):
        gpu.solve_bracelets(dev(planted(gpu.ALG1_MAX_N + 1, 0.3, 4)))


def test_literal_rule_misses_where_the_oracle_says(gpu, orc):
    """The printed rank rule, run on the GPU, misses the optimum exactly on
    the sets where the oracle's literal reading does."""
    st = Stream(6, 60)
    misses = 0
    for _ in range(40):
        xy = st.uniform(32, -100, 100).reshape(16, 2)
        lit = gpu.solve_bracelets(dev(xy), rule=gpu.RULE_LITERAL)
        tied = gpu.solve_bracelets(dev(xy), rule=gpu.RULE_TIED)
        assert lit.width == orc.bracelets(xy, rule=orc.RULE_LITERAL).width
        misses += lit.width > tied.width
    assert misses > 0
