"""Adversarial numerics, GPU path against the oracle through the C ABI:
huge coordinate offsets, power-of-two scalings by 2^+-200, pairs whose x
differ by about 1e-12, and lines of slope about 1e8. The FP32 screen's error
bound, the FP64 hand-off of steep or near-vertical pairs and the FP64
recheck must keep the answer exact in each case."""
import numpy as np
import pytest
import torch

from workloads.gen import Stream, planted

pytestmark = pytest.mark.gpu


def dev(xy):
    return torch.from_numpy(np.ascontiguousarray(xy)).to("cuda:0")


def check(gpu, orc, xy, bitwise=True, **kw):
    """Exact parity where the FP64 evaluation of F resolves the candidates;
    with huge coordinates it carries an absolute rounding of up to
    4 * 2^-53 * max|z| per window, and near-optimal slopes whose widths differ
    by less than that can swap places in the oracle's FP64 order. Then the
    widths agree to 1e-9 relative plus 8 * 2^-53 * max|z|, and the oracle
    certifies the GPU's window at its own slope."""
    r = gpu.solve(dev(xy), **kw)
    o = orc.solve(xy)
    print(len(xy), r.width, o.width, r.theta1, o.theta1, flush=True)
    assert r.status == o.status
    zmax = np.abs(xy[:, 1]).max() + abs(o.theta1) * np.abs(xy[:, 0]).max()
    tol = 1e-9 * max(r.width, o.width) + 8 * 2.0 ** -53 * zmax
    assert abs(r.width - o.width) <= tol or r.width == o.width
    if bitwise:
        assert (r.width, r.theta1, r.z_lo, r.z_hi) == (o.width, o.theta1, o.z_lo, o.z_hi)
    else:
        assert orc.window(xy, r.theta1) == (r.width, r.z_lo, r.z_hi)
    assert r.vertical == o.vertical and r.candidates == o.candidates
    return r, o


@pytest.mark.parametrize("n", [300, 1500])
def test_huge_offsets(gpu, orc, n):
    xy = planted(n, 0.45, 3100 + n) + np.array([1e6, 1e6])
    check(gpu, orc, xy)
    xy = planted(n, 0.45, 3200 + n) + np.array([-3e9, 7e9])
    check(gpu, orc, xy, bitwise=False)


@pytest.mark.parametrize("k", [-200, -60, 60, 200])
def test_power_of_two_scalings(gpu, orc, k):
    base = planted(700, 0.45, 3300)
    sx, sy = 2.0 ** k, 2.0 ** (-k // 2)
    xy = base * np.array([sx, sy])
    r, o = check(gpu, orc, xy)
    # exact scalings: the unscaled answer maps over bit for bit
    b = gpu.solve(dev(base))
    assert r.width == b.width * sy and r.theta1 == b.theta1 * sy / sx


def test_near_equal_x(gpu, orc):
    """Pairs whose x differ by about 1e-12 (relative 1e-13): their slopes are
    huge and their FP32 bound useless; they must go to the FP64 path."""
    st = Stream(34, 340)
    base = planted(600, 0.4, 3400)
    twins = base[:150].copy()
    twins[:, 0] += st.uniform(150, 0.5e-12, 2e-12)
    twins[:, 1] += st.uniform(150, -1.0, 1.0)
    xy = np.concatenate([base, twins])[Stream(35, 350).permutation(750)]
    check(gpu, orc, xy, bitwise=False)


@pytest.mark.parametrize("slope", [1e8, -3e8, 1e12])
def test_very_steep_lines(gpu, orc, slope):
    st = Stream(36, 360)
    n = 500
    n_in = 300
    x = st.uniform(n, -10.0, 10.0)
    y = slope * x + st.normal(n) * abs(slope) * 1e-3
    y[n_in:] = st.uniform(n - n_in, -20.0, 20.0) * abs(slope)
    xy = np.stack([x, y], 1)[st.permutation(n)]
    check(gpu, orc, xy, bitwise=False)
