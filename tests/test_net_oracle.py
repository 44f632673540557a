"""Pins for the network reference (oracle/net.py): its backward pass against
central finite differences of its own forward pass (exact arithmetic, no BF16
rounding, where the loss is smooth), and the BF16 rounding against known
values."""
import numpy as np

from oracle import net
from workloads.gen import Stream, planted


def small_batch(seed, n=40, B=3):
    sets, targets = [], []
    st = Stream(seed, 5)
    for b in range(B):
        xy = planted(n, 0.3, seed * 10 + b)
        pts, c, s = net.normalise(xy)
        sets.append(pts)
        targets.append(net.target_from_slope(0.7, s[0], s[1]))
    return sets, np.array(targets), st


def test_backward_matches_finite_differences():
    params = net.init_params(3)
    for k in params:
        if k.startswith("b"):
            params[k] = Stream(4, hash(k) % 1000).uniform(params[k].size, -0.1, 0.1)
    sets, targets, _ = small_batch(7)
    loss, grad, _ = net.loss_and_grad(params, sets, targets, round_bf16=False)
    st = Stream(8, 80)
    eps = 1e-6
    for k in net.ORDER:
        flat = params[k].reshape(-1)
        idx = st.integers(min(12, flat.size), 0, flat.size - 1)
        for i in idx:
            old = flat[i]
            flat[i] = old + eps
            lp, _, _ = net.loss_and_grad(params, sets, targets, round_bf16=False)
            flat[i] = old - eps
            lm, _, _ = net.loss_and_grad(params, sets, targets, round_bf16=False)
            flat[i] = old
            fd = (lp - lm) / (2 * eps)
            an = grad[k].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 + 1e-5 * abs(fd), (k, i, fd, an)


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -9, -3.14159265, 0.0])
    r = net.bf16(v)
    assert r[0] == 1.0
    assert r[1] == 1.0 + 2 ** -7 or r[1] == 1.0  # 2^-8 is exactly half an ulp: ties to even
    assert r[1] == 1.0  # 1.0 has an even mantissa
    assert r[2] == 1.0
    assert r[3] == 1.0 + 2 ** -7
    assert r[4] == -3.140625
    assert r[5] == 0.0


def test_target_roundtrip():
    for th in (0.0, 0.7, -3.0, 250.0, -1e-3):
        t = net.target_from_slope(th, 2.0, 5.0)
        assert abs(net.slope_from_output(t, 2.0, 5.0) - th) <= 1e-9 * max(1, abs(th))
    # a line and its reverse direction give the same target
    a = net.target_from_slope(1e12, 1.0, 1.0)
    b = net.target_from_slope(-1e12, 1.0, 1.0)
    assert np.allclose(a, b)
