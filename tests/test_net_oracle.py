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


def _tiny_params():
    """Weights chosen by hand, all exactly representable in BF16, so that the
    forward pass below can be followed on paper."""
    p = {k: np.zeros(net.SHAPES[k]) for k in net.ORDER}
    # layer 1: channel 0 = relu(x), channel 1 = relu(-x + 1), channel 2 = relu(y - 0.5)
    p["W1"][0] = (1.0, 0.0)
    p["W1"][1] = (-1.0, 0.0)
    p["b1"][1] = 1.0
    p["W1"][2] = (0.0, 1.0)
    p["b1"][2] = -0.5
    # layer 2: channel 0 = relu(h1_0 + 2 h1_2), channel 1 = relu(h1_1 - h1_0 - 0.25)
    p["W2"][0, 0], p["W2"][0, 2] = 1.0, 2.0
    p["W2"][1, 1], p["W2"][1, 0] = 1.0, -1.0
    p["b2"][1] = -0.25
    # head: h3_0 = relu(g0 - g1), h3_1 = relu(g1 + 1); out = (h3_0 - 0.5, 2 h3_1 - h3_0)
    p["W3"][0, 0], p["W3"][0, 1] = 1.0, -1.0
    p["W3"][1, 1] = 1.0
    p["b3"][1] = 1.0
    p["W4"][0, 0] = 1.0
    p["b4"][0] = -0.5
    p["W4"][1, 1], p["W4"][1, 0] = 2.0, -1.0
    return p


def test_forward_by_hand():
    """Three points worked through the layers on paper:
    (0.5, 1.0):  h1 = (0.5, 0.5, 0.5)   h2 = (1.5, 0)
    (-1.0, 0.0): h1 = (0, 2, 0)         h2 = (0, 1.75)
    (2.0, 0.75): h1 = (2, 0, 0.25)      h2 = (2.5, 0)
    max-pool g = (2.5, 1.75); h3 = (0.75, 2.75); out = (0.25, 4.75)."""
    p = _tiny_params()
    pts = np.array([[0.5, 1.0], [-1.0, 0.0], [2.0, 0.75]])
    out, cache = net.forward(p, pts)
    assert cache["g"][0] == 2.5 and cache["g"][1] == 1.75
    assert np.all(cache["g"][2:] == 0.0)
    assert list(cache["h3"][:2]) == [0.75, 2.75]
    assert list(out) == [0.25, 4.75]
    # one point alone: (0.5, 1.0) gives g = (1.5, 0), h3 = (1.5, 1), out = (1.0, 0.5)
    out1, _ = net.forward(p, pts[:1])
    assert list(out1) == [1.0, 0.5]


def test_forward_is_a_set_function():
    """Permuting the points changes neither the output nor the loss."""
    params = net.init_params(11)
    xy = planted(300, 0.4, 12)
    pts, _, _ = net.normalise(xy)
    out, _ = net.forward(params, pts)
    perm = Stream(3, 30).permutation(len(pts))
    out2, _ = net.forward(params, pts[perm])
    assert np.array_equal(out, out2)


def test_maxpool_gradient_goes_to_first_argmax():
    """Two points with the same features (W1 ignores y) tie in every channel;
    the gradient must reach only the first of them. The W1[:, 1] gradient is
    the routed point's y times its channel gradient, so it tells which one."""
    p = _tiny_params()
    p["W1"][2] = (0.0, 0.0)  # no channel reads y any more
    p["b1"][2] = 0.0
    for first_y, other_y in ((0.0, 5.0), (5.0, 0.0)):
        # (2, y): h1 = (2, 0, 0), h2 = (2, 0); (0.5, 1): h1 = (0.5, 0.5, 0), h2 = (0.5, 0)
        pts = np.array([[2.0, first_y], [2.0, other_y], [0.5, 1.0]])
        out, cache = net.forward(p, pts)
        assert cache["arg"][0] == 0 and cache["g"][0] == 2.0
        # g = (2, 0): h3_0 = relu(2) = 2 is active, so d out0 / d g0 = 1, routed
        # to the first tied point; there dz1 = (1, 0, 0) and dW1[0] = (x, y)
        g = net.backward(cache, np.array([1.0, 0.0]))
        assert g["W1"][0, 0] == 2.0 and g["W1"][0, 1] == first_y


def test_target_at_known_angles():
    """(cos 2phi, sin 2phi) of the line angle phi in the normalised frame,
    where a slope theta1 becomes theta1 * sx / sy."""
    cases = [(0.0, 1.0, 1.0, (1.0, 0.0)),          # horizontal line
             (1.0, 1.0, 1.0, (0.0, 1.0)),          # 45 degrees: 2 phi = 90
             (-1.0, 2.0, 2.0, (0.0, -1.0)),        # -45 degrees
             (np.sqrt(3.0), 1.0, 1.0, (-0.5, np.sqrt(3.0) / 2)),  # 60 degrees
             (0.5, 2.0, 1.0, (0.0, 1.0)),          # slope 0.5 in a frame scaled 2:1 -> 45
             (1e300, 1.0, 1.0, (-1.0, 0.0))]       # near vertical: 2 phi -> 180
    for th, sx, sy, want in cases:
        t = net.target_from_slope(th, sx, sy)
        assert np.allclose(t, want, atol=1e-12), (th, sx, sy, t)
    assert abs(net.slope_from_output(np.array([0.0, 1.0]), 1.0, 1.0) - 1.0) < 1e-12
    assert abs(net.slope_from_output(np.array([0.0, 3.0]), 2.0, 6.0) - 3.0) < 1e-12
    assert net.slope_from_output(np.array([2.0, 0.0]), 1.0, 1.0) == 0.0


def test_normalise_by_hand():
    """Lower median and MAD, worked by hand."""
    # x: sorted 1 3 5 7 9 -> centre 5; |x - 5| sorted 0 2 2 4 4 -> scale 2
    # y: sorted 1 2 3 4 10 -> centre 3; |y - 3| sorted 0 1 1 2 7 -> scale 1
    xy = np.array([[5.0, 10.0], [1.0, 2.0], [9.0, 3.0], [3.0, 4.0], [7.0, 1.0]])
    pts, c, s = net.normalise(xy)
    assert list(c) == [5.0, 3.0] and list(s) == [2.0, 1.0]
    assert list(pts[:, 0]) == [0.0, -2.0, 2.0, -1.0, 1.0]
    assert list(pts[:, 1]) == [7.0, -1.0, 0.0, 1.0, -2.0]
    # even count: the lower of the two middle values; a zero MAD falls back to
    # the largest deviation; a constant coordinate to 1
    xy = np.array([[3.0, 4.0], [3.0, 4.0], [3.0, 4.0], [8.0, 4.0]])
    _, c, s = net.normalise(xy)
    assert list(c) == [3.0, 4.0] and list(s) == [5.0, 1.0]
    _, c, s = net.normalise(np.array([[4.0, 0.0], [1.0, 0.0], [3.0, 0.0], [2.0, 1.0]]))
    assert c[0] == 2.0 and s[0] == 1.0  # sorted 1 2 3 4 -> 2; |x - 2| 0 1 1 2 -> 1


def test_normalise_uses_the_strided_sample():
    """510 points: the frame comes from points 0, 2, 4, ... (floor(k 510 / 255)
    = 2k), so the odd points, huge here, move neither centre nor scale. The
    sampled x are 0, 2, ..., 508: centre 254 (rank 127); deviations 0, 2, 2,
    4, 4, ...: rank 127 is 128."""
    n = 510
    x = np.where(np.arange(n) % 2 == 0, np.arange(n, dtype=np.float64), 1e9)
    xy = np.stack([x, np.zeros(n)], 1)
    assert list(net.frame_sample(n)[:4]) == [0, 2, 4, 6]
    _, c, s = net.normalise(xy)
    assert c[0] == 254.0 and s[0] == 128.0
