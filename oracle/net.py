"""FP64 reference of the point-set network that proposes a seed slope.

TEST INFRASTRUCTURE ONLY. Used to check the GPU forward and backward kernels.
It shares no code with them.

The network is not in the paper. It is the learned incumbent of this build:
any slope it proposes only sets the exact search's initial width bound, since
F(theta) >= the optimum for every theta (Eq. (1)). The search stays exact
whatever the network predicts.

Architecture, for one set of n points p_k in the set's robust frame (see
normalise: coordinate-wise median and MAD of a fixed sample of the points):
    h1_k = relu(W1 p_k + b1)            (64)
    h2_k = relu(W2 bf16(h1_k) + b2)     (64)
    g    = max_k h2_k                   (64, per channel)
    h3   = relu(W3 g + b3)              (64)
    out  = W4 h3 + b4                   (2)  ~ (cos 2phi, sin 2phi)
phi is the line angle in the normalised frame; doubling it makes lines of
angle phi and phi + pi the same target. The weights are BF16 copies of FP32
masters, and h1 is rounded to BF16 before the second product. Everything else
is FP64 here (FP32 on the GPU). Loss: mean over sets of 0.5 ||out - target||^2.
The gradient passes straight through the BF16 roundings, and the max-pool sends
each channel's gradient to the first point attaining the maximum.
"""
from __future__ import annotations

import numpy as np

HIDDEN = 64
SHAPES = {"W1": (HIDDEN, 2), "b1": (HIDDEN,), "W2": (HIDDEN, HIDDEN), "b2": (HIDDEN,),
          "W3": (HIDDEN, HIDDEN), "b3": (HIDDEN,), "W4": (2, HIDDEN), "b4": (2,)}
ORDER = ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4")


def bf16(a: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), via the float32 bits."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


SAMPLE = 255  # points of a set that fix its frame


def frame_sample(n: int) -> np.ndarray:
    """Indices that fix a set's frame: all points up to SAMPLE of them, else
    floor(k n / SAMPLE) for k = 0 .. SAMPLE - 1."""
    if n <= SAMPLE:
        return np.arange(n)
    return (np.arange(SAMPLE, dtype=np.int64) * n) // SAMPLE


def _lower_median(v: np.ndarray) -> float:
    """The value of rank floor((m - 1) / 2) among m values."""
    return float(np.sort(v, kind="stable")[(len(v) - 1) // 2])


def normalise(xy: np.ndarray):
    """Robust frame per coordinate: centre = the lower median of the sampled
    values, scale = the lower median of their absolute deviations from it (the
    MAD), else the largest deviation, else 1. Outliers, up to half of the
    points, move neither. Returns (points in that frame, centre, scale)."""
    smp = xy[frame_sample(len(xy))]
    c = np.empty(2)
    s = np.empty(2)
    for a in range(2):
        c[a] = _lower_median(smp[:, a])
        dev = np.abs(smp[:, a] - c[a])
        s[a] = _lower_median(dev)
        if not s[a] > 0:
            s[a] = dev.max()
        if not s[a] > 0:
            s[a] = 1.0
    return (xy - c) / s, c, s


def target_from_slope(theta1: float, sx: float, sy: float) -> np.ndarray:
    """(cos 2phi, sin 2phi) of the line's angle in the normalised frame."""
    phi = np.arctan(theta1 * sx / sy)
    return np.array([np.cos(2 * phi), np.sin(2 * phi)])


def slope_from_output(out: np.ndarray, sx: float, sy: float) -> float:
    phi = 0.5 * np.arctan2(out[1], out[0])
    return float(np.tan(phi) * sy / sx)


def forward(params: dict, pts: np.ndarray, round_bf16: bool = True):
    """Forward pass of one set; returns out and the cache the backward needs."""
    q = bf16 if round_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    W1, W2, W3, W4 = (q(params[k]) for k in ("W1", "W2", "W3", "W4"))
    z1 = pts @ W1.T + params["b1"]
    h1 = np.maximum(z1, 0.0)
    h1q = q(h1)
    z2 = h1q @ W2.T + params["b2"]
    h2 = np.maximum(z2, 0.0)
    arg = np.argmax(h2, axis=0)  # first maximiser per channel
    g = h2[arg, np.arange(HIDDEN)]
    z3 = W3 @ g + params["b3"]
    h3 = np.maximum(z3, 0.0)
    out = W4 @ h3 + params["b4"]
    cache = dict(pts=pts, W1=W1, W2=W2, W3=W3, W4=W4, z1=z1, h1q=h1q, z2=z2, arg=arg, g=g,
                 z3=z3, h3=h3)
    return out, cache


def backward(cache: dict, dout: np.ndarray) -> dict:
    """Gradients of a loss with d loss / d out = dout for one set."""
    c = cache
    gr = {}
    gr["W4"] = np.outer(dout, c["h3"])
    gr["b4"] = dout.copy()
    dh3 = c["W4"].T @ dout
    dz3 = dh3 * (c["z3"] > 0)
    gr["W3"] = np.outer(dz3, c["g"])
    gr["b3"] = dz3
    dg = c["W3"].T @ dz3
    n = c["pts"].shape[0]
    dz2 = np.zeros((n, HIDDEN))
    ch = np.arange(HIDDEN)
    dz2[c["arg"], ch] = dg * (c["z2"][c["arg"], ch] > 0)
    gr["W2"] = dz2.T @ c["h1q"]
    gr["b2"] = dz2.sum(0)
    dh1 = dz2 @ c["W2"]
    dz1 = dh1 * (c["z1"] > 0)
    gr["W1"] = dz1.T @ c["pts"]
    gr["b1"] = dz1.sum(0)
    return gr


def loss_and_grad(params: dict, sets: list, targets: np.ndarray, round_bf16: bool = True):
    """Mean loss over sets and its gradient (dict of arrays)."""
    tot = {k: np.zeros(SHAPES[k]) for k in ORDER}
    loss = 0.0
    B = len(sets)
    outs = []
    for pts, t in zip(sets, targets):
        out, cache = forward(params, pts, round_bf16)
        outs.append(out)
        loss += 0.5 * np.sum((out - t) ** 2) / B
        gr = backward(cache, (out - t) / B)
        for k in ORDER:
            tot[k] += gr[k]
    return loss, tot, np.array(outs)


def init_params(seed: int) -> dict:
    """He-style uniform initialisation from a SplitMix64 stream."""
    from workloads.gen import Stream
    st = Stream(seed, 4242)
    p = {}
    for k in ORDER:
        shp = SHAPES[k]
        if k.startswith("W"):
            fan_in = shp[1]
            lim = np.sqrt(6.0 / fan_in)
            p[k] = st.uniform(int(np.prod(shp)), -lim, lim).reshape(shp)
        else:
            p[k] = np.zeros(shp)
    return p


def predict(params: dict, xy: np.ndarray, max_points: int = 2048):
    """Inference on one raw set: the frame of the whole set (normalise), the
    features pooled over at most max_points points (a larger set is read at
    indices floor(j n / max_points)), the head; returns (out, slope in the
    original frame)."""
    pts, c, s = normalise(xy)
    n = len(xy)
    if n > max_points:
        pts = pts[(np.arange(max_points, dtype=np.int64) * n) // max_points]
    # the GPU rounds the framed points to FP32
    pts = pts.astype(np.float32).astype(np.float64)
    out, _ = forward(params, pts)
    return out, slope_from_output(out, s[0], s[1])
