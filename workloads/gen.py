"""Seeded synthetic point sets for the exact 2D LMS line search.

This module holds only input generation. It contains none of the estimator's
arithmetic, and it is the one piece shared by the CPU oracle's tests and the
GPU path's tests and benchmark.

Determinism across machines
---------------------------
Every value comes from a counter-based SplitMix64 stream (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014) and is
turned into coordinates with IEEE basic operations only (+, -, *, /, sqrt,
frexp and integer ops). Those are correctly rounded everywhere, so a seed gives
the same bytes on any x86 host, whatever SIMD level numpy picks. Normal
deviates use Marsaglia's polar method with a natural log written below from
the atanh series, instead of libm's log, whose last bit may differ between
builds.

Workloads
---------
The paper times exact LMS on random point sets of 128, 256 and 512 points
(Section 4, Table 1) and motivates the batched form with one LMS per Hough
peak on edge images (Section 5). Neither data set is published, so these
generators stand in for them:

* ``planted``: a line y = 0.7x + 2 with N(0, 0.05^2) vertical noise, plus a
  fraction of uniform outliers in [-10,10]x[-20,20].
* ``degenerate_int``: integer coordinates in [0,1023]^2 with a noisy planted
  line, uniform points, and 30 % of the points copying another point's x.
  This gives many vertical pairs, coincident points and exact width ties.
* ``hough_patches``: many small 64x64-pixel edge patches, each holding one
  rasterised line with +-1 px jitter plus 30-45 % salt noise, packed as CSR.
"""
from __future__ import annotations

import numpy as np

_M64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15
_LN2 = 0.6931471805599453  # nearest double to ln 2


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = z.astype(np.uint64, copy=True)
    z ^= z >> np.uint64(30)
    z *= np.uint64(0xBF58476D1CE4E5B9)
    z ^= z >> np.uint64(27)
    z *= np.uint64(0x94D049BB133111EB)
    z ^= z >> np.uint64(31)
    return z


def splitmix64(state: int, count: int) -> np.ndarray:
    """The first `count` outputs of SplitMix64 started at `state`: output k
    (0-based) is mix64(state + (k+1) * gamma)."""
    k = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(state & _M64) + k * np.uint64(_GAMMA)
    return _mix64(z)


def _key(seed: int, stream: int) -> int:
    """Starting state of an independent stream for (seed, stream)."""
    s = np.array([(seed * 0x2545F4914F6CDD1D + stream * _GAMMA + 0x1234567) & _M64],
                 dtype=np.uint64)
    return int(_mix64(s)[0])


class Stream:
    """A counter-based SplitMix64 stream: value k is mix64(key + (k+1)*gamma)."""

    def __init__(self, seed: int, stream: int):
        self.key = _key(seed, stream)
        self.pos = 0

    def u64(self, count: int) -> np.ndarray:
        k = np.arange(self.pos + 1, self.pos + 1 + count, dtype=np.uint64)
        self.pos += count
        with np.errstate(over="ignore"):
            z = np.uint64(self.key) + k * np.uint64(_GAMMA)
        return _mix64(z)

    def uniform(self, count: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
        """Uniform doubles on [lo, hi) from the top 53 bits."""
        u = (self.u64(count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
        return lo + (hi - lo) * u

    def integers(self, count: int, lo: int, hi: int) -> np.ndarray:
        """Uniform integers on [lo, hi] (inclusive), as int64."""
        span = np.uint64(hi - lo + 1)
        return (self.u64(count) % span).astype(np.int64) + lo

    def normal(self, count: int) -> np.ndarray:
        """Standard normal deviates (Marsaglia polar method)."""
        out = np.empty(count, dtype=np.float64)
        have = 0
        while have < count:
            need = count - have
            m = need // 2 + 1
            tries = int(m * 1.35) + 16
            u = self.uniform(tries, -1.0, 1.0)
            v = self.uniform(tries, -1.0, 1.0)
            s = u * u + v * v
            ok = (s > 0.0) & (s < 1.0)
            u, v, s = u[ok], v[ok], s[ok]
            f = np.sqrt(-2.0 * ln(s) / s)
            pair = np.empty(2 * len(s), dtype=np.float64)
            pair[0::2] = u * f
            pair[1::2] = v * f
            take = min(need, len(pair))
            out[have:have + take] = pair[:take]
            have += take
        return out

    def permutation(self, count: int) -> np.ndarray:
        """A uniformly random permutation of range(count)."""
        keys = self.u64(count)
        return np.argsort(keys, kind="stable")


def ln(s: np.ndarray) -> np.ndarray:
    """Natural log of positive doubles using basic operations only.

    s = m * 2^e with m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(t) with
    t = (m-1)/(m+1), |t| <= 0.1716, summed to 14 odd terms (error < 1e-19).
    """
    s = np.asarray(s, dtype=np.float64)
    m, e = np.frexp(s)
    small = m < 0.7071067811865476
    m = np.where(small, m * 2.0, m)
    e = np.where(small, e - 1, e).astype(np.float64)
    t = (m - 1.0) / (m + 1.0)
    t2 = t * t
    acc = np.zeros_like(t)
    for k in range(27, 0, -2):
        acc = acc * t2 + 1.0 / k
    return e * _LN2 + 2.0 * t * acc


# --------------------------------------------------------------------------
# Generators
# --------------------------------------------------------------------------

def planted(n: int, f_out: float, seed: int) -> np.ndarray:
    """Planted line y = 0.7x + 2 + N(0, 0.05^2) with uniform outliers.

    n_out = round(f_out * n) outliers uniform in [-10,10]x[-20,20]; the other
    points have x ~ U(-10,10). Returned as an (n, 2) float64 array, shuffled.
    """
    n_out = int(round(f_out * n))
    n_in = n - n_out
    st = Stream(seed, 1)
    xi = st.uniform(n_in, -10.0, 10.0)
    yi = 0.7 * xi + 2.0 + 0.05 * st.normal(n_in)
    xo = st.uniform(n_out, -10.0, 10.0)
    yo = st.uniform(n_out, -20.0, 20.0)
    xy = np.empty((n, 2), dtype=np.float64)
    xy[:n_in, 0], xy[:n_in, 1] = xi, yi
    xy[n_in:, 0], xy[n_in:, 1] = xo, yo
    return np.ascontiguousarray(xy[st.permutation(n)])


def degenerate_int(n: int, seed: int, dup_frac: float = 0.30) -> np.ndarray:
    """Integer points in [0,1023]^2 with duplicated x values and exact ties.

    55 % of the points follow y = clamp(round(0.7x + 150 + N(0, 2^2))), the
    rest are uniform; then a random dup_frac of the points take the x of a
    random point, so vertical pairs and coincident points are common.
    """
    n_line = int(round(0.55 * n))
    n_uni = n - n_line
    st = Stream(seed, 2)
    xl = st.integers(n_line, 0, 1023).astype(np.float64)
    yl = np.clip(np.round(0.7 * xl + 150.0 + 2.0 * st.normal(n_line)), 0.0, 1023.0)
    xu = st.integers(n_uni, 0, 1023).astype(np.float64)
    yu = st.integers(n_uni, 0, 1023).astype(np.float64)
    xy = np.empty((n, 2), dtype=np.float64)
    xy[:n_line, 0], xy[:n_line, 1] = xl, yl
    xy[n_line:, 0], xy[n_line:, 1] = xu, yu
    xy = xy[st.permutation(n)]
    m = int(round(dup_frac * n))
    copiers = st.permutation(n)[:m]
    sources = st.integers(m, 0, n - 1)
    x = xy[:, 0].copy()
    x[copiers] = xy[sources, 0]
    xy[:, 0] = x
    return np.ascontiguousarray(xy)


def _unit_upper(st: Stream, count: int) -> tuple[np.ndarray, np.ndarray]:
    """Unit vectors with angle uniform on [0, pi): rejection from the disk."""
    cx = np.empty(count)
    cy = np.empty(count)
    have = 0
    while have < count:
        need = count - have
        t = int(need * 1.35) + 16
        u = st.uniform(t, -1.0, 1.0)
        v = st.uniform(t, -1.0, 1.0)
        r2 = u * u + v * v
        ok = (r2 > 1e-6) & (r2 < 1.0)
        u, v, r2 = u[ok], v[ok], r2[ok]
        r = np.sqrt(r2)
        u, v = u / r, v / r
        flip = (v < 0.0) | ((v == 0.0) & (u < 0.0))
        u = np.where(flip, -u, u)
        v = np.where(flip, -v, v)
        take = min(need, len(u))
        cx[have:have + take] = u[:take]
        cy[have:have + take] = v[:take]
        have += take
    return cx, cy


def hough_patches(B: int, seed: int, n_lo: int = 32, n_hi: int = 512,
                  side: int = 64) -> tuple[np.ndarray, np.ndarray]:
    """B independent edge-pixel patches of a side x side image, CSR-packed.

    Per problem: n_b ~ U{n_lo..n_hi}; noise fraction f ~ U[0.30, 0.45] with
    round(f n_b) salt pixels uniform on the grid; the other pixels lie on one
    line through c ~ U([16,47]^2) at angle phi ~ U[0, pi), rasterised as
    round(c + t (cos phi, sin phi) + j (-sin phi, cos phi)) with t ~ U(-45,45)
    and j in {-1, 0, 1}, redrawn until inside the patch. Duplicate pixels are
    allowed. Returns (xy float64 (N,2), offsets int64 (B+1,)).
    """
    st = Stream(seed, 3)
    nb = st.integers(B, n_lo, n_hi)
    fb = st.uniform(B, 0.30, 0.45)
    n_noise = np.round(fb * nb).astype(np.int64)
    n_line = nb - n_noise
    dx, dy = _unit_upper(st, B)
    c = st.uniform(2 * B, 16.0, 47.0).reshape(B, 2)
    offsets = np.zeros(B + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(nb)
    N = int(offsets[-1])

    # line pixels, all problems at once, redrawn in rounds until inside
    pid = np.repeat(np.arange(B), n_line)
    L = len(pid)
    lx = np.empty(L)
    ly = np.empty(L)
    todo = np.arange(L)
    hi = float(side - 1)
    while len(todo):
        p = pid[todo]
        t = st.uniform(len(todo), -45.0, 45.0)
        j = st.integers(len(todo), -1, 1).astype(np.float64)
        px = np.round(c[p, 0] + t * dx[p] - j * dy[p])
        py = np.round(c[p, 1] + t * dy[p] + j * dx[p])
        ok = (px >= 0.0) & (px <= hi) & (py >= 0.0) & (py <= hi)
        lx[todo[ok]] = px[ok]
        ly[todo[ok]] = py[ok]
        todo = todo[~ok]

    npid = np.repeat(np.arange(B), n_noise)
    nx = st.integers(len(npid), 0, side - 1).astype(np.float64)
    ny = st.integers(len(npid), 0, side - 1).astype(np.float64)

    allp = np.concatenate([pid, npid])
    allx = np.concatenate([lx, nx])
    ally = np.concatenate([ly, ny])
    order = np.lexsort((st.u64(N), allp))  # by problem, random inside it
    xy = np.empty((N, 2), dtype=np.float64)
    xy[:, 0] = allx[order]
    xy[:, 1] = ally[order]
    return np.ascontiguousarray(xy), offsets


def rotated_line(count: int, n: int, seed: int, f_lo: float = 0.0, f_hi: float = 0.45):
    """count sets of n points around a line at a random angle (training data).

    Per set: outlier fraction f ~ U[f_lo, f_hi]; round(f n) outliers uniform in
    [-10,10]x[-20,20]; the other points c + t (cos phi, sin phi) +
    e (-sin phi, cos phi) with phi ~ U[-pi/2, pi/2), c ~ U([-2,2]^2),
    t ~ U(-10,10), e ~ N(0, 0.05^2). Returns (xy (count*n, 2), offsets).
    """
    st = Stream(seed, 6)
    f = st.uniform(count, f_lo, f_hi)
    n_out = np.round(f * n).astype(np.int64)
    # direction with cos phi >= 0: uniform angle on [-pi/2, pi/2)
    dx = np.empty(count)
    dy = np.empty(count)
    have = 0
    while have < count:
        need = count - have
        t = int(need * 1.35) + 16
        u = st.uniform(t, -1.0, 1.0)
        v = st.uniform(t, -1.0, 1.0)
        r2 = u * u + v * v
        ok = (r2 > 1e-6) & (r2 < 1.0)
        u, v, r2 = u[ok], v[ok], r2[ok]
        r = np.sqrt(r2)
        u, v = u / r, v / r
        flip = u < 0.0
        u = np.where(flip, -u, u)
        v = np.where(flip, -v, v)
        take = min(need, len(u))
        dx[have:have + take] = u[:take]
        dy[have:have + take] = v[:take]
        have += take
    c = st.uniform(2 * count, -2.0, 2.0).reshape(count, 2)
    N = count * n
    pid = np.repeat(np.arange(count), n)
    k = np.tile(np.arange(n), count)
    is_out = k < n_out[pid]
    t = st.uniform(N, -10.0, 10.0)
    e = 0.05 * st.normal(N)
    x = c[pid, 0] + t * dx[pid] - e * dy[pid]
    y = c[pid, 1] + t * dy[pid] + e * dx[pid]
    ox = st.uniform(N, -10.0, 10.0)
    oy = st.uniform(N, -20.0, 20.0)
    x = np.where(is_out, ox, x)
    y = np.where(is_out, oy, y)
    order = np.lexsort((st.u64(N), pid))
    xy = np.empty((N, 2), dtype=np.float64)
    xy[:, 0] = x[order]
    xy[:, 1] = y[order]
    offsets = np.arange(count + 1, dtype=np.int64) * n
    return np.ascontiguousarray(xy), offsets


def line_image(p_noise: float, seed: int, size: int = 1024, p_line: float = 0.5,
               min_len: float = 400.0, margin: int = 16):
    """Edge pixels of a synthetic size x size image: one line segment whose
    pixels are kept with probability p_line, plus salt noise, each pixel on
    with probability p_noise (the line-detection images of Section 5.1).

    The segment joins two points uniform in [margin, size-1-margin]^2, redrawn
    until it is at least min_len long; it is rasterised at unit steps along its
    longer axis. Returns (pix int32 (N, 2) of (x, y) in raster order,
    on_line bool (N,), segment (x0, y0, x1, y1) float64).
    """
    st = Stream(seed, 7)
    lo, hi = float(margin), float(size - 1 - margin)
    while True:
        x0, y0, x1, y1 = st.uniform(4, lo, hi)
        if (x1 - x0) ** 2 + (y1 - y0) ** 2 >= min_len ** 2:
            break
    steps = int(np.ceil(max(abs(x1 - x0), abs(y1 - y0))))
    t = np.arange(steps + 1, dtype=np.float64) / steps
    lx = np.round(x0 + t * (x1 - x0)).astype(np.int64)
    ly = np.round(y0 + t * (y1 - y0)).astype(np.int64)
    keep = st.uniform(steps + 1) < p_line
    on = np.zeros(size * size, dtype=bool)
    on[(ly * size + lx)[keep]] = True
    line_mask = on.copy()
    on |= st.uniform(size * size) < p_noise
    idx = np.flatnonzero(on)
    pix = np.stack([idx % size, idx // size], 1).astype(np.int32)
    return np.ascontiguousarray(pix), line_mask[idx], np.array([x0, y0, x1, y1])


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

CONFIGS = {
    # n=256, 40 % outliers, h=129: the small case the oracle finishes in seconds
    "c1": dict(kind="planted", n=256, f_out=0.40, seeds=(101, 102, 103)),
    # n=4096, 45 % outliers: the headline throughput workload
    "c2": dict(kind="planted", n=4096, f_out=0.45, seeds=(201, 202, 203)),
    # n=16384 planted, and its integer variant with duplicated x and ties
    "c3a": dict(kind="planted", n=16384, f_out=0.45, seeds=(301,)),
    "c3b": dict(kind="degenerate_int", n=16384, seeds=(302,)),
    # 20,000 Hough-style patches with n ~ U{32..512}
    "c4": dict(kind="hough_patches", B=20000, seeds=(401,)),
}


def make(name: str, seed: int | None = None):
    """Build a named workload; returns an (n,2) array, or (xy, offsets) for c4."""
    cfg = CONFIGS[name]
    s = cfg["seeds"][0] if seed is None else seed
    if cfg["kind"] == "planted":
        return planted(cfg["n"], cfg["f_out"], s)
    if cfg["kind"] == "degenerate_int":
        return degenerate_int(cfg["n"], s)
    if cfg["kind"] == "hough_patches":
        return hough_patches(cfg["B"], s)
    raise KeyError(name)


def default_h(n: int) -> int:
    """Low median: h = floor(n/2) + 1."""
    return n // 2 + 1
