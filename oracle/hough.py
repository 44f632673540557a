"""Reference of the line detector: coarse Hough transform, then one exact LMS
fit per accumulator peak (Section 5). TEST INFRASTRUCTURE ONLY; it shares no
code with the GPU library.

Steps, as Section 5 describes them, with the readings the GPU library states
in its header:
1. Polar accumulator: angle bins theta_b = b * (d_theta * pi/180),
   b = 0 .. ceil(180/d_theta) - 1; every pixel votes once per angle bin, into
   rho bin floor((x cos theta_b + y sin theta_b + width - 1) / d_rho).
2. Peaks: cells with at least min_votes votes that are local maxima of their
   3x3 neighbourhood (above earlier neighbours in cell order, at least equal to
   later ones), strongest first by (votes, then lower cell index).
3. Each peak's supporting set: the pixels that voted for it, in pixel order;
   larger than max_support: the max_support pixels with the smallest
   SplitMix64 keys (random sampling of a cell's points).
4. A steep line (|cos theta_b| > |sin theta_b|) is fitted as x = a y + b.
5. The exact LMS line of each set (oracle.solve).
"""
from __future__ import annotations

import math

import numpy as np

DEG = 0.017453292519943295  # pi / 180 rounded to double


def grid(width: int, height: int, d_rho: float, d_theta_deg: float):
    n_theta = math.ceil(180.0 / d_theta_deg)
    n_rho = math.floor(float(2 * (width - 1) + (height - 1)) / d_rho) + 1
    step = d_theta_deg * DEG
    th = [float(b) * step for b in range(n_theta)]
    c = np.array([math.cos(t) for t in th])
    s = np.array([math.sin(t) for t in th])
    return n_theta, n_rho, -float(width - 1), c, s


def rho_bins(pix: np.ndarray, c: np.ndarray, s: np.ndarray, rho_min: float, d_rho: float):
    """(N, n_theta) rho bin of every pixel at every angle."""
    x = pix[:, 0].astype(np.float64)[:, None]
    y = pix[:, 1].astype(np.float64)[:, None]
    rho = x * c[None, :] + y * s[None, :]
    return np.floor((rho - rho_min) / d_rho).astype(np.int64)


def accumulator(pix, width, height, d_rho, d_theta_deg):
    n_theta, n_rho, rho_min, c, s = grid(width, height, d_rho, d_theta_deg)
    acc = np.zeros((n_theta, n_rho), dtype=np.int64)
    if len(pix):
        r = rho_bins(pix, c, s, rho_min, d_rho)
        b = np.broadcast_to(np.arange(n_theta)[None, :], r.shape)
        ok = (r >= 0) & (r < n_rho)
        np.add.at(acc, (b[ok], r[ok]), 1)
    return acc


def peaks(acc: np.ndarray, min_votes: int, max_lines: int):
    """[(cell, votes)] strongest first."""
    n_theta, n_rho = acc.shape
    out = []
    for b in range(n_theta):
        for r in range(n_rho):
            v = acc[b, r]
            if v < min_votes:
                continue
            cell = b * n_rho + r
            ok = True
            for db in (-1, 0, 1):
                for dr in (-1, 0, 1):
                    if (db, dr) == (0, 0):
                        continue
                    bb, rr = b + db, r + dr
                    if not (0 <= bb < n_theta and 0 <= rr < n_rho):
                        continue
                    u = acc[bb, rr]
                    if u > v or (u == v and bb * n_rho + rr < cell):
                        ok = False
            if ok:
                out.append((cell, int(v)))
    out.sort(key=lambda cv: (-cv[1], cv[0]))
    return out[:max_lines]


def detect(pix, width, height, d_rho, d_theta_deg, max_lines, min_votes, max_support, seed):
    """Per peak: dict(theta_bin, rho_bin, votes, support, fitted, transposed,
    xy (the fitted set), result (oracle.solve of it))."""
    import oracle
    from workloads.gen import splitmix64

    n_theta, n_rho, rho_min, c, s = grid(width, height, d_rho, d_theta_deg)
    acc = accumulator(pix, width, height, d_rho, d_theta_deg)
    r_all = rho_bins(pix, c, s, rho_min, d_rho) if len(pix) else None
    keys = splitmix64(seed, len(pix))
    lines = []
    for cell, votes in peaks(acc, min_votes, max_lines):
        b, r = divmod(cell, n_rho)
        idx = np.flatnonzero(r_all[:, b] == r)
        support = len(idx)
        if support > max_support:
            order = np.lexsort((idx, keys[idx]))
            idx = np.sort(idx[order[:max_support]])
        steep = abs(c[b]) > abs(s[b])
        xy = pix[idx].astype(np.float64)
        if steep:
            xy = xy[:, ::-1]
        xy = np.ascontiguousarray(xy)
        lines.append(dict(theta_bin=b, rho_bin=r, votes=votes, support=support,
                          fitted=len(idx), transposed=int(steep), xy=xy,
                          result=oracle.solve(xy) if len(xy) >= 2 else None))
    return acc, lines
