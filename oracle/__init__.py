"""CPU oracle for the exact 2D LMS line (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package. The GPU library does not call it, and the two
share no code. The C source is ``lms_oracle.c``, which documents the steps and
the paper sections they follow (arXiv 1510.01041, Sections 1, 3.1-3.4).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lms_oracle.c")
_LIB = os.path.join(_HERE, "liblms_oracle.so")

OK, OK_DEGENERATE, ERR_ARG, ERR_NONFINITE = 0, 1, -1, -2
RULE_TIED, RULE_LITERAL = 0, 1


def build(verbose: bool = False, src: str = _SRC, out: str = _LIB) -> str:
    """Compile liblms_oracle.so with gcc (FP64, no contraction, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-I", _HERE, "-o", out + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


class _Result(ctypes.Structure):
    _fields_ = [("theta1", ctypes.c_double), ("theta2", ctypes.c_double),
                ("half_width", ctypes.c_double), ("width", ctypes.c_double),
                ("z_lo", ctypes.c_double), ("z_hi", ctypes.c_double),
                ("pair_i", ctypes.c_int64), ("pair_j", ctypes.c_int64),
                ("candidates", ctypes.c_int64), ("vertical", ctypes.c_int64),
                ("status", ctypes.c_int32), ("h", ctypes.c_int32)]


@dataclass
class OracleResult:
    theta1: float
    theta2: float
    half_width: float
    width: float
    z_lo: float
    z_hi: float
    pair_i: int
    pair_j: int
    candidates: int
    vertical: int
    status: int
    h: int


_lib = None


def bind(path: str):
    """Load an oracle library from path and declare its entry points."""
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    L.lms_oracle_solve.argtypes = [dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                   ctypes.POINTER(_Result)]
    L.lms_oracle_solve.restype = ctypes.c_int
    L.lms_oracle_solve_bounded.argtypes = [dp, ctypes.c_int64, ctypes.c_int64,
                                           ctypes.c_int, ctypes.POINTER(_Result),
                                           ctypes.POINTER(ctypes.c_int64)]
    L.lms_oracle_solve_bounded.restype = ctypes.c_int
    L.lms_oracle_window.argtypes = [dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                    dp, dp, dp]
    L.lms_oracle_window.restype = ctypes.c_int
    L.lms_oracle_eval_pairs.argtypes = [dp, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.POINTER(ctypes.c_int64), ctypes.c_int64,
                                        ctypes.c_int, dp, dp, dp, dp]
    L.lms_oracle_eval_pairs.restype = ctypes.c_int
    L.lms_oracle_anchored.argtypes = [dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_int64, dp, dp]
    L.lms_oracle_anchored.restype = ctypes.c_int
    L.lms_oracle_hth_abs_residual.argtypes = [dp, ctypes.c_int64, ctypes.c_int64,
                                              ctypes.c_double, ctypes.c_double]
    L.lms_oracle_hth_abs_residual.restype = ctypes.c_double
    L.lms_oracle_bracelets.argtypes = [dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                       ctypes.c_int, ctypes.POINTER(_Result)]
    L.lms_oracle_bracelets.restype = ctypes.c_int
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = bind(_LIB)
    return _lib


def _xy(xy) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(xy, dtype=np.float64))
    if a.ndim != 2 or a.shape[1] != 2:
        raise ValueError("xy must be an (n, 2) array")
    return a


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def solve(xy, h: int = 0, nthreads: int = 0) -> OracleResult:
    """Exhaustive FP64 LMS over all pair slopes (h=0 means floor(n/2)+1)."""
    a = _xy(xy)
    r = _Result()
    lib().lms_oracle_solve(_dp(a), a.shape[0], h, nthreads, ctypes.byref(r))
    return OracleResult(**{f: getattr(r, f) for f, _ in _Result._fields_})


def solve_bounded(xy, h: int = 0, nthreads: int = 0):
    """Same result as solve(), skipping slopes the Lipschitz bound rules out.

    Returns (OracleResult, number of distinct slopes evaluated)."""
    a = _xy(xy)
    r = _Result()
    ev = ctypes.c_int64()
    lib().lms_oracle_solve_bounded(_dp(a), a.shape[0], h, nthreads, ctypes.byref(r),
                                   ctypes.byref(ev))
    return OracleResult(**{f: getattr(r, f) for f, _ in _Result._fields_}), ev.value


def window(xy, theta: float, h: int = 0) -> tuple[float, float, float]:
    """F(theta): (width, z_lo, z_hi) of the narrowest h-window at one slope."""
    a = _xy(xy)
    w, lo, hi = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    st = lib().lms_oracle_window(_dp(a), a.shape[0], h, float(theta),
                                 ctypes.byref(w), ctypes.byref(lo), ctypes.byref(hi))
    if st != OK:
        raise ValueError(f"oracle window status {st}")
    return w.value, lo.value, hi.value


def eval_pairs(xy, pairs, h: int = 0, nthreads: int = 0):
    """F at each pair's slope: returns (theta, width, z_lo, z_hi) arrays."""
    a = _xy(xy)
    p = np.ascontiguousarray(np.asarray(pairs, dtype=np.int64).reshape(-1, 2))
    m = p.shape[0]
    th, w, lo, hi = (np.empty(m) for _ in range(4))
    st = lib().lms_oracle_eval_pairs(_dp(a), a.shape[0], h,
                                     p.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), m,
                                     nthreads, _dp(th), _dp(w), _dp(lo), _dp(hi))
    if st != OK:
        raise ValueError(f"oracle eval_pairs status {st}")
    return th, w, lo, hi


def anchored(xy, i: int, j: int, h: int = 0) -> tuple[float, float]:
    """Anchored (up, dn) widths of pair (i, j)."""
    a = _xy(xy)
    up, dn = ctypes.c_double(), ctypes.c_double()
    st = lib().lms_oracle_anchored(_dp(a), a.shape[0], h, i, j, ctypes.byref(up),
                                   ctypes.byref(dn))
    if st != OK:
        raise ValueError(f"oracle anchored status {st}")
    return up.value, dn.value


def hth_abs_residual(xy, theta1: float, theta2: float, h: int = 0) -> float:
    a = _xy(xy)
    return lib().lms_oracle_hth_abs_residual(_dp(a), a.shape[0], h, theta1, theta2)


def bracelets(xy, h: int = 0, rule: int = RULE_TIED, nthreads: int = 0) -> OracleResult:
    """Algorithm 1 as stated: the minimum over vertices of the bracelet hanging
    from each, with the tied-rank reading (RULE_TIED, exact) or the printed
    rank offset from the lowest tied rank (RULE_LITERAL)."""
    a = _xy(xy)
    r = _Result()
    lib().lms_oracle_bracelets(_dp(a), a.shape[0], h, rule, nthreads, ctypes.byref(r))
    return OracleResult(**{f: getattr(r, f) for f, _ in _Result._fields_})


def sample_indices(n: int, m: int, seed: int) -> np.ndarray:
    """Indices (ascending) of the m points with the smallest SplitMix64 keys,
    key_k = output k of SplitMix64 started at `seed`; equal keys go to the
    lower index. The random draw of the sampled solve."""
    from workloads.gen import splitmix64
    keys = splitmix64(seed, n)
    order = np.lexsort((np.arange(n), keys))
    return np.sort(order[:m])


def solve_sampled(xy, m: int, seed: int, h: int = 0) -> OracleResult:
    """Exact LMS line of the m-point sample (h = 0: the sample's low median;
    else ceil(h m / n), at least 2), pair indices in the input's numbering."""
    a = _xy(xy)
    n = a.shape[0]
    idx = sample_indices(n, m, seed)
    hm = 0 if h == 0 else max(2, -(-h * m // n))
    r = solve(a[idx], h=hm)
    if r.pair_i >= 0:
        r.pair_i, r.pair_j = int(idx[r.pair_i]), int(idx[r.pair_j])
    return r
