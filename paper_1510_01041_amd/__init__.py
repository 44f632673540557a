"""Exact 2D least-median-of-squares line search on MI355X (gfx950).

Thin ctypes binding over liblms.so (C ABI in include/lms.h). Every step of
the search runs in the library's HIP kernels; this module only marshals
arguments. PyTorch supplies device memory and streams, and the library shares
torch's HIP runtime. If the library is missing, the call fails: there is no
CPU fallback.

Method: arXiv 1510.01041, Eq. (1) and Algorithm 1. The LMS line
y = theta1*x + theta2 minimises the h-th smallest squared residual. It
bisects the thinnest vertical slab holding h points, and its slope is the
slope of a pair of points.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblms.so")

LMS_OK, LMS_OK_DEGENERATE = 0, 1
LMS_ERR_ARG, LMS_ERR_NONFINITE, LMS_ERR_DEVICE, LMS_ERR_NOMEM, LMS_ERR_CAPACITY = -1, -2, -3, -4, -5
LMS_F_NO_PRUNE = 1
LMS_F_GRAPH = 2
LMS_F_RANGE = 4
LMS_F_NO_RANGE = 8
BATCH_MAX_N = 4096
ALG1_MAX_N = 2048
RULE_TIED, RULE_LITERAL = 0, 1
MAX_N = 16384
RESULT_BYTES = 128


class _Result(ctypes.Structure):
    _fields_ = [("theta1", ctypes.c_double), ("theta2", ctypes.c_double),
                ("half_width", ctypes.c_double), ("width", ctypes.c_double),
                ("z_lo", ctypes.c_double), ("z_hi", ctypes.c_double),
                ("pair_i", ctypes.c_int32), ("pair_j", ctypes.c_int32),
                ("status", ctypes.c_int32), ("h", ctypes.c_int32),
                ("candidates", ctypes.c_uint64), ("vertical", ctypes.c_uint64),
                ("survivors", ctypes.c_uint64), ("point_evals", ctypes.c_uint64),
                ("dir_evals", ctypes.c_uint64), ("band_pass", ctypes.c_uint64),
                ("bin_pass", ctypes.c_uint64), ("bins", ctypes.c_uint64)]


assert ctypes.sizeof(_Result) == RESULT_BYTES


class _Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("seed_pairs", ctypes.c_int32), ("tile_regs", ctypes.c_int32),
                ("d_seed_theta", ctypes.c_void_p), ("n_seed_theta", ctypes.c_int64),
                ("tile_batches", ctypes.c_int32), ("window_pairs", ctypes.c_int32),
                ("bins_log2", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("max_workspace", ctypes.c_uint64), ("d_net_params", ctypes.c_void_p)]


class _Tuning(ctypes.Structure):
    _fields_ = [("tile_regs", ctypes.c_int32), ("tile_batches", ctypes.c_int32),
                ("seed_pairs", ctypes.c_int32), ("bins_log2", ctypes.c_int32),
                ("ms", ctypes.c_double), ("range", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _HoughParams(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("max_lines", ctypes.c_int32),
                ("d_rho", ctypes.c_double), ("d_theta_deg", ctypes.c_double),
                ("min_votes", ctypes.c_int32), ("max_support", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


class _Line(ctypes.Structure):
    _fields_ = [("theta_bin", ctypes.c_int32), ("rho_bin", ctypes.c_int32),
                ("votes", ctypes.c_int32), ("support", ctypes.c_int32),
                ("fitted", ctypes.c_int32), ("transposed", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2), ("result", _Result)]


@dataclass
class LmsResult:
    theta1: float
    theta2: float
    half_width: float
    width: float
    z_lo: float
    z_hi: float
    pair_i: int
    pair_j: int
    status: int
    h: int
    candidates: int
    vertical: int
    survivors: int
    point_evals: int
    dir_evals: int
    band_pass: int
    bin_pass: int
    bins: int


class LmsError(RuntimeError):
    pass


_lib = None


def load():
    """Load liblms.so (built by __graft_entry__.build()); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LmsError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    L.lms_solve.argtypes = [vp, i64, i64, vp, ctypes.POINTER(_Options), vp]
    L.lms_solve.restype = i32
    L.lms_solve_host.argtypes = [vp, i64, i64, ctypes.POINTER(_Result), ctypes.POINTER(_Options)]
    L.lms_solve_host.restype = i32
    L.lms_solve_batched.argtypes = [vp, vp, vp, i64, vp, vp, ctypes.POINTER(_Options), vp]
    L.lms_solve_batched.restype = i32
    L.lms_autotune.argtypes = [vp, i64, i64, ctypes.c_int32, vp, ctypes.POINTER(_Tuning)]
    L.lms_autotune.restype = i32
    L.lms_autotune_batched.argtypes = [vp, vp, vp, i64, vp, vp, ctypes.c_int32, vp,
                                       ctypes.POINTER(_Tuning)]
    L.lms_autotune_batched.restype = i32
    L.lms_eval_slopes.argtypes = [vp, i64, i64, vp, i64, vp, vp]
    L.lms_eval_slopes.restype = i32
    L.lms_screen_pairs.argtypes = [vp, i64, i64, ctypes.c_double, vp, i64, vp, vp]
    L.lms_screen_pairs.restype = i32
    L.lms_status_str.argtypes = [i32]
    L.lms_status_str.restype = ctypes.c_char_p
    L.lms_last_error.argtypes = []
    L.lms_last_error.restype = ctypes.c_char_p
    L.lms_profile_begin.argtypes = []
    L.lms_profile_begin.restype = None
    L.lms_profile_end.argtypes = [ctypes.POINTER(ctypes.c_double)]
    L.lms_profile_end.restype = ctypes.c_int64
    L.lms_solve_bracelets.argtypes = [vp, i64, i64, ctypes.c_int32, vp, vp]
    L.lms_solve_bracelets.restype = i32
    L.lms_solve_sampled.argtypes = [vp, i64, i64, i64, ctypes.c_uint64, vp,
                                    ctypes.POINTER(_Options), vp]
    L.lms_solve_sampled.restype = i32
    L.lms_detect_lines.argtypes = [vp, i64, ctypes.POINTER(_HoughParams), vp,
                                   ctypes.POINTER(_Line), ctypes.POINTER(ctypes.c_int32), vp]
    L.lms_detect_lines.restype = i32
    L.lms_workspace_size.argtypes = [i64, i64, ctypes.POINTER(_Options),
                                     ctypes.POINTER(ctypes.c_uint64)]
    L.lms_workspace_size.restype = i32
    L.lms_solve_noalloc.argtypes = [vp, i64, i64, vp, ctypes.POINTER(_Options), vp]
    L.lms_solve_noalloc.restype = i32
    L.lms_tuning_clear.argtypes = []
    L.lms_tuning_clear.restype = None
    L.lms_shutdown.argtypes = []
    L.lms_shutdown.restype = None
    _lib = L
    return L


def status_str(s: int) -> str:
    return load().lms_status_str(s).decode()


def last_error() -> str:
    return load().lms_last_error().decode()


def _check(st: int):
    if st < 0:
        raise LmsError(f"{status_str(st)}: {last_error()}")


def _points(xy: torch.Tensor) -> torch.Tensor:
    if not (isinstance(xy, torch.Tensor) and xy.is_cuda and xy.dtype == torch.float64
            and xy.dim() == 2 and xy.shape[1] == 2):
        raise ValueError("xy must be a CUDA float64 tensor of shape (n, 2)")
    return xy.contiguous()


def _stream(stream) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _options(flags=0, seed_pairs=None, seed_theta: torch.Tensor | None = None, tile_regs=0,
             tile_batches=0, window_pairs=0, bins_log2=0, max_workspace=0,
             net_params: torch.Tensor | None = None):
    o = _Options()
    o.max_workspace = int(max_workspace)
    if net_params is not None:
        if not (net_params.is_cuda and net_params.dtype == torch.float32
                and net_params.is_contiguous() and net_params.numel() == 8642):
            raise ValueError("net_params must be a contiguous CUDA float32 vector of 8642")
        o.d_net_params = net_params.data_ptr()
    o.struct_size = ctypes.sizeof(_Options)
    o.flags = flags
    o.tile_regs = int(tile_regs)
    o.tile_batches = int(tile_batches)
    o.window_pairs = int(window_pairs)
    o.bins_log2 = int(bins_log2)
    o.seed_pairs = -1 if seed_pairs is None else int(seed_pairs)
    if seed_theta is not None:
        if not (seed_theta.is_cuda and seed_theta.dtype == torch.float64 and seed_theta.dim() == 1
                and seed_theta.is_contiguous()):
            raise ValueError("seed_theta must be a contiguous CUDA float64 vector")
        o.d_seed_theta = seed_theta.data_ptr()
        o.n_seed_theta = seed_theta.numel()
    return o


def parse(raw: torch.Tensor) -> LmsResult:
    """Decode a 128-byte lms_result (device or host uint8 tensor)."""
    b = bytes(raw.detach().to("cpu").numpy().tobytes())
    r = _Result.from_buffer_copy(b)
    return LmsResult(**{f: getattr(r, f) for f, _ in _Result._fields_})


def solve_async(xy: torch.Tensor, h: int = 0, out: torch.Tensor | None = None, *,
                no_prune: bool = False, seed_pairs: int | None = None,
                seed_theta: torch.Tensor | None = None, tile_regs: int = 0,
                tile_batches: int = 0, window_pairs: int = 0, bins_log2: int = 0,
                graph: bool = False, slope_range: bool | None = None,
                max_workspace: int = 0, net_params: torch.Tensor | None = None,
                stream=None) -> torch.Tensor:
    """Enqueue one exact LMS solve; returns the device uint8[128] result buffer.

    seed_theta: optional CUDA float64 slopes whose exact widths seed the bound;
    window_pairs: with seed_theta, pairs drawn from the best seed line's window
    (two rounds) as further seeds. bins_log2: slope bins per anchor of the
    first screen (0 automatic, -1 off). net_params: the seed network's packed
    FP32 parameters (CUDA); its slope, computed inside the solve, is the seed
    slope (exclusive with seed_theta). graph=True captures the solve in a
    hipGraph on the first call and replays it on later calls with the same
    buffers and options. slope_range: None automatic (above 4096 points),
    True at any n, False never."""
    xy = _points(xy)
    if out is None:
        out = torch.empty(RESULT_BYTES, dtype=torch.uint8, device=xy.device)
    flags = (LMS_F_NO_PRUNE if no_prune else 0) | (LMS_F_GRAPH if graph else 0)
    if slope_range is not None:
        flags |= LMS_F_RANGE if slope_range else LMS_F_NO_RANGE
    opt = _options(flags, seed_pairs, seed_theta, tile_regs, tile_batches, window_pairs,
                   bins_log2, max_workspace, net_params)
    st = load().lms_solve(xy.data_ptr(), xy.shape[0], h, out.data_ptr(), ctypes.byref(opt),
                          _stream(stream))
    _check(st)
    return out


def solve_noalloc_async(xy: torch.Tensor, h: int = 0, out: torch.Tensor | None = None,
                        stream=None, **kw) -> torch.Tensor:
    """lms_solve_noalloc: the same solve in the library's static workspace (no
    device allocation by the library); kw as solve_async except graph."""
    xy = _points(xy)
    if out is None:
        out = torch.empty(RESULT_BYTES, dtype=torch.uint8, device=xy.device)
    opt = _options(0, **kw)
    _check(load().lms_solve_noalloc(xy.data_ptr(), xy.shape[0], h, out.data_ptr(),
                                    ctypes.byref(opt), _stream(stream)))
    return out


def workspace_size(n: int, h: int = 0, max_workspace: int = 0, **kw) -> int:
    """Device bytes lms_solve's workspace takes for n points (and options)."""
    flags = 0
    opt = _options(flags, max_workspace=max_workspace, **kw)
    b = ctypes.c_uint64(0)
    _check(load().lms_workspace_size(n, h, ctypes.byref(opt), ctypes.byref(b)))
    return b.value


def solve(xy: torch.Tensor, h: int = 0, **kw) -> LmsResult:
    """Exact LMS line of an (n, 2) CUDA float64 point tensor (synchronises)."""
    return parse(solve_async(xy, h, **kw))


RESULT_DTYPE = None


def _result_dtype():
    import numpy as np
    global RESULT_DTYPE
    if RESULT_DTYPE is None:
        RESULT_DTYPE = np.dtype([(f, "f8" if t is ctypes.c_double else
                                  "i4" if t is ctypes.c_int32 else "u8")
                                 for f, t in _Result._fields_])
        assert RESULT_DTYPE.itemsize == RESULT_BYTES
    return RESULT_DTYPE


def parse_batch(raw: torch.Tensor):
    """Decode B results (device or host uint8[B, 128]) into a numpy record array."""
    import numpy as np
    a = raw.detach().to("cpu").contiguous().numpy()
    return np.frombuffer(a.tobytes(), dtype=_result_dtype()).view(np.recarray)


def solve_batched_async(xy: torch.Tensor, offsets, h: torch.Tensor | None = None,
                        out: torch.Tensor | None = None, *, graph: bool = False,
                        seed_pairs: int | None = None, bins_log2: int = 0,
                        max_workspace: int = 0, stream=None) -> torch.Tensor:
    """Enqueue exact LMS fits of B point sets; problem b is xy[offsets[b]:offsets[b+1]].

    offsets: B+1 int64 (host array or tensor; a device copy is made if needed).
    h: optional CUDA int32 tensor of B values. graph=True captures the kernels in
    a hipGraph on the first call and replays it on later calls with the same
    buffers. Returns the device uint8[B, 128] result buffer."""
    import numpy as np
    xy = _points(xy)
    if isinstance(offsets, torch.Tensor):
        off_h = offsets.detach().to("cpu", torch.int64).contiguous().numpy()
        off_d = offsets if (offsets.is_cuda and offsets.dtype == torch.int64
                            and offsets.is_contiguous()) else \
            torch.from_numpy(off_h).to(xy.device)
    else:
        off_h = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        off_d = torch.from_numpy(off_h).to(xy.device)
    B = off_h.shape[0] - 1
    if out is None:
        out = torch.empty((B, RESULT_BYTES), dtype=torch.uint8, device=xy.device)
    if h is not None and not (h.is_cuda and h.dtype == torch.int32 and h.numel() == B):
        raise ValueError("h must be a CUDA int32 tensor with B values")
    opt = _options(LMS_F_GRAPH if graph else 0, seed_pairs, bins_log2=bins_log2,
                   max_workspace=max_workspace)
    st = load().lms_solve_batched(xy.data_ptr(), off_d.data_ptr(), off_h.ctypes.data, B,
                                  None if h is None else h.data_ptr(), out.data_ptr(),
                                  ctypes.byref(opt), _stream(stream))
    _check(st)
    # keep the device offsets alive while the work is queued
    out._lms_offsets = off_d
    return out


def autotune(xy: torch.Tensor, h: int = 0, reps: int = 3, stream=None) -> dict:
    """Time the screen tiles on this point set and keep the fastest for its
    size class (used by later solves with automatic tiles)."""
    xy = _points(xy)
    t = _Tuning()
    _check(load().lms_autotune(xy.data_ptr(), xy.shape[0], h, reps, _stream(stream),
                               ctypes.byref(t)))
    return {f: getattr(t, f) for f, _ in _Tuning._fields_}


def tuning_clear():
    """Forget every tuned choice of this process."""
    load().lms_tuning_clear()


def autotune_batched(xy: torch.Tensor, offsets, h=None, reps: int = 3, stream=None) -> dict:
    """Tune lms_solve_batched on this batch: seed pairs per problem and the small
    classes' bins (kept only if every width equals the default's)."""
    import numpy as np
    xy = _points(xy)
    off_h = np.ascontiguousarray(np.asarray(offsets.cpu() if isinstance(offsets, torch.Tensor)
                                            else offsets, dtype=np.int64))
    off_d = torch.from_numpy(off_h).to(xy.device)
    B = off_h.shape[0] - 1
    out = torch.empty((B, RESULT_BYTES), dtype=torch.uint8, device=xy.device)
    t = _Tuning()
    _check(load().lms_autotune_batched(xy.data_ptr(), off_d.data_ptr(), off_h.ctypes.data, B,
                                       None if h is None else h.data_ptr(), out.data_ptr(), reps,
                                       _stream(stream), ctypes.byref(t)))
    return {f: getattr(t, f) for f, _ in _Tuning._fields_}


def solve_batched(xy: torch.Tensor, offsets, h=None, **kw):
    """Exact LMS fits of B point sets (synchronises); a numpy record array."""
    return parse_batch(solve_batched_async(xy, offsets, h, **kw))


def solve_host(xy, h: int = 0) -> LmsResult:
    """Synchronous solve of a host (n, 2) float64 array via lms_solve_host."""
    import numpy as np
    a = np.ascontiguousarray(np.asarray(xy, dtype=np.float64))
    r = _Result()
    o = _options()
    st = load().lms_solve_host(a.ctypes.data, a.shape[0], h, ctypes.byref(r), ctypes.byref(o))
    res = LmsResult(**{f: getattr(r, f) for f, _ in _Result._fields_})
    if st < 0 and res.status >= 0:
        _check(st)
    return res


def eval_slopes(xy: torch.Tensor, theta: torch.Tensor, h: int = 0, stream=None) -> torch.Tensor:
    """F(theta) per slope: an (m, 3) tensor of (width, z_lo, z_hi)."""
    xy = _points(xy)
    theta = theta.to(device=xy.device, dtype=torch.float64).contiguous()
    out = torch.empty((theta.numel(), 3), dtype=torch.float64, device=xy.device)
    st = load().lms_eval_slopes(xy.data_ptr(), xy.shape[0], h, theta.data_ptr(), theta.numel(),
                                out.data_ptr(), _stream(stream))
    _check(st)
    return out


def screen_pairs(xy: torch.Tensor, pairs: torch.Tensor, W: float, h: int = 0,
                 stream=None) -> torch.Tensor:
    """FP32 screen verdicts (1 keep, 0 reject, 2 vertical) for (m, 2) pairs."""
    xy = _points(xy)
    pairs = pairs.to(device=xy.device, dtype=torch.int32).contiguous()
    out = torch.empty(pairs.shape[0], dtype=torch.int32, device=xy.device)
    st = load().lms_screen_pairs(xy.data_ptr(), xy.shape[0], h, float(W), pairs.data_ptr(),
                                 pairs.shape[0], out.data_ptr(), _stream(stream))
    _check(st)
    return out


def solve_bracelets_async(xy: torch.Tensor, h: int = 0, rule: int = RULE_TIED,
                          out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Enqueue Algorithm 1 as stated: every vertex materialised, one sort per
    vertex, the bracelet hanging from it, a min-reduction (n <= 2048).
    rule RULE_TIED (exact) or RULE_LITERAL (the printed rank offset)."""
    xy = _points(xy)
    if out is None:
        out = torch.empty(RESULT_BYTES, dtype=torch.uint8, device=xy.device)
    _check(load().lms_solve_bracelets(xy.data_ptr(), xy.shape[0], h, rule, out.data_ptr(),
                                      _stream(stream)))
    return out


def solve_bracelets(xy: torch.Tensor, h: int = 0, rule: int = RULE_TIED) -> LmsResult:
    """Algorithm 1 as stated (synchronises); see solve_bracelets_async."""
    return parse(solve_bracelets_async(xy, h, rule))


def solve_sampled_async(xy: torch.Tensor, m: int, seed: int = 0, h: int = 0,
                        out: torch.Tensor | None = None, stream=None, **kw) -> torch.Tensor:
    """Enqueue the exact LMS of m points drawn without replacement (an
    estimate of the whole set's line); kw as for solve_async."""
    xy = _points(xy)
    if out is None:
        out = torch.empty(RESULT_BYTES, dtype=torch.uint8, device=xy.device)
    flags = (LMS_F_GRAPH if kw.pop("graph", False) else 0)
    opt = _options(flags, **kw)
    _check(load().lms_solve_sampled(xy.data_ptr(), xy.shape[0], h, m, seed & ((1 << 64) - 1),
                                    out.data_ptr(), ctypes.byref(opt), _stream(stream)))
    return out


def solve_sampled(xy: torch.Tensor, m: int, seed: int = 0, h: int = 0, **kw) -> LmsResult:
    """Exact LMS line of a random m-point sample (synchronises)."""
    return parse(solve_sampled_async(xy, m, seed, h, **kw))


def detect_lines(pix: torch.Tensor, width: int, height: int, d_rho: float = 20.0,
                 d_theta_deg: float = 2.0, max_lines: int = 1, min_votes: int = 2,
                 max_support: int = BATCH_MAX_N, seed: int = 0, acc: torch.Tensor | None = None,
                 stream=None) -> list[dict]:
    """Coarse Hough transform of edge pixels (CUDA int32 (N, 2) of (x, y)),
    then the exact LMS line of each peak's supporting pixels (synchronous).
    Returns per peak: theta_bin, rho_bin, votes, support, fitted, transposed
    and the LmsResult of the fit (x = theta1 y + theta2 when transposed).
    acc: optional CUDA int32 tensor (n_theta, n_rho) for the accumulator."""
    if not (pix.is_cuda and pix.dtype == torch.int32 and pix.dim() == 2 and pix.shape[1] == 2):
        raise ValueError("pix must be a CUDA int32 tensor of shape (N, 2)")
    pix = pix.contiguous()
    p = _HoughParams()
    p.struct_size = ctypes.sizeof(_HoughParams)
    p.width, p.height, p.max_lines = width, height, max_lines
    p.d_rho, p.d_theta_deg = float(d_rho), float(d_theta_deg)
    p.min_votes, p.max_support, p.seed = min_votes, max_support, seed & ((1 << 64) - 1)
    lines = (_Line * max_lines)()
    n = ctypes.c_int32(0)
    if acc is not None and not (acc.is_cuda and acc.dtype == torch.int32 and acc.is_contiguous()):
        raise ValueError("acc must be a contiguous CUDA int32 tensor")
    _check(load().lms_detect_lines(pix.data_ptr(), pix.shape[0], ctypes.byref(p),
                                   None if acc is None else acc.data_ptr(), lines,
                                   ctypes.byref(n), _stream(stream)))
    out = []
    for k in range(n.value):
        L = lines[k]
        r = L.result
        out.append(dict(theta_bin=L.theta_bin, rho_bin=L.rho_bin, votes=L.votes,
                        support=L.support, fitted=L.fitted, transposed=L.transposed,
                        result=LmsResult(**{f: getattr(r, f) for f, _ in _Result._fields_})))
    return out


def hough_grid(width: int, height: int, d_rho: float, d_theta_deg: float) -> tuple[int, int]:
    """(n_theta, n_rho) of the accumulator lms_detect_lines uses."""
    import math
    return (math.ceil(180.0 / d_theta_deg),
            math.floor(float(2 * (width - 1) + (height - 1)) / d_rho) + 1)


STAGES = ("prep", "seed", "bins", "screen", "recheck", "finalize")


def profile_begin():
    """Start recording HIP events around each solve's stages."""
    load().lms_profile_begin()


def profile_end() -> tuple[int, dict]:
    """Stop recording; returns (solves timed, {stage: summed ms})."""
    ms = (ctypes.c_double * len(STAGES))()
    n = load().lms_profile_end(ms)
    _check(int(n) if n < 0 else 0)
    return int(n), {k: ms[i] for i, k in enumerate(STAGES)}


def shutdown():
    if _lib is not None:
        _lib.lms_shutdown()
