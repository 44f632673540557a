"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/*.h, and rejects bad arguments on the host before any
device work."""
import ctypes
import glob
import os
import re

import pytest

import paper_1510_01041_amd as lms

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        for m in re.finditer(r"\b(lms_\w+)\s*\(", src):
            names.add(m.group(1))
    return sorted(names)


def test_headers_declare_entry_points():
    names = declared_functions()
    for want in ("lms_solve", "lms_solve_host", "lms_eval_slopes", "lms_screen_pairs",
                 "lms_status_str", "lms_last_error", "lms_shutdown"):
        assert want in names


def test_library_exports_every_declared_symbol():
    L = lms.load()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings():
    assert lms.status_str(0) == "ok"
    assert "non-finite" in lms.status_str(-2)
    assert lms.status_str(12345) == "unknown status"


def _solve_raw(ptr, n, h, out, opt=None):
    L = lms.load()
    o = opt if opt is not None else lms._options()
    return L.lms_solve(ptr, n, h, out, ctypes.byref(o), None)


def test_argument_errors_are_synchronous():
    """Bad arguments return LMS_ERR_ARG from the host check, with a message."""
    fake = 0x1000  # never dereferenced: validation fails first
    assert _solve_raw(None, 10, 0, fake) == lms.LMS_ERR_ARG
    assert _solve_raw(fake, 1, 0, fake) == lms.LMS_ERR_ARG
    assert "n must be" in lms.last_error()
    assert _solve_raw(fake, lms.MAX_N + 1, 0, fake) == lms.LMS_ERR_ARG
    assert _solve_raw(fake, 10, 1, fake) == lms.LMS_ERR_ARG
    assert _solve_raw(fake, 10, 11, fake) == lms.LMS_ERR_ARG
    assert "h must be" in lms.last_error()
    assert _solve_raw(fake, 10, 0, None) == lms.LMS_ERR_ARG
    bad = lms._options()
    bad.struct_size = 4
    assert _solve_raw(fake, 10, 0, fake, bad) == lms.LMS_ERR_ARG
    neg = lms._options(seed_pairs=-2)
    assert _solve_raw(fake, 10, 0, fake, neg) == lms.LMS_ERR_ARG
    L = lms.load()
    assert L.lms_eval_slopes(fake, 10, 0, None, 5, fake, None) == lms.LMS_ERR_ARG
    assert L.lms_screen_pairs(fake, 10, 0, -1.0, fake, 3, fake, None) == lms.LMS_ERR_ARG
    assert L.lms_screen_pairs(fake, 10, 0, float("nan"), fake, 3, fake, None) == lms.LMS_ERR_ARG


def test_binding_rejects_non_cuda_input():
    import torch
    with pytest.raises(ValueError):
        lms.solve(torch.zeros((10, 2), dtype=torch.float64))


def test_batched_argument_errors():
    L = lms.load()
    import numpy as np
    fake = 0x1000
    opt = lms._options()
    off = np.array([0, 10, 20], dtype=np.int64)
    assert L.lms_solve_batched(fake, fake, off.ctypes.data, 0, None, fake, ctypes.byref(opt),
                               None) == lms.LMS_ERR_ARG
    assert L.lms_solve_batched(None, fake, off.ctypes.data, 2, None, fake, ctypes.byref(opt),
                               None) == lms.LMS_ERR_ARG
    big = np.array([0, 5000], dtype=np.int64)
    assert L.lms_solve_batched(fake, fake, big.ctypes.data, 1, None, fake, ctypes.byref(opt),
                               None) == lms.LMS_ERR_ARG
    assert "4096" in lms.last_error()
    dec = np.array([0, 10, 5], dtype=np.int64)
    assert L.lms_solve_batched(fake, fake, dec.ctypes.data, 2, None, fake, ctypes.byref(opt),
                               None) == lms.LMS_ERR_ARG


def test_tile_and_tuning_argument_errors():
    L = lms.load()
    fake = 0x1000
    bad = lms._options(tile_regs=65)
    assert _solve_raw(fake, 100, 0, fake, bad) == lms.LMS_ERR_ARG
    bad = lms._options(tile_batches=65)
    assert _solve_raw(fake, 100, 0, fake, bad) == lms.LMS_ERR_ARG
    bad = lms._options(window_pairs=-1)
    assert _solve_raw(fake, 100, 0, fake, bad) == lms.LMS_ERR_ARG
    assert "window_pairs" in lms.last_error()
    bad = lms._options(window_pairs=(1 << 16) + 1)
    assert _solve_raw(fake, 100, 0, fake, bad) == lms.LMS_ERR_ARG
    t = lms._Tuning()
    assert L.lms_autotune(None, 100, 0, 3, None, ctypes.byref(t)) == lms.LMS_ERR_ARG
    assert L.lms_autotune(fake, 100, 0, 0, None, ctypes.byref(t)) == lms.LMS_ERR_ARG


def test_result_decoding_on_host_buffers():
    """parse/parse_batch decode every lms_result field (host tensors suffice)."""
    import numpy as np
    import torch
    r = lms._Result()
    r.width, r.status, r.bin_pass, r.band_pass = 2.5, 1, 7, 9
    raw = torch.from_numpy(np.frombuffer(bytes(r), dtype=np.uint8).copy())
    assert raw.numel() == lms.RESULT_BYTES
    p = lms.parse(raw)
    assert (p.width, p.status, p.bin_pass, p.band_pass) == (2.5, 1, 7, 9)
    rb = lms.parse_batch(torch.stack([raw, raw]))
    assert rb.shape == (2,) and list(rb.bin_pass) == [7, 7]
    assert list(lms.STAGES) == ["prep", "seed", "bins", "screen", "recheck", "finalize"]


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU only: asked for more it exits at once with a
    message (before touching a GPU)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in (p.stdout + p.stderr)
