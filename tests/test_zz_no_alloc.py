"""lms_solve_noalloc (the allocation-free variant of lms_solve, its
workspace a static device array) against lms_solve, through the C ABI: two
calls in a row, the second on a smaller input, each bit for bit equal to
lms_solve on the same points (the array keeps the last call's contents, so
the second call shows that every call initialises what it reads)."""
import ctypes

import numpy as np
import pytest
import torch

from workloads import gen
from workloads.gen import planted

pytestmark = pytest.mark.gpu


def fields(r):
    return (r.width, r.theta1, r.theta2, r.z_lo, r.z_hi, r.pair_i, r.pair_j, r.status,
            r.candidates, r.vertical, r.survivors, r.band_pass, r.bin_pass)


def call_noalloc(gpu, d, h=0):
    """lms_solve_noalloc through ctypes, default options (NULL)."""
    L = gpu.load()
    out = torch.empty(gpu.RESULT_BYTES, dtype=torch.uint8, device=d.device)
    st = L.lms_solve_noalloc(d.data_ptr(), d.shape[0], h, out.data_ptr(), None,
                             torch.cuda.current_stream().cuda_stream)
    assert st == 0, gpu.last_error()
    torch.cuda.synchronize()
    return gpu.parse(out)


def test_noalloc_equals_solve_on_two_calls():
    import paper_1510_01041_amd as gpu
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    gpu.load()
    big = torch.from_numpy(gen.make("c2", 202)).to("cuda:0")
    small = torch.from_numpy(planted(700, 0.45, 4400)).to("cuda:0")
    for d in (big, small):
        a = call_noalloc(gpu, d)
        b = gpu.solve(d)
        print(d.shape[0], a.width, b.width, flush=True)
        assert fields(a) == fields(b)
    # the largest size fits too, and options pass through
    c3 = torch.from_numpy(gen.make("c3a", 301)).to("cuda:0")
    a = gpu.parse(gpu.solve_noalloc_async(c3))
    torch.cuda.synchronize()
    b = gpu.solve(c3)
    assert (a.width, a.theta1, a.z_lo, a.z_hi) == (b.width, b.theta1, b.z_lo, b.z_hi)
    a = gpu.parse(gpu.solve_noalloc_async(small, seed_pairs=7))
    b = gpu.solve(small, seed_pairs=7)
    assert fields(a) == fields(b)
    # LMS_F_GRAPH is refused before anything is enqueued
    out = torch.empty(gpu.RESULT_BYTES, dtype=torch.uint8, device="cuda:0")
    o = gpu._options(gpu.LMS_F_GRAPH)
    st = gpu.load().lms_solve_noalloc(small.data_ptr(), 700, 0, out.data_ptr(), ctypes.byref(o),
                                      torch.cuda.current_stream().cuda_stream)
    assert st == gpu.LMS_ERR_ARG
