"""Workspace limits and list overflow, through the C ABI: an exact solver
must return the exact answer for every valid problem whatever its lists hold.

* A batch whose shared survivor list is limited so far that problems lose
  survivors: those problems are re-solved one by one, and every problem of
  the batch still matches the oracle.
* A single solve whose slope-bin pass list is limited: the list overflows, the
  exhaustive FP32 screen runs instead, and the answer is the oracle's.
* A limit below what a solve needs at the least: LMS_ERR_NOMEM, nothing
  enqueued.
"""
import numpy as np
import pytest
import torch

from workloads import gen
from workloads.gen import planted

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def smallest_batch_limit(gpu, d, off, **kw):
    """The smallest power of two of bytes the batch accepts as max_workspace."""
    for k in range(14, 34):
        try:
            res = gpu.solve_batched(d, off, max_workspace=1 << k, **kw)
            return 1 << k, res
        except gpu.LmsError as e:
            assert "out of device memory" in str(e), e
    raise AssertionError("no limit accepted")


def test_batch_survivor_overflow_is_resolved(gpu, orc):
    # few seeds: a loose bound, so thousands of survivors per problem
    xy, off = gen.hough_patches(48, 31, n_lo=200, n_hi=400)
    d = dev(xy)
    full = gpu.solve_batched(d, off, seed_pairs=0)
    assert int(full.survivors.sum()) > 20_000, int(full.survivors.sum())
    limit, res = smallest_batch_limit(gpu, d, off, seed_pairs=0)
    print("limit", limit, "survivors", int(full.survivors.sum()), flush=True)
    # problems re-solved on their own carry lms_solve's bin count
    resolved = int((res.bins != full.bins).sum())
    assert resolved > 0, "the limit did not make any problem overflow"
    for b in range(len(off) - 1):
        p = xy[off[b]:off[b + 1]]
        r = res[b]
        assert r.status == 0, (b, r.status)
        o = orc.solve(p)
        assert abs(r.width - o.width) <= 1e-9 * max(r.width, o.width) or r.width == o.width
        assert orc.window(p, float(r.theta1)) == (r.width, r.z_lo, r.z_hi)
        assert r.width == full[b].width
    # graph replays take the same path
    for _ in range(2):
        g = gpu.solve_batched(d, off, seed_pairs=0, max_workspace=limit, graph=True)
        assert np.array_equal(g.width, res.width) and np.array_equal(g.status, res.status)


def test_single_solve_pass_list_overflow_runs_exhaustive_screen(gpu, orc):
    """Under a workspace limit the survivor list keeps 65536 slots and the
    slope-bin pass list shrinks; with a bound loose enough that more pairs
    pass the bins than the list holds, the exhaustive FP32 screen runs, and
    the answer is still the oracle's."""
    n = 1500
    xy = planted(n, 0.45, 32)
    d = dev(xy)
    for sp in (31, 15, 7, 3, 1):
        base = gpu.solve(d, seed_pairs=sp)
        fp32_only = gpu.solve(d, seed_pairs=sp, bins_log2=-1)
        if base.bin_pass > 4096 and fp32_only.survivors < 60000:
            break
    print("seed pairs", sp, "bin passes", base.bin_pass, "fp32 survivors", fp32_only.survivors,
          flush=True)
    assert base.bin_pass > 4096 and fp32_only.survivors < 60000
    full = gpu.workspace_size(n, seed_pairs=sp)
    pairs = n * (n - 1) // 2
    # default lists: `pairs` pass slots of 8 bytes, `pairs` survivor slots of
    # 40; the limit leaves about 2000 pass slots (alignment slack included)
    fixed = full - 48 * pairs
    limit = fixed + 40 * 65536 + 8 * 1024 + 8192
    assert gpu.workspace_size(n, seed_pairs=sp, max_workspace=limit) <= limit
    r = gpu.solve(d, seed_pairs=sp, max_workspace=limit)
    o = orc.solve(xy)
    assert r.status == 0
    assert (r.width, r.theta1, r.z_lo, r.z_hi) == (o.width, o.theta1, o.z_lo, o.z_hi)
    # the exhaustive FP32 screen tested far more pairs than the list held
    assert r.point_evals > base.point_evals
    assert r.bin_pass == base.bin_pass


def test_too_small_limit_is_nomem(gpu):
    xy = dev(planted(500, 0.4, 33))
    for call in (lambda: gpu.solve(xy, max_workspace=4096),
                 lambda: gpu.solve_batched(xy, np.array([0, 250, 500]), max_workspace=4096)):
        with pytest.raises(gpu.LmsError) as e:
            call()
        assert "out of device memory" in str(e.value)
    with pytest.raises(gpu.LmsError):
        gpu.workspace_size(500, max_workspace=4096)
