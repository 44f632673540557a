"""The autotuner sweeps the hot path's parameters on the device (the
slope-bin screen's bins, the slope range, the seeds, the FP32 screen's
tiles), persists its choice, and solves that use it return the same line."""
import json
import os

import numpy as np
import pytest
import torch

from workloads import gen
from workloads.gen import planted

pytestmark = pytest.mark.gpu


@pytest.fixture
def clean_table(gpu):
    yield
    os.environ.pop("LMS_TUNE_FILE", None)
    gpu.tuning_clear()


@pytest.mark.parametrize("n", [2500, 6000])
def test_autotune_single_and_persist(gpu, tmp_path, clean_table, n):
    os.environ["LMS_TUNE_FILE"] = str(tmp_path / "tune.json")
    xy = planted(n, 0.45, 4500 + n)
    d = torch.from_numpy(np.ascontiguousarray(xy)).cuda()
    before = gpu.solve(d)
    t = gpu.autotune(d, reps=2)
    print(n, t, flush=True)
    # tiles: the size's default or a swept one; bins down to n / 2 (below 2 n
    # the screen takes its WIDE form)
    assert 1 <= t["tile_regs"] <= 64 and 1 <= t["tile_batches"] <= 8 and t["ms"] > 0
    assert 11 <= t["bins_log2"] <= 15 and (1 << t["bins_log2"]) >= n // 2
    assert t["range"] in (-1, 0, 1) and t["seed_pairs"] in (63, 127, 255)
    after = gpu.solve(d)
    assert (after.width, after.theta1, after.z_lo, after.z_hi) == \
           (before.width, before.theta1, before.z_lo, before.z_hi)
    rows = json.load(open(tmp_path / "tune.json"))
    cls = 4096 if n <= 4096 else 8192
    assert any(r[1] == 0 and r[2] == cls and r[8] == t["range"] for r in rows)
    # the tuned choice is used: with the range tuned off the full screen runs
    if t["range"] < 0:
        assert after.bins != 2048


def test_autotune_batched(gpu, clean_table):
    xy, off = gen.hough_patches(400, 31)
    d = torch.from_numpy(xy).cuda()
    a = gpu.solve_batched(d, off)
    t = gpu.autotune_batched(d, off, reps=2)
    assert t["seed_pairs"] in (15, 31, 63) and t["bins_log2"] in (11, 12)
    b = gpu.solve_batched(d, off)
    # the tuned choice gives every problem the default width bit for bit
    # (integer patches have exact width ties; another tied line may be chosen)
    assert np.all(b.status == 0)
    assert np.array_equal(a.width, b.width)
    assert set(np.unique(b.bins[np.diff(off) <= 1024])) == {(1 << t["bins_log2"]) + 64}
