"""Line detection (lms_detect_lines) against the reference detector
(oracle/hough.py), through the C ABI: the accumulator bit for bit, the same
peaks, supporting sets and sampling, and the LMS fit of every set equal to
the oracle's exhaustive search (width to 1e-9, window certified by the oracle
at the GPU's slope: pixel data ties exactly)."""
import numpy as np
import pytest
import torch

from oracle import hough
from workloads.gen import line_image

pytestmark = pytest.mark.gpu


def run(gpu, orc, pix, W=1024, H=1024, d_rho=20.0, d_theta=2.0, max_lines=1, min_votes=2,
        max_support=4096, seed=0):
    n_theta, n_rho = gpu.hough_grid(W, H, d_rho, d_theta)
    acc = torch.zeros((n_theta, n_rho), dtype=torch.int32, device="cuda:0")
    got = gpu.detect_lines(torch.from_numpy(pix).to("cuda:0"), W, H, d_rho, d_theta, max_lines,
                           min_votes, max_support, seed, acc=acc)
    oacc, want = hough.detect(pix, W, H, d_rho, d_theta, max_lines, min_votes, max_support, seed)
    assert np.array_equal(acc.cpu().numpy().astype(np.int64), oacc)
    assert len(got) == len(want)
    for g, w in zip(got, want):
        for k in ("theta_bin", "rho_bin", "votes", "support", "fitted", "transposed"):
            assert g[k] == w[k], k
        r, o = g["result"], w["result"]
        print(g["theta_bin"], g["rho_bin"], g["votes"], r.width, o.width, flush=True)
        assert r.status == o.status
        assert abs(r.width - o.width) <= 1e-9 * max(r.width, o.width) or r.width == o.width
        assert orc.window(w["xy"], r.theta1) == (r.width, r.z_lo, r.z_hi)
    return got, want


@pytest.mark.parametrize("p_noise,seed", [(0.001, 1), (0.002, 2), (0.004, 3), (0.006, 4)])
def test_single_line_images(gpu, orc, p_noise, seed):
    pix, on, seg = line_image(p_noise, seed)
    got, _ = run(gpu, orc, pix)
    assert got and got[0]["votes"] >= 2


def test_many_peaks_and_coarse_grid(gpu, orc):
    pix, _, _ = line_image(0.003, 11)
    run(gpu, orc, pix, d_rho=20.0, d_theta=20.0, max_lines=8)
    run(gpu, orc, pix, d_rho=5.0, d_theta=2.0, max_lines=40, min_votes=5)


def test_sampled_supporting_sets(gpu, orc):
    pix, _, _ = line_image(0.02, 12)
    got, _ = run(gpu, orc, pix, max_lines=4, max_support=64, seed=7)
    assert any(g["support"] > g["fitted"] == 64 for g in got)


def test_empty_and_tiny_images(gpu, orc):
    for pix in (np.zeros((0, 2), dtype=np.int32),
                np.array([[3, 4]], dtype=np.int32),
                np.array([[3, 4], [3, 4], [5, 4]], dtype=np.int32)):
        run(gpu, orc, pix, W=16, H=16, d_rho=1.0, d_theta=45.0, max_lines=3)
