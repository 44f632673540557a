"""Random sampling before the exact search (lms_solve_sampled), through the C
ABI, against the oracle's exact search on the same sample.

The draw is SplitMix64 keys per point, the m smallest taken in index order;
the oracle implements the draw from the generator's definition and solves
the sample exhaustively. Results must agree bit for bit (general position),
and m = n must reproduce the exact solve.
"""
import numpy as np
import pytest
import torch

from workloads.gen import degenerate_int, planted

pytestmark = pytest.mark.gpu


def dev(xy):
    return torch.from_numpy(np.ascontiguousarray(xy)).to("cuda:0")


def key(r):
    return (r.width, r.theta1, r.theta2, r.z_lo, r.z_hi, r.pair_i, r.pair_j, r.status)


@pytest.mark.parametrize("n,m,seed", [(3000, 64, 1), (3000, 500, 2), (3000, 2000, 3),
                                      (777, 2, 4), (777, 3, 5), (100_000, 300, 6),
                                      (40_000, 1000, 7)])
def test_sampled_matches_oracle(gpu, orc, n, m, seed):
    xy = planted(n, 0.45, 2000 + n + m)
    r = gpu.solve_sampled(dev(xy), m, seed)
    o = orc.solve_sampled(xy, m, seed)
    print(n, m, seed, r.width, o.width, flush=True)
    assert key(r) == key(o)
    assert r.candidates == o.candidates


def test_sampled_general_h_and_integer_data(gpu, orc):
    xy = planted(2000, 0.3, 21)
    for h in (2, 700, 1500, 2000):
        r = gpu.solve_sampled(dev(xy), 400, 9, h=h)
        o = orc.solve_sampled(xy, 400, 9, h=h)
        assert key(r) == key(o) and r.h == max(2, -(-h * 400 // 2000)), h
    xi = degenerate_int(1500, 22)
    r = gpu.solve_sampled(dev(xi), 600, 10)
    o = orc.solve_sampled(xi, 600, 10)
    assert r.width == o.width and r.status == o.status


def test_full_sample_is_the_exact_solve(gpu):
    xy = planted(1000, 0.45, 23)
    a = gpu.solve_sampled(dev(xy), 1000, 12345)
    b = gpu.solve(dev(xy))
    assert key(a) == key(b)


def test_sampled_arguments(gpu):
    xy = dev(planted(100, 0.3, 24))
    for m in (1, 101):
        with pytest.raises(gpu.LmsError):
            gpu.solve_sampled(xy, m, 0)
