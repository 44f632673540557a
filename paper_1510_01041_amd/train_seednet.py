"""Train the seed network on exact LMS solutions.

    python -m paper_1510_01041_amd.train_seednet --sets 200000 --n 2048 --epochs 20 \\
        --out paper_1510_01041_amd/seednet_weights.npy

Training data: seeded rotated-line sets (workloads.gen.rotated_line: outlier
fraction U[0, 0.45], line angle U[-pi/2, pi/2)). Each set is labelled by the
exact batched GPU solver and kept resident in HBM. Each batch trains on one
random subset of m points of its sets, m drawn log-uniformly from
[min_points, n], so that the network works at every size it will see
(inference reads larger sets strided, at seednet.MAX_POINTS points). Each set's
frame is its robust one (coordinate-wise median and MAD of a fixed sample of
its points), so that the outliers do not set it. Forward, backward
and Adam run in the library's kernels. PyTorch only holds the buffers and
gathers each batch into one contiguous block.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_1510_01041_amd as lms  # noqa: E402
from paper_1510_01041_amd import seednet  # noqa: E402
from workloads import gen  # noqa: E402


def label(d: torch.Tensor, off: np.ndarray, log=print):
    """Exact LMS slope of every set in one batch (FP64, host array). The
    batched solver re-solves on its own any set whose survivors did not fit
    its shared list, so every set gets its exact answer."""
    res = lms.solve_batched(d, off)
    st = np.asarray(res.status)
    if np.any(st < 0):
        raise RuntimeError(f"labelling failed with status {np.unique(st[st < 0]).tolist()}")
    return np.asarray(res.theta1, dtype=np.float64)


def build_dataset(n_sets, n, seed, chunk, net, log=print):
    """Generate and label (exact solver) n_sets sets of n points: raw FP32
    points on the device and the exact slopes on the host."""
    dev = net.device
    xy_all = torch.empty((n_sets * n, 2), dtype=torch.float32, device=dev)
    theta_all = np.empty(n_sets)
    t0 = time.time()
    for c0 in range(0, n_sets, chunk):
        cn = min(chunk, n_sets - c0)
        xy, off = gen.rotated_line(cn, n, seed * 1000 + c0 // chunk)
        d = torch.from_numpy(xy).to(dev)
        theta_all[c0:c0 + cn] = label(d, np.asarray(off, dtype=np.int64), log)
        xy_all[c0 * n:(c0 + cn) * n] = d.to(torch.float32)
        log(f"labelled {c0 + cn}/{n_sets} sets ({time.time() - t0:.1f} s)")
    return xy_all, theta_all


def batch_inputs(net, xy_sets: torch.Tensor, theta: np.ndarray, pts_idx: torch.Tensor):
    """Normalised points and targets of sets (B, n, 2) restricted to pts_idx."""
    B = xy_sets.shape[0]
    sub = xy_sets.index_select(1, pts_idx).reshape(-1, 2).to(torch.float64).contiguous()
    m = pts_idx.numel()
    off = torch.arange(B + 1, dtype=torch.int64, device=net.device) * m
    pts, scale, off = net.prepare(sub, off)
    tgt = seednet.targets_from_slopes(theta, scale.cpu().numpy())
    return pts, off, torch.from_numpy(tgt).to(net.device)


def angle_error(out: np.ndarray, tgt: np.ndarray) -> np.ndarray:
    """|phi_hat - phi| in radians, modulo pi (from the doubled-angle outputs)."""
    d = np.arctan2(out[:, 1], out[:, 0]) - np.arctan2(tgt[:, 1], tgt[:, 0])
    d = (d + np.pi) % (2 * np.pi) - np.pi
    return np.abs(d) / 2


def train(n_sets=200000, n=2048, epochs=20, batch=256, lr=2e-3, seed=1, chunk=4096,
          test_frac=0.05, min_points=256, log=print, net=None):
    net = net or seednet.SeedNet(seed=seed)
    xy, theta = build_dataset(n_sets, n, seed, chunk, net, log)
    n_test = max(1, int(n_sets * test_frac))
    n_train = n_sets - n_test
    view = xy.view(n_sets, n, 2)
    g = torch.Generator(device="cpu").manual_seed(seed)
    hist = {"loss": [], "test_loss": [], "test_angle_err_deg": []}
    all_pts = torch.arange(n, device=net.device)
    tpts, toff, ttgt = batch_inputs(net, view[n_train:], theta[n_train:], all_pts)
    t0 = time.time()
    for ep in range(epochs):
        perm = torch.randperm(n_train, generator=g)
        tot, cnt = torch.zeros((), device=net.device), 0
        lr_ep = lr * 0.5 * (1 + np.cos(np.pi * ep / max(epochs, 1)))  # cosine schedule
        for s0 in range(0, n_train - batch + 1, batch):
            idx = perm[s0:s0 + batch]
            m = int(round(np.exp(np.log(min_points) + (np.log(n) - np.log(min_points)) *
                                 torch.rand((), generator=g).item())))
            sub = torch.randperm(n, generator=g)[:m].to(net.device)
            pts, off, tgt = batch_inputs(net, view.index_select(0, idx.to(net.device)),
                                         theta[idx.numpy()], sub)
            loss = net.train_step(pts, off, tgt, lr=lr_ep)
            tot = tot + loss.sum()
            cnt += 1
        hist["loss"].append(float(tot) / max(cnt, 1))
        # held-out split, all n points
        out, _ = net.forward(tpts, toff, want_g=False)
        o = out.cpu().numpy().astype(np.float64)
        t = ttgt.cpu().numpy().astype(np.float64)
        hist["test_loss"].append(float(0.5 * np.mean(np.sum((o - t) ** 2, 1))))
        hist["test_angle_err_deg"].append(float(np.degrees(np.median(angle_error(o, t)))))
        log(f"epoch {ep}: train loss {hist['loss'][-1]:.5f}, test loss "
            f"{hist['test_loss'][-1]:.5f}, median angle error "
            f"{hist['test_angle_err_deg'][-1]:.3f} deg ({time.time() - t0:.1f} s)")
    return net, hist


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sets", type=int, default=200000)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--min-points", type=int, default=256)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "seednet_weights.npy"))
    args = ap.parse_args()
    t0 = time.time()
    net, hist = train(args.sets, args.n, args.epochs, args.batch, args.lr, args.seed,
                      min_points=args.min_points, log=lambda s: print(s, flush=True))
    net.save(args.out)
    print(json.dumps({"weights": args.out, "sets": args.sets, "n": args.n, "epochs": args.epochs,
                      "seconds": time.time() - t0, **{k: v[-1] for k, v in hist.items()},
                      "history": hist}), flush=True)


if __name__ == "__main__":
    main()
