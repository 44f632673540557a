"""Train the seed network on exact LMS solutions.

    python -m paper_1510_01041_amd.train_seednet --sets 65536 --n 2048 --epochs 20 \\
        --out paper_1510_01041_amd/seednet_weights.npy

Training data: seeded rotated-line sets (workloads.gen.rotated_line: outlier
fraction U[0, 0.45], line angle U[-pi/2, pi/2)). Each set is labelled by the
exact batched GPU solver, normalised on the device and kept resident in HBM.
Forward, backward and Adam run in the library's kernels. PyTorch only holds
the buffers and gathers each batch's sets into one contiguous block.
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
    """Exact LMS slope of every set in one batch (FP64, host array).

    A batch whose survivor list overflows (every set then reports
    LMS_ERR_CAPACITY) is split in halves and solved again; a single set that
    still overflows goes to the single-problem solver."""
    B = off.shape[0] - 1
    res = lms.solve_batched(d, off)
    st = np.asarray(res.status)
    if np.all(st >= 0):
        return np.asarray(res.theta1, dtype=np.float64)
    if np.any((st < 0) & (st != lms.LMS_ERR_CAPACITY)):
        bad = np.unique(st[st < 0]).tolist()
        raise RuntimeError(f"labelling failed with status {bad}")
    if B == 1:
        r = lms.solve(d[int(off[0]):int(off[1])].contiguous())
        if r.status < 0:
            raise RuntimeError(f"labelling failed with status {r.status}")
        return np.array([r.theta1])
    log(f"survivor list overflow on a batch of {B} sets: splitting it")
    m = B // 2
    a = off[:m + 1]
    b = off[m:]
    ta = label(d[int(a[0]):int(a[-1])].contiguous(), a - a[0], log)
    tb = label(d[int(b[0]):int(b[-1])].contiguous(), b - b[0], log)
    return np.concatenate([ta, tb])


def build_dataset(n_sets, n, seed, chunk, net, log=print):
    """Generate, label (exact solver) and normalise n_sets sets of n points."""
    dev = net.device
    pts_all = torch.empty((n_sets * n, 2), dtype=torch.float32, device=dev)
    tgt_all = np.empty((n_sets, 2), dtype=np.float32)
    theta_all = np.empty(n_sets)
    t0 = time.time()
    for c0 in range(0, n_sets, chunk):
        cn = min(chunk, n_sets - c0)
        xy, off = gen.rotated_line(cn, n, seed * 1000 + c0 // chunk)
        d = torch.from_numpy(xy).to(dev)
        theta = label(d, np.asarray(off, dtype=np.int64), log)
        pts, scale, _ = net.prepare(d, off)
        pts_all[c0 * n:(c0 + cn) * n] = pts
        sc = scale.cpu().numpy()
        theta_all[c0:c0 + cn] = theta
        tgt_all[c0:c0 + cn] = seednet.targets_from_slopes(theta, sc)
        log(f"labelled {c0 + cn}/{n_sets} sets ({time.time() - t0:.1f} s)")
    return pts_all, torch.from_numpy(tgt_all).to(dev), theta_all


def angle_error(out: np.ndarray, tgt: np.ndarray) -> np.ndarray:
    """|phi_hat - phi| in radians, modulo pi (from the doubled-angle outputs)."""
    d = np.arctan2(out[:, 1], out[:, 0]) - np.arctan2(tgt[:, 1], tgt[:, 0])
    d = (d + np.pi) % (2 * np.pi) - np.pi
    return np.abs(d) / 2


def train(n_sets=65536, n=2048, epochs=20, batch=256, lr=2e-3, seed=1, chunk=4096,
          test_frac=0.05, log=print, net=None):
    net = net or seednet.SeedNet(seed=seed)
    pts, tgt, _ = build_dataset(n_sets, n, seed, chunk, net, log)
    n_test = max(1, int(n_sets * test_frac))
    n_train = n_sets - n_test
    view = pts.view(n_sets, n, 2)
    g = torch.Generator(device="cpu").manual_seed(seed)
    off_b = torch.arange(batch + 1, dtype=torch.int64, device=net.device) * n
    hist = {"loss": [], "test_loss": [], "test_angle_err_deg": []}
    t0 = time.time()
    for ep in range(epochs):
        perm = torch.randperm(n_train, generator=g)
        tot, cnt = torch.zeros((), device=net.device), 0
        lr_ep = lr * 0.5 * (1 + np.cos(np.pi * ep / max(epochs, 1)))  # cosine schedule
        for s0 in range(0, n_train - batch + 1, batch):
            idx = perm[s0:s0 + batch].to(net.device)
            bp = view.index_select(0, idx).reshape(-1, 2).contiguous()
            loss = net.train_step(bp, off_b, tgt.index_select(0, idx), lr=lr_ep)
            tot = tot + loss.sum()
            cnt += 1
        hist["loss"].append(float(tot) / max(cnt, 1))
        # held-out split
        tp = view[n_train:].reshape(-1, 2).contiguous()
        toff = torch.arange(n_test + 1, dtype=torch.int64, device=net.device) * n
        out, _ = net.forward(tp, toff, want_g=False)
        o = out.cpu().numpy().astype(np.float64)
        t = tgt[n_train:].cpu().numpy().astype(np.float64)
        hist["test_loss"].append(float(0.5 * np.mean(np.sum((o - t) ** 2, 1))))
        hist["test_angle_err_deg"].append(float(np.degrees(np.median(angle_error(o, t)))))
        log(f"epoch {ep}: train loss {hist['loss'][-1]:.5f}, test loss "
            f"{hist['test_loss'][-1]:.5f}, median angle error "
            f"{hist['test_angle_err_deg'][-1]:.3f} deg ({time.time() - t0:.1f} s)")
    return net, hist


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sets", type=int, default=65536)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "seednet_weights.npy"))
    args = ap.parse_args()
    t0 = time.time()
    net, hist = train(args.sets, args.n, args.epochs, args.batch, args.lr, args.seed,
                      log=lambda s: print(s, flush=True))
    net.save(args.out)
    print(json.dumps({"weights": args.out, "sets": args.sets, "n": args.n, "epochs": args.epochs,
                      "seconds": time.time() - t0, **{k: v[-1] for k, v in hist.items()},
                      "history": hist}), flush=True)


if __name__ == "__main__":
    main()
