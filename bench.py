"""Throughput of the exact 2D LMS search on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]

A step is one complete solve (prep, seed evaluation, FP32 screen, FP64
recheck, finalize) of one point set whose coordinates are already resident in
HBM. The default workload is the headline one: a planted line with n = 4096
points, 45 % uniform outliers and h = 2049. That is 8,386,560 candidate pair
slopes per step. The input is synthetic: the paper's random point sets are not
published.

Printed as one JSON line: candidate slopes per second (the headline value),
solves per second, the screen kernel's fraction of the VALU issue peak
measured with HIP events on the solve's stream, and the CPU oracle timed on a
bounded sample of the same workload on the host's cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "candidate slopes/sec and LMS solves/sec at n=4096; learned vs plain speedup"

# VALU issue peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one 32-bit
# (or FP64) lane-op per lane per clock (packed FP32 is not used).
VALU_PEAK_LANE_OPS = 256 * 64 * 2.4e9
# Algorithmic lane-ops of the FP32 test per residual: band test = FMA + |d| <= t
# compare; one-sided tests = FMA + four compares.
OPS_BAND, OPS_DIR = 2, 5
# Algorithmic lane-ops of the slope-bin screen: per (anchor, point) insertion,
# the reciprocal of dx, two sums and three products for the interval ends,
# three bin maps and four histogram increments (13); per (anchor, bin), one
# prefix-sum add; per (anchor, partner) query, the slope, its bin map, the
# lookup and two compares (5).
OPS_INSERT, OPS_BIN, OPS_QUERY = 13, 1, 5
PRUNED_BINS = 2048


def roofline(stage_ms, n, pairs, r):
    """Roofline of the dominant screen kernel (slope bins or the FP32 test),
    timed by the library's HIP events on the solve's stream."""
    kernels = {}
    # r.bins == 2048: the slope range ran and the pruned screen visited only
    # the anchors and points it left; its ops are then counted as the full
    # screen's (an equivalent rate, not executed work)
    pruned = r.bins == PRUNED_BINS
    if r.bins:
        nb = 1 << max(11, min(15, (2 * n - 1).bit_length())) if pruned else r.bins
        ops = OPS_INSERT * n * (n - 1) + OPS_BIN * n * nb + OPS_QUERY * pairs
        kernels["k_bins_pruned" if pruned else "k_bins"] = (ops, stage_ms["bins"])
    ops = OPS_BAND * r.point_evals + OPS_DIR * r.dir_evals
    kernels["k_screen_list" if r.bins else "k_screen"] = (ops, stage_ms["screen"])
    name = max(kernels, key=lambda k: kernels[k][1])
    ops, ms = kernels[name]
    achieved = ops / (ms * 1e-3)
    return {"bound": "alu", "kernel": name, "achieved": achieved / 1e12,
            "ops_basis": "full-screen equivalent" if name == "k_bins_pruned" else "algorithmic",
            "peak": VALU_PEAK_LANE_OPS / 1e12, "unit": "T lane-op/s",
            "frac": achieved / VALU_PEAK_LANE_OPS, "traffic": None, "ops_per_launch": ops,
            "kernels": {k: {"ms": v[1], "ops": v[0], "frac": v[0] / (v[1] * 1e-3) /
                            VALU_PEAK_LANE_OPS} for k, v in kernels.items()}}


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3a", "c3b", "c4"])
    ap.add_argument("--seed", type=int, default=None)
    ap.add_argument("--tile-regs", type=int, default=0,
                    help="64-point chunks of the screen kept in registers (0 = automatic)")
    ap.add_argument("--bins-log2", type=int, default=0,
                    help="slope bins per anchor, 2^k (0 = automatic, -1 = no slope-bin screen)")
    ap.add_argument("--seed-pairs", type=int, default=None,
                    help="random seed pairs of a single solve (default: the library's)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the seeding comparison")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target wall time of the CPU-oracle sample (0 = skip)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this size (HBM counter scale)")
    return ap.parse_args()


def cpu_baseline(xy, target_s):
    """The oracle as it stands, on a random sample of the workload's pairs."""
    import numpy as np
    import oracle
    from workloads.gen import Stream

    n = len(xy)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    st = Stream(99, 990)

    def sample(m):
        a = st.integers(m, 0, n - 1)
        b = st.integers(m, 0, n - 2)
        b = b + (b >= a)
        return np.stack([a, b], 1)

    probe = max(threads * 8, 64)
    t = time.perf_counter()
    oracle.eval_pairs(xy, sample(probe), nthreads=threads)
    rate = probe / max(time.perf_counter() - t, 1e-6)
    m = int(min(max(rate * target_s, probe), 5_000_000))
    t = time.perf_counter()
    oracle.eval_pairs(xy, sample(m), nthreads=threads)
    dt = time.perf_counter() - t
    return {"value": m / dt, "unit": "candidate slopes/s", "cores": threads, "kind": "oracle",
            "sample": f"{m} random pairs of the same n={n} input, full FP64 sort per pair "
                      f"({dt:.1f} s wall)"}


def main():
    args = parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (one problem "
              "would shard by anchor range, each GPU screening its share against the same "
              "width bound).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1510_01041_amd as lms
    from workloads import gen

    dev = torch.device("cuda:0")
    if args.calibrate_copy_mib:
        nb = args.calibrate_copy_mib << 20
        a = torch.empty(nb // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": nb, "bytes_written": nb,
                          "launches": args.steps}))
        return

    if args.workload == "c4":
        return bench_batched(args)

    cfg = gen.CONFIGS[args.workload]
    seed = cfg["seeds"][0] if args.seed is None else args.seed
    xy = gen.make(args.workload, seed)
    n = len(xy)
    h = gen.default_h(n)
    pairs = n * (n - 1) // 2
    d = torch.from_numpy(xy).to(dev)
    out = torch.empty(lms.RESULT_BYTES, dtype=torch.uint8, device=dev)

    kw = dict(tile_regs=args.tile_regs, bins_log2=args.bins_log2, seed_pairs=args.seed_pairs)
    for _ in range(args.warmup):
        lms.solve_async(d, 0, out, graph=True, **kw)
    torch.cuda.synchronize()
    first = lms.parse(out)
    if first.status < 0:
        raise SystemExit(f"solve failed: {lms.status_str(first.status)}")

    # timed: the whole solve replayed from a captured hipGraph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lms.solve_async(d, 0, out, graph=True, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    r = lms.parse(out)
    ms_step = (t1 - t0) * 1e3 / args.steps

    # stage split: eager launches with HIP events on the solve's stream
    eager_steps = max(3, min(args.steps, 20))
    lms.solve_async(d, 0, out, **kw)
    lms.profile_begin()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(eager_steps):
        lms.solve_async(d, 0, out, **kw)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    n_prof, stage_ms = lms.profile_end()
    stages = {k: v / max(n_prof, 1) for k, v in stage_ms.items()}
    ms_eager = (t3 - t2) * 1e3 / eager_steps
    re = lms.parse(out)
    if (re.width, re.theta1, re.z_lo) != (r.width, r.theta1, r.z_lo):
        raise SystemExit("graph replay and eager solve differ")

    parity = "not checked"
    gold_path = os.path.join(ROOT, "tests", "golden", "oracle_results.json")
    if os.path.exists(gold_path):
        g = json.load(open(gold_path)).get(f"{args.workload}/{seed}")
        if g:
            same = (r.width == float.fromhex(g["width"]) and r.theta1 == float.fromhex(g["theta1"]))
            parity = "bitwise equal to stored oracle" if same else \
                f"MISMATCH vs stored oracle width {float.fromhex(g['width'])!r}"

    line = {
        "metric": METRIC,
        "value": pairs / (ms_step * 1e-3),
        "unit": "candidate slopes/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 screen, f64 recheck", "data": "synthetic",
        "config": {"workload": f"{args.workload}: " + (
            f"planted line y=0.7x+2+N(0,0.05^2), n={n}, {cfg.get('f_out', 0):.0%} uniform "
            f"outliers" if cfg["kind"] == "planted" else
            f"integer points in [0,1023]^2, n={n}, 30% duplicated x"),
            "n": n, "h": h, "pairs": pairs, "seed": seed, "tile_regs": args.tile_regs,
            "bins_log2": args.bins_log2, "seed_pairs": args.seed_pairs},
        "solves_per_sec": 1e3 / ms_step,
        "mode": "hipGraph replay of the whole solve",
        "eager_ms_per_step": ms_eager,
        "stages_ms_per_solve": stages,
        "roofline": roofline(stages, n, pairs, r),
        "search": {"survivors": r.survivors, "band_pass": r.band_pass, "bin_pass": r.bin_pass,
                   "vertical": r.vertical, "band_evals": r.point_evals,
                   "dir_evals": r.dir_evals,
                   "evals_per_pair": r.point_evals / max(r.candidates, 1)},
        "result": {"half_width": r.half_width, "theta1": r.theta1, "theta2": r.theta2,
                   "parity": parity},
    }
    if not args.no_compare:
        line["learned_vs_plain"] = seeding_comparison(lms, d, r, max(3, args.steps // 5))
    if args.cpu_seconds > 0:
        line["cpu_baseline"] = cpu_baseline(xy, args.cpu_seconds)
    print(json.dumps(line), flush=True)


def seeding_comparison(lms, d, ref, steps):
    """Time the same solve under different initial width bounds.

    plain: 255 random pair slopes (the default). learned: the seed network's
    slope, then two rounds of 63 pairs drawn from the narrowest window found
    (from the network's line, then from the best of those pairs), with network
    inference inside the timed region. Also reported: the network slope alone,
    the learned seeds plus the random pairs, no seed at all (only the
    extreme-x pair), 63 random pairs, and the exact LMS slope itself (the
    tightest bound any seed can give). Every variant must return the same
    line. pruned: the fraction of candidate slopes that the band test rejects
    early."""
    import numpy as np
    import torch
    from paper_1510_01041_amd import seednet

    wpath = os.path.join(ROOT, "paper_1510_01041_amd", "seednet_weights.npy")
    net = seednet.SeedNet.load_weights(wpath) if os.path.exists(wpath) else None
    off = np.array([0, d.shape[0]], dtype=np.int64)
    plan = net.plan(off) if net else None  # built once: no copies in the timed loop
    out = torch.empty(lms.RESULT_BYTES, dtype=torch.uint8, device=d.device)
    exact = torch.tensor([ref.theta1], dtype=torch.float64, device=d.device)

    def run(kind):
        def once():
            if kind == "plain":
                lms.solve_async(d, 0, out)
            elif kind == "no_seed":
                lms.solve_async(d, 0, out, seed_pairs=0)
            elif kind == "control63":
                lms.solve_async(d, 0, out, seed_pairs=63)
            elif kind == "exact_slope":
                lms.solve_async(d, 0, out, seed_pairs=0, seed_theta=exact)
            else:
                th = net.predict_slopes(d, plan=plan)
                lms.solve_async(d, 0, out, seed_pairs=None if kind == "learned+pairs" else 0,
                                seed_theta=th,
                                window_pairs=0 if kind == "learned_slope_only" else 63)
        once()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            once()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        r = lms.parse(out)
        return {"ms": ms, "survivors": r.survivors, "band_pass": r.band_pass,
                "pruned": 1.0 - r.band_pass / max(r.candidates, 1),
                "band_evals_per_pair": r.point_evals / max(r.candidates, 1),
                "same_result": (r.width, r.theta1, r.z_lo) == (ref.width, ref.theta1, ref.z_lo)}

    kinds = ["plain", "no_seed", "control63", "exact_slope"]
    if net:
        kinds += ["learned", "learned_slope_only", "learned+pairs"]
    res = {k: run(k) for k in kinds}
    res["mismatches"] = sum(not v["same_result"] for v in res.values() if isinstance(v, dict))
    if net:
        th = float(net.predict_slopes(d, plan=plan)[0])
        res["learned_angle_error_deg"] = abs(np.degrees(np.arctan(th) - np.arctan(ref.theta1)))
        res["speedup_learned_vs_plain"] = res["plain"]["ms"] / res["learned"]["ms"]
        res["speedup_learned_vs_no_seed"] = res["no_seed"]["ms"] / res["learned"]["ms"]
    else:
        res["note"] = "no trained seed network weights found"
    return res


def bench_batched(args):
    """20,000 Hough-style patches (n ~ U{32..512}): one graph replay of the
    batched pipeline per step, against one lms_solve launch per problem."""
    import numpy as np
    import torch

    import paper_1510_01041_amd as lms
    from workloads import gen

    dev = torch.device("cuda:0")
    seed = gen.CONFIGS["c4"]["seeds"][0] if args.seed is None else args.seed
    xy, off = gen.hough_patches(gen.CONFIGS["c4"]["B"], seed)
    B = len(off) - 1
    pairs = int((np.diff(off) * (np.diff(off) - 1) // 2).sum())
    d = torch.from_numpy(xy).to(dev)
    out = torch.empty((B, lms.RESULT_BYTES), dtype=torch.uint8, device=dev)
    for _ in range(args.warmup):
        lms.solve_batched_async(d, off, out=out, graph=True)
    torch.cuda.synchronize()
    lms.profile_begin()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lms.solve_batched_async(d, off, out=out, graph=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lms.profile_end()
    res = lms.parse_batch(out)
    ms_batched = (t1 - t0) * 1e3 / args.steps

    # eager (no graph) batched pass, for the per-stage split
    lms.profile_begin()
    lms.solve_batched_async(d, off, out=out)
    torch.cuda.synchronize()
    n_prof, stage_ms = lms.profile_end()

    # one launch per problem on one stream, on the same resident data
    outs = torch.empty((B, lms.RESULT_BYTES), dtype=torch.uint8, device=dev)
    views = [d[off[b]:off[b + 1]] for b in range(B)]
    for b in range(min(B, 200)):
        lms.solve_async(views[b], 0, outs[b])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in range(B):
        lms.solve_async(views[b], 0, outs[b])
    torch.cuda.synchronize()
    ms_loop = (time.perf_counter() - t0) * 1e3
    single = lms.parse_batch(outs)
    same = bool(np.all(single.width == res.width) and np.all(single.theta1 == res.theta1))

    nb = np.diff(off).astype(np.int64)
    kernels = {"k_bscreen_list": (OPS_BAND * int(res.point_evals.sum()) +
                                  OPS_DIR * int(res.dir_evals.sum()), stage_ms["screen"])}
    if int(res.bins.max()) > 0:
        kernels["k_bbins"] = (int((OPS_INSERT * nb * (nb - 1) + OPS_BIN * nb * res.bins.astype(np.int64)
                                   + OPS_QUERY * (nb * (nb - 1) // 2)).sum()), stage_ms["bins"])
    name = max(kernels, key=lambda k: kernels[k][1])
    ops, kms = kernels[name]
    line = {
        "metric": "LMS solves/sec, batched Hough patches",
        "value": B / (ms_batched * 1e-3), "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_batched,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 screen, f64 recheck", "data": "synthetic",
        "config": {"workload": f"c4: {B} patches of 64x64 px, n~U{{32..512}}, 30-45% salt noise",
                   "B": B, "points": int(off[-1]), "pairs": pairs, "seed": seed},
        "candidate_slopes_per_sec": pairs / (ms_batched * 1e-3),
        "one_launch_per_problem": {"ms": ms_loop, "solves_per_sec": B / (ms_loop * 1e-3),
                                   "bitwise_equal": same},
        "speedup_vs_per_problem": ms_loop / ms_batched,
        "stages_ms_eager": stage_ms,
        "roofline": {"bound": "alu", "kernel": name, "achieved": ops / (kms * 1e-3) / 1e12,
                     "peak": VALU_PEAK_LANE_OPS / 1e12, "unit": "T lane-op/s",
                     "frac": ops / (kms * 1e-3) / VALU_PEAK_LANE_OPS, "traffic": None,
                     "ops_per_launch": ops,
                     "kernels": {k: {"ms": v[1], "ops": v[0],
                                     "frac": v[0] / (v[1] * 1e-3) / VALU_PEAK_LANE_OPS}
                                 for k, v in kernels.items()}},
        "search": {"survivors": int(res.survivors.sum()), "band_pass": int(res.band_pass.sum()),
                   "bin_pass": int(res.bin_pass.sum()),
                   "vertical": int(res.vertical.sum())},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
