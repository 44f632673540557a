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
# LDS instruction issue: one LDS instruction per CU per clock (the LDS pipe of
# each CU accepts one wavefront instruction per cycle)
LDS_INST_PEAK = 256 * 2.4e9


COUNTERS = os.path.join(ROOT, "profiles", "counters.json")


def kernel_source_sha():
    """SHA-256 of the HIP sources (csrc/*.hip, *.h in name order): the
    counters in profiles/counters.json hold only for the sources they were
    taken from."""
    import hashlib
    d = os.path.join(ROOT, "paper_1510_01041_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def _counters():
    """The committed counter summary, or None if absent or taken from other
    kernel sources than these."""
    if not os.path.exists(COUNTERS):
        return None
    c = json.load(open(COUNTERS))
    return c if c.get("source_sha256") == kernel_source_sha() else None


def issued(kernel, workload, ms):
    """Issued-VALU and LDS fractions of a kernel: its per-launch instruction
    counts (rocprofv3 --pmc, committed under profiles/) over the launch time
    measured here, and its HBM traffic per launch (FETCH_SIZE and WRITE_SIZE
    scaled by what they read for a plain copy of known size). None if the
    counters are absent or stale."""
    cs = _counters()
    c = cs and cs["kernels"].get(kernel, {}).get(workload)
    if not c or not ms:
        return None
    t = ms * 1e-3
    out = {"source": "profiles/counters.json", "counters": c}
    if "SQ_INSTS_VALU" in c:
        out["valu_lane_ops_per_s"] = c["SQ_INSTS_VALU"] * 64 / t
        out["valu_frac"] = c["SQ_INSTS_VALU"] * 64 / t / VALU_PEAK_LANE_OPS
    if "SQ_INSTS_LDS" in c:
        # one LDS instruction per CU per clock
        out["lds_insts_per_s"] = c["SQ_INSTS_LDS"] / t
        out["lds_frac_of_issue"] = c["SQ_INSTS_LDS"] / t / (LDS_INST_PEAK)
    if "SQ_LDS_BANK_CONFLICT" in c and "SQ_INSTS_LDS" in c:
        out["bank_conflict_cycles_per_lds_inst"] = c["SQ_LDS_BANK_CONFLICT"] / max(
            c["SQ_INSTS_LDS"], 1)
    if "SQ_ACTIVE_INST_VALU" in c and "SQ_BUSY_CYCLES" in c:
        out["valu_active_per_busy_cycle"] = c["SQ_ACTIVE_INST_VALU"] / max(c["SQ_BUSY_CYCLES"], 1)
    tr = traffic(kernel, workload)
    if tr is not None:
        out["hbm_bytes_per_launch"] = tr
        out["hbm_gb_per_s"] = tr / t / 1e9
    return out


def traffic(kernel, workload):
    """HBM bytes per launch from the counter summary (None if absent)."""
    cs = _counters()
    c = cs and cs["kernels"].get(kernel, {}).get(workload)
    cal = cs and cs.get("copy")
    if not c or not cal or "FETCH_SIZE" not in c or "WRITE_SIZE" not in c:
        return None
    return 1024.0 * (c["FETCH_SIZE"] * cal["fetch_scale"] + c["WRITE_SIZE"] * cal["write_scale"])


def roofline(stage_ms, n, pairs, r, workload):
    """Roofline of the dominant screen kernel (slope bins or the FP32 test),
    timed by the library's HIP events on the solve's stream. `achieved` counts
    the method's algorithmic lane-ops of the full slope-bin screen (the
    pruned screen after a slope range is reported by its issued counters
    only: its work depends on the range, not on a formula of n)."""
    kernels = {}
    pruned = r.bins == PRUNED_BINS
    if r.bins and not pruned:
        ops = OPS_INSERT * n * (n - 1) + OPS_BIN * n * r.bins + OPS_QUERY * pairs
        kernels["k_bins"] = (ops, stage_ms["bins"])
    ops = OPS_BAND * r.point_evals + OPS_DIR * r.dir_evals
    kernels["k_screen_list" if r.bins else "k_screen"] = (ops, stage_ms["screen"])
    name = max(kernels, key=lambda k: kernels[k][1])
    ops, ms = kernels[name]
    achieved = ops / (ms * 1e-3)
    out = {"bound": "alu", "kernel": name, "achieved": achieved / 1e12,
           "peak": VALU_PEAK_LANE_OPS / 1e12, "unit": "T lane-op/s",
           "frac": achieved / VALU_PEAK_LANE_OPS, "traffic": traffic(name, workload),
           "ops_per_launch": ops,
           "kernel_ms": ms,
           "kernels": {k: {"ms": v[1], "ops": v[0], "frac": v[0] / (v[1] * 1e-3) /
                           VALU_PEAK_LANE_OPS} for k, v in kernels.items()}}
    out["issued"] = issued(name, workload, ms)
    if pruned:
        out["k_bins_pruned"] = {"ms": stage_ms["bins"],
                                "issued": issued("k_bins_pruned", workload, stage_ms["bins"])}
    return out


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
    ap.add_argument("--slope-range", choices=["auto", "on", "off"], default="auto",
                    help="slope-range pruning before the slope-bin screen (auto: the library's)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the seeding comparison")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the named workload (skip the n = 16384 sets, the batch, "
                         "Algorithm 1, sampling and line detection blocks)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target wall time of the CPU-oracle sample (0 = skip)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this size (HBM counter scale)")
    return ap.parse_args()


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


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
            "cpu_model": cpu_model(),
            "sample": f"{m} random pairs of the same n={n} input, full FP64 sort per pair "
                      f"({dt:.1f} s wall)"}


def graph_ms(lms, d, out, steps, warmup=2, **kw):
    """Mean wall time of `steps` solves replayed from one captured hipGraph."""
    import torch
    for _ in range(max(warmup, 1)):
        lms.solve_async(d, 0, out, graph=True, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        lms.solve_async(d, 0, out, graph=True, **kw)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps, lms.parse(out)


def stored_parity(name, seed, r):
    gold_path = os.path.join(ROOT, "tests", "golden", "oracle_results.json")
    if not os.path.exists(gold_path):
        return "not checked"
    g = json.load(open(gold_path)).get(f"{name}/{seed}")
    if not g:
        return "no stored oracle result"
    w = float.fromhex(g["width"])
    if r.width == w and r.theta1 == float.fromhex(g["theta1"]):
        return "bitwise equal to stored oracle"
    if abs(r.width - w) <= 1e-9 * w:
        return "width within 1e-9 of stored oracle (tied slope)"
    return f"MISMATCH vs stored oracle width {w!r}"


def measure_single(lms, name, seed, steps, warmup, kw):
    """One workload of single solves: graph replays (timed), then an eager
    pass with the library's stage events."""
    import torch
    from workloads import gen
    cfg = gen.CONFIGS[name]
    xy = gen.make(name, seed)
    n = len(xy)
    pairs = n * (n - 1) // 2
    d = torch.from_numpy(xy).to("cuda:0")
    out = torch.empty(lms.RESULT_BYTES, dtype=torch.uint8, device=d.device)
    ms, r = graph_ms(lms, d, out, steps, warmup, **kw)
    if r.status < 0:
        raise SystemExit(f"solve failed: {lms.status_str(r.status)}")
    eager_steps = max(3, min(steps, 20))
    lms.solve_async(d, 0, out, **kw)
    lms.profile_begin()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(eager_steps):
        lms.solve_async(d, 0, out, **kw)
    torch.cuda.synchronize()
    ms_eager = (time.perf_counter() - t2) * 1e3 / eager_steps
    n_prof, stage_ms = lms.profile_end()
    stages = {k: v / max(n_prof, 1) for k, v in stage_ms.items()}
    re = lms.parse(out)
    if (re.width, re.theta1, re.z_lo) != (r.width, r.theta1, r.z_lo):
        raise SystemExit("graph replay and eager solve differ")
    return dict(xy=xy, d=d, r=r, n=n, pairs=pairs, cfg=cfg, ms=ms, ms_eager=ms_eager,
                stages=stages, roofline=roofline(stages, n, pairs, r, name),
                parity=stored_parity(name, seed, r))


def search_counts(r):
    return {"survivors": r.survivors, "band_pass": r.band_pass, "bin_pass": r.bin_pass,
            "bins": r.bins, "vertical": r.vertical, "band_evals": r.point_evals,
            "dir_evals": r.dir_evals, "evals_per_pair": r.point_evals / max(r.candidates, 1)}


def main():
    args = parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (one problem "
              "would shard by anchor range, each GPU screening its share against the same "
              "width bound).", file=sys.stderr)
        sys.exit(2)

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
        print(json.dumps(bench_batched(args, per_problem=not args.no_extra)), flush=True)
        return

    seed = gen.CONFIGS[args.workload]["seeds"][0] if args.seed is None else args.seed
    kw = dict(tile_regs=args.tile_regs, bins_log2=args.bins_log2, seed_pairs=args.seed_pairs,
              slope_range={"auto": None, "on": True, "off": False}[args.slope_range])
    M = measure_single(lms, args.workload, seed, args.steps, args.warmup, kw)
    r, n, cfg = M["r"], M["n"], M["cfg"]
    line = {
        "metric": METRIC,
        "value": M["pairs"] / (M["ms"] * 1e-3),
        "unit": "candidate slopes/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": M["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 screen, f64 recheck", "data": "synthetic",
        "config": {"workload": f"{args.workload}: " + (
            f"planted line y=0.7x+2+N(0,0.05^2), n={n}, {cfg.get('f_out', 0):.0%} uniform "
            f"outliers" if cfg["kind"] == "planted" else
            f"integer points in [0,1023]^2, n={n}, 30% duplicated x"),
            "n": n, "h": gen.default_h(n), "pairs": M["pairs"], "seed": seed,
            "tile_regs": args.tile_regs, "bins_log2": args.bins_log2,
            "seed_pairs": args.seed_pairs},
        "solves_per_sec": 1e3 / M["ms"],
        "mode": "hipGraph replay of the whole solve",
        "eager_ms_per_step": M["ms_eager"],
        "stages_ms_per_solve": M["stages"],
        "roofline": M["roofline"],
        "search": search_counts(r),
        "result": {"half_width": r.half_width, "theta1": r.theta1, "theta2": r.theta2,
                   "parity": M["parity"]},
    }
    net = load_net(lms)
    if not args.no_compare:
        line["learned_vs_plain"] = {args.workload: seeding_comparison(
            lms, M["d"], r, max(3, args.steps // 5), net, with_no_seed=True)}
    if args.workload == "c2" and not args.no_extra:
        # the n = 16384 workloads and the batch, measured by the same run
        for name in ("c3a", "c3b"):
            X = measure_single(lms, name, gen.CONFIGS[name]["seeds"][0], 10, 2, {})
            line[name] = {"ms_per_solve": X["ms"], "candidate_slopes_per_sec":
                          X["pairs"] / (X["ms"] * 1e-3), "stages_ms_per_solve": X["stages"],
                          "roofline": X["roofline"], "search": search_counts(X["r"]),
                          "parity": X["parity"]}
            if name == "c3a":
                if not args.no_compare:
                    line["learned_vs_plain"]["c3a"] = seeding_comparison(
                        lms, X["d"], X["r"], 5, net, with_no_seed=False)
                line["sampling"] = sampling_block(lms, X["d"], X["r"])
        line["c4"] = bench_batched(args, steps=5, warmup=2, per_problem=True)
        line["paper_alg1"] = alg1_block(lms)
        line["line_detection"] = line_detection_block(lms)
    if args.cpu_seconds > 0:
        line["cpu_baseline"] = cpu_baseline(M["xy"], args.cpu_seconds)
    print(json.dumps(line), flush=True)


def load_net(lms):
    wpath = os.path.join(ROOT, "paper_1510_01041_amd", "seednet_weights.npy")
    if not os.path.exists(wpath):
        return None
    from paper_1510_01041_amd import seednet
    return seednet.SeedNet.load_weights(wpath)


def seeding_comparison(lms, d, ref, steps, net, with_no_seed=True):
    """The same solve under different initial width bounds, each replayed from
    its own hipGraph (network inference, when used, runs inside the graph).

    plain: 127 random pair slopes (the default). no_seed: only the extreme-x
    pair. learned: no random pairs; the seed network's slope, computed inside
    the solve, is the only seed. learned+window: the same, then two rounds of
    63 pairs drawn from the narrowest window found. exact_slope: the LMS slope
    itself as the only seed (the tightest bound any seed can give). Every
    variant must return the same line. pruned: the fraction of candidate
    slopes the screens reject before the FP32 band test passes them."""
    import numpy as np
    import torch
    out = torch.empty(lms.RESULT_BYTES, dtype=torch.uint8, device=d.device)
    exact = torch.tensor([ref.theta1], dtype=torch.float64, device=d.device)
    variants = {"plain": {}, "exact_slope": dict(seed_pairs=0, seed_theta=exact)}
    if with_no_seed:
        variants["no_seed"] = dict(seed_pairs=0)
    if net is not None:
        variants["learned"] = dict(seed_pairs=0, net_params=net.P)
        variants["learned+window"] = dict(seed_pairs=0, net_params=net.P, window_pairs=63)
    res = {}
    for k, kw in variants.items():
        st = 1 if k == "no_seed" else steps
        ms, r = graph_ms(lms, d, out, st, 1, **kw)
        res[k] = {"ms": ms, "survivors": r.survivors, "band_pass": r.band_pass,
                  "bin_pass": r.bin_pass, "pruned": 1.0 - r.band_pass / max(r.candidates, 1),
                  "band_evals_per_pair": r.point_evals / max(r.candidates, 1),
                  "same_result": (r.width, r.theta1, r.z_lo) == (ref.width, ref.theta1, ref.z_lo)}
    res["mismatches"] = sum(not v["same_result"] for v in res.values() if isinstance(v, dict))
    if net is not None:
        th = float(net.predict_slopes(d, np.array([0, d.shape[0]]))[0])
        res["learned_angle_error_deg"] = float(abs(np.degrees(np.arctan(th) -
                                                              np.arctan(ref.theta1))))
        res["speedup_learned_vs_plain"] = res["plain"]["ms"] / res["learned"]["ms"]
        res["speedup_learned_window_vs_plain"] = res["plain"]["ms"] / res["learned+window"]["ms"]
        if with_no_seed:
            res["speedup_learned_vs_no_seed"] = res["no_seed"]["ms"] / res["learned"]["ms"]
            res["band_pass_no_seed_over_learned"] = (res["no_seed"]["band_pass"] /
                                                     max(res["learned"]["band_pass"], 1))
    else:
        res["note"] = "no trained seed network weights found"
    return res


def sampling_block(lms, d, ref, ms=(1024, 2048, 4096), steps=5):
    """Random sampling before the exact search: the exact LMS of m of the n
    points (lms_solve_sampled), its time and its error against the exact
    result: the slope's angle, and the whole set's narrowest window at that
    slope over the exact one (>= 1)."""
    import numpy as np
    import torch
    out = torch.empty(lms.RESULT_BYTES, dtype=torch.uint8, device=d.device)
    res = {}
    for m in ms:
        lms.solve_sampled_async(d, m, 12345, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            lms.solve_sampled_async(d, m, 12345, out=out)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) * 1e3 / steps
        r = lms.parse(out)
        w_full = float(lms.eval_slopes(d, torch.tensor([r.theta1]))[0, 0])
        res[str(m)] = {"ms": t, "angle_error_deg": float(abs(np.degrees(
            np.arctan(r.theta1) - np.arctan(ref.theta1)))), "width_ratio": w_full / ref.width}
    return res


PAPER_TABLE1_MS = {128: 0.98, 256: 4.22, 512: 35.3}  # the paper's GPU, Section 4, Table 1


def alg1_block(lms, steps=5):
    """Algorithm 1 as stated (every vertex sorted) against lms_solve, on the
    paper's set sizes; and how often the printed rank rule misses."""
    import torch
    from workloads.gen import Stream, planted
    res = {}
    for n in (128, 256, 512):
        d = torch.from_numpy(planted(n, 0.4, 1600 + n)).to("cuda:0")
        row = {"paper_table1_ms": PAPER_TABLE1_MS[n]}
        for rule, key in ((lms.RULE_TIED, "alg1_tied"), (lms.RULE_LITERAL, "alg1_literal")):
            out = lms.solve_bracelets_async(d, 0, rule)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                lms.solve_bracelets_async(d, 0, rule, out=out)
            torch.cuda.synchronize()
            row[key + "_ms"] = (time.perf_counter() - t0) * 1e3 / steps
            row[key + "_width"] = lms.parse(out).width
        out = torch.empty(lms.RESULT_BYTES, dtype=torch.uint8, device=d.device)
        row["lms_solve_ms"], r = graph_ms(lms, d, out, 20)
        row["lms_solve_width"] = r.width
        row["speedup_solve_vs_alg1"] = row["alg1_tied_ms"] / row["lms_solve_ms"]
        res[str(n)] = row
    # the printed rule on small general-position sets: how often it misses
    st = Stream(8, 80)
    misses = 0
    for _ in range(100):
        d = torch.from_numpy(st.uniform(32, -100, 100).reshape(16, 2)).to("cuda:0")
        a = lms.solve_bracelets(d, 0, lms.RULE_TIED)
        b = lms.solve_bracelets(d, 0, lms.RULE_LITERAL)
        misses += b.width > a.width
    res["literal_rule_misses_of_100_sets_n16"] = misses
    return res


def line_detection_block(lms, noise=(0.001, 0.002, 0.004, 0.006, 0.01), seeds=(1, 2, 3, 4)):
    """Hough then LMS on synthetic 1024^2 edge images (one segment kept with
    probability 0.5, salt noise with probability p), d_rho = 20 px,
    d_theta = 2 degrees: the angle error of the LMS line and of the
    accumulator cell's own line against the true segment, per noise level."""
    import numpy as np
    import torch
    from workloads.gen import line_image
    res = {}
    for p in noise:
        e_lms, e_cell, ms = [], [], []
        for s in seeds:
            pix, on, seg = line_image(p, s)
            d = torch.from_numpy(pix).to("cuda:0")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            got = lms.detect_lines(d, 1024, 1024, 20.0, 2.0, 1)
            ms.append((time.perf_counter() - t0) * 1e3)
            true = np.degrees(np.arctan2(seg[3] - seg[1], seg[2] - seg[0])) % 180.0
            L = got[0]
            r = L["result"]
            ang = (np.degrees(np.arctan2(1.0, r.theta1)) if L["transposed"]
                   else np.degrees(np.arctan(r.theta1))) % 180.0
            cell = (L["theta_bin"] * 2.0 + 90.0) % 180.0

            def err(a):
                e = abs(a - true) % 180.0
                return min(e, 180.0 - e)
            e_lms.append(err(ang))
            e_cell.append(err(cell))
        res[str(p)] = {"lms_angle_error_deg_median": float(np.median(e_lms)),
                       "cell_angle_error_deg_median": float(np.median(e_cell)),
                       "ms_per_image": float(np.median(ms))}
    return res


def bench_batched(args, steps=None, warmup=None, per_problem=True):
    """20,000 Hough-style patches (n ~ U{32..512}): one graph replay of the
    batched pipeline per step, against one lms_solve launch per problem."""
    import numpy as np
    import torch

    import paper_1510_01041_amd as lms
    from workloads import gen

    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    dev = torch.device("cuda:0")
    seed = gen.CONFIGS["c4"]["seeds"][0] if args.seed is None or args.workload != "c4" \
        else args.seed
    xy, off = gen.hough_patches(gen.CONFIGS["c4"]["B"], seed)
    B = len(off) - 1
    pairs = int((np.diff(off) * (np.diff(off) - 1) // 2).sum())
    d = torch.from_numpy(xy).to(dev)
    out = torch.empty((B, lms.RESULT_BYTES), dtype=torch.uint8, device=dev)
    for _ in range(max(warmup, 1)):
        lms.solve_batched_async(d, off, out=out, graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        lms.solve_batched_async(d, off, out=out, graph=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    res = lms.parse_batch(out)
    ms_batched = (t1 - t0) * 1e3 / steps

    # eager (no graph) batched pass, for the per-stage split
    lms.profile_begin()
    lms.solve_batched_async(d, off, out=out)
    torch.cuda.synchronize()
    n_prof, stage_ms = lms.profile_end()

    line = {
        "metric": "LMS solves/sec, batched Hough patches",
        "value": B / (ms_batched * 1e-3), "unit": "solves/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": ms_batched,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 screen, f64 recheck", "data": "synthetic",
        "config": {"workload": f"c4: {B} patches of 64x64 px, n~U{{32..512}}, 30-45% salt noise",
                   "B": B, "points": int(off[-1]), "pairs": pairs, "seed": seed},
        "candidate_slopes_per_sec": pairs / (ms_batched * 1e-3),
        "stages_ms_eager": stage_ms,
    }
    if per_problem:
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
        line["one_launch_per_problem"] = {"ms": ms_loop, "solves_per_sec": B / (ms_loop * 1e-3),
                                          "bitwise_equal": same}
        line["speedup_vs_per_problem"] = ms_loop / ms_batched
    # every problem against the oracle's stored result (written by
    # tests/golden/make_golden.py from the oracle alone)
    gold = os.path.join(ROOT, "tests", "golden", "c4_401_oracle.npz")
    if os.path.exists(gold) and seed == 401:
        g = np.load(gold)
        w = g["rec"][:, 0]
        ok = np.abs(res.width - w) <= 1e-9 * np.maximum(np.abs(res.width), np.abs(w))
        line["parity"] = {"problems": B, "width_within_1e-9": int(ok.sum()),
                          "status_ok": int((res.status >= 0).sum())}

    nb = np.diff(off).astype(np.int64)
    # problems up to 512 points take the one-pair-per-lane FP32 screen
    sname = "k_bscreen_lanes" if int(nb.max()) <= 512 else "k_bscreen_list"
    kernels = {sname: (OPS_BAND * int(res.point_evals.sum()) +
                       OPS_DIR * int(res.dir_evals.sum()), stage_ms["screen"])}
    if int(res.bins.max()) > 0:
        # problems up to 1024 points take the one-wavefront-per-anchor kernel
        bname = "k_bbins_wave" if int(nb.max()) <= 1024 else "k_bbins"
        kernels[bname] = (int((OPS_INSERT * nb * (nb - 1) + OPS_BIN * nb * res.bins.astype(np.int64)
                                   + OPS_QUERY * (nb * (nb - 1) // 2)).sum()), stage_ms["bins"])
    name = max(kernels, key=lambda k: kernels[k][1])
    ops, kms = kernels[name]
    line["roofline"] = {"bound": "alu", "kernel": name, "achieved": ops / (kms * 1e-3) / 1e12,
                        "peak": VALU_PEAK_LANE_OPS / 1e12, "unit": "T lane-op/s",
                        "frac": ops / (kms * 1e-3) / VALU_PEAK_LANE_OPS,
                        "traffic": traffic(name, "c4"),
                        "ops_per_launch": ops, "kernel_ms": kms,
                        "issued": issued(name, "c4", kms),
                        "kernels": {k: {"ms": v[1], "ops": v[0],
                                        "frac": v[0] / (v[1] * 1e-3) / VALU_PEAK_LANE_OPS}
                                    for k, v in kernels.items()}}
    line["search"] = {"survivors": int(res.survivors.sum()), "band_pass": int(res.band_pass.sum()),
                      "bin_pass": int(res.bin_pass.sum()), "vertical": int(res.vertical.sum())}
    return line


if __name__ == "__main__":
    main()
