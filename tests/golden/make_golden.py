"""Write the stored expected values under tests/golden/ (calls only the oracle).

    python tests/golden/make_golden.py inputs          # generator SHA-256 digests
    python tests/golden/make_golden.py oracle c2 c3s   # oracle results per config
    python tests/golden/make_golden.py bounded c3 mid  # same, by the bounded search
    python tests/golden/make_golden.py c4 [workers]    # every problem of the batch

Oracle results are the exhaustive FP64 search of oracle/lms_oracle.c on the
seeded inputs of workloads/gen.py. Above a few thousand points the exhaustive
search takes days on a few cores; there the stored result comes from the
oracle's bounded search (lms_oracle_solve_bounded), which returns the same
fields bitwise (pinned against the exhaustive search in the oracle's tests,
at 4096 points among others) and is recorded with "method": "bounded".
Nothing here touches the GPU library.
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from workloads import gen  # noqa: E402

# cases whose oracle result is stored: name -> (generator call, seeds)
ORACLE_CASES = {
    "c1": [("c1", s) for s in (101, 102, 103)],
    "c2": [("c2", s) for s in (201, 202, 203)],
    # a 4096-point slice of the integer, duplicated-x workload (full size is
    # beyond the oracle's reach on a few cores)
    "c3s": [("degenerate_int_4096", 302)],
    # the 16384-point workloads: planted, and integer with duplicated x
    "c3": [("c3a", 301), ("c3b", 302)],
    # sizes where the slope range (one and two grids) prunes the screen
    "mid": [("planted_6000", 601), ("planted_9000", 901),
            ("degenerate_int_6000", 602), ("degenerate_int_9000", 902)],
}


def inputs(name, seed):
    if name.startswith("degenerate_int_"):
        return gen.degenerate_int(int(name.rsplit("_", 1)[1]), seed)
    if name.startswith("planted_"):
        return gen.planted(int(name.rsplit("_", 1)[1]), 0.45, seed)
    return gen.make(name, seed)


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def write_inputs():
    out = {}
    for name, cfg in gen.CONFIGS.items():
        for s in cfg["seeds"]:
            v = gen.make(name, s)
            if isinstance(v, tuple):
                out[f"{name}/{s}"] = {"xy": digest(v[0]), "offsets": digest(v[1])}
            else:
                out[f"{name}/{s}"] = {"xy": digest(v)}
    out["degenerate_int_4096/302"] = {"xy": digest(gen.degenerate_int(4096, 302))}
    with open(os.path.join(HERE, "inputs_sha256.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


def write_oracle(names, bounded=False):
    path = os.path.join(HERE, "oracle_results.json")
    for name in names:
        for gname, seed in ORACLE_CASES[name]:
            xy = inputs(gname, seed)
            t = time.time()
            if bounded:
                r, evaluated = oracle.solve_bounded(xy)
            else:
                r, evaluated = oracle.solve(xy), None
            dt = time.time() - t
            store = json.load(open(path)) if os.path.exists(path) else {}
            store[f"{gname}/{seed}"] = {
                "n": int(xy.shape[0]), "h": r.h, "status": r.status,
                "width": r.width.hex(), "theta1": r.theta1.hex(), "theta2": r.theta2.hex(),
                "z_lo": r.z_lo.hex(), "z_hi": r.z_hi.hex(),
                "half_width": r.half_width.hex(),
                "pair": [r.pair_i, r.pair_j], "candidates": r.candidates,
                "vertical": r.vertical, "input_sha256": digest(xy),
                "seconds": round(dt, 2),
                "method": "bounded" if bounded else "exhaustive",
                **({"slopes_evaluated": evaluated} if bounded else {}),
                "readable": {"half_width": r.half_width, "theta1": r.theta1,
                             "theta2": r.theta2},
            }
            print(gname, seed, store[f"{gname}/{seed}"]["readable"], f"{dt:.1f}s", flush=True)
            with open(path, "w") as f:
                json.dump(store, f, indent=1, sort_keys=True)


def _c4_shard(args):
    """Exhaustive oracle on problems [b0, b1) of the 20,000-patch batch."""
    b0, b1, path = args
    if os.path.exists(path):
        return path
    xy, off = gen.make("c4", 401)
    rec = np.zeros((b1 - b0, 4), dtype=np.float64)
    meta = np.zeros((b1 - b0, 5), dtype=np.int64)
    for b in range(b0, b1):
        r = oracle.solve(xy[off[b]:off[b + 1]], nthreads=1)
        rec[b - b0] = (r.width, r.theta1, r.z_lo, r.z_hi)
        meta[b - b0] = (r.pair_i, r.pair_j, r.candidates, r.vertical, r.status)
    np.savez(path + ".tmp.npz", rec=rec, meta=meta)
    os.replace(path + ".tmp.npz", path)
    return path


def write_c4(workers=6, shard=250, ckpt="/tmp/lms_golden_c4"):
    """Oracle result of all 20,000 problems of c4 (seed 401), sharded with
    per-shard checkpoint files so that an interrupted run resumes."""
    from multiprocessing import Pool
    os.makedirs(ckpt, exist_ok=True)
    xy, off = gen.make("c4", 401)
    B = len(off) - 1
    jobs = [(b, min(B, b + shard), os.path.join(ckpt, f"shard_{b:05d}.npz"))
            for b in range(0, B, shard)]
    # the biggest shards first would not help: sizes are i.i.d. per problem
    t = time.time()
    with Pool(workers) as pool:
        for k, path in enumerate(pool.imap_unordered(_c4_shard, jobs)):
            print(f"shard {k + 1}/{len(jobs)} {os.path.basename(path)} {time.time() - t:.0f}s",
                  flush=True)
    rec = np.concatenate([np.load(j[2])["rec"] for j in jobs])
    meta = np.concatenate([np.load(j[2])["meta"] for j in jobs])
    np.savez_compressed(os.path.join(HERE, "c4_401_oracle.npz"), rec=rec, meta=meta,
                        offsets_sha256=np.array(digest(off)), xy_sha256=np.array(digest(xy)))


if __name__ == "__main__":
    if sys.argv[1] == "inputs":
        write_inputs()
    elif sys.argv[1] == "oracle":
        write_oracle(sys.argv[2:])
    elif sys.argv[1] == "bounded":
        write_oracle(sys.argv[2:], bounded=True)
    elif sys.argv[1] == "c4":
        write_c4(int(sys.argv[2]) if len(sys.argv) > 2 else 6)
