"""Write the stored expected values under tests/golden/ (calls only the oracle).

    python tests/golden/make_golden.py inputs          # generator SHA-256 digests
    python tests/golden/make_golden.py oracle c2 c3s   # oracle results per config

Oracle results are the exhaustive FP64 search of oracle/lms_oracle.c on the
seeded inputs of workloads/gen.py. Nothing here touches the GPU library.
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
}


def inputs(name, seed):
    if name == "degenerate_int_4096":
        return gen.degenerate_int(4096, seed)
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


def write_oracle(names):
    path = os.path.join(HERE, "oracle_results.json")
    store = json.load(open(path)) if os.path.exists(path) else {}
    for name in names:
        for gname, seed in ORACLE_CASES[name]:
            xy = inputs(gname, seed)
            t = time.time()
            r = oracle.solve(xy)
            dt = time.time() - t
            store[f"{gname}/{seed}"] = {
                "n": int(xy.shape[0]), "h": r.h, "status": r.status,
                "width": r.width.hex(), "theta1": r.theta1.hex(), "theta2": r.theta2.hex(),
                "z_lo": r.z_lo.hex(), "z_hi": r.z_hi.hex(),
                "half_width": r.half_width.hex(),
                "pair": [r.pair_i, r.pair_j], "candidates": r.candidates,
                "vertical": r.vertical, "input_sha256": digest(xy),
                "seconds": round(dt, 2),
                "readable": {"half_width": r.half_width, "theta1": r.theta1,
                             "theta2": r.theta2},
            }
            print(gname, seed, store[f"{gname}/{seed}"]["readable"], f"{dt:.1f}s", flush=True)
            with open(path, "w") as f:
                json.dump(store, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    if sys.argv[1] == "inputs":
        write_inputs()
    elif sys.argv[1] == "oracle":
        write_oracle(sys.argv[2:])
