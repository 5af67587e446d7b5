"""Writes the expected results of the full-size workloads, from the CPU oracle
only: tests/golden/full_<workload>.json.

    python tests/golden/make_full.py stencil160 powerlaw1m [rmat24]

Each record holds the SHA-256 of the generated input arrays (so a test can
tell a generator change from a partitioner change), the number of levels,
the lambda-1 objective, the block weights and the SHA-256 of the final
partition (uint32, little endian) of one oracle run with seed 0.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2303_17679_amd import workloads as W  # noqa: E402


def input_sha(h) -> str:
    d = hashlib.sha256()
    for a, dt in ((h.pin_off, np.uint32), (h.pins, np.uint32), (h.vwgt, np.int32), (h.nwgt, np.int32)):
        d.update(np.ascontiguousarray(a, dt).tobytes())
    return d.hexdigest()


def main(names):
    for name in names:
        t = time.time()
        h, k = W.workload(name)
        print(f"{name}: generated in {time.time() - t:.1f} s", flush=True)
        seed = 0
        t = time.time()
        part, f, levels = oracle.partition(h, oracle.params(k, seed=seed))
        print(f"{name}: oracle in {time.time() - t:.1f} s, levels {levels}, objective {f}", flush=True)
        _, bw = oracle.objective(h, k, part)
        rec = {"workload": name, "k": k, "seed": seed, "n": int(h.n), "m": int(h.m), "p": int(h.p),
               "input_sha256": input_sha(h), "levels": levels, "objective": f,
               "block_weights": [int(x) for x in bw],
               "part_sha256": hashlib.sha256(np.ascontiguousarray(part, np.uint32).tobytes()).hexdigest()}
        with open(os.path.join(HERE, f"full_{name}.json"), "w") as fh:
            json.dump(rec, fh, indent=1)
            fh.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:] or ["stencil160", "powerlaw1m"])
