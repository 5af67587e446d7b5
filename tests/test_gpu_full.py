"""Full-size parity: hgp_partition on the full workloads, in the configuration
the benchmark times, against the expected results that the oracle wrote
(tests/golden/full_*.json, made by tests/golden/make_full.py).

Checks: identical final partition (SHA-256), objective, number of levels and
block weights, and the balance bound recomputed on the host.
"""
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np
import pytest

from paper_2303_17679_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
RECORDS = sorted(glob.glob(os.path.join(HERE, "golden", "full_*.json")))


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def input_sha(h) -> str:
    d = hashlib.sha256()
    for a, dt in ((h.pin_off, np.uint32), (h.pins, np.uint32), (h.vwgt, np.int32), (h.nwgt, np.int32)):
        d.update(np.ascontiguousarray(a, dt).tobytes())
    return d.hexdigest()


def lmax(W_, k, num=3, den=100):
    return (den + num) * (-(-W_ // k)) // den


@pytest.mark.parametrize("path", RECORDS, ids=[os.path.basename(p)[5:-5] for p in RECORDS])
def test_full_size_partition(path):
    import torch
    import paper_2303_17679_amd as H
    rec = json.load(open(path))
    name, k = rec["workload"], rec["k"]
    t = time.time()
    h, k2 = W.workload(name)
    assert k2 == k
    say(f"[{name}] generated n={h.n} m={h.m} p={h.p} in {time.time() - t:.1f} s")
    assert input_sha(h) == rec["input_sha256"], "the input generator changed"
    G = H.Hypergraph.from_host(h)
    P = H.Partitioner(G, H.params(k, seed=rec["seed"]))
    say(f"[{name}] partition")
    levels = P.run()
    torch.cuda.synchronize()
    f = int(P.f.item())
    part = P.part.cpu().numpy().view(np.uint32)
    say(f"[{name}] levels {levels} objective {f} (expected {rec['levels']}, {rec['objective']})")
    assert levels == rec["levels"]
    assert f == rec["objective"]
    assert hashlib.sha256(part.tobytes()).hexdigest() == rec["part_sha256"]
    bw = np.bincount(part, weights=h.vwgt.astype(np.float64), minlength=k).astype(np.int64)
    assert bw.tolist() == rec["block_weights"]
    assert int(bw.max()) <= lmax(int(h.vwgt.sum()), k)
    f2, bw2 = H.objective(G, k, P.part)
    assert f2 == f and bw2.cpu().numpy().tolist() == rec["block_weights"]
