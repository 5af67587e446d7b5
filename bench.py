#!/usr/bin/env python3
"""Throughput of the multilevel partitioning hot path on one MI355X.

One step = one whole hgp_partition call on a device-resident hypergraph:
every coarsening pass and contraction, the greedy initial partition, and
projection + label-propagation refinement on every level.  The metric is
input pins per second (pins of the finest level divided by the step time).

Prints one JSON line.  The CPU baseline is the sequential oracle on the
host, timed on the same workload (one core).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2303_17679_amd import workloads as W  # noqa: E402

WORKLOADS = {
    # name: (description, k)
    "stencil160": "row-net model of a 3D 7-point stencil on a 160^3 grid (4,096,000 vertices and nets, "
                  "28,518,400 pins), unit weights, k=64, eps=0.03",
    "powerlaw1m": "power-law hypergraph, seed 2, n=m=1,000,000, Zipf(2.1) net sizes in [2,1000], Zipf(2.3) "
                  "vertex degrees, net weights in [1,4], k=8, eps=0.03",
    "random10k": "random hypergraph, seed 1, n=m=10,000, net sizes in [2,8], k=2, eps=0.03",
}


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 PMC runs
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or None
    when no such record exists or the kernel sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(f"{workload}:{kernel}")
    if not rec:
        return None
    src = os.path.join(ROOT, "paper_2303_17679_amd", "csrc", rec["source"])
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["source_sha256"]:
        return None
    return rec["bytes_per_launch"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="stencil160", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain elementwise copy of 1 GiB (read 1 GiB, write 1 GiB) three times, "
                         "the reference for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2303_17679_amd as H

    if args.copy_calibration:
        n = 1 << 28  # int32 elements: 1 GiB each way
        src = torch.arange(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read": 4 * n, "bytes_written": 4 * n, "launches": 3}}),
              flush=True)
        return

    h, k = W.workload(args.workload)
    G = H.Hypergraph.from_host(h)
    prm = H.params(k, seed=args.seed)
    P = H.Partitioner(G, prm)
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        P.run()
    torch.cuda.synchronize()
    roof, dom, acc, KT = None, None, None, None
    if not args.no_roofline:
        # untimed: (1) which kernel dominates one step, (2) its compulsory bytes
        KT = H.KernelTimer(h.n, h.m)
        KT.begin((1 << len(H.KERNELS)) - 1, account=False)
        P.run()
        disc = KT.end()
        dom = max(range(len(disc)), key=lambda i: disc[i]["ms"])
        KT.begin(1 << dom, account=True)
        P.run()
        acc = KT.end()[dom]
        KT.begin(1 << dom, account=False)  # events on the dominant kernel only
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        levels = P.run()
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    if KT is not None:
        tim = KT.end()[dom]
        avg_s = tim["ms"] / 1e3 / max(tim["launches"], 1)
        per_launch = acc["bytes"] / max(acc["launches"], 1)
        achieved = per_launch / avg_s / 1e9 if avg_s > 0 else 0.0
        roof = {"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s", "frac": achieved / 8000.0,
                "traffic": measured_traffic(H.KERNELS[dom], args.workload),
                "kernel": H.KERNELS[dom], "avg_launch_us": avg_s * 1e6,
                "launches_per_step": tim["launches"] / args.steps,
                "alg_bytes_per_launch": per_launch,
                "kernel_share_of_step": tim["ms"] / 1e3 / T}
    f_gpu = int(P.f.item())
    value = h.p * args.steps / T

    cpu = None
    oracle_match = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build()
        t1 = time.perf_counter()
        part_o, f_o, L_o = oracle.partition(h, oracle.params(k, seed=args.seed))
        To = time.perf_counter() - t1
        cpu = {"value": h.p / To, "unit": "pins/s", "cores": 1, "kind": "oracle",
               "sample": f"the whole {args.workload} partition (all levels), one run, single thread, "
                         f"{To:.1f} s"}
        import numpy as np
        oracle_match = bool(f_o == f_gpu and L_o == levels and
                            np.array_equal(P.part.cpu().numpy().view(np.uint32), part_o))

    line = {
        "metric": "pins/s for coarsen+LP refine (HBM GB/s vs peak)",
        "value": value,
        "unit": "pins/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * T / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32/int64 (integer only)",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload], "k": k,
                   "n": h.n, "m": h.m, "pins": h.p, "levels": levels, "objective": f_gpu,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "oracle_match": oracle_match,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
