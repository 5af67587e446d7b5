"""Summaries of rocprofv3 CSV output for the committed profile records.

    python -m paper_2303_17679_amd.rocprof_summary stats DIR --cmd "..." [--runs R]
        Markdown table of the kernel-trace statistics in DIR/*_kernel_stats.csv.

    python -m paper_2303_17679_amd.rocprof_summary traffic --workload W --kernel K --source FILE \
        --copy-fetch D1 --copy-write D2 --fetch D3 --write D4 --cmd-copy "..." --cmd "..."
        HBM bytes per launch of kernel K from two PMC runs (FETCH_SIZE, WRITE_SIZE,
        KiB per dispatch), each scaled by what the same counter reads for a plain
        elementwise copy of known size (bench.py --copy-calibration).  Prints a
        Markdown summary and updates profiles/traffic.json.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _csv(d: str, suffix: str):
    files = sorted(glob.glob(os.path.join(d, f"*{suffix}")))
    if not files:
        raise SystemExit(f"no *{suffix} under {d}")
    rows = []
    for f in files:
        rows += list(csv.DictReader(open(f)))
    return rows


def short(name: str) -> str:
    s = name.replace("(anonymous namespace)::", "").split("(")[0]
    return s.replace("void ", "").strip()


def stats(d: str, cmd: str, runs: int, top: int = 40) -> str:
    rows = _csv(d, "_kernel_stats.csv")
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    out = [f"Command (run from /tmp with TMPDIR=/tmp, repository at $R):", "", f"    {cmd}", "",
           f"Kernel time over the whole program: {tot / 1e6:.2f} ms; per partition run "
           f"(÷ {runs} runs of the hot path in the program): {tot / 1e6 / runs:.2f} ms.", "",
           "| kernel | calls | calls/run | total ms | ms/run | avg us | min us | max us | % |",
           "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for r in rows[:top]:
        c = int(r["Calls"])
        t = float(r["TotalDurationNs"]) / 1e6
        out.append(f"| `{short(r['Name'])}` | {c} | {c / runs:.1f} | {t:.3f} | {t / runs:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                   f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out) + "\n"


def _counter(d: str, counter: str, match: str):
    vals = [float(r["Counter_Value"]) for r in _csv(d, "_counter_collection.csv")
            if r["Counter_Name"] == counter and match in r["Kernel_Name"]]
    if not vals:
        raise SystemExit(f"no {counter} records for kernels matching {match!r} under {d}")
    return vals


def traffic(a) -> str:
    cal = json.loads(a.copy_json) if a.copy_json else {"bytes_read": 1 << 30, "bytes_written": 1 << 30}
    cf = _counter(a.copy_fetch, "FETCH_SIZE", a.copy_kernel)
    cw = _counter(a.copy_write, "WRITE_SIZE", a.copy_kernel)
    sf = cal["bytes_read"] / (statistics.mean(cf) * 1024.0)
    sw = cal["bytes_written"] / (statistics.mean(cw) * 1024.0)
    kf = _counter(a.fetch, "FETCH_SIZE", a.kernel)
    kw = _counter(a.write, "WRITE_SIZE", a.kernel)
    fb = statistics.mean(kf) * 1024.0 * sf
    wb = statistics.mean(kw) * 1024.0 * sw
    src = os.path.join(HERE, "csrc", a.source)
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    path = os.path.join(ROOT, "profiles", "traffic.json")
    db = json.load(open(path)) if os.path.exists(path) else {}
    db[f"{a.workload}:{a.kernel}"] = {
        "source": a.source, "source_sha256": sha, "bytes_per_launch": fb + wb,
        "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb, "launches": len(kf),
        "fetch_scale": sf, "write_scale": sw}
    with open(path, "w") as fh:
        json.dump(db, fh, indent=1, sort_keys=True)
        fh.write("\n")
    return "\n".join([
        f"HBM traffic of `{a.kernel}` on {a.workload}", "",
        "Calibration (plain elementwise copy, 1 GiB read + 1 GiB written per launch):", "",
        f"    {a.cmd_copy.replace('COUNTER', 'FETCH_SIZE')}",
        f"    {a.cmd_copy.replace('COUNTER', 'WRITE_SIZE')}", "",
        f"- FETCH_SIZE reads {statistics.mean(cf):.1f} KiB per copy launch -> scale {sf:.4f}",
        f"- WRITE_SIZE reads {statistics.mean(cw):.1f} KiB per copy launch -> scale {sw:.4f}", "",
        "Kernel passes:", "",
        f"    {a.cmd.replace('COUNTER', 'FETCH_SIZE')}",
        f"    {a.cmd.replace('COUNTER', 'WRITE_SIZE')}", "",
        f"- launches: {len(kf)}",
        f"- FETCH_SIZE mean {statistics.mean(kf):.1f} KiB (min {min(kf):.1f}, max {max(kf):.1f}) "
        f"-> {fb / 1e6:.2f} MB per launch",
        f"- WRITE_SIZE mean {statistics.mean(kw):.1f} KiB (min {min(kw):.1f}, max {max(kw):.1f}) "
        f"-> {wb / 1e6:.3f} MB per launch",
        f"- traffic per launch: {(fb + wb) / 1e6:.2f} MB", "",
        f"Source `{a.source}` sha256 {sha} (the benchmark drops this record once the file changes).", ""])


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--cmd", required=True)
    s.add_argument("--runs", type=int, default=1)
    s.add_argument("--top", type=int, default=40)
    t = sub.add_parser("traffic")
    for k in ("workload", "kernel", "source", "copy_fetch", "copy_write", "fetch", "write", "cmd_copy", "cmd"):
        t.add_argument("--" + k.replace("_", "-"), required=True)
    t.add_argument("--copy-kernel", default="elementwise")
    t.add_argument("--copy-json", default="")
    a = ap.parse_args()
    print(stats(a.dir, a.cmd, a.runs, a.top) if a.what == "stats" else traffic(a), end="")


if __name__ == "__main__":
    main()
