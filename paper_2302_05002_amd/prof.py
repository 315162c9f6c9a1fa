"""Summaries of rocprofv3 output for the benchmark's kernels.

    python3 -m paper_2302_05002_amd.prof stats  <kernel_stats.csv> <builds>
        per-kernel device time per build (from a --kernel-trace --stats run)
    python3 -m paper_2302_05002_amd.prof pmc    <counter_collection.csv> <counter>
        per-build sum of one counter for each timed kernel group
    python3 -m paper_2302_05002_amd.prof traffic <fetch.csv> <write.csv> <workload> <out.json> [chunk_passes]
        FETCH_SIZE and WRITE_SIZE per build of every timed kernel group, with
        the digest of the HIP sources they were taken on, merged into out.json

Counter files come from runs of bench.py under ``rocprofv3 --pmc FETCH_SIZE``
(then ``WRITE_SIZE``); builds are delimited by the bounding-box kernel, which
every non-empty build launches exactly once.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))

# Plain-copy calibration of the two counters on MI355X: a copy of 256 MiB
# read back FETCH_SIZE = 131,100 KiB and WRITE_SIZE = 262,100 KiB, so actual
# bytes = FETCH_SIZE * 2.0 (reads) and WRITE_SIZE * 1.0 (writes).
READ_FACTOR = 2.0
WRITE_FACTOR = 1.0


def source_digest() -> str:
    """Hash of the HIP sources (counter readings apply only to the code they were taken on)."""
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    return name.split("(")[0].replace("void ", "").strip()


def stats(path: str, builds: int) -> str:
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    out = ["| kernel | calls/build | avg us | ms/build | % |", "|---|---:|---:|---:|---:|"]
    for r in rows:
        t = float(r["TotalDurationNs"])
        out.append(f"| {_short(r['Name'])} | {int(r['Calls']) / builds:g} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{t / 1e6 / builds:.4f} | {100 * t / tot:.1f} |")
    out.append(f"| **all kernels** | | | {tot / 1e6 / builds:.4f} | 100 |")
    return "\n".join(out)


def _dispatches(path: str, counter: str):
    """[(dispatch_id, kernel, value)] in dispatch order, summed over the counter's instances."""
    acc = defaultdict(float)
    names = {}
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter:
            continue
        d = int(r["Dispatch_Id"])
        acc[d] += float(r["Counter_Value"])
        names[d] = r["Kernel_Name"]
    return [(d, names[d], acc[d]) for d in sorted(acc)]


def groups_per_build(path: str, counter: str, chunk_passes: int = 1):
    """Per build, the counter summed over each timed kernel group (averaged over builds)."""
    seq = _dispatches(path, counter)
    starts = [i for i, (_, k, _) in enumerate(seq) if "k_bbox" in k]
    sums = defaultdict(float)
    nb = 0
    for bi, s0 in enumerate(starts):
        s1 = starts[bi + 1] if bi + 1 < len(starts) else len(seq)
        # the build's preview kernels come before its bounding box
        b = seq[s0:s1]
        nb += 1
        after_quant = in_counts = False
        chunk_left = chunk_passes
        for _, k, v in b:
            if "k_bbox" in k:
                sums["bbox"] += v
            elif "k_quantize" in k:
                sums["quantize"] += v
                after_quant = True
            elif "k_subsample" in k or "k_list_classes" in k:
                sums["subsample"] += v
            elif "k_np_pieces" in k:
                sums["node_counts"] += v
                in_counts = True
            elif "k_np_shared" in k:
                sums["node_counts"] += v
            elif "k_np_count" in k:
                sums["node_counts"] += v
                in_counts = False
            elif in_counts and "k_scan" in k:
                sums["node_counts"] += v
            elif "k_np_place" in k:
                sums["node_place"] += v
            elif "k_np_sort" in k or "k_np_merge" in k:
                sums["node_sort"] += v
            elif "k_ms_scatter<false" in k:
                if after_quant and chunk_left > 0:
                    sums["chunk_scatter"] += v
                    chunk_left -= 1
    return {k: v / nb for k, v in sums.items()}, nb


def traffic(fetch_csv: str, write_csv: str, workload: str, out_json: str, chunk_passes: int = 1):
    f, nf = groups_per_build(fetch_csv, "FETCH_SIZE", chunk_passes)
    w, nw = groups_per_build(write_csv, "WRITE_SIZE", chunk_passes)
    data = {"read_factor": READ_FACTOR, "write_factor": WRITE_FACTOR, "unit": "KiB per build", "kernels": {}}
    if os.path.exists(out_json):
        with open(out_json) as fh:
            data["kernels"] = json.load(fh).get("kernels", {})
    dig = source_digest()
    for k in sorted(set(f) | set(w)):
        data["kernels"][f"{workload}/{k}"] = {"fetch_kib": f.get(k, 0.0), "write_kib": w.get(k, 0.0),
                                              "builds": min(nf, nw), "source_digest": dig}
    with open(out_json, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    return data


def main(argv):
    if argv[0] == "stats":
        print(stats(argv[1], int(argv[2])))
    elif argv[0] == "pmc":
        g, nb = groups_per_build(argv[1], argv[2])
        print(f"{nb} builds; {argv[2]} per build (KiB):")
        for k, v in sorted(g.items()):
            print(f"  {k:14s} {v:14.1f}")
    elif argv[0] == "traffic":
        extra = [int(a) for a in argv[5:6]]
        d = traffic(argv[1], argv[2], argv[3], argv[4], *extra)
        for k, v in sorted(d["kernels"].items()):
            hbm = (v["fetch_kib"] * d["read_factor"] + v["write_kib"] * d["write_factor"]) / 1024
            print(f"  {k:30s} fetch {v['fetch_kib']:12.1f} KiB  write {v['write_kib']:12.1f} KiB  -> {hbm:9.1f} MiB")
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
