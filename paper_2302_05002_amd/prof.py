"""Summaries of rocprofv3 output for the benchmark's kernels.

    python3 -m paper_2302_05002_amd.prof stats   <kernel_stats.csv> <builds>
        per-kernel device time per build (from a --kernel-trace --stats run)
    python3 -m paper_2302_05002_amd.prof groups  <kernel_trace.csv> [chunk_passes]
        device time per build of every timed region (the groups bench.py
        reports), from the dispatch timestamps
    python3 -m paper_2302_05002_amd.prof traffic <fetch.csv> <write.csv> <workload> <out.json> [chunk_passes]
        FETCH_SIZE and WRITE_SIZE per build of every region, with the digest of
        the HIP sources they were taken on, merged into out.json
    python3 -m paper_2302_05002_amd.prof calibrate
        three plain device copies of 256 MiB, to be run under rocprofv3 --pmc
        (the counters' calibration: bytes moved per FETCH_SIZE / WRITE_SIZE unit)
    python3 -m paper_2302_05002_amd.prof calibration <fetch.csv> <write.csv>
        the factors from such a run

Every dispatch of a build is attributed to the region the library's timers
bracket (include/fpo.h, fpo_timer): preview, bbox, quantize, cut,
chunk_split, subsample, node_counts, node_place, node_sort.  The attribution
follows the launch order of a build with the hash or stride preview; builds
are delimited by the preview kernel, which every non-empty build launches
once.  Host-to-device and device-to-host copies (runtime blit kernels) belong
to no region.
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

REGIONS = ("preview", "bbox", "quantize", "cut", "chunk_split", "subsample", "node_counts", "node_place",
           "node_sort")


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


# kernels of the chunk split (its passes and scans); the first other kernel
# after it begins the subsample region
CHUNK_SPLIT_KERNELS = ("k_ms_count<false", "k_ms_scatter<false", "k_scan_", "k_u32_to_u64", "k_fill_u32")


def attribute(names, chunk_passes: int = 0):
    """Region of every dispatch in `names` (kernel names in dispatch order),
    or None for runtime copies.  Transitions follow a build's launch order:
    preview (counters' fill, preview kernels) -> bbox -> quantize (through
    k_qz_bin_grid in the binned form) -> cut
    (through k_wc_segs) -> chunk_split (its count, scan and scatter kernels, in
    one or two passes; with chunk_passes > 0, exactly that many scatters) ->
    subsample -> node_counts (k_np_pieces .. k_np_count) -> node_place ->
    node_sort (from the first k_np_sort)."""
    out = []
    state, prev, left = None, "", 0
    for i, k in enumerate(names):
        if "__amd_rocclr" in k:
            out.append(None)
            continue
        nxt = next((m for m in names[i + 1:] if "__amd_rocclr" not in m), "")
        if "k_preview_bits" in k or ("k_fill_u32" in k and "k_preview_bits" in nxt):
            state = "preview"
        elif state == "preview" and "k_bits_write" in prev:
            state = "bbox"
        elif "k_quantize" in k or "k_qz_bin" in k:
            state = "quantize"
        elif state == "quantize" and ("k_quantize" in prev or "k_qz_bin_grid" in prev):
            state = "cut"
        elif state == "cut" and "k_wc_segs" in prev:
            state, left = "chunk_split", chunk_passes
        elif state == "chunk_split" and (left == 0 if chunk_passes else
                                         not any(c in k for c in CHUNK_SPLIT_KERNELS)):
            state = "subsample"
        elif "k_np_pieces" in k:
            state = "node_counts"
        elif state == "node_counts" and "k_np_count" in prev:
            state = "node_place"
        elif "k_np_sort" in k and state != "node_sort":
            state = "node_sort"
        out.append(state)
        if state == "chunk_split" and "k_ms_scatter<false" in k:
            left -= 1
        prev = k
    return out


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


def _builds(names) -> int:
    return sum(1 for k in names if "k_preview_bits" in k)


def trace_groups(path: str, chunk_passes: int = 0):
    """(region -> (ms per build, kernels per build)), builds, from a kernel trace."""
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    names = [r["Kernel_Name"] for r in rows]
    regs = attribute(names, chunk_passes)
    nb = _builds(names)
    ms = defaultdict(float)
    cnt = defaultdict(int)
    for r, g in zip(rows, regs):
        if g is None:
            continue
        ms[g] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
        cnt[g] += 1
    return {g: (ms[g] / nb, cnt[g] / nb) for g in ms}, nb


def _dispatches(path: str, counter: str):
    """[(kernel, value)] in dispatch order, summed over the counter's instances."""
    acc = defaultdict(float)
    names = {}
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter:
            continue
        d = int(r["Dispatch_Id"])
        acc[d] += float(r["Counter_Value"])
        names[d] = r["Kernel_Name"]
    return [(names[d], acc[d]) for d in sorted(acc)]


def groups_per_build(path: str, counter: str, chunk_passes: int = 0):
    """Per build, the counter summed over each region (averaged over builds)."""
    seq = _dispatches(path, counter)
    names = [k for k, _ in seq]
    regs = attribute(names, chunk_passes)
    nb = _builds(names)
    sums = defaultdict(float)
    for (_, v), g in zip(seq, regs):
        if g is not None:
            sums[g] += v
    return {k: v / nb for k, v in sums.items()}, nb


def traffic(fetch_csv: str, write_csv: str, workload: str, out_json: str, chunk_passes: int = 0):
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


def calibrate():
    """Three device-to-device copies of 256 MiB (the copy kernel of the HIP runtime)."""
    import torch
    src = torch.empty(1 << 26, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print("copied 3 x 256 MiB", flush=True)


def calibration(fetch_csv: str, write_csv: str):
    """(read factor, write factor): bytes a 256 MiB copy moves each way per counter unit (KiB)."""
    out = []
    for path, counter in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        vals = [v for k, v in _dispatches(path, counter) if "copyBuffer" in k]
        if not vals:
            raise SystemExit(f"no copy kernel in {path}")
        per = sorted(vals)[len(vals) // 2]   # median copy, KiB
        out.append(256 * 1024 / per)
    return tuple(out)


def main(argv):
    if not argv:
        raise SystemExit(__doc__)
    if argv[0] == "calibrate":
        calibrate()
        return
    if argv[0] == "calibration":
        r, w = calibration(argv[1], argv[2])
        print(f"read factor {r:.3f}, write factor {w:.3f} (bytes = FETCH_SIZE KiB x {r:.3f} + WRITE_SIZE KiB x {w:.3f}, in KiB)")
        return
    if argv[0] == "stats":
        print(stats(argv[1], int(argv[2])))
    elif argv[0] == "groups":
        g, nb = trace_groups(argv[1], *[int(a) for a in argv[2:3]])
        print(f"{nb} builds; device time per build of every region:")
        print("| region | kernels/build | ms/build |")
        print("|---|---:|---:|")
        for k in REGIONS:
            if k in g:
                print(f"| {k} | {g[k][1]:g} | {g[k][0]:.4f} |")
        print(f"| **all regions** | {sum(v[1] for v in g.values()):g} | {sum(v[0] for v in g.values()):.4f} |")
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
