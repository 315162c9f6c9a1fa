#!/usr/bin/env python3
"""Benchmark of the octree build + preview on one MI355X.

A step is one whole build (all five steps of the path: bbox + quantise +
count, pyramid + chunk cut, stable scatter, node subsample, preview) of one
synthetic cloud whose coordinates are already resident in HBM.  Default
workload: 20,000,000 points on 200 random planes (count grid 128^3, chunks of
at most 1,000,000 points, subsample grid 128^3, leaf capacity 10,000, preview
modulus 64).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s

WORKLOADS = {
    # name: (generator, params attribute, description)
    "planes20m": ("config2", "CONFIG2", "20M points on 200 planes, G=128, C=1M, S=128, L=10k, M=64"),
    "uniform1m": ("config1", "CONFIG1", "1M uniform points, G=64, C=100k, S=32, L=10k, M=64"),
}


def algorithmic_bytes(n: int, G: int, M: int) -> int:
    """Bytes the path must move: bbox read 12/pt, quantise+count read 12/pt,
    scatter read 12 + write 4 /pt, subsample read perm 4 + gather 12 + write
    node_points 4 /pt, histogram written and read once (8 G^3), preview
    4 N/M."""
    return 60 * n + 8 * G ** 3 + 4 * n // M


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="planes20m", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="CPU work budget of the oracle baseline")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): this build has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2302_05002_amd as fpo
    import synth

    gen, pname, desc = WORKLOADS[args.workload]
    p = getattr(synth, pname)
    t = time.perf_counter()
    cloud = getattr(synth, gen)()
    print(f"[bench] generated {cloud.n} points in {time.perf_counter() - t:.1f}s", file=sys.stderr, flush=True)
    n = cloud.n
    dev = torch.device("cuda", 0)
    x = torch.from_numpy(cloud.x).to(dev)
    y = torch.from_numpy(cloud.y).to(dev)
    z = torch.from_numpy(cloud.z).to(dev)
    params = fpo.Params(p.count_grid, p.max_points_per_chunk, p.subsample_grid, p.leaf_capacity, p.preview_modulus)
    ctx = fpo.Context(0)
    ws = torch.empty(fpo.workspace_size(n, params), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step():
        job = ctx.submit(x, y, z, params, workspace=ws, stream=stream)
        job.wait()
        job.release()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1000.0 / args.steps
    value = n / (ms / 1000.0)
    b_alg = algorithmic_bytes(n, p.count_grid, p.preview_modulus)
    out = {
        "metric": "octree-build points/s (bit-exact) + %HBM peak; batched/served vs plain",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+u32",
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "count_grid": p.count_grid, "max_points_per_chunk": p.max_points_per_chunk,
                   "subsample_grid": p.subsample_grid, "leaf_capacity": p.leaf_capacity,
                   "preview_modulus": p.preview_modulus, "parallelism": "single GPU"},
        "path_hbm_frac": b_alg / (ms / 1000.0) / (HBM_PEAK_GBS * 1e9),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
