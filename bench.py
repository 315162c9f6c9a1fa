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
    """Bytes the whole path must move: bbox read 12/pt, quantise+count read
    12/pt, scatter read 12 + write 4 /pt, subsample read perm 4 + gather 12 +
    write node_points 4 /pt, histogram written and read once (8 G^3), preview
    4 N/M."""
    return 60 * n + 8 * G ** 3 + 4 * n // M


# Algorithmic bytes of each timed kernel per build, from the per-step figures
# above: (bytes(n, G, M), what they are).
KERNEL_BYTES = {
    "bbox": (lambda n, G, M: 12 * n, "read x, y, z once: 12 B/pt"),
    "quantize": (lambda n, G, M: 12 * n + 4 * G ** 3, "read x, y, z again: 12 B/pt; write the count grid: 4 B/cell"),
    "chunk_scatter": (lambda n, G, M: 16 * n, "re-read the points 12 B/pt, write perm 4 B/pt"),
    "subsample": (lambda n, G, M: 16 * n, "read perm 4 B/pt, gather the coordinates once 12 B/pt"),
    "node_counts": (None, "rows per (depth, work chunk), not per point"),
    "node_place": (lambda n, G, M: 9 * n, "read each point's depth 1 B and original index 4 B, write it 4 B"),
    "node_sort": (lambda n, G, M: 8 * n, "read and write every node's points once: 8 B/pt"),
}

KERNEL_NAMES = {
    "bbox": "fpo::k_bbox",
    "quantize": "fpo::k_quantize",
    "chunk_scatter": "fpo::k_ms_scatter<false, 8> (split into chunks)",
    "subsample": "fpo::k_subsample_* (all size classes)",
    "node_counts": "fpo::k_np_pieces + scan + fpo::k_np_shared + fpo::k_np_count",
    "node_place": "fpo::k_np_place",
    "node_sort": "fpo::k_np_sort (four tile sizes) + fpo::k_np_merge",
}


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per build of `kernel` from the committed FETCH_SIZE /
    WRITE_SIZE readings (profiles/traffic.json), scaled by the plain-copy
    calibration factors; None when there is no reading for this kernel and
    workload or the sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    from paper_2302_05002_amd.prof import source_digest
    e = t.get("kernels", {}).get(f"{workload}/{kernel}")
    if not e or e.get("source_digest") != source_digest():
        return None
    kib = e["fetch_kib"] * t["read_factor"] + e["write_kib"] * t["write_factor"]
    return kib * 1024.0


def cpu_baseline(cloud, p, seconds: float) -> dict:
    """The CPU oracle as it stands (single thread) on the same workload,
    repeated until `seconds` of work are done."""
    import oracle
    op = oracle.Params(p.count_grid, p.max_points_per_chunk, p.subsample_grid, p.leaf_capacity, p.preview_modulus)
    runs, t_total = 0, 0.0
    while runs == 0 or t_total < seconds:
        t = time.perf_counter()
        r = oracle.build_octree(cloud.x, cloud.y, cloud.z, op)
        t_total += time.perf_counter() - t
        assert r["status"] == oracle.OK
        runs += 1
    return {"value": runs * cloud.n / t_total, "unit": "points/s", "cores": 1, "kind": "oracle",
            "sample": f"the whole {cloud.n}-point workload, built {runs} times in {t_total:.1f} s "
                      f"(single-threaded C, host CPU)"}


def fpo_params_of(fpo, p):
    return fpo.Params(p.count_grid, p.max_points_per_chunk, p.subsample_grid, p.leaf_capacity, p.preview_modulus)


def to_device(torch, c):
    return tuple(torch.from_numpy(a).to("cuda") for a in (c.x, c.y, c.z))


def plain_loop(fpo, torch, ctx, items, ws):
    """Serial plain builds (submit, wait, release), one workspace reused."""
    for (x, y, z), p in items:
        job = ctx.submit(x, y, z, p, workspace=ws)
        job.wait()
        job.release()


def bench_batched(fpo, torch, ctx, rounds: int = 3) -> dict:
    """The batched workload at reduced scale: a pool of 32 clouds, sizes
    log-uniform in [10k, 4M], kinds uniform / planes (5-200) / clusters
    (10-500), per-size parameters; the batch is the pool repeated `rounds`
    times.  One fpo_build_batch call against the serial loop of plain builds
    over the same clouds."""
    import synth
    mix = synth.batch_mix(32, seed=4)
    pool = [(to_device(torch, c), fpo_params_of(fpo, p)) for c, p in mix]
    items = pool * rounds
    points = sum(int(x.shape[0]) for (x, _, _), _ in items)
    ws = torch.empty(max(fpo.workspace_size(int(x.shape[0]), p) for (x, _, _), p in pool), dtype=torch.uint8,
                     device="cuda")
    plain_loop(fpo, torch, ctx, pool, ws)   # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    plain_loop(fpo, torch, ctx, items, ws)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t
    del ws
    clouds = [c for c, _ in items]
    params = [p for _, p in items]
    jobs = ctx.build_batch(clouds, params)   # warm-up (also sizes the workspace)
    bws = jobs[0].workspace
    for j in jobs:
        j.wait()
        j.release()
    torch.cuda.synchronize()
    t = time.perf_counter()
    jobs = ctx.build_batch(clouds, params, workspace=bws)
    for j in jobs:
        j.wait()
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t
    for j in jobs:
        j.release()
    return {"workload": f"{len(items)} builds: a pool of 32 clouds (10k-4M points, log-uniform; uniform, planes, "
                        f"clusters) repeated {rounds} times", "points": points,
            "plain_points_per_s": points / t_plain, "batched_points_per_s": points / t_batch,
            "speedup": t_plain / t_batch}


def bench_served(fpo, torch, ctx, num_requests: int = 64, load: float = 1.25, slots: int = 4) -> dict:
    """The served workload at reduced scale: requests drawn from a pool of 12
    clouds (100k-8M points, log-uniform, mixed kinds), Poisson arrivals at
    `load` times the measured capacity of the serial plain loop.  Latency =
    completion - arrival; throughput = points / makespan."""
    import numpy as np
    import synth
    mix = synth.batch_mix(12, seed=5, lo=100_000, hi=8_000_000)
    pool = [(to_device(torch, c), fpo_params_of(fpo, p)) for c, p in mix]
    rng = np.random.default_rng(5)
    reqs = [pool[int(k)] for k in rng.integers(0, len(pool), num_requests)]
    points = sum(int(x.shape[0]) for (x, _, _), _ in reqs)
    need = [fpo.workspace_size(int(x.shape[0]), p) for (x, _, _), p in reqs]
    ws = torch.empty(max(need), dtype=torch.uint8, device="cuda")
    plain_loop(fpo, torch, ctx, pool, ws)   # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    plain_loop(fpo, torch, ctx, reqs, ws)
    torch.cuda.synchronize()
    t_serial = time.perf_counter() - t
    del ws
    serial_pps = points / t_serial
    rate = load * serial_pps / (points / num_requests)   # requests per second
    gaps = rng.exponential(1.0 / rate, num_requests)
    budget = int(min(64 << 30, 8 * sum(sorted(need)[-slots:])))
    srv = fpo.Server(ctx, budget, slots)
    for (x, y, z), p in pool[:slots]:            # warm-up of the slot streams
        j = srv.submit(x, y, z, p)
        j.wait()
        j.release()
    # a client thread collects the results in arrival order and releases them
    # at once (a request holds its share of the budget until then), while
    # this thread submits on the arrival schedule
    import queue
    import threading
    pending = queue.Queue()
    lat = []
    span = [None, None]

    def collect():
        for _ in range(num_requests):
            j = pending.get()
            j.wait()
            sub, _, done = j.timestamps()
            j.release()
            lat.append((done - sub) / 1e6)
            span[0] = sub if span[0] is None else min(span[0], sub)
            span[1] = done if span[1] is None else max(span[1], done)

    client = threading.Thread(target=collect)
    client.start()
    due = time.monotonic()
    for ((x, y, z), p), g in zip(reqs, gaps):
        due += g
        rest = due - time.monotonic()
        if rest > 1e-3:
            time.sleep(rest - 5e-4)   # (sleeping lets the client thread run)
        while time.monotonic() < due:
            pass
        pending.put(srv.submit(x, y, z, p))
    client.join()
    first, last = span
    srv.close()
    lat = np.array(lat)
    return {"workload": f"{num_requests} requests from a pool of 12 clouds (100k-8M points, log-uniform; uniform, "
                        f"planes, clusters), Poisson arrivals at {load}x the serial capacity, {slots} slots",
            "points": points, "serial_points_per_s": serial_pps, "served_points_per_s": points / ((last - first) / 1e9),
            "speedup": points / ((last - first) / 1e9) / serial_pps,
            "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99))}


def bench_streamed(fpo, torch, ctx, steps: int = 3) -> dict:
    """The out-of-core workload: 200M points of terrain plus clusters in
    pinned host memory, copied to the device in 16M-point batches with the
    exact box given as a header (G=512, C=2M, S=128, L=10k, M=64).  Bound by
    the host link: reported against a plain pinned copy of the same bytes.
    Also the time until the preview is ready (it depends only on n)."""
    import synth
    c = synth.config3()
    p = synth.CONFIG3
    box = ((float(c.x.min()), float(c.y.min()), float(c.z.min())),
           (float(c.x.max()), float(c.y.max()), float(c.z.max())))
    params = fpo.Params(p.count_grid, p.max_points_per_chunk, p.subsample_grid, p.leaf_capacity, p.preview_modulus,
                        box)
    host = [torch.from_numpy(a).pin_memory() for a in (c.x, c.y, c.z)]
    del c
    n = int(host[0].shape[0])
    dev = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(3)]
    for d, h in zip(dev, host):   # warm-up
        d.copy_(h, non_blocking=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for d, h in zip(dev, host):
        d.copy_(h, non_blocking=True)
    torch.cuda.synchronize()
    link = 12 * n / (time.perf_counter() - t)
    del dev
    torch.cuda.empty_cache()
    job = ctx.submit(*host, params, stream_batch=16_000_000)   # warm-up, sizes the workspace
    job.wait()
    ws = job.workspace
    job.release()
    times, previews = [], []
    for _ in range(steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        job = ctx.submit(*host, params, workspace=ws, stream_batch=16_000_000)
        while not job.preview_ready():
            pass
        previews.append(time.perf_counter() - t)
        job.wait()
        times.append(time.perf_counter() - t)
        job.release()
    t_build = sorted(times)[len(times) // 2]
    return {"workload": "200M points (terrain + 5000 clusters) in pinned host memory, 16M-point batches, box given; "
                        "G=512, C=2M, S=128, L=10k, M=64",
            "points_per_s": n / t_build, "ms_per_build": 1000 * t_build,
            "h2d_GBps": link / 1e9, "link_frac": (12 * n / link) / t_build,
            "preview_ready_ms": 1000 * sorted(previews)[len(previews) // 2]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="planes20m", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="CPU work budget of the oracle baseline")
    ap.add_argument("--no-mix", action="store_true", help="skip the batched and served comparisons")
    ap.add_argument("--no-stream", action="store_true", help="skip the streamed 200M-point build")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the LAS decode, preview variant, gather and node selection legs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the library builds on one GPU (no multi-GPU path); "
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

    for _ in range(args.warmup):
        job = ctx.submit(x, y, z, params, workspace=ws, stream=stream)
        job.wait()
        job.release()

    def bench_gather(reps: int = 10) -> dict:
        """Node-ordered points of one build (the export step after the tree):
        read the index 4 B, gather the coordinates 12 B, write 12 B per point."""
        job = ctx.submit(x, y, z, params, workspace=ws, stream=stream)
        job.wait()
        job.gather(x, y, z)   # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            job.gather(x, y, z)
        torch.cuda.synchronize()
        ms_g = (time.perf_counter() - t) * 1000.0 / reps
        job.release()
        gbs = 28 * n / (ms_g / 1000.0) / 1e9
        return {"what": "xyz of every point gathered into node order (28 B/pt)", "ms": ms_g, "GBps": gbs,
                "hbm_frac": gbs / HBM_PEAK_GBS}

    def bench_preview_variants(reps: int = 5) -> dict:
        """The three previews on the same workload: device time of the preview
        kernels per build (timer 'preview'), of the quantise pass (which keeps
        the per-cell hash minima for the grid preview) and of the whole build.
        Algorithmic bytes of the preview kernels: hash and stride write 4 B per
        pick (index-only predicates); grid reads the per-cell minima (8 B/cell)
        and writes 4 B per pick."""
        res = {}
        ctx.set_timing(True)
        for mode in ("hash", "stride", "grid"):
            pm = fpo.Params(p.count_grid, p.max_points_per_chunk, p.subsample_grid, p.leaf_capacity,
                            p.preview_modulus, None, mode)
            wsm = torch.empty(fpo.workspace_size(n, pm), dtype=torch.uint8, device=dev)
            tot = pv = qz = 0.0
            picks = 0
            for r in range(reps + 1):
                torch.cuda.synchronize()
                t = time.perf_counter()
                job = ctx.submit(x, y, z, pm, workspace=wsm, stream=stream)
                job.wait()
                el = (time.perf_counter() - t) * 1000.0
                if r:
                    tot += el
                    pv += job.timer("preview")[0]
                    qz += job.timer("quantize")[0]
                picks = int(job.result().preview_count)
                job.release()
            del wsm
            pv /= reps
            alg = 4 * picks + (8 * p.count_grid ** 3 if mode == "grid" else 0)
            res[mode] = {"preview_ms": pv, "quantize_ms": qz / reps, "build_ms": tot / reps, "picks": picks,
                         "GBps": alg / (pv / 1000.0) / 1e9, "hbm_frac": alg / (pv / 1000.0) / 1e9 / HBM_PEAK_GBS}
        ctx.set_timing(False)
        return res

    def bench_las_decode(reps: int = 10) -> dict:
        """The same points as LAS 1.2 point format 3 records (34 B: X, Y, Z int32,
        attributes, GPS time, R, G, B), decoded to float32 x, y, z and uint16
        R, G, B on the device.  Algorithmic bytes: read 34 B, write 12 + 6 B
        per point.  Timed with events on the stream the decode runs on."""
        from synth.las import write_las
        t = time.perf_counter()
        f = write_las(cloud.x + 330_000.0, cloud.y + 4_200_000.0, cloud.z, scale=(1e-4, 1e-4, 1e-4),
                      offset=(330_000.0, 4_200_000.0, 0.0), point_format=3)
        h = fpo.las_parse_header(f)
        recs = torch.frombuffer(bytearray(f[h.offset_to_points:]), dtype=torch.uint8).to(dev)
        del f
        print(f"[bench] LAS records ready in {time.perf_counter() - t:.1f}s", file=sys.stderr, flush=True)
        origin = (330_000.0, 4_200_000.0, 0.0)
        ctx.las_decode(recs, h, origin, rgb=True, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            out = ctx.las_decode(recs, h, origin, rgb=True, stream=stream)
        e1.record(stream)
        e1.synchronize()
        ms_d = e0.elapsed_time(e1) / reps
        del out, recs
        b = (34 + 12 + 6) * n
        return {"what": "LAS point format 3 records (34 B) to float32 xyz + uint16 rgb", "ms": ms_d,
                "points_per_s": n / (ms_d / 1000.0), "GBps": b / (ms_d / 1000.0) / 1e9,
                "hbm_frac": b / (ms_d / 1000.0) / 1e9 / HBM_PEAK_GBS}

    def bench_copy(reps: int = 20) -> dict:
        """A plain device-to-device copy of 1 GiB (read + write), the practical
        HBM ceiling the kernels are compared against."""
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            dst.copy_(src)
        e1.record()
        e1.synchronize()
        ms_c = e0.elapsed_time(e1) / reps
        del src, dst
        gbs = 2 * (1 << 30) / (ms_c / 1000.0) / 1e9
        return {"what": "torch copy of 1 GiB on the device (2 GiB moved)", "ms": ms_c, "GBps": gbs,
                "frac_of_peak": gbs / HBM_PEAK_GBS}

    def bench_atomics(reps: int = 5) -> dict:
        """Device atomic throughput, the secondary ceiling of the histogram and
        winner passes: int32 scatter-add (global atomics) of 64M updates into
        a 1M-entry table, uniform random and sorted (neighbouring lanes on
        neighbouring words) targets."""
        m = 1 << 26
        g = torch.Generator(device=dev)
        g.manual_seed(9)
        idx = torch.randint(0, 1 << 20, (m,), device=dev, generator=g)
        one = torch.ones(m, dtype=torch.int32, device=dev)
        res = {}
        for name, ix in (("random", idx), ("sorted", torch.sort(idx).values)):
            tab = torch.zeros(1 << 20, dtype=torch.int32, device=dev)
            tab.scatter_add_(0, ix, one)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                tab.scatter_add_(0, ix, one)
            e1.record()
            e1.synchronize()
            res[name + "_per_s"] = m * reps / (e0.elapsed_time(e1) / 1000.0)
        del idx, one
        res["what"] = "torch scatter_add_ of 64M int32 updates into 1M counters (global atomics)"
        return res

    extras = {}
    if not args.no_extras:
        extras["hbm_copy"] = bench_copy()
        extras["atomics"] = bench_atomics()
        extras["las_decode"] = las_stats = bench_las_decode()
        print(f"[bench] LAS decode {las_stats['ms']:.3f} ms, {las_stats['hbm_frac']:.2f} of HBM peak",
              file=sys.stderr, flush=True)
        extras["preview_variants"] = preview_stats = bench_preview_variants()
        print(f"[bench] preview variants: " + ", ".join(f"{k} {v['preview_ms']:.3f} ms ({v['picks']} picks)"
                                                        for k, v in preview_stats.items()),
              file=sys.stderr, flush=True)
        extras["node_ordered_points"] = bench_gather()

    def bench_select(reps: int = 20) -> dict:
        """Node selection for one perspective view of the built tree (eye outside
        the cloud, 60 degree field of view, 1080-pixel viewport, nodes refined
        above 100 pixels): time per view from the host (launches, compaction
        and the read-back of the two totals)."""
        job = ctx.submit(x, y, z, params, workspace=ws, stream=stream)
        job.wait()
        res = job.result()
        lo = [float(v) for v in res.bbox_min]
        side = float(res.cube_size)
        eye = (lo[0] - 0.5 * side, lo[1] - 0.5 * side, lo[2] + 1.5 * side)
        tgt = tuple(lo[a] + 0.5 * side for a in range(3))
        f = [tgt[a] - eye[a] for a in range(3)]
        fl = sum(v * v for v in f) ** 0.5
        f = [v / fl for v in f]
        up = (0.0, 0.0, 1.0)
        r = [f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2], f[0] * up[1] - f[1] * up[0]]
        rl = sum(v * v for v in r) ** 0.5
        r = [v / rl for v in r]
        u = [r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]]
        th = 0.5773502691896257   # tan(30 degrees)
        tw = th * 16 / 9
        planes = []
        for nrm, pt in (([tw * f[a] + r[a] for a in range(3)], eye), ([tw * f[a] - r[a] for a in range(3)], eye),
                        ([th * f[a] + u[a] for a in range(3)], eye), ([th * f[a] - u[a] for a in range(3)], eye),
                        (f, eye), ([-v for v in f], [eye[a] + 10 * side * f[a] for a in range(3)])):
            planes.append((*nrm, -sum(nrm[a] * pt[a] for a in range(3))))
        view = fpo.make_view(eye, planes, 1080.0 / (2 * th), 100.0)
        sel = ctx.select_nodes(res.node_depth, res.node_key, res.node_count, res.bbox_min, res.cube_size, view)
        t = time.perf_counter()
        for _ in range(reps):
            sel = ctx.select_nodes(res.node_depth, res.node_key, res.node_count, res.bbox_min, res.cube_size, view)
        ms_s = (time.perf_counter() - t) * 1000.0 / reps
        out = {"what": "drawn nodes of one perspective view (frustum + 100-pixel refinement)", "ms": ms_s,
               "nodes": res.num_nodes, "drawn_nodes": int(sel[0].shape[0]), "drawn_points": int(sel[1])}
        job.release()
        return out

    if not args.no_extras:
        extras["node_selection"] = bench_select()
    def timed_builds(k: int, only=None):
        """k builds submitted back to back (same stream and workspace, so they
        run one after another on the device) and waited for together: the host
        work of a build (its two read-backs and launches) overlaps the end of
        the one before, as for any caller with more than one cloud to build.
        Returns (seconds, {timer: [ms summed over the builds, launches]})."""
        ctx.set_timing(True, only)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        jobs = [ctx.submit(x, y, z, params, workspace=ws, stream=stream) for _ in range(k)]
        for job in jobs:
            job.wait()
        torch.cuda.synchronize()
        tb = time.perf_counter()
        acc = {name: [0.0, 0] for name in KERNEL_BYTES}
        for job in jobs:
            for name in KERNEL_BYTES:
                ms_k, nl = job.timer(name)
                acc[name][0] += ms_k
                acc[name][1] += nl
            job.release()
        ctx.set_timing(False)
        return tb - ta, acc

    # kernel timers (HIP events on the build's stream): every group on a few
    # builds to find the dominant one and the split, then the timed region
    # with events around the dominant group only (fewer events, less
    # perturbation), its duration measured live there
    split_builds = max(2, min(args.steps, 5))
    _, split = timed_builds(split_builds)
    dom = max(split, key=lambda k: split[k][0])
    secs, timers = timed_builds(args.steps, [dom])
    ms = secs * 1000.0 / args.steps
    value = n / (ms / 1000.0)
    b_alg = algorithmic_bytes(n, p.count_grid, p.preview_modulus)

    # dominant kernel: the most device time per build (from the split builds)
    dom_ms = timers[dom][0] / args.steps
    dom_launches = timers[dom][1] / args.steps
    fn = KERNEL_BYTES[dom][0]
    dom_bytes = fn(n, p.count_grid, p.preview_modulus) if fn else None
    achieved = dom_bytes / (dom_ms / 1000.0) / 1e9 if dom_bytes else None
    traffic = measured_traffic(dom, args.workload)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": traffic,
                "kernel": KERNEL_NAMES[dom], "algorithmic_bytes": dom_bytes, "bytes_rule": KERNEL_BYTES[dom][1],
                "ms_per_build": dom_ms, "launches_per_build": dom_launches,
                "kernels_ms_per_build": {k: v[0] / split_builds for k, v in split.items()},
                "split_builds": split_builds}

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
        "roofline": roofline,
        **extras,
    }
    if not args.no_mix:
        del ws
        torch.cuda.empty_cache()
        out["batched"] = bench_batched(fpo, torch, ctx)
        print(f"[bench] batched {out['batched']['speedup']:.2f}x the plain loop", file=sys.stderr, flush=True)
        out["served"] = bench_served(fpo, torch, ctx)
        print(f"[bench] served {out['served']['speedup']:.2f}x serial, p99 {out['served']['latency_ms_p99']:.1f} ms",
              file=sys.stderr, flush=True)
        # the same trace at half the serial capacity: latency without queueing
        out["served_half_load"] = bench_served(fpo, torch, ctx, load=0.5)
        print(f"[bench] served at 0.5x load: p50 {out['served_half_load']['latency_ms_p50']:.1f} ms, "
              f"p99 {out['served_half_load']['latency_ms_p99']:.1f} ms", file=sys.stderr, flush=True)
    if not args.no_stream:
        if not args.no_mix:
            torch.cuda.empty_cache()
        out["streamed"] = bench_streamed(fpo, torch, ctx)
        print(f"[bench] streamed {out['streamed']['points_per_s'] / 1e9:.2f} G points/s, "
              f"{out['streamed']['link_frac']:.2f} of the host link", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cloud, p, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
