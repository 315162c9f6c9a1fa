#!/usr/bin/env python3
"""Benchmark of the octree build + preview on one MI355X.

A step is one whole build (all five steps of the path: bbox + quantise +
count, pyramid + chunk cut, stable scatter, node subsample, preview) of one
synthetic cloud whose coordinates are already resident in HBM.  Default
workload: 20,000,000 points on 200 random planes (count grid 128^3, chunks of
at most 1,000,000 points, subsample grid 128^3, leaf capacity 10,000, preview
modulus 64).  The same line reports the plain 1M-point build, the 256-cloud
batch against the plain loop, the 2,000-request served trace against serial
plain builds, the streamed 200M-point build, and the CPU oracle on the host's
cores.  Prints one JSON line.
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
    "planes20m": ("planes_20m", "PLANES_20M", "20M points on 200 planes, G=128, C=1M, S=128, L=10k, M=64"),
    "uniform1m": ("uniform_1m", "UNIFORM_1M", "1M uniform points, G=64, C=100k, S=32, L=10k, M=64"),
    # the out-of-core workload built from device memory (profiling of the G = 512 path)
    "terrain200m": ("terrain_200m", "TERRAIN_200M", "200M points of terrain and clusters in device memory, G=512, C=2M, S=128, "
                                          "L=10k, M=64"),
}


def algorithmic_bytes(n: int, G: int, M: int, given: bool = False) -> int:
    """Bytes the whole path must move: bbox read 12/pt (none with a given
    box), quantise+count read 12/pt, scatter read 12 + write 4 /pt, subsample
    read perm 4 + gather 12 + write node_points 4 /pt, histogram written and
    read once (8 G^3), preview 4 per kept index (about n/M)."""
    return (48 if given else 60) * n + 8 * G ** 3 + 4 * -(-n // M)


# The path's steps as groups of the library's timed regions (fpo_timer), each
# with its share of the algorithmic bytes above, so that the groups add up to
# the whole path: (regions, bytes(n, G, M, given), what the bytes are).
GROUPS = {
    "a1 bbox": (("bbox",), lambda n, G, M, gv: 0 if gv else 12 * n, "read x, y, z once: 12 B/pt"),
    "a1 quantize + count": (("quantize",), lambda n, G, M, gv: 12 * n + 4 * G ** 3,
                            "read x, y, z again 12 B/pt; write the count grid 4 B/cell"),
    "a2 pyramid + chunk cut": (("cut",), lambda n, G, M, gv: 4 * G ** 3, "read the count grid once: 4 B/cell"),
    "a3 stable scatter": (("chunk_split",), lambda n, G, M, gv: 16 * n,
                          "re-read the points 12 B/pt; write perm 4 B/pt"),
    "a4 node subsample": (("subsample",), lambda n, G, M, gv: 16 * n,
                          "read perm 4 B/pt; gather the coordinates once 12 B/pt"),
    "a4 node_points": (("node_counts", "node_place", "node_sort"), lambda n, G, M, gv: 4 * n,
                       "write node_points once: 4 B/pt"),
    "a5 preview": (("preview",), lambda n, G, M, gv: 4 * -(-n // M), "write every kept index: 4 B each"),
}

GROUP_KERNELS = {
    "a1 bbox": "fpo::k_fill_u32 (count grid), fpo::k_bbox, fpo::k_setup",
    "a1 quantize + count": "fpo::k_quantize<false>",
    "a2 pyramid + chunk cut": "fpo::k_pyr_*, k_grid_export, k_cut_flags, scans, k_cut_table, k_cell_ids, k_wc_chunks*",
    "a3 stable scatter": "chunk begins (scans, k_u32_to_u64), fpo::k_ms_count<false, 8>, scan, fpo::k_ms_scatter<false, 8>",
    "a4 node subsample": "work-chunk split (fpo::k_ms_*<true, 12>), fpo::k_gdepth_*, fpo::k_wc_alive_rows, "
                         "fpo::k_list_classes, fpo::k_subsample_*, fpo::k_decide, fpo::k_node_counts, scans",
    "a4 node_points": "fpo::k_np_pieces/k_np_shared/k_np_count, fpo::k_node_fill, fpo::k_np_lists, fpo::k_np_place, "
                      "fpo::k_np_sort, fpo::k_np_merge",
    "a5 preview": "fpo::k_preview_bits, fpo::k_bits_count, scan, fpo::k_bits_write",
}


def measured_traffic(group: str, workload: str):
    """HBM bytes per build of a group from the committed FETCH_SIZE /
    WRITE_SIZE readings of its regions (profiles/traffic.json), scaled by the
    plain-copy calibration factors; None when a region has no reading for
    this workload or the sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    from paper_2302_05002_amd.prof import source_digest
    dig = source_digest()
    total = 0.0
    for reg in GROUPS[group][0]:
        e = t.get("kernels", {}).get(f"{workload}/{reg}")
        if not e or e.get("source_digest") != dig:
            return None
        total += e["fetch_kib"] * t["read_factor"] + e["write_kib"] * t["write_factor"]
    return total * 1024.0


def host_cpu() -> dict:
    """The host's CPU model and the cores this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": len(os.sched_getaffinity(0)), "os_cpu_count": os.cpu_count()}


def _oracle_worker(args):
    """One all-cores worker: builds its own copy of the workload `builds`
    times with the oracle; returns (points built, seconds)."""
    gen, pname, builds, barrier_at = args
    import synth
    import oracle
    c = getattr(synth, gen)()
    p = getattr(synth, pname)
    op = oracle.Params(p.count_grid, p.max_points_per_chunk, p.subsample_grid, p.leaf_capacity, p.preview_modulus)
    while time.time() < barrier_at:   # start together
        time.sleep(0.001)
    t = time.perf_counter()
    for _ in range(builds):
        r = oracle.build_octree(c.x, c.y, c.z, op)
        assert r["status"] == oracle.OK
    return c.n * builds, time.perf_counter() - t


def cpu_baseline(cloud, p, seconds: float, gen: str, pname: str) -> dict:
    """The CPU oracle as it stands on the same workload: one thread, repeated
    until `seconds` of work are done; then all cores, as independent
    single-threaded oracle processes (one per core this process may use, at
    most 16), each building its own copy of the workload twice.  The oracle
    itself is unchanged: all-cores is throughput over concurrent builds."""
    import oracle
    op = oracle.Params(p.count_grid, p.max_points_per_chunk, p.subsample_grid, p.leaf_capacity, p.preview_modulus)
    runs, t_total = 0, 0.0
    while runs == 0 or t_total < seconds:
        t = time.perf_counter()
        r = oracle.build_octree(cloud.x, cloud.y, cloud.z, op)
        t_total += time.perf_counter() - t
        assert r["status"] == oracle.OK
        runs += 1
    single = runs * cloud.n / t_total
    cpu = host_cpu()
    procs = max(1, min(16, cpu["nproc"]))
    import multiprocessing as mp
    builds = 2
    with mp.get_context("spawn").Pool(procs) as pool:
        start = time.time() + 4.0 + 0.05 * procs   # time for every worker to generate its copy
        res = pool.map(_oracle_worker, [(gen, pname, builds, start)] * procs)
    pts = sum(a for a, _ in res)
    wall = max(b for _, b in res)
    return {"value": pts / wall, "unit": "points/s", "cores": procs, "kind": "oracle",
            "sample": f"{procs} concurrent single-threaded oracle builds of the whole {cloud.n}-point workload, "
                      f"{builds} each ({procs * builds} builds in {wall:.1f} s of wall time)",
            "cpu": cpu,
            "single_thread": {"value": single, "unit": "points/s", "cores": 1,
                              "sample": f"the whole workload built {runs} times in {t_total:.1f} s"}}


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


def tune_classes(fpo, ctx, items, reps: int = 2) -> dict:
    """The quantise shape of every (size class, count grid) in `items`
    ([((x, y, z), Params)]), tuned on the first cloud of each."""
    seen = {}
    for (x, y, z), p in items:
        n = int(x.shape[0])
        key = (n.bit_length() - 1, p.count_grid)
        if key in seen or n < 1:
            continue
        t = ctx.autotune(x, y, z, p, reps=reps)
        seen[key] = t["quantize_variant"]
    return {f"2^{k}:G{g}": v for (k, g), v in sorted(seen.items())}


def bench_batched(fpo, torch, ctx) -> dict:
    """The batched workload: 256 clouds, sizes log-uniform in [10k, 4M],
    kinds uniform / planes (5-200) / clusters (10-500), per-size parameters
    (about 150M points).  One fpo_build_batch call against the serial loop of
    plain builds (submit, wait, release) over the same clouds."""
    import synth
    t = time.perf_counter()
    mix = synth.batch_mix(256, seed=4)
    items = [(to_device(torch, c), fpo_params_of(fpo, p)) for c, p in mix]
    del mix
    print(f"[bench] batched workload ready in {time.perf_counter() - t:.1f}s", file=sys.stderr, flush=True)
    points = sum(int(x.shape[0]) for (x, _, _), _ in items)
    t = time.perf_counter()
    tuned = tune_classes(fpo, ctx, items)
    print(f"[bench] tuned {len(tuned)} size classes in {time.perf_counter() - t:.1f}s", file=sys.stderr, flush=True)
    ws = torch.empty(max(fpo.workspace_size(int(x.shape[0]), p) for (x, _, _), p in items), dtype=torch.uint8,
                     device="cuda")
    plain_loop(fpo, torch, ctx, items, ws)   # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    plain_loop(fpo, torch, ctx, items, ws)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t
    del ws
    torch.cuda.empty_cache()
    clouds = [c for c, _ in items]
    params = [p for _, p in items]
    jobs = ctx.build_batch(clouds, params)   # warm-up (also sizes the workspace)
    bws = jobs[0].workspace
    for j in jobs:
        j.wait()
        j.release()
    workers = ctx.autotune_batch(clouds, params, workspace=bws, reps=2)
    torch.cuda.synchronize()
    reps = 3
    t_batch = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        jobs = ctx.build_batch(clouds, params, workspace=bws)
        for j in jobs:
            j.wait()
        torch.cuda.synchronize()
        t_batch.append(time.perf_counter() - t)
        for j in jobs:
            j.release()
    tb = sorted(t_batch)[reps // 2]
    return {"workload": "256 clouds (10k-4M points, log-uniform; uniform, planes, clusters; per-size G, C, S)",
            "clouds": len(items), "points": points, "batch_workspace_bytes": int(bws.numel()),
            "plain_points_per_s": points / t_plain, "batched_points_per_s": points / tb,
            "plain_ms": 1000 * t_plain, "batched_ms": 1000 * tb, "speedup": t_plain / tb,
            "autotuned": {"quantize_shape_by_class": tuned, "batch_workers": workers["workers"],
                          "batch_ms_by_workers": workers["batch_ms"]}}


class ServedTrace:
    """The served workload, generated once: 2,000 requests with sizes
    log-uniform in [100k, 50M] (about 16G points), each the first n points of
    one of three 50M-point pool clouds (uniform, planes, clusters) resident on
    the device, per-size parameters."""

    def __init__(self, fpo, torch):
        import synth
        t = time.perf_counter()
        pool, self.reqs = synth.serve_trace(2000, seed=5)
        self.dev = [to_device(torch, c) for c in pool]
        del pool
        self.params = [fpo_params_of(fpo, synth.params_for_size(r.n)) for r in self.reqs]
        self.points = sum(r.n for r in self.reqs)
        self.need = [fpo.workspace_size(r.n, p) for r, p in zip(self.reqs, self.params)]
        print(f"[bench] served trace ready in {time.perf_counter() - t:.1f}s ({self.points} points)",
              file=sys.stderr, flush=True)

    def cloud(self, i):
        r = self.reqs[i]
        return tuple(a[:r.n] for a in self.dev[r.kind])

    def serial(self, fpo, torch, ctx) -> float:
        """Points/s of the serial plain loop over the whole trace (one
        workspace, sized for the largest request)."""
        ws = torch.empty(max(self.need), dtype=torch.uint8, device="cuda")
        items = [(self.cloud(i), p) for i, p in enumerate(self.params)]
        plain_loop(fpo, torch, ctx, items[:50], ws)   # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        plain_loop(fpo, torch, ctx, items, ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        del ws
        torch.cuda.empty_cache()
        return self.points / dt


def bench_served(fpo, torch, ctx, trace: ServedTrace, serial_pps: float, load, slots: int = 4,
                 budget: int = 200 * 10 ** 9) -> dict:
    """Requests submitted on their Poisson schedule, rescaled so that the
    offered load is `load` times the serial plain loop's capacity (None: all
    at once, the server's capacity), into a
    server with `slots` slots and an HBM budget of `budget` bytes.  A client
    thread collects results in arrival order and releases each at once (a
    request holds its share of the budget until then).  Latency = completion
    - arrival; throughput = points / makespan."""
    import numpy as np
    import queue
    import threading
    reqs = trace.reqs
    num = len(reqs)
    if load is None:
        scale = 0.0
    else:
        rate = load * serial_pps / (trace.points / num)   # requests per second
        mean_gap = reqs[-1].arrival / max(num - 1, 1)
        scale = (1.0 / rate) / mean_gap
    srv = fpo.Server(ctx, budget, slots)
    for i in range(slots):   # warm-up of the slot streams
        j = srv.submit(*trace.cloud(i), trace.params[i])
        j.wait()
        j.release()
    pending = queue.Queue()
    lat = []
    span = [None, None]

    def collect():
        for _ in range(num):
            j = pending.get()
            j.wait()
            sub, _, done = j.timestamps()
            j.release()
            lat.append((done - sub) / 1e6)
            span[0] = sub if span[0] is None else min(span[0], sub)
            span[1] = done if span[1] is None else max(span[1], done)

    client = threading.Thread(target=collect)
    client.start()
    t0 = time.monotonic()
    for i, r in enumerate(reqs):
        due = t0 + r.arrival * scale
        rest = due - time.monotonic()
        if rest > 1e-3:
            time.sleep(rest - 5e-4)   # (sleeping lets the client thread run)
        while time.monotonic() < due:
            pass
        pending.put(srv.submit(*trace.cloud(i), trace.params[i]))
    client.join()
    srv.close()
    first, last = span
    lat = np.array(lat)
    served = trace.points / ((last - first) / 1e9)
    arrivals = "all submitted at once" if load is None else f"Poisson arrivals at {load}x the serial capacity"
    return {"workload": f"{num} requests (100k-50M points, log-uniform; uniform, planes, clusters), {arrivals}, "
                        f"{slots} slots, {budget / 1e9:.0f} GB budget",
            "requests": num, "points": trace.points, "serial_points_per_s": serial_pps,
            "served_points_per_s": served, "speedup": served / serial_pps,
            "makespan_s": (last - first) / 1e9,
            "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99))}


def bench_streamed(fpo, torch, ctx, steps: int = 3) -> dict:
    """The out-of-core workload: 200M points of terrain plus clusters in
    pinned host memory, copied to the device in 16M-point batches with the
    exact box given as a header (G=512, C=2M, S=128, L=10k, M=64).  Bound by
    the host link: reported against a plain pinned copy of the same bytes.
    Also the time until the preview is ready (it depends only on n)."""
    import synth
    c = synth.terrain_200m()
    p = synth.TERRAIN_200M
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


def measure(fpo, torch, ctx, xyz, params, ws, stream, steps: int, workload: str, p, given: bool = False) -> dict:
    """Timed plain builds of one workload.

    A few builds with every region timed give the split per group and the
    dominant group (most device time per build).  Then `steps` builds are
    submitted back to back on one stream and workspace and waited for
    together (a build's host round trips overlap the device work of the one
    before), with HIP events around the dominant group's regions only, so
    its duration is measured live over the timed region."""
    x, y, z = xyz
    n = int(x.shape[0])
    G, M = p.count_grid, p.preview_modulus

    def timed_builds(k: int, only):
        ctx.set_timing(True, only)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        jobs = [ctx.submit(x, y, z, params, workspace=ws, stream=stream) for _ in range(k)]
        for job in jobs:
            job.wait()
        torch.cuda.synchronize()
        tb = time.perf_counter()
        acc = {name: [0.0, 0] for name in fpo.TIMERS}
        for job in jobs:
            for name in only:
                ms_k, nl = job.timer(name)
                acc[name][0] += ms_k
                acc[name][1] += nl
            job.release()
        ctx.set_timing(False)
        return tb - ta, acc

    split_builds = max(2, min(steps, 5))
    _, split = timed_builds(split_builds, list(fpo.TIMERS))
    group_ms = {g: sum(split[r][0] for r in regs) / split_builds for g, (regs, _, _) in GROUPS.items()}
    dom = max(group_ms, key=group_ms.get)
    secs, timers = timed_builds(steps, list(GROUPS[dom][0]))
    ms = secs * 1000.0 / steps
    b_alg = algorithmic_bytes(n, G, M, given)
    dom_ms = sum(timers[r][0] for r in GROUPS[dom][0]) / steps
    dom_brackets = sum(timers[r][1] for r in GROUPS[dom][0]) / steps
    dom_bytes = GROUPS[dom][1](n, G, M, given)
    achieved = dom_bytes / (dom_ms / 1000.0) / 1e9
    groups = {}
    for g, (regs, fn, rule) in GROUPS.items():
        b = fn(n, G, M, given)
        t = group_ms[g]
        groups[g] = {"ms": t, "algorithmic_bytes": b, "GBps": b / (t / 1000.0) / 1e9 if t > 0 else None,
                     "frac": b / (t / 1000.0) / 1e9 / HBM_PEAK_GBS if t > 0 else None, "bytes_rule": rule,
                     "regions": list(regs)}
    device_ms = sum(group_ms.values())
    assert sum(fn(n, G, M, given) for _, fn, _ in GROUPS.values()) == b_alg
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom, workload),
                "kernel": f"{dom}: {GROUP_KERNELS[dom]}", "algorithmic_bytes": dom_bytes,
                "bytes_rule": GROUPS[dom][2], "ms_per_build": dom_ms, "brackets_per_build": dom_brackets,
                "groups": groups, "split_builds": split_builds}
    path = {"algorithmic_bytes": b_alg, "bytes_rule": "60 B/pt + 8 B per count-grid cell + 4 B per kept index "
                                                      "(48 B/pt with a given box)",
            "device_ms_per_build": device_ms, "achieved_device_GBps": b_alg / (device_ms / 1000.0) / 1e9,
            "frac_of_device_time": b_alg / (device_ms / 1000.0) / 1e9 / HBM_PEAK_GBS,
            "ms_per_build": ms, "frac_of_step": b_alg / (ms / 1000.0) / 1e9 / HBM_PEAK_GBS}
    return {"ms_per_build": ms, "roofline": roofline, "path": path}


def bench_uniform1m(fpo, torch, ctx, steps: int) -> dict:
    """The plain 1M-point build (uniform cube, G=64, C=100k, S=32, L=10k,
    M=64): ms per build and the fraction of HBM peak for the whole path."""
    import synth
    p = synth.UNIFORM_1M
    c = synth.uniform_1m()
    xyz = to_device(torch, c)
    params = fpo_params_of(fpo, p)
    ws = torch.empty(fpo.workspace_size(c.n, params), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    tuned = ctx.autotune(*xyz, params, workspace=ws, reps=5)
    for _ in range(3):
        job = ctx.submit(*xyz, params, workspace=ws, stream=stream)
        job.wait()
        job.release()
    res = measure(fpo, torch, ctx, xyz, params, ws, stream, max(steps, 50), "uniform1m", p)
    return {"workload": "1M uniform points, G=64, C=100k, S=32, L=10k, M=64", "n": c.n,
            "ms_per_build": res["ms_per_build"], "points_per_s": c.n / (res["ms_per_build"] / 1000.0),
            "path": res["path"], "roofline": res["roofline"], "autotuned": tuned,
            "target": "<= 15.5 us per build (50% of HBM peak for the path's algorithmic bytes)"}


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
    ap.add_argument("--no-tune", action="store_true", help="keep the default kernel shapes (profiling runs)")
    ap.add_argument("--no-uniform1m", action="store_true", help="skip the 1M-point leg (profiling runs)")
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

    tuned = None
    if not args.no_tune:
        tuned = ctx.autotune(x, y, z, params, workspace=ws, reps=3)
        print(f"[bench] autotuned quantise shape {tuned['quantize_variant']} "
              f"(ms per shape {['%.3f' % v for v in tuned['quantize_ms']]})", file=sys.stderr, flush=True)
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
    res = measure(fpo, torch, ctx, (x, y, z), params, ws, stream, args.steps, args.workload, p)
    ms = res["ms_per_build"]
    value = n / (ms / 1000.0)

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
        "path_hbm_frac": res["path"]["frac_of_step"],
        "roofline": res["roofline"],
        "path": res["path"],
        "autotuned": tuned,
        **extras,
    }
    if args.workload != "uniform1m" and not args.no_uniform1m:
        out["uniform1m"] = bench_uniform1m(fpo, torch, ctx, args.steps)
        print(f"[bench] 1M uniform: {out['uniform1m']['ms_per_build']:.3f} ms per build, "
              f"{out['uniform1m']['path']['frac_of_step']:.4f} of HBM peak", file=sys.stderr, flush=True)
    if not args.no_mix:
        del ws
        torch.cuda.empty_cache()
        out["batched"] = bench_batched(fpo, torch, ctx)
        print(f"[bench] batched {out['batched']['speedup']:.2f}x the plain loop", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        trace = ServedTrace(fpo, torch)
        tuned = {}
        if not args.no_tune:
            t = time.perf_counter()
            tuned = tune_classes(fpo, ctx, [(trace.cloud(i), p) for i, p in enumerate(trace.params)])
            torch.cuda.empty_cache()
            print(f"[bench] tuned {len(tuned)} size classes of the trace in {time.perf_counter() - t:.1f}s",
                  file=sys.stderr, flush=True)
        serial_pps = trace.serial(fpo, torch, ctx)
        print(f"[bench] serial plain loop over the trace: {serial_pps / 1e9:.2f} G points/s", file=sys.stderr,
              flush=True)
        out["served"] = bench_served(fpo, torch, ctx, trace, serial_pps, 1.25)
        out["served"]["autotuned"] = {"quantize_shape_by_class": tuned}
        print(f"[bench] served {out['served']['speedup']:.2f}x serial, p99 {out['served']['latency_ms_p99']:.1f} ms",
              file=sys.stderr, flush=True)
        # every request at once: the server's capacity against the serial loop
        out["served_saturated"] = bench_served(fpo, torch, ctx, trace, serial_pps, None)
        print(f"[bench] served, all requests at once: {out['served_saturated']['speedup']:.2f}x serial",
              file=sys.stderr, flush=True)
        # the same trace at half the serial capacity: latency without queueing
        out["served_half_load"] = bench_served(fpo, torch, ctx, trace, serial_pps, 0.5)
        print(f"[bench] served at 0.5x load: p50 {out['served_half_load']['latency_ms_p50']:.1f} ms, "
              f"p99 {out['served_half_load']['latency_ms_p99']:.1f} ms", file=sys.stderr, flush=True)
        del trace
        torch.cuda.empty_cache()
    if not args.no_stream:
        if not args.no_mix:
            torch.cuda.empty_cache()
        out["streamed"] = bench_streamed(fpo, torch, ctx)
        print(f"[bench] streamed {out['streamed']['points_per_s'] / 1e9:.2f} G points/s, "
              f"{out['streamed']['link_frac']:.2f} of the host link", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cloud, p, args.cpu_seconds, gen, pname)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
