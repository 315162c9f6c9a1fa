"""The autotuner's candidates change speed only: every shape of the quantise
+ count pass gives the oracle's result bit for bit (device and streamed
inputs, computed and given boxes, scans and uniform clouds, the binned shape
from G = 32 to 512, with a given box that leaves points outside), the tuner keeps
its choice in the context and in the FPO_AUTOTUNE_CACHE file, and the batch
tuner's worker counts give identical batches."""
import os

import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import compare

pytestmark = pytest.mark.gpu


def _oracle(c, G, C, S, L, M, bbox=None):
    r = oracle.build_octree(c.x, c.y, c.z, oracle.Params(G, C, S, L, M, bbox))
    assert r["status"] == oracle.OK
    return r


CLOUDS = [("uniform", lambda: synth.uniform(300_000, seed=31), (64, 20_000, 32, 1_000, 64)),
          ("planes", lambda: synth.planes(500_000, seed=32, num_planes=30), (128, 50_000, 64, 2_000, 16)),
          ("clusters", lambda: synth.clusters(200_000, seed=33, num_clusters=12), (32, 5_000, 16, 300, 7)),
          # G = 512: few points per cell, the regime of the two-points-per-thread
          # shape; 2^20 points and more: the binned shape runs for device input
          ("sparse", lambda: synth.planes(1_100_000, seed=34, num_planes=40), (512, 1_000_000, 128, 10_000, 64)),
          ("g256", lambda: synth.clusters(1_200_000, seed=35, num_clusters=30), (256, 200_000, 32, 2_000, 16))]


@pytest.mark.parametrize("name,make,case", CLOUDS, ids=[c[0] for c in CLOUDS])
def test_every_quantize_shape_gives_the_same_result(name, make, case):
    import torch
    import paper_2302_05002_amd as fpo
    c = make()
    exp = _oracle(c, *case)
    box = ((float(c.x.min()), float(c.y.min()), float(c.z.min())), (float(c.x.max()), float(c.y.max()),
                                                                   float(c.z.max())))
    exp_box = _oracle(c, *case, bbox=box)
    ctx = fpo.Context(0)
    try:
        dev = [torch.from_numpy(a).cuda() for a in (c.x, c.y, c.z)]
        pinned = [torch.from_numpy(a).pin_memory() for a in (c.x, c.y, c.z)]
        for v in range(fpo.QUANTIZE_VARIANTS):
            ctx.force_quantize_variant(v)
            compare(ctx.build(*dev, fpo.Params(*case)).to_numpy(), exp, label=f"{name} shape {v}: ")
            compare(ctx.build(*dev, fpo.Params(*case, box)).to_numpy(), exp_box, label=f"{name} shape {v} box: ")
            job = ctx.submit(*pinned, fpo.Params(*case, box), stream_batch=1 << 20)
            job.wait()
            compare(job.result().to_numpy(), exp_box, label=f"{name} shape {v} streamed: ")
            job.release()
        ctx.force_quantize_variant(-1)
    finally:
        ctx.close()


def test_binned_shape_edges():
    """The binned shape with a given box smaller than the cloud (points clamp
    to its faces and are counted outside), at exactly 2^20 points, and with
    a non-finite coordinate (rejected with a given box and a computed one)."""
    import torch
    import paper_2302_05002_amd as fpo
    c = synth.clusters(1 << 20, seed=36, num_clusters=9)
    lo = (float(c.x.min()), float(c.y.min()), float(c.z.min()))
    hi = (float(c.x.max()), float(c.y.max()), float(c.z.max()))
    box = (tuple(a + 0.1 * (b - a) for a, b in zip(lo, hi)), tuple(b - 0.1 * (b - a) for a, b in zip(lo, hi)))
    ctx = fpo.Context(0)
    try:
        ctx.force_quantize_variant(4)
        dev = [torch.from_numpy(a).cuda() for a in (c.x, c.y, c.z)]
        for G in (256, 512):
            case = (G, 300_000, 32, 5_000, 9)
            got = ctx.build(*dev, fpo.Params(*case, box)).to_numpy()
            assert got["n_outside"] > 0
            compare(got, _oracle(c, *case, bbox=box), label=f"binned G={G} given box: ")
            compare(ctx.build(*dev, fpo.Params(*case)).to_numpy(), _oracle(c, *case), label=f"binned G={G}: ")
        c.z[777_777] = np.nan
        dev = [torch.from_numpy(a).cuda() for a in (c.x, c.y, c.z)]
        for b in (None, box):
            with pytest.raises(fpo.FpoError) as e:
                ctx.build(*dev, fpo.Params(512, 300_000, 32, 5_000, 9, b))
            assert e.value.status == fpo.FPO_ERR_NONFINITE
    finally:
        ctx.close()


def test_autotune_with_the_binned_shape():
    """At G = 512 and 2^20 points or more the tuner times five shapes; below
    2^16 points the binned one is not a candidate."""
    import torch
    import paper_2302_05002_amd as fpo
    c = synth.planes(1_100_000, seed=37, num_planes=60)
    case = (512, 1_000_000, 128, 10_000, 64)
    ctx = fpo.Context(0)
    try:
        dev = [torch.from_numpy(a).cuda() for a in (c.x, c.y, c.z)]
        t = ctx.autotune(*dev, fpo.Params(*case), reps=2)
        assert len(t["quantize_ms"]) == fpo.QUANTIZE_VARIANTS and all(ms > 0 for ms in t["quantize_ms"])
        assert t["quantize_ms"][t["quantize_variant"]] == min(t["quantize_ms"])
        compare(ctx.build(*dev, fpo.Params(*case)).to_numpy(), _oracle(c, *case), label="tuned at G = 512: ")
        small = synth.uniform(60_000, seed=38)
        dev = [torch.from_numpy(a).cuda() for a in (small.x, small.y, small.z)]
        t = ctx.autotune(*dev, fpo.Params(64, 100_000, 32, 1_000, 8), reps=1)
        assert len(t["quantize_ms"]) == fpo.QUANTIZE_VARIANTS - 1
    finally:
        ctx.close()


def test_autotune_keeps_and_stores_its_choice(tmp_path):
    import torch
    import paper_2302_05002_amd as fpo
    c = synth.planes(400_000, seed=34, num_planes=40)
    case = (64, 40_000, 32, 1_000, 64)
    exp = _oracle(c, *case)
    cache = tmp_path / "tune.txt"
    os.environ["FPO_AUTOTUNE_CACHE"] = str(cache)
    try:
        ctx = fpo.Context(0)
        try:
            dev = [torch.from_numpy(a).cuda() for a in (c.x, c.y, c.z)]
            t = ctx.autotune(*dev, fpo.Params(*case), reps=2)
            assert t["quantize_variant"] in range(fpo.QUANTIZE_VARIANTS)
            assert len(t["quantize_ms"]) == fpo.QUANTIZE_VARIANTS   # the binned shape too (64 bins)
            assert all(ms > 0 for ms in t["quantize_ms"])
            assert t["size_class"] == 18 and t["count_grid_log2"] == 6   # 2^18 <= 400k < 2^19
            assert t["quantize_ms"][t["quantize_variant"]] == min(t["quantize_ms"])
            compare(ctx.build(*dev, fpo.Params(*case)).to_numpy(), exp, label="after tuning: ")
        finally:
            ctx.close()
        lines = cache.read_text().splitlines()
        assert lines[0] == "fpo-autotune 1"
        assert f"qz 18 6 {t['quantize_variant']}" in lines
        # a new context reads the file and builds the same result
        ctx = fpo.Context(0)
        try:
            compare(ctx.build(*dev, fpo.Params(*case)).to_numpy(), exp, label="from the cache: ")
        finally:
            ctx.close()
    finally:
        del os.environ["FPO_AUTOTUNE_CACHE"]


def test_autotune_batch_workers():
    import torch
    import paper_2302_05002_amd as fpo
    mix = synth.batch_mix(10, seed=35, lo=10_000, hi=300_000)
    ctx = fpo.Context(0)
    try:
        dev = [tuple(torch.from_numpy(a).cuda() for a in (c.x, c.y, c.z)) for c, _ in mix]
        params = [fpo.Params(p.count_grid, p.max_points_per_chunk, p.subsample_grid, p.leaf_capacity,
                             p.preview_modulus) for _, p in mix]
        t = ctx.autotune_batch(dev, params, reps=1)
        assert t["workers"] in (2, 4, 8) and all(v > 0 for v in t["batch_ms"].values())
        jobs = ctx.build_batch(dev, params)
        for j, (c, p) in zip(jobs, mix):
            j.wait()
            compare(j.result().to_numpy(), _oracle(c, p.count_grid, p.max_points_per_chunk, p.subsample_grid,
                                                   p.leaf_capacity, p.preview_modulus), label="tuned batch: ")
            j.release()
    finally:
        ctx.close()
