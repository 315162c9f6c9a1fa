"""Preview variants on the GPU (stride of the fixed-target decimation, one
pick per occupied count-grid cell) against the oracle, element by element,
plus the full-size 200-plane workload against numpy's per-cell minimum."""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from checks import h64_numpy, quantize_emulated
from test_gpu_parity import compare

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2302_05002_amd as fpo
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = fpo.Context(0)
    yield c
    c.close()


def dev(c):
    import torch
    return tuple(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (c.x, c.y, c.z))


def both(ctx, c, G, C, S, L, M, preview, bbox=None, label=""):
    import torch
    import paper_2302_05002_amd as fpo
    print(f"[preview] {label} n={c.n} G={G} M={M} mode={preview}", flush=True)
    exp = oracle.build_octree(c.x, c.y, c.z, oracle.Params(G, C, S, L, M, bbox, preview))
    assert exp["status"] == oracle.OK
    got = ctx.build(*dev(c), fpo.Params(G, C, S, L, M, bbox, preview)).to_numpy()
    torch.cuda.synchronize()
    compare(got, exp, label=f"{label} {preview}: ")
    return got, exp


def test_worked_example(ctx):
    ex = json.load(open(os.path.join(GOLD, "preview_grid_example.json")))
    pts = np.array(ex["points"], dtype=np.float32)
    c = synth.Cloud(pts[:, 0].copy(), pts[:, 1].copy(), pts[:, 2].copy())
    p = ex["params"]
    for mode, key in (("grid", "preview_grid"), ("stride", "preview_stride_m4"), ("hash", "preview_hash_m4")):
        got, _ = both(ctx, c, p["count_grid"], p["max_points_per_chunk"], p["subsample_grid"], p["leaf_capacity"],
                      p["preview_modulus"], mode, label="worked")
        assert got["preview_index"].tolist() == ex[key]


CASES = [
    # (kind, n, seed, G, M)
    ("uniform", 5_000, 1, 8, 4),
    ("planes", 30_001, 3, 32, 64),
    ("clusters", 40_000, 4, 64, 3),
    ("planes", 65_537, 5, 128, 1),
    ("uniform", 7_777, 8, 1, 7_777),
    ("planes", 20_000, 9, 512, 9),
    ("clusters", 250_000, 12, 256, 100),
]


def make(kind, n, seed):
    if kind == "uniform":
        return synth.uniform(n, seed=seed)
    if kind == "planes":
        return synth.planes(n, seed=seed, num_planes=12)
    return synth.clusters(n, seed=seed, num_clusters=9)


@pytest.mark.parametrize("mode", ["stride", "grid"])
@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[1]}-G{c[3]}-M{c[4]}" for c in CASES])
def test_parity(ctx, case, mode):
    kind, n, seed, G, M = case
    c = make(kind, n, seed)
    both(ctx, c, G, max(n // 8, 1), 32, 1_000, M, mode, label=str(case))


def test_grid_table_flushes(ctx):
    """3M uniform points over a 128^3 count grid: the grid preview's cell
    table (per-cell hash minima) is flushed between the quantise rounds of
    every block, since each round of 2,048 points meets about 2,000 new
    cells."""
    c = synth.uniform(3_000_000, seed=91)
    both(ctx, c, 128, 1_000_000, 32, 10_000, 64, "grid", label="flushes")


def test_empty_single_and_identical(ctx):
    e = synth.Cloud(np.zeros(0, np.float32), np.zeros(0, np.float32), np.zeros(0, np.float32))
    one = np.array([3.5], np.float32)
    same = np.full(5_000, -2.25, np.float32)
    for mode in ("stride", "grid"):
        import paper_2302_05002_amd as fpo
        got = ctx.build(*dev(e), fpo.Params(8, 10, 8, 10, 4, None, mode)).to_numpy()
        assert got["preview_index"].shape[0] == 0
        both(ctx, synth.Cloud(one, one.copy(), one.copy()), 8, 10, 8, 10, 4, mode, label="single")
        got, _ = both(ctx, synth.Cloud(same, same.copy(), same.copy()), 64, 100, 8, 10, 4, mode, label="same")
        if mode == "grid":
            assert got["preview_index"].tolist() == [0]


def test_given_box_and_streamed(ctx):
    """The grid preview follows the count pass, also when the points arrive in
    batches from pinned host memory with a box given as a header."""
    import torch
    import paper_2302_05002_amd as fpo
    c = synth.terrain_clusters(1_500_000, seed=17, colors=False)
    box = ((float(c.x.min()), float(c.y.min()), float(c.z.min())),
           (float(c.x.max()), float(c.y.max()), float(c.z.max())))
    x, y, z = (torch.from_numpy(np.ascontiguousarray(a)).pin_memory() for a in (c.x, c.y, c.z))
    # G = 64: picks by inverse hash (cells < 2n); G = 256: by the per-point predicate
    for G, bbox in ((64, None), (64, box), (256, None), (256, box)):
        exp = oracle.build_octree(c.x, c.y, c.z, oracle.Params(G, 100_000, 64, 5_000, 16, bbox, "grid"))
        print(f"[preview] streamed grid n={c.n} G={G} bbox={bbox is not None}", flush=True)
        job = ctx.submit(x, y, z, fpo.Params(G, 100_000, 64, 5_000, 16, bbox, "grid"), stream_batch=400_000)
        job.wait()
        assert job.preview_ready()
        got = job.result().to_numpy()
        job.release()
        compare(got, exp, label=f"streamed grid G={G} bbox={bbox is not None}: ")


def test_fixed_target_modulus(ctx):
    """The paper's decimation to a fixed target count: M from the target, then
    a stride preview of at most that many points."""
    import paper_2302_05002_amd as fpo
    c = synth.planes(2_500_001, seed=23, num_planes=40)
    M = fpo.preview_modulus(c.n, 100_000)
    assert M == 26
    got, _ = both(ctx, c, 128, 300_000, 128, 10_000, M, "stride", label="target")
    assert got["preview_index"].shape[0] == -(-c.n // M) <= 100_000


def test_full_size_planes(ctx):
    """The 200-plane workload at 20M points with G = 128: the grid preview
    equals the per-cell minimum of the hash computed by numpy from the points
    (cells from the parity-tested box and scale), and the stride preview is
    the closed form."""
    import torch
    import paper_2302_05002_amd as fpo
    c = synth.planes_20m()
    p = synth.PLANES_20M
    x, y, z = dev(c)
    print(f"[preview] full-size planes n={c.n} G={p.count_grid}", flush=True)
    got = ctx.build(x, y, z, fpo.Params(p.count_grid, p.max_points_per_chunk, p.subsample_grid, p.leaf_capacity,
                                        p.preview_modulus, None, "grid")).to_numpy()
    torch.cuda.synchronize()
    G = p.count_grid
    sh = 21 - int(np.log2(G))
    cell = np.zeros(c.n, np.int64)
    for k, a in enumerate((c.x, c.y, c.z)):
        cell = cell * G + (quantize_emulated(a, got["bbox_min"][k], got["scale"]) >> sh).astype(np.int64)
    h = h64_numpy(np.arange(c.n, dtype=np.uint64))
    best = np.full(G ** 3, np.iinfo(np.uint64).max, np.uint64)
    np.minimum.at(best, cell, h)
    exp = np.nonzero(h == best[cell])[0]
    np.testing.assert_array_equal(got["preview_index"].astype(np.int64), exp)
    assert exp.shape[0] == int(np.count_nonzero(got["count_grid"]))
    got = ctx.build(x, y, z, fpo.Params(p.count_grid, p.max_points_per_chunk, p.subsample_grid, p.leaf_capacity,
                                        p.preview_modulus, None, "stride")).to_numpy()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got["preview_index"], np.arange(0, c.n, p.preview_modulus, dtype=np.uint32))


@pytest.mark.parametrize("mode", ["hash", "stride", "grid"])
def test_ragged_sizes_multi_kernel(mode):
    """The multi-kernel preview (bit map per wave of 1024 indices, 4096-index
    compaction tiles) at sizes around its word, wave and tile boundaries, with
    single-workgroup builds turned off."""
    import paper_2302_05002_amd as fpo
    ctx = fpo.Context(0)
    try:
        ctx.set_single_block_max(0)
        for n in (1, 31, 33, 63, 65, 1023, 1025, 4095, 4097, 5121, 70_001):
            c = synth.uniform(n, seed=n)
            both(ctx, c, 16, 2_000, 8, 100, 7 if mode != "grid" else 3, mode, label=f"ragged {n}")
    finally:
        ctx.close()
