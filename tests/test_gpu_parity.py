"""GPU path (through the C ABI) versus the CPU oracle, element by element.

Every array is integer or index data, so the bar is bit-exact equality; the
float scalars (box, cube side, scale) are compared bit for bit too, since both
sides follow the same IEEE operations."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from checks import check_chunks, check_octree_invariants, check_preview

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
KEYS = ("count_grid", "chunk_level", "chunk_key", "chunk_count", "chunk_begin", "perm", "node_depth", "node_key",
        "node_child_mask", "node_begin", "node_count", "node_points", "preview_index")


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2302_05002_amd as fpo
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = fpo.Context(0)
    yield c
    c.close()


def gpu_build(ctx, cloud, G, C, S, L, M, bbox=None):
    import torch
    import paper_2302_05002_amd as fpo
    print(f"[gpu_build] n={cloud.n} G={G} C={C} S={S} L={L} M={M} bbox={bbox is not None}", flush=True)
    x = torch.from_numpy(np.ascontiguousarray(cloud.x)).cuda()
    y = torch.from_numpy(np.ascontiguousarray(cloud.y)).cuda()
    z = torch.from_numpy(np.ascontiguousarray(cloud.z)).cuda()
    res = ctx.build(x, y, z, fpo.Params(G, C, S, L, M, bbox))
    torch.cuda.synchronize()
    return res.to_numpy()


def compare(got, exp, label=""):
    for k in ("bbox_min", "bbox_max"):
        np.testing.assert_array_equal(got[k].view(np.uint32), exp[k].view(np.uint32), err_msg=label + k)
    assert np.float32(got["cube_size"]).view(np.uint32) == np.float32(exp["cube_size"]).view(np.uint32), label
    assert np.float32(got["scale"]).view(np.uint32) == np.float32(exp["scale"]).view(np.uint32), label
    assert got["n_outside"] == exp["n_outside"], label
    assert got["chunk_oversized_any"] == exp["chunk_oversized_any"], label
    for k in KEYS:
        a, b = np.asarray(got[k]), np.asarray(exp[k])
        assert a.shape == b.shape, f"{label}{k}: shape {a.shape} vs {b.shape}"
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0]
            raise AssertionError(f"{label}{k}: {bad.size} mismatches, first at {bad[:5]}: {a[bad[:5]]} vs {b[bad[:5]]}")


def run_both(ctx, cloud, G, C, S, L, M, bbox=None, label=""):
    exp = oracle.build_octree(cloud.x, cloud.y, cloud.z, oracle.Params(G, C, S, L, M, bbox))
    assert exp["status"] == oracle.OK
    got = gpu_build(ctx, cloud, G, C, S, L, M, bbox)
    compare(got, exp, label)
    return got, exp


def test_worked_example(ctx):
    ex = json.load(open(os.path.join(GOLD, "worked_example.json")))
    pts = np.array(ex["points"], dtype=np.float32)
    p = ex["params"]
    c = synth.Cloud(pts[:, 0].copy(), pts[:, 1].copy(), pts[:, 2].copy())
    got = gpu_build(ctx, c, p["count_grid"], p["max_points_per_chunk"], p["subsample_grid"], p["leaf_capacity"],
                    p["preview_modulus"])
    for k in KEYS:
        np.testing.assert_array_equal(np.asarray(got[k]).astype(np.int64), np.array(ex[k], dtype=np.int64), err_msg=k)
    assert float(got["scale"]) == ex["scale"] and float(got["cube_size"]) == ex["cube_size"]


SMALL_CASES = [
    # (kind, n, seed, G, C, S, L, M)
    ("uniform", 5_000, 1, 8, 700, 8, 100, 4),
    ("uniform", 12_345, 2, 16, 3_000, 16, 500, 7),
    ("planes", 30_001, 3, 32, 5_000, 32, 1_000, 64),
    ("clusters", 40_000, 4, 64, 10_000, 16, 2_000, 3),
    ("planes", 65_537, 5, 128, 20_000, 128, 10_000, 64),
    ("uniform", 100_000, 6, 64, 100_000, 32, 10_000, 64),
    ("clusters", 50_000, 7, 4, 1_000, 4, 50, 5),
    ("uniform", 7_777, 8, 1, 10, 2, 10, 1),
    ("planes", 20_000, 9, 512, 300, 256, 64, 9),
    ("clusters", 25_000, 10, 2, 100_000, 1, 30, 2),
]


def make(kind, n, seed):
    if kind == "uniform":
        return synth.uniform(n, seed=seed)
    if kind == "planes":
        return synth.planes(n, seed=seed, num_planes=12)
    return synth.clusters(n, seed=seed, num_clusters=9)


@pytest.mark.parametrize("case", SMALL_CASES, ids=[f"{c[0]}-{c[1]}-G{c[3]}-S{c[5]}" for c in SMALL_CASES])
def test_small_parity(ctx, case):
    kind, n, seed, G, C, S, L, M = case
    c = make(kind, n, seed)
    got, _ = run_both(ctx, c, G, C, S, L, M, label=f"{case}: ")
    check_preview(got, n, M)


def test_empty_and_single(ctx):
    e = synth.Cloud(np.zeros(0, np.float32), np.zeros(0, np.float32), np.zeros(0, np.float32))
    got = gpu_build(ctx, e, 8, 10, 8, 10, 4)
    assert got["node_depth"].shape[0] == 0 and got["perm"].shape[0] == 0 and got["preview_index"].shape[0] == 0
    assert int(got["count_grid"].sum()) == 0
    one = np.array([3.5], np.float32)
    run_both(ctx, synth.Cloud(one, one.copy(), one.copy()), 8, 10, 8, 10, 4)


def test_identical_points_deep_chain(ctx):
    """All points equal: a chain of one-point nodes down to depth 21 - s; with
    more than 4096 points the single work chunk takes the global-memory path."""
    for n, S in ((300, 4), (9_000, 32)):
        v = np.full(n, 2.5, np.float32)
        run_both(ctx, synth.Cloud(v, v.copy(), v.copy()), 4, 50, S, 10, 7, label=f"n={n} S={S}: ")


def test_big_work_chunks(ctx):
    """Dense blobs deeper than the work-chunk level cap give work chunks of
    more than 4096 points (global-memory hash path)."""
    c = synth.clusters(120_000, seed=21, num_clusters=3, sigma_frac=0.001)
    run_both(ctx, c, 64, 5_000, 4, 200, 64)
    c = synth.clusters(200_000, seed=22, num_clusters=5, sigma_frac=0.002)
    run_both(ctx, c, 512, 2_000, 128, 1_000, 64)


def test_given_bbox(ctx):
    c = synth.planes(40_000, seed=31, num_planes=8)
    lo = (float(c.x.min()), float(c.y.min()), float(c.z.min()))
    hi = (float(c.x.max()), float(c.y.max()), float(c.z.max()))
    run_both(ctx, c, 32, 4_000, 16, 400, 8, bbox=(lo, hi))
    mid = tuple((a + b) / 2 for a, b in zip(lo, hi))
    got, exp = run_both(ctx, c, 32, 4_000, 16, 400, 8, bbox=(lo, mid))
    assert got["n_outside"] > 0


def test_signed_zero_extremes(ctx):
    for xs in ([-0.0, 0.0, 1.0], [0.0, -0.0, 1.0], [1.0, -0.0, 0.0]):
        x = np.array(xs, np.float32)
        m = np.array([-1.0, -0.0, -0.0], np.float32)
        got, _ = run_both(ctx, synth.Cloud(x, m, x.copy()), 4, 10, 4, 1, 2)
        assert not np.signbit(got["bbox_min"][0]) and not np.signbit(got["bbox_max"][1])


def test_nonfinite_rejected(ctx):
    import torch
    import paper_2302_05002_amd as fpo
    x = torch.tensor([0.0, 1.0, float("nan"), 2.0], device="cuda")
    with pytest.raises(fpo.FpoError) as e:
        ctx.build(x, x.clone(), x.clone(), fpo.Params(8, 10, 8, 10, 4))
    assert e.value.status == fpo.FPO_ERR_NONFINITE


def test_nonfinite_rejected_with_given_box(ctx):
    """With a given box there is no bounding-box pass: the quantise pass flags
    NaN and infinities, in any coordinate and anywhere in the input."""
    import torch
    import paper_2302_05002_amd as fpo
    box = ((0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    c = synth.uniform(300_000, seed=77)
    for bad in (float("nan"), float("inf"), float("-inf")):
        for axis in range(3):
            for at in (0, 123_457, c.n - 1):
                a = [np.ascontiguousarray(v).copy() for v in (c.x, c.y, c.z)]
                a[axis][at] = bad
                x, y, z = (torch.from_numpy(v).cuda() for v in a)
                with pytest.raises(fpo.FpoError) as e:
                    ctx.build(x, y, z, fpo.Params(16, 10_000, 8, 100, 4, box))
                assert e.value.status == fpo.FPO_ERR_NONFINITE, (bad, axis, at)
    # finite points outside the given box are fine (counted, clamped)
    a = [np.ascontiguousarray(v).copy() for v in (c.x, c.y, c.z)]
    a[1][5] = 7.0
    run_both(ctx, synth.Cloud(*a), 16, 10_000, 8, 100, 4, box, label="outside: ")


def test_uniform_1m_full(ctx):
    """The uniform 1M-point workload, every output compared."""
    c = synth.uniform_1m()
    p = synth.UNIFORM_1M
    got, exp = run_both(ctx, c, p.count_grid, p.max_points_per_chunk, p.subsample_grid, p.leaf_capacity,
                        p.preview_modulus)
    assert got["preview_index"].shape[0] == 15761
    assert np.bincount(got["node_depth"]).tolist() == [1, 8, 64, 512]


def test_quantize_table_flushes(ctx):
    """3M uniform points over a 128^3 count grid: each block of the quantise
    pass meets about 8,000 new cells in its first round of 8,192 points,
    more than its LDS cell table keeps between rounds, so the table is
    flushed to the global histogram between rounds."""
    c = synth.uniform(3_000_000, seed=91)
    run_both(ctx, c, 128, 1_000_000, 32, 10_000, 64)


def test_planes_20m_reduced_with_invariants(ctx):
    """The 200-plane workload at 2M points: full comparison plus invariants."""
    c = synth.planes(2_000_000, seed=2)
    p = synth.PLANES_20M
    got, _ = run_both(ctx, c, p.count_grid, p.max_points_per_chunk, p.subsample_grid, p.leaf_capacity,
                      p.preview_modulus)
    u = oracle.build_octree(c.x, c.y, c.z, oracle.Params(p.count_grid, p.max_points_per_chunk, p.subsample_grid,
                                                         p.leaf_capacity, p.preview_modulus))["u"]
    check_chunks(got, u, p.count_grid, p.max_points_per_chunk)
    check_octree_invariants(got, u, p.subsample_grid, p.leaf_capacity)


def test_planes_20m_full(ctx):
    """The 200-plane workload at its full 20M points, in the configuration the
    benchmark times: every output compared with the oracle."""
    c = synth.planes_20m()
    p = synth.PLANES_20M
    run_both(ctx, c, p.count_grid, p.max_points_per_chunk, p.subsample_grid, p.leaf_capacity, p.preview_modulus)


def test_repeatable(ctx):
    c = synth.planes(300_000, seed=41, num_planes=30)
    a = gpu_build(ctx, c, 64, 50_000, 32, 2_000, 64)
    b = gpu_build(ctx, c, 64, 50_000, 32, 2_000, 64)
    for k in KEYS:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def spike_cloud(levels=7, dense=5000, seed=3):
    """A dense cell at the minimum corner of the finest work-chunk level and one
    point in each of the 7 sibling octants along its path at every level:
    after the dense work chunk come about 7 * levels one-point work chunks,
    far more than one 2048-position tile of the node-id pass caches."""
    rng = np.random.default_rng(seed)
    pts = [rng.uniform(0.0, 2.0 ** -levels, (dense, 3))]
    for l in range(1, levels + 1):
        for o in range(1, 8):
            org = np.array([(o >> 2) & 1, (o >> 1) & 1, o & 1], float) * 2.0 ** -l
            pts.append((org + 2.0 ** -(l + 1))[None, :])
    pts.append(np.array([[1.0, 1.0, 1.0]]))
    p = np.concatenate(pts).astype(np.float32)
    return synth.Cloud(p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy())


def test_many_tiny_work_chunks(ctx):
    """Tiles of the node-id pass overlapping more work chunks than they cache."""
    c = spike_cloud()
    run_both(ctx, c, 128, 100_000, 128, 10_000, 8)
    run_both(ctx, c, 128, 1_000, 128, 300, 8)


def test_oversized_work_chunks(ctx):
    """Dense clusters inside one cell of the deepest work-chunk level: work
    chunks of 4097-8192 points whose root is a leaf (wide LDS instance), and
    of more than 8192 points (global-memory path)."""
    c = synth.clusters(100_000, seed=23, num_clusters=15, sigma_frac=0.0005)   # 14 of 6667 points
    run_both(ctx, c, 128, 1_000_000, 128, 10_000, 64)
    c = synth.clusters(120_000, seed=24, num_clusters=12, sigma_frac=0.0004)   # 10 of 10000 points
    run_both(ctx, c, 128, 1_000_000, 128, 12_000, 64)


def test_node_points_odd_tile_count(ctx):
    """A root above two sort tiles of 16384 values (41,307 points: three
    tiles, so two merge rounds, the first with an unpaired run)."""
    c = synth.uniform(45_000, seed=41)
    got, exp = run_both(ctx, c, 16, 1_000_000, 64, 10_000, 7)
    assert int(exp["node_count"][0]) > 2 * 16384


def test_node_points_many_own_nodes(ctx):
    """A dense blob inside one count-grid cell (a single work chunk of 30,000
    points taking the global-memory path) with L = 1: more than 4096 own nodes,
    beyond the per-work-chunk LDS counters of the node sizes and placement."""
    rng = np.random.default_rng(42)
    p = rng.random((30_000, 3), dtype=np.float32)
    p = np.concatenate([p, np.array([[1000.0, 1000.0, 1000.0]], np.float32)])
    c = synth.Cloud(p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy())
    got, exp = run_both(ctx, c, 4, 1_000_000, 2, 1, 5)
    assert exp["node_depth"].shape[0] > 4096 + 1000


LARGEST_GRID_CASES = [
    # (label, cloud, G, C, S, L, M): the largest subsample grid (2^24 cells per
    # node: general subsample classes, hashed cell tables) at millions of points
    ("planes 2M G128 S256", lambda: synth.planes(2_000_000, seed=61, num_planes=30), 128, 200_000, 256, 10_000, 64),
    ("clusters 1M G64 S256 L1000", lambda: synth.clusters(1_000_000, 62, 25), 64, 100_000, 256, 1_000, 16),
    ("uniform 3M G256 S256", lambda: synth.uniform(3_000_000, seed=63), 256, 500_000, 256, 20_000, 64),
    ("planes 2M G512 S256", lambda: synth.planes(2_000_000, seed=64, num_planes=30), 512, 100_000, 256, 5_000, 64),
    ("clusters 2M G256 S256 tight", lambda: synth.clusters(2_000_000, 65, 8, sigma_frac=0.002), 256, 300_000, 256,
     1_000, 64),
]


@pytest.mark.parametrize("case", LARGEST_GRID_CASES, ids=[c[0] for c in LARGEST_GRID_CASES])
def test_largest_subsample_grid(ctx, case):
    label, make_cloud, G, C, S, L, M = case
    run_both(ctx, make_cloud(), G, C, S, L, M, label=f"{label}: ")
