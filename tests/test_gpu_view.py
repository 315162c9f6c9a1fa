"""View-dependent node selection on the GPU against the oracle's top-down
traversal: the hand-worked tree, random perspective views of real trees
(including eyes inside the cloud, no size limit and an infinite one), exact
axis-aligned clipping at cube faces, an empty table, and the 20M-point
workload's tree straight from a GPU build."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import view as V

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
OPEN = ((0.0, 0.0, 0.0, 1.0),) * 6


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2302_05002_amd as fpo
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = fpo.Context(0)
    yield c
    c.close()


def gpu_select(ctx, depth, key, count, bmin, side, v: V.View):
    import torch
    import paper_2302_05002_amd as fpo
    d = torch.from_numpy(np.asarray(depth, dtype=np.uint8)).cuda()
    k = torch.from_numpy(np.asarray(key, dtype=np.uint64).view(np.int64)).cuda()
    c = torch.from_numpy(np.asarray(count, dtype=np.uint32).view(np.int32)).cuda()
    idx, pts = ctx.select_nodes(d, k, c, bmin, side, fpo.make_view(v.eye, v.planes, v.proj_factor, v.min_size))
    return idx.cpu().numpy().astype(np.int64).tolist(), pts


def check(ctx, depth, key, count, bmin, side, v, label=""):
    exp, epts = V.select_nodes(depth, key, count, bmin, side, v)
    got, pts = gpu_select(ctx, depth, key, count, bmin, side, v)
    assert got == exp, f"{label}: {len(got)} vs {len(exp)} nodes"
    assert pts == epts, label
    return got


def test_worked_example(ctx):
    ex = json.load(open(os.path.join(GOLD, "view_worked_example.json")))
    args = (ex["node_depth"], ex["node_key"], ex["node_count"], ex["bbox_min"], ex["cube_size"])
    clip = (tuple(ex["clip"]),) + OPEN[:5]
    for key, planes, mn in (("selected_min40_clip", clip, 40.0), ("selected_min20_clip", clip, 20.0),
                            ("selected_min20_noclip", OPEN, 20.0), ("selected_min50_noclip", OPEN, 50.0)):
        got = check(ctx, *args, V.View(tuple(ex["eye"]), planes, ex["proj_factor"], mn), key)
        assert got == ex[key]


def random_views(lo, side, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for t in range(count):
        eye = [lo[a] + side * float(rng.uniform(-1.5, 2.5)) for a in range(3)]
        if t % 5 == 0:   # inside the cloud
            eye = [lo[a] + side * float(rng.uniform(0.3, 0.7)) for a in range(3)]
        tgt = [lo[a] + side * float(rng.uniform(0.1, 0.9)) for a in range(3)]
        mn = float(rng.choice([0.0, 10.0, 60.0, 200.0, 800.0, math.inf]))
        out.append(V.perspective_view(eye, tgt, (0.0, 0.0, 1.0), float(rng.uniform(15, 100)),
                                      float(rng.uniform(0.8, 2.0)), 0.01 * side, 8 * side,
                                      float(rng.choice([720.0, 1080.0, 2160.0])), mn))
    return out


@pytest.mark.parametrize("kind,n,G,S,L", [("clusters", 60_000, 32, 16, 300), ("planes", 200_000, 64, 64, 1_000),
                                          ("uniform", 100_000, 16, 8, 100)])
def test_random_views(ctx, kind, n, G, S, L):
    c = {"clusters": lambda: synth.clusters(n, seed=3, num_clusters=7),
         "planes": lambda: synth.planes(n, seed=4, num_planes=20), "uniform": lambda: synth.uniform(n, seed=5)}[kind]()
    r = oracle.build_octree(c.x, c.y, c.z, oracle.Params(G, n // 4, S, L, 64))
    assert r["status"] == oracle.OK
    lo = [float(v) for v in r["bbox_min"]]
    side = float(r["cube_size"])
    print(f"[view] {kind} n={n} nodes={r['node_depth'].shape[0]}", flush=True)
    sizes = []
    for i, v in enumerate(random_views(lo, side, 40, seed=n)):
        got = check(ctx, r["node_depth"], r["node_key"], r["node_count"], r["bbox_min"], r["cube_size"], v,
                    f"{kind} view {i}")
        sizes.append(len(got))
    assert min(sizes) < max(sizes)   # the views really differ


def test_exact_clipping_at_faces(ctx):
    c = synth.uniform(20_000, seed=3, lo=0.0, hi=64.0)
    x = c.x.copy(); x[0] = 0.0; x[1] = 64.0
    r = oracle.build_octree(x, c.y, c.z, oracle.Params(8, 2_000, 4, 100, 64))
    assert float(r["cube_size"]) == 64.0
    for t in (0.0, 16.0, 31.5, 32.0, 48.0, 64.0):
        for sign in (1.0, -1.0):
            for axis in range(3):
                q = [0.0, 0.0, 0.0, -sign * t]
                q[axis] = sign
                v = V.View((-1e3, 0.0, 0.0), (tuple(q),) + OPEN[:5], 1.0, 0.0)
                check(ctx, r["node_depth"], r["node_key"], r["node_count"], r["bbox_min"], 64.0, v, f"clip {t}")


def test_empty_table(ctx):
    got, pts = gpu_select(ctx, [], [], [], (0.0, 0.0, 0.0), 1.0, V.View((0.0, 0.0, 0.0), OPEN, 1.0, 0.0))
    assert got == [] and pts == 0


def test_full_size_planes_tree_from_gpu_build(ctx):
    """The 20M-point planes workload: the GPU build's node table (device
    arrays, no copy) selected for several views against the oracle traversal
    over the same table."""
    import torch
    import paper_2302_05002_amd as fpo
    c = synth.planes_20m()
    p = synth.PLANES_20M
    x, y, z = (torch.from_numpy(a).cuda() for a in (c.x, c.y, c.z))
    res = ctx.build(x, y, z, fpo.Params(p.count_grid, p.max_points_per_chunk, p.subsample_grid, p.leaf_capacity,
                                        p.preview_modulus))
    h = res.to_numpy()
    lo = [float(v) for v in h["bbox_min"]]
    side = float(h["cube_size"])
    print(f"[view] planes20m nodes={res.num_nodes}", flush=True)
    for i, v in enumerate(random_views(lo, side, 8, seed=77)):
        fv = fpo.make_view(v.eye, v.planes, v.proj_factor, v.min_size)
        idx, pts = ctx.select_nodes(res.node_depth, res.node_key, res.node_count, h["bbox_min"], h["cube_size"], fv)
        exp, epts = V.select_nodes(h["node_depth"], h["node_key"], h["node_count"], h["bbox_min"], side, v)
        assert idx.cpu().numpy().astype(np.int64).tolist() == exp, f"view {i}"
        assert pts == epts
