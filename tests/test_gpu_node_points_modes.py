"""node_points by a split of perm order, chunk by chunk, against the oracle
and against the placement in work-chunk order: uniform, planes and clustered
clouds, hundreds of chunks, nodes spanning chunks at several depths, and
builds the split cannot take (a chunk with points of more than 2048 nodes, the
global-memory subsample path, work chunks spanning chunks), which fall back.
Each build's statistics tell which form ran."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

KEYS = ("count_grid", "chunk_level", "chunk_key", "chunk_count", "chunk_begin", "perm", "node_depth", "node_key",
        "node_child_mask", "node_begin", "node_count", "node_points", "preview_index")


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2302_05002_amd as fpo
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = fpo.Context(0)
    c.set_single_block_max(0)   # every build through the multi-kernel path
    yield c
    c.close()


def build(ctx, cloud, G, C, S, L, M, by_chunk):
    import torch
    import paper_2302_05002_amd as fpo
    print(f"[node_points] n={cloud.n} G={G} C={C} S={S} L={L} M={M} by_chunk={by_chunk}", flush=True)
    ctx.set_node_points_by_chunk(by_chunk)
    try:
        x, y, z = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (cloud.x, cloud.y, cloud.z))
        job = ctx.submit(x, y, z, fpo.Params(G, C, S, L, M))
        job.wait()
        out = job.to_numpy()
        st = job.stats()
        job.release()
        torch.cuda.synchronize()
    finally:
        ctx.set_node_points_by_chunk(True)
    return out, st


def compare(got, exp, label):
    for k in KEYS:
        a, b = np.asarray(got[k]), np.asarray(exp[k])
        assert a.shape == b.shape, f"{label}{k}: shape {a.shape} vs {b.shape}"
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0]
            raise AssertionError(f"{label}{k}: {bad.size} mismatches, first at {bad[:5]}: {a[bad[:5]]} vs {b[bad[:5]]}")


def nodes_spanning_chunks(exp):
    """Nodes whose points lie in more than one chunk (computed from the
    oracle's arrays)."""
    n = exp["perm"].shape[0]
    nc = np.asarray(exp["node_count"], np.int64)
    node_of = np.empty(n, np.int64)
    node_of[np.asarray(exp["node_points"], np.int64)] = np.repeat(np.arange(nc.shape[0]), nc)
    cc = np.asarray(exp["chunk_count"], np.int64)
    chunk_of = np.empty(n, np.int64)
    chunk_of[np.asarray(exp["perm"], np.int64)] = np.repeat(np.arange(cc.shape[0]), cc)
    pairs = np.unique(node_of * cc.shape[0] + chunk_of)
    return int((np.bincount(pairs // cc.shape[0], minlength=nc.shape[0]) > 1).sum())


CASES = [
    # kind, n, seed, G, C, S, L, M, split expected (None: either)
    ("uniform", 1_000_000, 1, 64, 100_000, 32, 10_000, 64, True),
    ("planes", 300_000, 3, 64, 20_000, 32, 1_000, 64, True),
    ("clusters", 500_000, 4, 128, 30_000, 16, 500, 64, True),
    ("planes", 2_000_000, 5, 128, 200_000, 128, 10_000, 64, True),
    ("uniform", 200_000, 6, 32, 1_000, 8, 50, 64, None),        # 512 chunks (C below the work-chunk cap)
    ("uniform", 70_000, 7, 16, 1_000_000, 64, 10_000, 7, True),  # one chunk: every node ascends after the split
    ("clusters", 200_000, 8, 64, 1_000_000, 8, 20, 64, False),  # one chunk with thousands of nodes
]


def make(kind, n, seed):
    if kind == "uniform":
        return synth.uniform(n, seed=seed)
    if kind == "planes":
        return synth.planes(n, seed=seed, num_planes=40)
    return synth.clusters(n, seed=seed, num_clusters=40)


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[1]}-G{c[3]}-C{c[4]}-S{c[5]}" for c in CASES])
def test_both_forms_match_the_oracle(ctx, case):
    kind, n, seed, G, C, S, L, M, split = case
    cloud = make(kind, n, seed)
    exp = oracle.build_octree(cloud.x, cloud.y, cloud.z, oracle.Params(G, C, S, L, M))
    assert exp["status"] == oracle.OK
    got, st = build(ctx, cloud, G, C, S, L, M, True)
    compare(got, exp, f"{case} by chunk: ")
    print(f"  by_chunk={st['node_points_by_chunk']}", flush=True)
    if split is not None:
        assert st["node_points_by_chunk"] == (1 if split else 0), st
    got, st = build(ctx, cloud, G, C, S, L, M, False)
    compare(got, exp, f"{case} placed: ")
    assert st["node_points_by_chunk"] == 0
    if split and exp["chunk_level"].shape[0] > 1:
        assert nodes_spanning_chunks(exp) > 0   # the sort of spanning nodes is exercised


def test_fallbacks(ctx):
    """Builds the split does not take: the global-memory subsample path (a dense
    blob in one count-grid cell), and work chunks spanning several chunks
    (chunks finer than the work-chunk levels' first level)."""
    rng = np.random.default_rng(42)
    p = rng.random((30_000, 3), dtype=np.float32)
    p = np.concatenate([p, np.array([[1000.0, 1000.0, 1000.0]], np.float32)])
    blob = synth.Cloud(p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy())
    for cloud, prm in ((blob, (4, 1_000_000, 2, 1, 5)), (synth.uniform(100_000, seed=9), (64, 500, 8, 100, 16))):
        exp = oracle.build_octree(cloud.x, cloud.y, cloud.z, oracle.Params(*prm))
        got, st = build(ctx, cloud, *prm, True)
        compare(got, exp, f"{prm}: ")
        print(f"  by_chunk={st['node_points_by_chunk']}", flush=True)
