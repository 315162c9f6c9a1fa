"""Node-ordered points and the one-file export of a completed build, against
the oracle's node table: the points of node k are the input points listed by
node_points in node k's range, in that order."""
import os

import numpy as np
import pytest

import oracle
import synth
from checks import quantize_emulated

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2302_05002_amd as fpo
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = fpo.Context(0)
    yield c
    c.close()


CASES = [("planes", 200_000, 101, 64, 20_000, 32, 1_000, 64, 3), ("clusters", 50_000, 102, 128, 5_000, 16, 300, 8, 4),
         ("uniform", 7, 103, 4, 10, 4, 2, 2, 0)]


def make(kind, n, seed):
    if kind == "planes":
        return synth.planes(n, seed=seed, num_planes=10)
    if kind == "clusters":
        return synth.clusters(n, seed=seed, num_clusters=7)
    return synth.uniform(n, seed=seed)


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[1]}" for c in CASES])
def test_gather_and_file(ctx, case, tmp_path):
    import torch
    import paper_2302_05002_amd as fpo
    kind, n, seed, G, C, S, L, M, stride = case
    c = make(kind, n, seed)
    print(f"[export] {case}", flush=True)
    exp = oracle.build_octree(c.x, c.y, c.z, oracle.Params(G, C, S, L, M))
    rng = np.random.default_rng(seed)
    color = rng.integers(0, 256, size=(n, stride), dtype=np.uint8) if stride else None
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (c.x, c.y, c.z)]
    dcol = torch.from_numpy(color).cuda() if stride else None
    job = ctx.submit(*dev, fpo.Params(G, C, S, L, M))
    job.wait()
    xyz, col = job.gather(*dev, dcol)
    torch.cuda.synchronize()
    order = exp["node_points"].astype(np.int64)
    want = np.stack([c.x, c.y, c.z], 1)[order]
    np.testing.assert_array_equal(xyz.cpu().numpy().view(np.uint32), want.view(np.uint32))
    if stride:
        np.testing.assert_array_equal(col.cpu().numpy(), color[order])
    path = os.path.join(tmp_path, "tree.fpo")
    job.write_file(path, *dev, dcol)
    f = fpo.read_file(path)
    assert f["n"] == n and f["num_nodes"] == exp["node_depth"].shape[0] and f["color_stride"] == stride
    assert f["count_grid"] == G and f["subsample_grid"] == S
    np.testing.assert_array_equal(f["nodes"]["depth"], exp["node_depth"])
    np.testing.assert_array_equal(f["nodes"]["key"], exp["node_key"])
    np.testing.assert_array_equal(f["nodes"]["child_mask"], exp["node_child_mask"])
    np.testing.assert_array_equal(f["nodes"]["begin"], exp["node_begin"])
    np.testing.assert_array_equal(f["nodes"]["count"], exp["node_count"])
    np.testing.assert_array_equal(f["xyz"].view(np.uint32), want.view(np.uint32))
    if stride:
        np.testing.assert_array_equal(f["color"], color[order])
    job.release()
