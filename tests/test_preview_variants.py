"""Pins of the oracle's preview variants (step 5): the exact stride of the
fixed-target decimation (section "Results" decimates to one million points)
and the spatially constrained sampler of section "Future Work" (one pick per
occupied count-grid cell, the point of least H64).  Checked against a
hand-worked fixture, closed forms, special cases and a brute force over
per-cell point lists on tiny clouds."""
import json
import os
from collections import defaultdict

import numpy as np
import pytest

import oracle
import synth
from checks import bbox_numpy, h64_numpy, quantize_emulated

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _run(c, G, M, preview, C=100_000, S=32, L=10_000):
    r = oracle.build_octree(c.x, c.y, c.z, oracle.Params(G, C, S, L, M, None, preview))
    assert r["status"] == oracle.OK
    return r


def test_worked_example_variants():
    ex = json.load(open(os.path.join(GOLD, "preview_grid_example.json")))
    pts = np.array(ex["points"], dtype=np.float32)
    c = synth.Cloud(pts[:, 0].copy(), pts[:, 1].copy(), pts[:, 2].copy())
    p = ex["params"]
    for mode, key in (("grid", "preview_grid"), ("stride", "preview_stride_m4"), ("hash", "preview_hash_m4")):
        r = _run(c, p["count_grid"], p["preview_modulus"], mode, p["max_points_per_chunk"], p["subsample_grid"],
                 p["leaf_capacity"])
        assert r["preview_index"].tolist() == ex[key], mode


@pytest.mark.parametrize("M", [1, 2, 7, 64, 10_007, 10_008, 99_999])
def test_stride_closed_form(M):
    n = 10_007
    c = synth.uniform(n, seed=3)
    r = _run(c, 16, M, "stride")
    idx = r["preview_index"]
    assert idx.shape[0] == -(-n // M)
    np.testing.assert_array_equal(idx, np.arange(0, n, M, dtype=np.uint32))


def _cells(c, G):
    """Row-major count-grid cell of every point, from the pinned numpy box and
    quantisation (checked against the oracle's fine coordinates)."""
    lo, _ = bbox_numpy(c.x, c.y, c.z)
    r = oracle.build_octree(c.x, c.y, c.z, oracle.Params(G, 10**9, 1, 10**9, 1))
    u = np.stack([quantize_emulated(a, lo[k], r["scale"]) for k, a in enumerate((c.x, c.y, c.z))], 1)
    np.testing.assert_array_equal(u, r["u"])
    sh = 21 - int(np.log2(G))
    cu = (u >> sh).astype(np.int64)
    return (cu[:, 0] * G + cu[:, 1]) * G + cu[:, 2]


@pytest.mark.parametrize("seed,G,kind", [(0, 4, "uniform"), (1, 8, "clusters"), (2, 2, "planes"), (3, 16, "uniform"),
                                         (4, 1, "clusters")])
def test_grid_brute_force(seed, G, kind):
    """Per-cell point lists built in plain Python; the pick of each list is its
    argmin of the (separately pinned) vectorised hash."""
    n = 700
    c = {"uniform": synth.uniform, "clusters": lambda n, seed: synth.clusters(n, seed=seed, num_clusters=3),
         "planes": lambda n, seed: synth.planes(n, seed=seed, num_planes=3)}[kind](n, seed=seed)
    cell = _cells(c, G)
    h = h64_numpy(np.arange(n, dtype=np.uint64))
    lists = defaultdict(list)
    for i in range(n):
        lists[int(cell[i])].append(i)
    exp = sorted(min(pts, key=lambda i: int(h[i])) for pts in lists.values())
    r = _run(c, G, 5, "grid")
    assert r["preview_index"].tolist() == exp
    assert r["preview_index"].shape[0] == int(np.count_nonzero(r["count_grid"]))


def test_grid_special_cases():
    c = synth.clusters(5_000, seed=11, num_clusters=4)
    # one cell: only index 0 (H64(0) = 0 is the least value)
    assert _run(c, 1, 3, "grid")["preview_index"].tolist() == [0]
    # index 0 is picked in every grid, whatever its cell holds
    for G in (2, 8, 64):
        assert _run(c, G, 3, "grid")["preview_index"][0] == 0
    # eight points at the cube corners, G = 2: every point alone in its cell
    k = np.array([[(a >> 2) & 1, (a >> 1) & 1, a & 1] for a in range(8)], np.float32)
    rng = np.random.default_rng(5)
    k = k[rng.permutation(8)]
    corners = synth.Cloud(k[:, 0].copy(), k[:, 1].copy(), k[:, 2].copy())
    assert _run(corners, 2, 3, "grid")["preview_index"].tolist() == list(range(8))
    # all points identical: one pick
    same = synth.Cloud(np.full(100, 2.5, np.float32), np.full(100, -1.0, np.float32), np.full(100, 7.0, np.float32))
    assert _run(same, 64, 3, "grid")["preview_index"].tolist() == [0]
    # empty cloud: empty preview in every mode
    e = synth.Cloud(np.zeros(0, np.float32), np.zeros(0, np.float32), np.zeros(0, np.float32))
    for mode in ("hash", "stride", "grid"):
        assert _run(e, 8, 3, mode)["preview_index"].shape[0] == 0


def test_variants_leave_the_tree_alone():
    c = synth.planes(20_000, seed=9, num_planes=5)
    base = _run(c, 32, 16, "hash")
    for mode in ("stride", "grid"):
        r = _run(c, 32, 16, mode)
        for k in ("perm", "node_key", "node_points", "chunk_key", "count_grid"):
            np.testing.assert_array_equal(r[k], base[k], err_msg=f"{mode}: {k}")


def test_grid_invariant_to_point_order_within_value():
    """The pick of a cell depends only on which indices the cell holds:
    swapping the coordinates of two points of one cell keeps the preview.
    Every pick is the least hash of its cell, and no two picks share one."""
    c = synth.uniform(2_000, seed=21)
    G = 4
    base = _run(c, G, 1, "grid")["preview_index"]
    cell = _cells(c, G)
    h = h64_numpy(np.arange(c.n, dtype=np.uint64))
    same_cell = np.nonzero(cell == cell[7])[0]
    j = int(same_cell[same_cell != 7][0])
    x, y, z = c.x.copy(), c.y.copy(), c.z.copy()
    for a in (x, y, z):
        a[[7, j]] = a[[j, 7]]
    sw = synth.Cloud(x, y, z)
    np.testing.assert_array_equal(_run(sw, G, 1, "grid")["preview_index"], base)
    # a pick is the least hash of its cell and no two picks share a cell
    assert len(set(cell[base].tolist())) == base.shape[0]
    for i in base.tolist():
        assert h[i] == h[cell == cell[i]].min()


def test_invalid_mode_rejected():
    with pytest.raises(KeyError):
        _run(synth.uniform(10, seed=1), 4, 2, "voxel")
