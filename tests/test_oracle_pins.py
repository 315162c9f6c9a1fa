"""Pins of the CPU oracle against values fixed outside it: the hand-worked
example, the hash known answers, numpy library routines, a brute-force
definitional octree on tiny clouds, closed forms of the uniform workload,
special cases and metamorphic relations."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from checks import (brute_force_octree, bbox_numpy, check_chunks, check_octree_invariants,
                    check_preview, count_grid_numpy, h64_numpy, octree_as_dict, quantize_emulated)

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _run(c, G, C, S, L, M, bbox=None):
    r = oracle.build_octree(c.x, c.y, c.z, oracle.Params(G, C, S, L, M, bbox))
    assert r["status"] == oracle.OK
    return r


def _full_check(c, r, G, C, S, L, M):
    lo, hi = bbox_numpy(c.x, c.y, c.z)
    np.testing.assert_array_equal(r["bbox_min"], lo)
    np.testing.assert_array_equal(r["bbox_max"], hi)
    u = np.stack([quantize_emulated(a, r["bbox_min"][k], r["scale"]) for k, a in enumerate((c.x, c.y, c.z))], 1)
    np.testing.assert_array_equal(r["u"], u)
    np.testing.assert_array_equal(r["count_grid"], count_grid_numpy(u, G))
    check_chunks(r, u, G, C)
    check_octree_invariants(r, u, S, L)
    check_preview(r, c.n, M)
    return u


def test_worked_example():
    ex = json.load(open(os.path.join(GOLD, "worked_example.json")))
    pts = np.array(ex["points"], dtype=np.float32)
    p = ex["params"]
    r = oracle.build_octree(pts[:, 0], pts[:, 1], pts[:, 2],
                            oracle.Params(p["count_grid"], p["max_points_per_chunk"], p["subsample_grid"],
                                          p["leaf_capacity"], p["preview_modulus"]))
    assert r["status"] == oracle.OK
    for k in ("bbox_min", "bbox_max", "u", "count_grid", "chunk_level", "chunk_key", "chunk_count",
              "chunk_begin", "perm", "node_depth", "node_key", "node_child_mask", "node_begin",
              "node_count", "node_points", "preview_index"):
        np.testing.assert_array_equal(np.asarray(r[k]).astype(np.int64), np.array(ex[k], dtype=np.int64), err_msg=k)
    assert float(r["cube_size"]) == ex["cube_size"]
    assert float(r["scale"]) == ex["scale"]
    assert [oracle.h64(i) % 4 for i in range(8)] == ex["h64_mod4_first8"]


def test_h64_known_answers():
    ka = json.load(open(os.path.join(GOLD, "h64_known_answers.json")))
    for i, h in ka["h64"].items():
        assert oracle.h64(int(i)) == int(h, 16)
        assert int(h64_numpy(np.array([int(i)], dtype=np.uint64))[0]) == int(h, 16)
    assert oracle.h64(0) == 0
    pv = ka["preview_n1000000_m64"]
    r = oracle.build_octree(np.zeros(1_000_000, np.float32), np.zeros(1_000_000, np.float32),
                            np.zeros(1_000_000, np.float32), oracle.Params(1, 10**9, 1, 10**9, 64))
    idx = r["preview_index"]
    assert idx.shape[0] == pv["count"]
    assert idx[:10].tolist() == pv["first10"] and idx[-3:].tolist() == pv["last3"]


def test_uniform_1m_closed_forms():
    """Uniform 1M points, G=64, C=100k, S=32, L=10k: all 64 level-2 chunks
    (level-2 cells hold ~15.6k <= C, level-1 ~125k > C); the root's 32^3 grid is
    fully occupied (P(empty) = e^-30.5 per cell); a depth-1 node receives
    125000 - 4096 points and keeps about 32768 (1 - e^-3.69); depth-2 nodes receive about 11.1k > L and keep about
    9.4k; the 512 depth-3 nodes are leaves of about 211 points: 585 nodes."""
    c = synth.uniform_1m()
    r = _run(c, 64, 100_000, 32, 10_000, 64)
    assert r["chunk_level"].shape[0] == 64 and np.all(r["chunk_level"] == 2)
    assert r["chunk_oversized_any"] == 0
    dep = r["node_depth"]
    assert np.bincount(dep).tolist() == [1, 8, 64, 512]
    assert r["node_count"][0] == 32768
    d1 = r["node_count"][dep == 1]
    assert np.all(np.abs(d1.astype(float) - 32768 * (1 - math.exp(-(1e6 / 8 - 4096) / 32768))) < 150)
    d3 = r["node_count"][dep == 3]
    assert 150 < d3.mean() < 280 and d3.max() <= 10_000
    assert r["preview_index"].shape[0] == 15761
    _full_check(c, r, 64, 100_000, 32, 10_000, 64)


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_tiny(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 400))
    kind = seed % 4
    if kind == 0:
        c = synth.uniform(n, seed=seed)
    elif kind == 1:
        c = synth.planes(n, seed=seed, num_planes=3)
    elif kind == 2:
        c = synth.clusters(n, seed=seed, num_clusters=4)
    else:  # heavy duplicates on a coarse lattice
        base = synth.uniform(n, seed=seed)
        q = np.float32(0.25)
        c = synth.Cloud(np.floor(base.x / q) * q, np.floor(base.y / q) * q, np.floor(base.z / q) * q)
    G = int(2 ** rng.integers(0, 4))
    C = int(rng.integers(1, max(2, n)))
    S = int(2 ** rng.integers(0, 3))
    L = int(rng.integers(1, 30))
    M = int(rng.integers(1, 9))
    r = _run(c, G, C, S, L, M)
    u = _full_check(c, r, G, C, S, L, M)
    nodes, masks = brute_force_octree(u, S, L)
    got, gmask = octree_as_dict(r)
    assert got == nodes
    assert gmask == masks


def test_special_cases():
    c = synth.uniform(5000, seed=7)
    # L >= N: one root leaf holding 0..N-1
    r = _run(c, 8, 100, 8, 5000, 3)
    assert r["node_depth"].tolist() == [0] and r["node_points"].tolist() == list(range(5000))
    # C >= N: one chunk (the root) and perm = identity
    r = _run(c, 8, 5000, 8, 10, 3)
    assert r["chunk_level"].tolist() == [0] and r["perm"].tolist() == list(range(5000))
    # S = 1: every inner node keeps exactly its lowest reaching index
    r = _run(c, 8, 100, 1, 10, 3)
    dep, cnt, beg = r["node_depth"], r["node_count"], r["node_begin"]
    inner = r["node_child_mask"] != 0
    assert np.all(cnt[inner] == 1)
    assert r["node_points"][beg[0]] == 0
    # M = 1: preview = 0..N-1
    r = _run(c, 8, 100, 8, 10, 1)
    assert r["preview_index"].tolist() == list(range(5000))
    # G = 1: one chunk
    r = _run(c, 1, 10, 8, 10, 3)
    assert r["chunk_level"].tolist() == [0] and r["chunk_oversized_any"] == 1


def test_empty_and_single():
    e = np.zeros(0, np.float32)
    r = oracle.build_octree(e, e, e, oracle.Params(8, 10, 8, 10, 4))
    assert r["status"] == oracle.OK
    assert r["node_depth"].shape[0] == 0 and r["chunk_level"].shape[0] == 0
    assert r["preview_index"].shape[0] == 0 and int(r["count_grid"].sum()) == 0
    one = np.array([3.5], np.float32)
    r = oracle.build_octree(one, one, one, oracle.Params(8, 10, 8, 10, 4))
    assert r["scale"] == 0 and r["u"].tolist() == [[0, 0, 0]]
    assert r["node_depth"].tolist() == [0] and r["node_points"].tolist() == [0]
    assert r["chunk_level"].tolist() == [0]


def test_identical_points_reach_deepest_depth():
    """All points equal: scale 0, every u = 0; each inner node keeps one point
    (one occupied cell) and the chain ends at depth 21 - s with the rest."""
    n = 300
    v = np.full(n, 1.25, np.float32)
    S, L = 4, 10
    r = _run(synth.Cloud(v, v, v), 4, 50, S, L, 7)
    dmax = 21 - 2
    assert r["node_depth"].tolist() == list(range(dmax + 1))
    assert r["node_count"].tolist() == [1] * dmax + [n - dmax]
    assert r["node_points"].tolist() == list(range(n))
    assert r["node_child_mask"].tolist() == [1] * dmax + [0]
    assert r["chunk_oversized_any"] == 1


def test_octree_independent_of_grid_and_chunk_size():
    c = synth.planes(20_000, seed=11, num_planes=6)
    ref = _run(c, 64, 100_000, 16, 500, 5)
    for G, C in ((1, 1), (4, 700), (32, 3000), (128, 20_000)):
        r = _run(c, G, C, 16, 500, 5)
        for k in ("node_depth", "node_key", "node_child_mask", "node_begin", "node_count", "node_points",
                  "preview_index"):
            np.testing.assert_array_equal(r[k], ref[k], err_msg=k)


def test_power_of_two_scaling_invariance():
    c = synth.clusters(20_000, seed=5, num_clusters=7)
    ref = _run(c, 16, 2000, 8, 300, 6)
    for k2 in (-3, 5):
        f = np.float32(2.0 ** k2)
        r = _run(synth.Cloud(c.x * f, c.y * f, c.z * f), 16, 2000, 8, 300, 6)
        for k in ("u", "count_grid", "perm", "node_key", "node_points", "node_count"):
            np.testing.assert_array_equal(r[k], ref[k], err_msg=k)


def test_given_bbox_equals_computed():
    c = synth.planes(30_000, seed=9, num_planes=10)
    lo, hi = bbox_numpy(c.x, c.y, c.z)
    a = _run(c, 32, 4000, 16, 400, 8)
    b = _run(c, 32, 4000, 16, 400, 8, bbox=(tuple(lo.tolist()), tuple(hi.tolist())))
    assert b["n_outside"] == 0
    for k in ("u", "count_grid", "perm", "node_key", "node_points"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    # a smaller box: outside points clamp and are counted
    mid = (lo + hi) / 2
    r = _run(c, 32, 4000, 16, 400, 8, bbox=(tuple(lo.tolist()), tuple(mid.tolist())))
    outside = np.any(np.stack([c.x > mid[0], c.y > mid[1], c.z > mid[2]]), axis=0).sum()
    assert r["n_outside"] == outside
    assert int(r["u"].max()) == (1 << 21) - 1


def test_errors():
    x = np.array([0.0, 1.0, np.nan], np.float32)
    r = oracle.build_octree(x, x, x, oracle.Params(8, 10, 8, 10, 4))
    assert r["status"] == oracle.ERR_NONFINITE
    x = np.array([0.0, np.inf], np.float32)
    assert oracle.build_octree(x, x, x, oracle.Params(8, 10, 8, 10, 4))["status"] == oracle.ERR_NONFINITE
    ok = np.zeros(4, np.float32)
    for p in (oracle.Params(3, 10, 8, 10, 4), oracle.Params(1024, 10, 8, 10, 4),
              oracle.Params(8, 0, 8, 10, 4), oracle.Params(8, 10, 512, 10, 4),
              oracle.Params(8, 10, 6, 10, 4), oracle.Params(8, 10, 8, 0, 4), oracle.Params(8, 10, 8, 10, 0)):
        assert oracle.build_octree(ok, ok, ok, p)["status"] == oracle.ERR_INVALID_ARG


def test_signed_zero_extremes_reported_as_plus_zero():
    """A box extreme of -0.0 is reported as +0.0 whatever the point order."""
    for xs in ([-0.0, 0.0, 1.0], [0.0, -0.0, 1.0], [1.0, -0.0, 0.0]):
        x = np.array(xs, np.float32)
        m = np.array([-1.0, -0.0, -0.0], np.float32)  # max of this axis is a zero
        r = oracle.build_octree(x, m, x.copy(), oracle.Params(4, 10, 4, 1, 2))
        assert r["status"] == oracle.OK
        assert np.signbit(r["bbox_min"][0]) == False and r["bbox_min"][0] == 0.0
        assert np.signbit(r["bbox_max"][1]) == False and r["bbox_max"][1] == 0.0


def test_node_ordered_points_inside_their_nodes():
    """The export order (the oracle's node_points) puts every point inside the
    cube of the node it is listed under: its fine coordinates shifted to the
    node's depth equal the node's key (checked on an independent numpy
    quantisation)."""
    from checks import morton_keys
    c = synth.planes(30_000, seed=7, num_planes=6)
    r = oracle.build_octree(c.x, c.y, c.z, oracle.Params(32, 4_000, 16, 500, 8))
    lo, hi = bbox_numpy(c.x, c.y, c.z)
    side = np.float32(max(hi - lo))
    scale = np.float32(2.0 ** 21 / float(side))
    u = np.stack([quantize_emulated(a, lo[k], scale) for k, a in enumerate((c.x, c.y, c.z))], 1)
    for k in range(r["node_depth"].shape[0]):
        d = int(r["node_depth"][k])
        b, cnt = int(r["node_begin"][k]), int(r["node_count"][k])
        pts = r["node_points"][b:b + cnt].astype(np.int64)
        q = u[pts] >> (21 - d)
        keys = morton_keys(q[:, 0], q[:, 1], q[:, 2], d)
        assert np.all(keys == r["node_key"][k]), k
