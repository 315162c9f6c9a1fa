"""Pins of the view-selection oracle (section "Octree Rendering"): a
hand-worked tree, closed forms (no clipping and no size limit draws every
node; an infinite limit draws the root alone), axis-aligned clipping against
exactly representable cube bounds, the perspective helper's planes, and the
traversal against a per-node rule (every ancestor visible and refined)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from checks import morton_decode
from oracle import view as V

GOLD = os.path.join(os.path.dirname(__file__), "golden")
OPEN = ((0.0, 0.0, 0.0, 1.0),) * 6   # six planes that keep everything


def test_worked_example():
    ex = json.load(open(os.path.join(GOLD, "view_worked_example.json")))
    args = (ex["node_depth"], ex["node_key"], ex["node_count"], ex["bbox_min"], ex["cube_size"])
    clip = (tuple(ex["clip"]),) + OPEN[:5]
    for k, (d, key) in enumerate(zip(ex["node_depth"][:4], ex["node_key"][:4])):
        _, _, ctr, r = V.node_box(d, V.cell_of(key, d), ex["bbox_min"], ex["cube_size"])
        s = V.screen_size(ctr, r, V.View(tuple(ex["eye"]), OPEN, ex["proj_factor"], 0.0))
        assert math.isclose(s, ex["sizes"][k], rel_tol=1e-9)
    for key, planes, mn in (("selected_min40_clip", clip, 40.0), ("selected_min20_clip", clip, 20.0),
                            ("selected_min20_noclip", OPEN, 20.0), ("selected_min50_noclip", OPEN, 50.0)):
        sel, pts = V.select_nodes(*args, V.View(tuple(ex["eye"]), planes, ex["proj_factor"], mn))
        assert sel == ex[key], key
        assert pts == sum(ex["node_count"][i] for i in sel)


@pytest.fixture(scope="module")
def tree():
    c = synth.clusters(30_000, seed=8, num_clusters=6)
    r = oracle.build_octree(c.x, c.y, c.z, oracle.Params(16, 5_000, 8, 200, 64))
    assert r["status"] == oracle.OK and r["node_depth"].shape[0] > 50
    return r


def _args(r):
    return r["node_depth"], r["node_key"], r["node_count"], r["bbox_min"], float(r["cube_size"])


def test_closed_forms(tree):
    n = tree["node_depth"].shape[0]
    eye = tuple(float(v) for v in tree["bbox_min"] - 1e6)
    sel, pts = V.select_nodes(*_args(tree), V.View(eye, OPEN, 1000.0, 0.0))
    assert sel == list(range(n)) and pts == tree["n"]
    sel, pts = V.select_nodes(*_args(tree), V.View(eye, OPEN, 1000.0, math.inf))
    assert sel == [0] and pts == int(tree["node_count"][0])
    # a plane that keeps nothing
    sel, _ = V.select_nodes(*_args(tree), V.View(eye, ((0.0, 0.0, 0.0, -1.0),) + OPEN[:5], 1000.0, 0.0))
    assert sel == []
    # eye inside the root's bounding sphere: infinite size, so even an infinite
    # limit refines the root
    mid = tuple(float(tree["bbox_min"][a]) + float(tree["cube_size"]) / 2 for a in range(3))
    sel, _ = V.select_nodes(*_args(tree), V.View(mid, OPEN, 1e-9, math.inf))
    assert sel[0] == 0 and any(tree["node_depth"][i] == 1 for i in sel)


def test_axis_aligned_clipping_exact():
    """Cube [0, 64]^3: node bounds are exact, so a half-space x >= t keeps
    exactly the nodes whose upper x bound reaches t (with no size limit)."""
    c = synth.uniform(20_000, seed=3, lo=0.0, hi=64.0)
    x = c.x.copy(); x[0] = 0.0; x[1] = 64.0
    r = oracle.build_octree(x, c.y, c.z, oracle.Params(8, 2_000, 4, 100, 64))
    assert r["status"] == oracle.OK and float(r["cube_size"]) == 64.0 and r["bbox_min"][0] == 0.0
    d, k = r["node_depth"], r["node_key"]
    for t in (0.0, 5.0, 16.0, 31.5, 32.0, 47.25, 63.0, 64.0, 64.5):
        for sign in (1.0, -1.0):
            plane = (sign, 0.0, 0.0, -sign * t)   # sign +1: x >= t, -1: x <= t
            sel, _ = V.select_nodes(d, k, r["node_count"], r["bbox_min"], 64.0,
                                    V.View((-1e3, 0.0, 0.0), (plane,) + OPEN[:5], 1.0, 0.0))
            exp = []
            for i in range(d.shape[0]):
                cx = morton_decode(int(k[i]), int(d[i]))[0]
                lo, hi = cx * 64.0 / 2 ** int(d[i]), (cx + 1) * 64.0 / 2 ** int(d[i])
                # a node is drawn iff it and all its ancestors touch the half-space;
                # ancestors contain it, so the node's own bounds decide
                exp.append(i) if (hi >= t if sign > 0 else lo <= t) else None
            assert sel == exp, (t, sign)


def test_perspective_planes():
    v = V.perspective_view((0.0, 0.0, 0.0), (0.0, 0.0, -1.0), (0.0, 1.0, 0.0), 60.0, 2.0, 0.5, 100.0, 1000.0, 1.0)

    def inside(p):
        return all(((a * p[0] + b * p[1]) + c * p[2]) + e >= 0 for a, b, c, e in v.planes)

    assert inside((0.0, 0.0, -10.0))
    assert not inside((0.0, 0.0, 10.0)) and not inside((0.0, 0.0, -0.1)) and not inside((0.0, 0.0, -101.0))
    th = math.tan(math.radians(30.0))
    assert inside((0.0, 0.99 * th * 10, -10.0)) and not inside((0.0, 1.01 * th * 10, -10.0))
    assert inside((1.98 * th * 10, 0.0, -10.0)) and not inside((2.02 * th * 10, 0.0, -10.0))
    assert math.isclose(v.proj_factor, 1000.0 / (2 * th))


def test_traversal_equals_per_node_rule(tree):
    """Drawn iff every ancestor is visible and refined, and the node is visible."""
    r = tree
    lo = [float(v) for v in r["bbox_min"]]
    side = float(r["cube_size"])
    rng = np.random.default_rng(1)
    for trial in range(6):
        eye = [lo[a] + side * float(rng.uniform(-1.0, 2.0)) for a in range(3)]
        tgt = [lo[a] + side * float(rng.uniform(0.2, 0.8)) for a in range(3)]
        v = V.perspective_view(eye, tgt, (0.0, 0.0, 1.0), float(rng.uniform(20, 90)), 1.5, 0.1, 10 * side, 1080.0,
                               float(rng.choice([0.0, 50.0, 150.0, 400.0])))
        sel, _ = V.select_nodes(*_args(r), v)
        exp = []
        for i in range(r["node_depth"].shape[0]):
            d, k = int(r["node_depth"][i]), int(r["node_key"][i])
            ok = True
            for j in range(d + 1):
                cell = list(morton_decode(k >> (3 * (d - j)), j))
                blo, bhi, ctr, rad = V.node_box(j, cell, lo, side)
                if not V.visible(blo, bhi, v.planes) or (j < d and V.screen_size(ctr, rad, v) < v.min_size):
                    ok = False
                    break
            if ok:
                exp.append(i)
        assert sel == exp, trial
        # closure: the parent of every drawn node is drawn
        drawn = {(int(r["node_depth"][i]), int(r["node_key"][i])) for i in sel}
        assert all(d == 0 or (d - 1, k >> 3) in drawn for d, k in drawn)
