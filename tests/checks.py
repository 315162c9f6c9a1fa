"""Independent checks of a build result (test helpers; import neither the oracle
nor the library).

* numpy reductions that pin individual steps: bounding box, float32
  quantisation (emulated through exact float64 arithmetic plus one rounding),
  count grid (np.bincount), pyramid (reshape-sum), chunk maximality,
  perm (np.argsort(kind="stable")), per-node winners (np.unique).
* a brute-force definitional octree for tiny clouds, written level by level
  with dictionaries (a different structure from the recursive oracle);
* the structural invariants every result must satisfy.
"""
from __future__ import annotations

from collections import defaultdict

import numpy as np

K = 21
UMAX = (1 << K) - 1


def ilog2(v: int) -> int:
    l = 0
    while (1 << l) < v:
        l += 1
    return l


# ---- step 1 ------------------------------------------------------------------

def bbox_numpy(x, y, z):
    lo = np.array([x.min(), y.min(), z.min()], dtype=np.float32)
    hi = np.array([x.max(), y.max(), z.max()], dtype=np.float32)
    return lo, hi


def quantize_emulated(a: np.ndarray, lo: np.float32, scale: np.float32) -> np.ndarray:
    """Fine coordinate through float64: a - lo and the product of two float32
    values are exact in float64 (for the magnitudes used here), so converting
    each to float32 once applies exactly one IEEE round-to-nearest-even, as a
    float32 subtraction and multiplication do."""
    d = (a.astype(np.float64) - np.float64(lo)).astype(np.float32)
    t = (d.astype(np.float64) * np.float64(scale)).astype(np.float32)
    with np.errstate(invalid="ignore"):
        f = np.floor(t.astype(np.float64))
    f = np.where(np.isnan(f) | (f < 0), 0, f)
    f = np.minimum(f, UMAX)
    return f.astype(np.uint32)


def morton_keys(cx: np.ndarray, cy: np.ndarray, cz: np.ndarray, level: int) -> np.ndarray:
    k = np.zeros(cx.shape[0], dtype=np.uint64)
    for b in range(level - 1, -1, -1):
        k = (k << np.uint64(3)) | (((cx >> b) & 1).astype(np.uint64) << np.uint64(2)) \
            | (((cy >> b) & 1).astype(np.uint64) << np.uint64(1)) | ((cz >> b) & 1).astype(np.uint64)
    return k


def morton_decode(key: int, level: int):
    cx = cy = cz = 0
    for b in range(level):
        cz |= ((key >> (3 * b)) & 1) << b
        cy |= ((key >> (3 * b + 1)) & 1) << b
        cx |= ((key >> (3 * b + 2)) & 1) << b
    return cx, cy, cz


def count_grid_numpy(u: np.ndarray, G: int) -> np.ndarray:
    g = ilog2(G)
    c = u >> np.uint32(K - g)
    flat = (c[:, 0].astype(np.int64) * G + c[:, 1]) * G + c[:, 2]
    return np.bincount(flat, minlength=G ** 3).astype(np.uint32)


def pyramid_numpy(count_grid: np.ndarray, G: int):
    g = ilog2(G)
    levels = [None] * (g + 1)
    levels[g] = count_grid.reshape(G, G, G).astype(np.int64)
    for l in range(g - 1, -1, -1):
        s = 1 << l
        levels[l] = levels[l + 1].reshape(s, 2, s, 2, s, 2).sum(axis=(1, 3, 5))
    return levels


# ---- step 2/3 -----------------------------------------------------------------

def check_chunks(res: dict, u: np.ndarray, G: int, C: int):
    """Chunks are the maximal pyramid nodes with 0 < count <= C (finest cells may
    exceed C), disjoint, covering, in Morton pre-order, begins = prefix sums;
    perm is exactly the stable argsort of the per-point chunk id."""
    g = ilog2(G)
    pyr = pyramid_numpy(res["count_grid"], G)
    lv = res["chunk_level"].astype(np.int64)
    ky = res["chunk_key"].astype(np.uint64)
    ct = res["chunk_count"].astype(np.int64)
    bg = res["chunk_begin"].astype(np.int64)
    n = u.shape[0]
    assert ct.sum() == n
    if lv.size:
        assert bg[0] == 0 and np.all(bg[1:] == np.cumsum(ct)[:-1])
    over = False
    for l, k, c in zip(lv.tolist(), ky.tolist(), ct.tolist()):
        cx, cy, cz = morton_decode(int(k), l)
        assert pyr[l][cx, cy, cz] == c and c > 0
        assert c <= C or l == g
        over |= c > C
        if l > 0:
            assert pyr[l - 1][cx // 2, cy // 2, cz // 2] > C
    assert bool(res["chunk_oversized_any"]) == over
    # pre-order: start of each chunk on the finest level strictly increases
    start = [int(k) << (3 * (g - l)) for l, k in zip(lv.tolist(), ky.tolist())]
    assert all(a < b for a, b in zip(start, start[1:]))
    # per-point chunk id from the chunk table (coverage + disjointness)
    fine = morton_keys(u[:, 0] >> (K - g), u[:, 1] >> (K - g), u[:, 2] >> (K - g), g)
    start_a = np.array(start, dtype=np.uint64)
    end_a = np.array([(int(k) + 1) << (3 * (g - l)) for l, k in zip(lv.tolist(), ky.tolist())], dtype=np.uint64)
    cid = np.searchsorted(start_a, fine, side="right") - 1
    assert np.all(cid >= 0) and np.all(fine < end_a[cid]) and np.all(fine >= start_a[cid])
    np.testing.assert_array_equal(res["perm"], np.argsort(cid, kind="stable").astype(np.uint32))


# ---- step 4 ------------------------------------------------------------------

def brute_force_octree(u: np.ndarray, S: int, L: int):
    """Membership rule applied level by level with dictionaries: at depth d the
    surviving points are grouped by node; a node with at most L points or at
    the deepest depth keeps them all; otherwise each occupied cell of its S^3
    grid keeps its lowest index and the rest survive to depth d + 1.
    Returns {(depth, morton key): sorted list of indices} and child masks."""
    s = ilog2(S)
    dmax = K - s
    n = u.shape[0]
    alive = list(range(n))
    final = {}
    d = 0
    while alive:
        groups = defaultdict(list)
        for i in alive:  # ascending
            groups[(int(u[i, 0]) >> (K - d), int(u[i, 1]) >> (K - d), int(u[i, 2]) >> (K - d))].append(i)
        nxt = []
        for nk, R in groups.items():
            if len(R) <= L or d == dmax:
                final.setdefault((d, nk), []).extend(R)
                continue
            winner = {}
            sh = K - d - s
            for i in R:
                c = ((int(u[i, 0]) >> sh) & (S - 1), (int(u[i, 1]) >> sh) & (S - 1), (int(u[i, 2]) >> sh) & (S - 1))
                if c not in winner:
                    winner[c] = i
                    final.setdefault((d, nk), []).append(i)
                else:
                    nxt.append(i)
        alive = sorted(nxt)
        d += 1
    nodes = {}
    for (dd, (cx, cy, cz)), pts in final.items():
        key = int(morton_keys(np.array([cx]), np.array([cy]), np.array([cz]), dd)[0])
        nodes[(dd, key)] = sorted(pts)
    masks = {}
    for (dd, key) in nodes:
        m = 0
        for o in range(8):
            if (dd + 1, key * 8 + o) in nodes:
                m |= 1 << o
        masks[(dd, key)] = m
    return nodes, masks


def octree_as_dict(res: dict):
    nodes = {}
    masks = {}
    for i in range(res["node_depth"].shape[0]):
        d = int(res["node_depth"][i])
        k = int(res["node_key"][i])
        b = int(res["node_begin"][i])
        c = int(res["node_count"][i])
        nodes[(d, k)] = res["node_points"][b:b + c].tolist()
        masks[(d, k)] = int(res["node_child_mask"][i])
    return nodes, masks


def check_octree_invariants(res: dict, u: np.ndarray, S: int, L: int):
    """I4 partition, I5 distinct kept cells, I6 minimality (np.unique winners of
    the reaching set), I7 inside node bounds, I8 leaf size, I9 masks/nesting,
    plus (depth, key) order, ascending lists and prefix-sum begins."""
    s = ilog2(S)
    dmax = K - s
    n = u.shape[0]
    dep = res["node_depth"].astype(np.int64)
    key = res["node_key"].astype(np.uint64)
    cnt = res["node_count"].astype(np.int64)
    beg = res["node_begin"].astype(np.int64)
    pts = res["node_points"]
    nn = dep.shape[0]
    assert cnt.sum() == n
    if nn:
        assert beg[0] == 0 and np.all(beg[1:] == np.cumsum(cnt)[:-1])
        order = np.lexsort((key, dep))
        assert np.all(order == np.arange(nn)), "nodes not in (depth, key) order"
        pairs = list(zip(dep.tolist(), key.tolist()))
        assert len(set(pairs)) == nn
    assert np.array_equal(np.sort(pts), np.arange(n, dtype=pts.dtype)), "I4: not a partition"
    assert np.all(cnt > 0)
    node_of = np.empty(n, dtype=np.int64)
    for i in range(nn):
        seg = pts[beg[i]:beg[i] + cnt[i]]
        assert np.all(np.diff(seg.astype(np.int64)) > 0), "points not ascending in a node"
        node_of[seg] = i
    # I7: every point lies inside its node
    d_of = dep[node_of]
    for d in np.unique(d_of).tolist():
        sel = np.nonzero(d_of == d)[0]
        kk = morton_keys(u[sel, 0] >> (K - d), u[sel, 1] >> (K - d), u[sel, 2] >> (K - d), d)
        assert np.array_equal(kk, key[node_of[sel]]), "I7: point outside its node"
    # I9: masks match the existing children and every non-root node has a parent
    index = {p: i for i, p in enumerate(zip(dep.tolist(), key.tolist()))}
    for i, (d, k) in enumerate(zip(dep.tolist(), key.tolist())):
        m = 0
        for o in range(8):
            if (d + 1, k * 8 + o) in index:
                m |= 1 << o
        assert m == int(res["node_child_mask"][i]), "I9: child mask"
        if d > 0:
            assert (d - 1, k >> 3) in index, "I9: orphan node"
    # I5/I6/I8 per node, using the reaching set R = the node's points plus every
    # point that ends deeper inside the node's cube
    node_index = {p: i for i, p in enumerate(zip(dep.tolist(), key.tolist()))}
    for d in np.unique(dep).tolist():
        sel = np.nonzero(d_of >= d)[0]
        kk = morton_keys(u[sel, 0] >> (K - d), u[sel, 1] >> (K - d), u[sel, 2] >> (K - d), d)
        order = np.argsort(kk, kind="stable")
        sel = sel[order]
        kk = kk[order]
        uniq, starts = np.unique(kk, return_index=True)
        ends = np.append(starts[1:], kk.shape[0])
        for k, a, b in zip(uniq.tolist(), starts.tolist(), ends.tolist()):
            i = node_index[(d, k)]
            R = np.sort(sel[a:b].astype(np.int64))
            seg = pts[beg[i]:beg[i] + cnt[i]].astype(np.int64)
            m = int(res["node_child_mask"][i])
            if R.size <= L or d == dmax:
                assert m == 0 and np.array_equal(R, seg), "I8: leaf must hold its whole reaching set"
                continue
            sh = K - d - s
            cell = (((u[R, 0] >> sh) & (S - 1)).astype(np.int64) * S + ((u[R, 1] >> sh) & (S - 1))) * S \
                + ((u[R, 2] >> sh) & (S - 1))
            _, first = np.unique(cell, return_index=True)
            assert np.array_equal(np.sort(R[first]), seg), "I5/I6: winners differ from the reaching set's"


def h64_numpy(i: np.ndarray) -> np.ndarray:
    """The preview hash, vectorised (pinned by the known answers)."""
    phi = np.uint64(0x9E3779B97F4A7C15)
    h = i.astype(np.uint64)
    with np.errstate(over="ignore"):
        h ^= h >> np.uint64(31)
        h *= phi
        h ^= h >> np.uint64(29)
        h *= phi
        h ^= h >> np.uint64(32)
    return h


def check_preview(res: dict, n: int, M: int):
    idx = res["preview_index"].astype(np.int64)
    exp = np.nonzero(h64_numpy(np.arange(n, dtype=np.uint64)) % np.uint64(M) == 0)[0]
    np.testing.assert_array_equal(idx, exp)
