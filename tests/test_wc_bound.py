"""The bound on the number of work chunks that sizes the library's per-(depth,
work chunk) tables, checked on the host against the work-chunk cut computed
here with numpy from its definition (maximal pyramid nodes of at most 4096
points, at levels d0 = max(0, g - s) to g, finest cells above 4096 points
included).  A work chunk deeper than d0 has a parent of more than 4096
points; those parents are disjoint within a level and have at most eight
children each, so there are at most 8^d0 + 8 (g - d0) floor(n / 4097)."""
import numpy as np
import pytest

import synth

CAP = 4096


def level_keys(u, l):
    return ((u[0] >> (21 - l)) << (2 * l)) | ((u[1] >> (21 - l)) << l) | (u[2] >> (21 - l))


def work_chunks(u, g, d0):
    """Number of work chunks of the cut, from the pyramid counts."""
    count = 0
    heavy_parent = None
    for l in range(d0, g + 1):
        k, c = np.unique(level_keys(u, l), return_counts=True)
        if l == d0:
            ok = np.ones(k.shape, bool)
        else:
            kx, ky, kz = k >> (2 * l), (k >> l) & ((1 << l) - 1), k & ((1 << l) - 1)
            pk = ((kx >> 1) << (2 * (l - 1))) | ((ky >> 1) << (l - 1)) | (kz >> 1)
            ok = np.isin(pk, heavy_parent)
        count += int(np.sum(ok & ((c <= CAP) | (l == g))))
        heavy_parent = k[ok & (c > CAP)]
    return count


def fine_coords(cloud):
    pts = [np.asarray(a, np.float64) for a in (cloud.x, cloud.y, cloud.z)]
    lo = [p.min() for p in pts]
    side = max(p.max() - m for p, m in zip(pts, lo)) or 1.0
    return [np.clip(np.floor((p - m) / side * (1 << 21)), 0, (1 << 21) - 1).astype(np.int64) for p, m in zip(pts, lo)]


@pytest.mark.parametrize("kind,n,g,s", [("clusters", 200_000, 7, 7), ("planes", 300_000, 6, 3),
                                        ("uniform", 150_000, 5, 5), ("clusters", 120_000, 9, 4)])
def test_work_chunk_bound(kind, n, g, s):
    if kind == "clusters":
        c = synth.clusters(n, seed=5, num_clusters=40, sigma_frac=0.002)
    elif kind == "planes":
        c = synth.planes(n, seed=6, num_planes=30)
    else:
        c = synth.uniform(n, seed=7)
    d0 = max(0, g - s)
    w = work_chunks(fine_coords(c), g, d0)
    bound = 8 ** d0 + 8 * (g - d0) * (n // (CAP + 1))
    assert 0 < w <= bound, (w, bound)
