"""Single-workgroup builds (fpo_context_set_single_block_max) against the
oracle, element by element, and against the multi-kernel path on the same
cloud: clouds of 1 to 65536 points of every kind, every subsample grid the
path takes, count grids 1 to 64, small leaf capacities (deep trees, many
nodes per depth), a given box with points outside it, both preview
predicates, n = C, the eligibility limits, non-finite inputs, and batches
that put many such clouds in one launch beside larger builds."""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import KEYS, compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctxs():
    import torch
    import paper_2302_05002_amd as fpo
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    on, off = fpo.Context(0), fpo.Context(0)
    on.set_single_block_max(fpo.SINGLE_BLOCK_MAX_POINTS)
    off.set_single_block_max(0)
    yield on, off
    on.close()
    off.close()


def _cloud(kind, n, seed):
    if kind == "uniform":
        return synth.uniform(n, seed=seed)
    if kind == "planes":
        return synth.planes(n, seed=seed, num_planes=7)
    if kind == "clusters":
        return synth.clusters(n, seed=seed, num_clusters=5, sigma_frac=0.002)
    if kind == "same":   # every point at one position: a chain of single-winner nodes down to the last depth
        v = np.full(n, 0.25, dtype=np.float32)
        return synth.Cloud(v.copy(), v.copy(), v.copy())
    if kind == "few":    # many duplicates of a few positions
        rng = np.random.default_rng(seed)
        pos = rng.random((7, 3), dtype=np.float32)
        pick = rng.integers(0, 7, n)
        return synth.Cloud(*(np.ascontiguousarray(pos[pick, a]) for a in range(3)))
    raise ValueError(kind)


def _dev(c):
    import torch
    return tuple(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (c.x, c.y, c.z))


def _both(ctxs, c, p, label):
    """The single-workgroup build equals the oracle and the multi-kernel build."""
    import paper_2302_05002_amd as fpo
    on, off = ctxs
    print(f"[single_block] {label}", flush=True)
    exp = oracle.build_octree(c.x, c.y, c.z, oracle.Params(p.count_grid, p.max_points_per_chunk, p.subsample_grid,
                                                           p.leaf_capacity, p.preview_modulus, p.bbox, p.preview))
    assert exp["status"] == oracle.OK
    x, y, z = _dev(c)
    on.set_timing(True, only=["fused"])
    job = on.submit(x, y, z, p)
    job.wait()
    fused = job.timer("fused")[1]
    got = job.to_numpy()
    job.release()
    on.set_timing(False)
    assert fused == 1, f"{label}: the build did not take the single-workgroup path"
    compare(got, exp, label=label + ": ")
    multi = off.build(x, y, z, p).to_numpy()
    for k in KEYS:
        assert np.array_equal(np.asarray(got[k]), np.asarray(multi[k])), f"{label}: {k} differs between the paths"
    return got


CASES = [
    # kind, n, G, C, S, L, M
    ("uniform", 1, 64, 100_000, 32, 10_000, 64),
    ("uniform", 2, 64, 100_000, 32, 1, 1),
    ("uniform", 63, 8, 100, 4, 1, 3),
    ("uniform", 64, 64, 64, 32, 1, 2),
    ("uniform", 65, 1, 65, 1, 1, 5),
    ("uniform", 1000, 16, 100_000, 8, 20, 7),
    ("uniform", 4097, 64, 100_000, 32, 100, 64),
    ("uniform", 30_000, 64, 100_000, 32, 10_000, 64),
    ("uniform", 65_536, 64, 100_000, 32, 10_000, 64),
    ("uniform", 65_536, 32, 65_536, 16, 1_100, 1),
    ("planes", 20_000, 64, 100_000, 32, 400, 64),
    ("planes", 50_000, 2, 100_000, 2, 10_000, 10),
    ("clusters", 40_000, 64, 100_000, 32, 700, 64),
    ("clusters", 60_000, 4, 100_000, 8, 1_000, 33),
    ("same", 5_000, 64, 100_000, 32, 100, 64),
    ("same", 3_000, 16, 100_000, 1, 50, 4),
    ("few", 20_000, 64, 100_000, 16, 400, 9),
]


@pytest.mark.parametrize("kind,n,G,C,S,L,M", CASES)
def test_single_block_parity(ctxs, kind, n, G, C, S, L, M):
    import paper_2302_05002_amd as fpo
    c = _cloud(kind, n, seed=n % 97 + G)
    _both(ctxs, c, fpo.Params(G, C, S, L, M), f"{kind} n={n} G={G} C={C} S={S} L={L} M={M}")


@pytest.mark.parametrize("S", [1, 2, 4, 8, 16, 32])
def test_every_subsample_grid(ctxs, S):
    import paper_2302_05002_amd as fpo
    c = _cloud("clusters", 25_000, seed=S)
    _both(ctxs, c, fpo.Params(64, 100_000, S, 500, 16), f"clusters S={S}")


@pytest.mark.parametrize("preview", ["hash", "stride"])
def test_given_box_and_previews(ctxs, preview):
    """A given box smaller than the cloud (points clamp to its faces) and both
    preview predicates."""
    import paper_2302_05002_amd as fpo
    c = _cloud("uniform", 12_345, seed=3)
    p = fpo.Params(32, 100_000, 16, 300, 6, ((0.2, 0.1, 0.3), (0.8, 0.7, 0.9)), preview)
    got = _both(ctxs, c, p, f"given box, {preview} preview")
    assert got["n_outside"] > 0


def test_limits_take_the_right_path(ctxs):
    """Just inside each limit the build is one launch; just outside it is the
    multi-kernel path; both equal the oracle."""
    import paper_2302_05002_amd as fpo
    on, _ = ctxs
    c = _cloud("uniform", 6_500, seed=11)
    x, y, z = _dev(c)

    def launches(p):
        on.set_timing(True, only=["fused"])
        job = on.submit(x, y, z, p)
        job.wait()
        k = job.timer("fused")[1]
        got = job.to_numpy()
        job.release()
        on.set_timing(False)
        exp = oracle.build_octree(c.x, c.y, c.z, oracle.Params(p.count_grid, p.max_points_per_chunk, p.subsample_grid,
                                                               p.leaf_capacity, p.preview_modulus))
        compare(got, exp, label=f"{p}: ")
        return k

    n = c.n
    assert launches(fpo.Params(64, n, 32, 200, 8)) == 1            # n = C
    assert launches(fpo.Params(64, n - 1, 32, 200, 8)) == 0        # n = C + 1
    assert launches(fpo.Params(64, n, 32, 99, 8)) == 0             # n / (L + 1) = 65: above 64 nodes per depth
    assert launches(fpo.Params(64, n, 32, 100, 8)) == 1            # n / (L + 1) = 64.4: at the limit
    assert launches(fpo.Params(128, n, 32, 200, 8)) == 0           # G above 64
    assert launches(fpo.Params(64, n, 64, 200, 8)) == 0            # S above 32
    on.set_single_block_max(n - 1)
    try:
        assert launches(fpo.Params(64, n, 32, 200, 8)) == 0        # above the context's limit
    finally:
        on.set_single_block_max(fpo.SINGLE_BLOCK_MAX_POINTS)
    with pytest.raises(fpo.FpoError) as e:
        on.set_single_block_max(fpo.SINGLE_BLOCK_MAX_POINTS + 1)
    assert e.value.status == fpo.FPO_ERR_INVALID_ARG


def test_largest_single_block_cloud(ctxs):
    import paper_2302_05002_amd as fpo
    c = _cloud("planes", fpo.SINGLE_BLOCK_MAX_POINTS, seed=5)
    _both(ctxs, c, fpo.Params(64, 1_000_000, 32, 10_000, 64), "n = 262143")


@pytest.mark.parametrize("given", [False, True])
def test_nonfinite_rejected(ctxs, given):
    import paper_2302_05002_amd as fpo
    on, _ = ctxs
    for bad, at in ((np.nan, 0), (np.inf, 777), (-np.inf, 999)):
        c = _cloud("uniform", 1000, seed=2)
        c.y[at] = bad
        x, y, z = _dev(c)
        box = ((0.0, 0.0, 0.0), (1.0, 1.0, 1.0)) if given else None
        with pytest.raises(fpo.FpoError) as e:
            on.build(x, y, z, fpo.Params(16, 100_000, 8, 100, 8, box))
        assert e.value.status == fpo.FPO_ERR_NONFINITE, (bad, at)


def test_batch_groups_many_small_clouds(ctxs):
    """70 single-workgroup clouds (three launches) among a few multi-kernel
    builds, one with a NaN: that one fails alone, every other equals the
    oracle."""
    import paper_2302_05002_amd as fpo
    on, _ = ctxs
    rng = np.random.default_rng(41)
    clouds, params = [], []
    kinds = ("uniform", "planes", "clusters", "few")
    for i in range(70):
        n = int(rng.integers(1, 40_000))
        clouds.append(_cloud(kinds[i % 4], n, seed=100 + i))
        params.append(fpo.Params(int(rng.choice([8, 32, 64])), 100_000, int(rng.choice([4, 16, 32])),
                                 max(1_000, n // 60), int(rng.integers(1, 50))))
    for i, n in enumerate((300_000, 150_000, 90_000)):
        clouds.append(_cloud(kinds[i], n, seed=7 + i))
        params.append(fpo.Params(64, 50_000, 32, 5_000, 64))
    bad = 17
    clouds[bad].x[clouds[bad].n // 2] = np.nan
    dev = [_dev(c) for c in clouds]
    jobs = on.build_batch(dev, params)
    for i, (c, p, j) in enumerate(zip(clouds, params, jobs)):
        if i == bad:
            with pytest.raises(fpo.FpoError) as e:
                j.wait()
            assert e.value.status == fpo.FPO_ERR_NONFINITE
            j.release()
            continue
        j.wait()
        exp = oracle.build_octree(c.x, c.y, c.z, oracle.Params(p.count_grid, p.max_points_per_chunk,
                                                               p.subsample_grid, p.leaf_capacity, p.preview_modulus))
        compare(j.result().to_numpy(), exp, label=f"cloud {i} (n={c.n}): ")
        j.release()


def test_plain_and_batch_limits_are_separate():
    """With the plain limit at 0 and the batch limit at its maximum, a plain
    build takes the multi-kernel path and the same clouds in a batch take the
    single-workgroup one (one launch, a fused timer bracket per job)."""
    import paper_2302_05002_amd as fpo
    ctx = fpo.Context(0)
    try:
        ctx.set_single_block_max(0, fpo.SINGLE_BLOCK_MAX_POINTS)
        ctx.set_timing(True, only=["fused"])
        clouds = [_cloud(k, n, seed=n) for k, n in (("uniform", 9_000), ("planes", 150_000), ("few", 3))]
        p = fpo.Params(64, 200_000, 32, 10_000, 16)
        dev = [_dev(c) for c in clouds]
        job = ctx.submit(*dev[0], p)
        job.wait()
        assert job.timer("fused")[1] == 0
        job.release()
        jobs = ctx.build_batch(dev, p)
        for c, j in zip(clouds, jobs):
            j.wait()
            assert j.timer("fused")[1] == 1
            exp = oracle.build_octree(c.x, c.y, c.z, oracle.Params(64, 200_000, 32, 10_000, 16))
            compare(j.result().to_numpy(), exp, label=f"batch n={c.n}: ")
            j.release()
    finally:
        ctx.close()
