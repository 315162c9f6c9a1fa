"""Builds from pinned host memory, streamed to the device in batches: the
result is the oracle's, with the box computed or given as a header."""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2302_05002_amd as fpo
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = fpo.Context(0)
    yield c
    c.close()


def pinned(c):
    import torch
    return tuple(torch.from_numpy(np.ascontiguousarray(a)).pin_memory() for a in (c.x, c.y, c.z))


def exact_box(c):
    return ((float(c.x.min()), float(c.y.min()), float(c.z.min())),
            (float(c.x.max()), float(c.y.max()), float(c.z.max())))


def streamed_vs_oracle(ctx, c, G, C, S, L, M, bbox, batch, label):
    import paper_2302_05002_amd as fpo
    print(f"[streamed] {label}: n={c.n} batch={batch} bbox={bbox is not None}", flush=True)
    exp = oracle.build_octree(c.x, c.y, c.z, oracle.Params(G, C, S, L, M, bbox))
    assert exp["status"] == oracle.OK
    x, y, z = pinned(c)
    job = ctx.submit(x, y, z, fpo.Params(G, C, S, L, M, bbox), stream_batch=batch)
    job.wait()
    got = job.result().to_numpy()
    job.release()
    compare(got, exp, label=label)
    return got


def test_streamed_terrain_batches(ctx):
    c = synth.terrain_clusters(3_000_000, seed=91, colors=False)
    a = streamed_vs_oracle(ctx, c, 512, 200_000, 128, 10_000, 64, None, 1_000_000, "computed box: ")
    b = streamed_vs_oracle(ctx, c, 512, 200_000, 128, 10_000, 64, exact_box(c), 1_000_000, "given box: ")
    # the exact box as a header gives the same tree
    np.testing.assert_array_equal(a["node_points"], b["node_points"])
    lo, hi = exact_box(c)
    mid = tuple((p + q) / 2 for p, q in zip(lo, hi))
    got = streamed_vs_oracle(ctx, c, 512, 200_000, 128, 10_000, 64, (lo, mid), 1_000_000, "half box: ")
    assert got["n_outside"] > 0


def test_streamed_rejects_pageable(ctx):
    import ctypes
    import torch
    import paper_2302_05002_amd as fpo
    lib = fpo.load_library()
    c = synth.uniform(10_000, seed=92)
    x, y, z = (torch.from_numpy(np.ascontiguousarray(a)) for a in (c.x, c.y, c.z))   # pageable, not pinned
    cloud = fpo._Cloud(c.n, x.data_ptr(), y.data_ptr(), z.data_ptr(), fpo.FPO_HOST_PINNED, 0)
    p = fpo.Params(16, 1_000, 16, 100, 8).to_c()
    need = ctypes.c_uint64()
    assert lib.fpo_workspace_size_cloud(ctypes.byref(cloud), ctypes.byref(p), ctypes.byref(need)) == fpo.FPO_OK
    ws = torch.empty(int(need.value), dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    st = lib.fpo_build_submit(ctx._h, ctypes.byref(cloud), ctypes.byref(p), ctypes.c_void_p(ws.data_ptr()),
                              ws.numel(), None, ctypes.byref(h))
    assert st == fpo.FPO_ERR_INVALID_ARG


def test_terrain_200m_streamed_full(ctx):
    """The 200M-point terrain workload as the benchmark runs it: pinned host
    input in 16M-point batches, the exact box given as a header, every output
    compared with the oracle; then the same build from device memory (the
    binned count, the default at G = 512, and the two-pass chunk split),
    compared with the streamed one."""
    import torch
    import paper_2302_05002_amd as fpo
    p = synth.TERRAIN_200M
    c = synth.terrain_200m()
    box = exact_box(c)
    got = streamed_vs_oracle(ctx, c, p.count_grid, p.max_points_per_chunk, p.subsample_grid, p.leaf_capacity,
                             p.preview_modulus, box, 16_000_000, "terrain 200M: ")
    print("[streamed] terrain 200M from device memory", flush=True)
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (c.x, c.y, c.z)]
    res = ctx.build(*dev, fpo.Params(p.count_grid, p.max_points_per_chunk, p.subsample_grid, p.leaf_capacity,
                                     p.preview_modulus, box)).to_numpy()
    for k in got:
        assert np.array_equal(np.asarray(res[k]), np.asarray(got[k])), f"terrain 200M resident: {k} differs"


def test_streamed_nonfinite_with_given_box(ctx):
    """A NaN in the last batch of a streamed build with a given box."""
    import paper_2302_05002_amd as fpo
    c = synth.uniform(1_000_000, seed=92)
    x = c.x.copy()
    x[-3] = float("nan")
    box = ((0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    hx, hy, hz = pinned(synth.Cloud(x, c.y, c.z))
    job = ctx.submit(hx, hy, hz, fpo.Params(16, 100_000, 8, 1_000, 4, box), stream_batch=300_000)
    with pytest.raises(fpo.FpoError) as e:
        job.wait()
    assert e.value.status == fpo.FPO_ERR_NONFINITE
    job.release()
