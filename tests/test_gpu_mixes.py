"""The batched and served workloads at their stated scale, through the C ABI.

* Batched: 256 independent clouds, sizes log-uniform in [10k, 4M] (about
  150M points), mixed uniform / planes / clusters, per-size parameters, built
  by one fpo_build_batch call; every cloud compared with the oracle.
* Served: a seeded trace of 2,000 requests with sizes log-uniform in
  [100k, 50M] (about 16G points) under a 200 GB budget.  Each request is the
  first n points of one of three 50M-point pool clouds (a prefix of a cloud
  is a cloud), which bounds host generation.  A seeded sample of 50 requests
  of at most 5M points is compared with the oracle run on exactly those
  points, and the three largest requests with the same build run alone.
"""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import KEYS, compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2302_05002_amd as fpo
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = fpo.Context(0)
    yield c
    c.close()


def _params(fpo, p):
    return fpo.Params(p.count_grid, p.max_points_per_chunk, p.subsample_grid, p.leaf_capacity, p.preview_modulus)


def _oracle(x, y, z, p):
    r = oracle.build_octree(x, y, z, oracle.Params(p.count_grid, p.max_points_per_chunk, p.subsample_grid,
                                                   p.leaf_capacity, p.preview_modulus))
    assert r["status"] == oracle.OK
    return r


def test_batch_of_256_clouds(ctx):
    import torch
    import paper_2302_05002_amd as fpo
    mix = synth.batch_mix(256, seed=4)
    total = sum(c.n for c, _ in mix)
    print(f"[batch] 256 clouds, {total} points", flush=True)
    assert 100_000_000 < total < 250_000_000
    dev = [tuple(torch.from_numpy(a).cuda() for a in (c.x, c.y, c.z)) for c, _ in mix]
    jobs = ctx.build_batch(dev, [_params(fpo, p) for _, p in mix])
    for i, ((c, p), j) in enumerate(zip(mix, jobs)):
        j.wait()
        compare(j.result().to_numpy(), _oracle(c.x, c.y, c.z, p), label=f"cloud {i} (n={c.n}): ")
        j.release()


def test_served_trace_of_2000_requests(ctx):
    import torch
    import paper_2302_05002_amd as fpo
    torch.cuda.empty_cache()   # the arena below takes 200 GB of the device
    pool, reqs = synth.serve_trace(2000, seed=5)
    points = sum(r.n for r in reqs)
    print(f"[served] 2000 requests, {points} points", flush=True)
    dev = [tuple(torch.from_numpy(a).cuda() for a in (c.x, c.y, c.z)) for c in pool]
    rng = np.random.default_rng(55)
    small = [i for i, r in enumerate(reqs) if r.n <= 5_000_000]
    sample = set(int(i) for i in rng.choice(small, 50, replace=False))
    largest = set(sorted(range(len(reqs)), key=lambda i: -reqs[i].n)[:3])
    srv = fpo.Server(ctx, hbm_budget_bytes=200 * 10 ** 9, max_slots=4)
    jobs = []
    for r in reqs:
        x, y, z = (a[:r.n] for a in dev[r.kind])
        jobs.append(srv.submit(x, y, z, _params(fpo, synth.params_for_size(r.n))))
    checked = 0
    for i, (r, j) in enumerate(zip(reqs, jobs)):
        j.wait()
        if i in sample or i in largest:
            got = j.to_numpy()
            p = synth.params_for_size(r.n)
            c = pool[r.kind]
            if i in sample:
                compare(got, _oracle(c.x[:r.n], c.y[:r.n], c.z[:r.n], p), label=f"request {i} (n={r.n}): ")
            else:
                # mix == alone: the same request built on its own
                x, y, z = (a[:r.n] for a in dev[r.kind])
                alone = ctx.build(x, y, z, _params(fpo, p)).to_numpy()
                for k in KEYS:
                    assert np.array_equal(got[k], alone[k]), f"request {i} (n={r.n}): {k} differs from alone"
            checked += 1
        j.release()   # frees its share of the budget for the requests behind it
        jobs[i] = None
    assert checked == len(sample | largest)
    srv.close()
