"""Handle lifetimes through the C ABI: jobs, contexts and servers may be
released in any order.  Destroying a context or a server never blocks and
never frees what a live job still uses; a job released afterwards (also one
whose build failed) finds its context and server intact, and its results are
still right."""
import ctypes
import gc

import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import compare

pytestmark = pytest.mark.gpu


def _dev(c):
    import torch
    return tuple(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (c.x, c.y, c.z))


def _expected(c, G, C, S, L, M):
    r = oracle.build_octree(c.x, c.y, c.z, oracle.Params(G, C, S, L, M))
    assert r["status"] == oracle.OK
    return r


def test_job_outlives_context():
    import paper_2302_05002_amd as fpo
    lib = fpo.load_library()
    c = synth.planes(80_000, seed=91, num_planes=6)
    x, y, z = _dev(c)
    ctx = fpo.Context(0)
    job = ctx.submit(x, y, z, fpo.Params(32, 8_000, 16, 500, 16))
    # the owner's handle goes first; the job still holds the context
    lib.fpo_context_destroy(ctx._h)
    ctx._h = None
    job.wait()
    compare(job.to_numpy(), _expected(c, 32, 8_000, 16, 500, 16), label="after context destroy: ")
    job.release()


def test_failed_job_released_after_context():
    """A build that failed (non-finite input) and is released only after its
    context was destroyed, as a job kept alive by a traceback is."""
    import torch
    import paper_2302_05002_amd as fpo
    lib = fpo.load_library()
    ctx = fpo.Context(0)
    bad = torch.tensor([0.0, 1.0, float("nan"), 2.0], device="cuda")
    job = ctx.submit(bad, bad.clone(), bad.clone(), fpo.Params(8, 10, 8, 10, 4))
    with pytest.raises(fpo.FpoError) as e:
        job.wait()
    assert e.value.status == fpo.FPO_ERR_NONFINITE
    lib.fpo_context_destroy(ctx._h)
    ctx._h = None
    del e
    job.release()
    gc.collect()


def test_build_error_releases_its_job():
    """Context.build releases the job when wait raises, so no job is left for
    a later garbage collection to release after the context is gone."""
    import torch
    import paper_2302_05002_amd as fpo
    ctx = fpo.Context(0)
    bad = torch.tensor([float("inf"), 1.0], device="cuda")
    with pytest.raises(fpo.FpoError):
        ctx.build(bad, bad.clone(), bad.clone(), fpo.Params(8, 10, 8, 10, 4))
    ctx.close()
    gc.collect()


def test_served_jobs_outlive_server():
    import paper_2302_05002_amd as fpo
    lib = fpo.load_library()
    ctx = fpo.Context(0)
    c = synth.clusters(120_000, seed=92, num_clusters=9)
    d = _dev(c)
    p = fpo.Params(64, 10_000, 32, 1_000, 64)
    need = fpo.workspace_size(c.n, p)
    # two fit at once: the later requests wait for memory the earlier hold
    srv = fpo.Server(ctx, hbm_budget_bytes=2 * need + 4096, max_slots=2)
    jobs = [srv.submit(*d, p) for _ in range(4)]
    lib.fpo_server_destroy(srv._h)   # returns at once: requests still queued
    srv._h = None
    lib.fpo_context_destroy(ctx._h)
    ctx._h = None
    exp = _expected(c, 64, 10_000, 32, 1_000, 64)
    for j in jobs:
        j.wait()
        compare(j.to_numpy(), exp, label="after server destroy: ")
        j.release()   # frees arena memory: the next waiting request is admitted


def test_unstarted_served_job_released_after_server():
    """A request still waiting for memory when its server and context are
    destroyed and it is released: taken out of the queue, nothing leaks or
    blocks."""
    import paper_2302_05002_amd as fpo
    lib = fpo.load_library()
    ctx = fpo.Context(0)
    c = synth.uniform(60_000, seed=93)
    d = _dev(c)
    p = fpo.Params(32, 10_000, 16, 1_000, 64)
    need = fpo.workspace_size(c.n, p)
    srv = fpo.Server(ctx, hbm_budget_bytes=need + 4096, max_slots=1)
    first, second = srv.submit(*d, p), srv.submit(*d, p)
    lib.fpo_server_destroy(srv._h)
    srv._h = None
    lib.fpo_context_destroy(ctx._h)
    ctx._h = None
    second.release()          # never admitted: removed from the queue
    first.wait()
    compare(first.to_numpy(), _expected(c, 32, 10_000, 16, 1_000, 64), label="first: ")
    first.release()


def test_owner_kept_alive_by_python_job():
    """Dropping the Python Context or Server object does not destroy it while
    one of its jobs is alive."""
    import paper_2302_05002_amd as fpo
    c = synth.uniform(30_000, seed=94)
    d = _dev(c)
    p = fpo.Params(16, 5_000, 8, 500, 8)
    ctx = fpo.Context(0)
    job = ctx.submit(*d, p)
    srv = fpo.Server(ctx, hbm_budget_bytes=1 << 30, max_slots=2)
    sjob = srv.submit(*d, p)
    del ctx, srv
    gc.collect()
    exp = _expected(c, 16, 5_000, 8, 500, 8)
    for j in (job, sjob):
        j.wait()
        compare(j.to_numpy(), exp, label="owner dropped: ")
        j.release()
