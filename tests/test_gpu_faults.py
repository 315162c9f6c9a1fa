"""Injected allocation failures (FPO_FAULT=alloc:<k>): for every k, the k-th
allocation a context makes (its stream, the issuing and worker streams,
pinned staging, events, a server's arena and slot streams) fails.  The call
that needed it reports FPO_ERR_OUT_OF_MEMORY, nothing else fails, and the
same operations succeed afterwards with results equal to the oracle's."""
import os

import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import compare

pytestmark = pytest.mark.gpu

CASE = (16, 5_000, 8, 500, 8)   # G, C, S, L, M


@pytest.fixture(scope="module")
def cloud():
    import torch
    c = synth.planes(40_000, seed=123, num_planes=5)
    r = oracle.build_octree(c.x, c.y, c.z, oracle.Params(*CASE))
    assert r["status"] == oracle.OK
    return tuple(torch.from_numpy(a).cuda() for a in (c.x, c.y, c.z)), r


def _ops(fpo, ctx, dev, exp):
    """Plain builds, a batch and a server; yields (name, outcome) with
    outcome None on success or the FpoError status."""
    p = fpo.Params(*CASE)

    def plain():
        compare(ctx.build(*dev, p).to_numpy(), exp, label="plain: ")

    def batch():
        jobs = ctx.build_batch([dev, dev], p)
        try:
            for j in jobs:
                j.wait()
                compare(j.result().to_numpy(), exp, label="batch: ")
        finally:
            for j in jobs:
                j.release()

    def served():
        srv = fpo.Server(ctx, 1 << 30, 2)
        try:
            jobs = [srv.submit(*dev, p) for _ in range(2)]
            for j in jobs:
                j.wait()
                compare(j.to_numpy(), exp, label="served: ")
                j.release()
        finally:
            srv.close()

    for name, op in (("plain", plain), ("plain again", plain), ("batch", batch), ("served", served)):
        try:
            op()
            yield name, None
        except fpo.FpoError as e:
            yield name, e.status


@pytest.mark.parametrize("k", list(range(1, 27)))
def test_injected_allocation_failure(cloud, k):
    import paper_2302_05002_amd as fpo
    dev, exp = cloud
    os.environ["FPO_FAULT"] = f"alloc:{k}"
    try:
        try:
            ctx = fpo.Context(0)
        except fpo.FpoError as e:
            assert k == 1 and e.status == fpo.FPO_ERR_OUT_OF_MEMORY
            return
    finally:
        del os.environ["FPO_FAULT"]
    try:
        # passes over the same operations: exactly one call in all of them
        # may fail (the one making allocation k), with FPO_ERR_OUT_OF_MEMORY,
        # and the pass after it is clean
        failed = []
        for _ in range(3):
            outcomes = list(_ops(fpo, ctx, dev, exp))
            bad = [(n, s) for n, s in outcomes if s is not None]
            if failed:
                assert not bad, outcomes
                break
            failed = bad
        assert len(failed) <= 1, failed
        assert all(s == fpo.FPO_ERR_OUT_OF_MEMORY for _, s in failed), failed
    finally:
        ctx.close()


def test_faults_hit_every_kind_of_call(cloud):
    """Over the range of k above, each of plain, batch and served has failed
    once (so the injection reaches every allocation path)."""
    import paper_2302_05002_amd as fpo
    dev, exp = cloud
    hit = set()
    for k in range(2, 27):
        os.environ["FPO_FAULT"] = f"alloc:{k}"
        try:
            ctx = fpo.Context(0)
        finally:
            del os.environ["FPO_FAULT"]
        try:
            hit |= {n.split()[0] for n, s in _ops(fpo, ctx, dev, exp) if s is not None}
        finally:
            ctx.close()
    assert hit == {"plain", "batch", "served"}, hit
