"""Paths that only large clouds take, against the oracle element by element:
the chunk split in two passes (at least 2^24 points and 128 chunks or
more), the binned quantise + count pass (G = 512, the default there from
2^20 points), and five global shared depths with their alternating cell
tables (G = 512, S = 16)."""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import compare

pytestmark = pytest.mark.gpu


def _build(c, case, variant=None):
    import torch
    import paper_2302_05002_amd as fpo
    ctx = fpo.Context(0)
    try:
        if variant is not None:
            ctx.force_quantize_variant(variant)
        dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (c.x, c.y, c.z)]
        return ctx.build(*dev, fpo.Params(*case)).to_numpy()
    finally:
        ctx.close()


def test_two_pass_chunk_split():
    c = synth.planes(17_000_000, seed=41, num_planes=60)
    case = (128, 100_000, 32, 2_000, 16)
    print(f"[large] 17M planes {case}", flush=True)
    exp = oracle.build_octree(c.x, c.y, c.z, oracle.Params(*case))
    assert exp["status"] == oracle.OK and len(exp["chunk_count"]) >= 128
    compare(_build(c, case), exp, label="17M planes, two-pass split: ")


@pytest.mark.parametrize("variant", [None, 0])
def test_binned_count_and_deep_global_depths(variant):
    c = synth.clusters(2_500_000, seed=42, num_clusters=40)
    case = (512, 300_000, 16, 1_000, 9)   # d0 = 9 - 4 = 5 global depths
    print(f"[large] 2.5M clusters {case} variant {variant}", flush=True)
    exp = oracle.build_octree(c.x, c.y, c.z, oracle.Params(*case))
    assert exp["status"] == oracle.OK
    compare(_build(c, case, variant), exp, label=f"2.5M clusters, G = 512, S = 16, shape {variant}: ")
