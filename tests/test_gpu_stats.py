"""fpo_job_get_stats of completed builds against the oracle's outputs: counts,
deepest node, oversized flag, clamped points, preview size, the workspace
plan, ordered timestamps, and the timed regions of a timed build."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind,n,G,C,S,L,M,box", [("clusters", 150_000, 32, 2_000, 16, 300, 16, False),
                                                   ("uniform", 80_000, 16, 10_000, 8, 100, 8, True)])
def test_stats_match_the_oracle(kind, n, G, C, S, L, M, box):
    import torch
    import paper_2302_05002_amd as fpo
    c = synth.clusters(n, seed=7, num_clusters=20) if kind == "clusters" else synth.uniform(n, seed=8)
    bbox = ((0.1, 0.1, 0.1), (0.9, 0.9, 0.9)) if box else None   # clamps some points
    exp = oracle.build_octree(c.x, c.y, c.z, oracle.Params(G, C, S, L, M, bbox))
    assert exp["status"] == oracle.OK
    ctx = fpo.Context(0)
    try:
        ctx.set_timing(True)
        x, y, z = (torch.from_numpy(a).cuda() for a in (c.x, c.y, c.z))
        p = fpo.Params(G, C, S, L, M, bbox)
        job = ctx.submit(x, y, z, p)
        job.wait()
        st = job.stats()
        job.release()
    finally:
        ctx.close()
    assert st["n"] == n
    assert st["num_chunks"] == exp["chunk_level"].shape[0]
    assert st["num_nodes"] == exp["node_depth"].shape[0]
    assert st["max_depth"] == int(exp["node_depth"].max())
    assert st["chunk_oversized_any"] == exp["chunk_oversized_any"]
    assert st["n_outside"] == exp["n_outside"] and (st["n_outside"] > 0) == box
    assert st["preview_count"] == exp["preview_index"].shape[0]
    assert st["workspace_bytes"] == fpo.workspace_size(n, p)
    assert st["submitted_ns"] <= st["started_ns"] <= st["completed_ns"]
    regions = st["region_ms"]
    assert set(regions) == set(fpo.TIMERS)
    assert all(v >= 0.0 for v in regions.values())
    assert sum(regions.values()) * 1e6 <= st["completed_ns"] - st["submitted_ns"]
