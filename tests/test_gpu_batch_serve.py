"""Batched builds and the request server, through the C ABI: every result is
the one the oracle (and a plain build of the same cloud) gives, alone or in a
mix of concurrent builds."""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import KEYS, compare, make

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2302_05002_amd as fpo
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = fpo.Context(0)
    yield c
    c.close()


MIX = [
    # (kind, n, seed, G, C, S, L, M)
    ("planes", 150_000, 51, 64, 20_000, 32, 2_000, 64),
    ("uniform", 3_000, 52, 8, 500, 8, 100, 7),
    ("clusters", 60_000, 53, 128, 5_000, 128, 1_000, 16),
    ("uniform", 1, 54, 4, 10, 4, 10, 2),
    ("planes", 40_000, 55, 32, 100_000, 16, 10_000, 64),
    ("clusters", 90_000, 56, 16, 2_000, 64, 300, 5),
    ("uniform", 20_000, 57, 64, 1_000, 2, 50, 3),
    ("planes", 9_000, 58, 512, 300, 256, 64, 9),
]


def device_cloud(c):
    import torch
    return tuple(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (c.x, c.y, c.z))


def oracle_of(c, case):
    _, _, _, G, C, S, L, M = case
    r = oracle.build_octree(c.x, c.y, c.z, oracle.Params(G, C, S, L, M))
    assert r["status"] == oracle.OK
    return r


def fpo_params(case):
    import paper_2302_05002_amd as fpo
    _, _, _, G, C, S, L, M = case
    return fpo.Params(G, C, S, L, M)


def test_batch_matches_oracle(ctx):
    import torch
    import paper_2302_05002_amd as fpo
    clouds = [make(k, n, s) for (k, n, s, *_rest) in MIX]
    dev = [device_cloud(c) for c in clouds]
    # an empty cloud and one with a NaN: the first builds, the second fails alone
    e = torch.zeros(0, device="cuda")
    bad = torch.tensor([0.0, 1.0, float("nan"), 2.0], device="cuda")
    dev_all = dev + [(e, e.clone(), e.clone()), (bad, bad.clone(), bad.clone())]
    params = [fpo_params(c) for c in MIX] + [fpo.Params(8, 10, 8, 10, 4)] * 2
    print(f"[batch] {len(dev_all)} clouds", flush=True)
    jobs = ctx.build_batch(dev_all, params)
    for i, (c, case) in enumerate(zip(clouds, MIX)):
        jobs[i].wait()
        got = jobs[i].result().to_numpy()
        compare(got, oracle_of(c, case), label=f"batch {case}: ")
        packed = jobs[i].to_numpy()
        for k in KEYS:
            np.testing.assert_array_equal(packed[k], got[k], err_msg=k)
    jobs[-2].wait()
    assert jobs[-2].result().to_numpy()["node_depth"].shape[0] == 0
    with pytest.raises(fpo.FpoError) as ei:
        jobs[-1].wait()
    assert ei.value.status == fpo.FPO_ERR_NONFINITE
    for j in jobs:
        j.release()


def test_batch_after_stream_work(ctx):
    """Inputs written on the caller's stream just before the batch call."""
    import torch
    import paper_2302_05002_amd as fpo
    case = ("planes", 50_000, 61, 64, 5_000, 32, 1_000, 64)
    c = make(*case[:3])
    x = torch.empty(c.n, device="cuda")
    y, z = torch.empty_like(x), torch.empty_like(x)
    host = [torch.from_numpy(a).pin_memory() for a in (c.x, c.y, c.z)]
    for d, h in zip((x, y, z), host):
        d.copy_(h, non_blocking=True)
    jobs = ctx.build_batch([(x, y, z)] * 3, fpo_params(case))
    exp = oracle_of(c, case)
    for j in jobs:
        j.wait()
        compare(j.result().to_numpy(), exp, label="after-stream: ")
        j.release()


def test_server_mix_equals_alone(ctx):
    import paper_2302_05002_amd as fpo
    clouds = [make(k, n, s) for (k, n, s, *_rest) in MIX]
    dev = [device_cloud(c) for c in clouds]
    alone = []
    for d, case in zip(dev, MIX):
        alone.append(ctx.build(*d, fpo_params(case)).to_numpy())
    srv = fpo.Server(ctx, hbm_budget_bytes=4 << 30, max_slots=3)   # G=512 alone needs 2.5 GB
    print(f"[server] {len(MIX)} requests, 3 slots", flush=True)
    jobs = [srv.submit(*d, fpo_params(case)) for d, case in zip(dev, MIX)]
    for j, a, case in zip(jobs, alone, MIX):
        j.wait()
        got = j.to_numpy()
        compare(got, a, label=f"served {case}: ")
        sub, start, done = j.timestamps()
        assert sub <= start <= done
    for j in jobs:
        j.release()
    srv.close()


def test_server_budget_admission(ctx):
    """A budget that holds about two requests: later ones wait for memory,
    admitted as earlier jobs are released; results unchanged."""
    import paper_2302_05002_amd as fpo
    case = ("planes", 80_000, 71, 64, 10_000, 32, 1_000, 64)
    c = make(*case[:3])
    d = device_cloud(c)
    p = fpo_params(case)
    need = fpo.workspace_size(c.n, p)
    srv = fpo.Server(ctx, hbm_budget_bytes=2 * need + 4096, max_slots=4)
    exp = oracle_of(c, case)
    jobs = [srv.submit(*d, p) for _ in range(6)]
    for j in jobs:
        j.wait()
        compare(j.to_numpy(), exp, label="budget: ")
        j.release()
    # larger than the whole budget: rejected at submit
    big = make("uniform", 400_000, 72)
    with pytest.raises(fpo.FpoError) as ei:
        srv.submit(*device_cloud(big), p)
    assert ei.value.status == fpo.FPO_ERR_REJECTED
    srv.close()


def test_server_cancel(ctx):
    import paper_2302_05002_amd as fpo
    case = ("planes", 60_000, 81, 64, 10_000, 32, 1_000, 64)
    c = make(*case[:3])
    d = device_cloud(c)
    p = fpo_params(case)
    need = fpo.workspace_size(c.n, p)
    srv = fpo.Server(ctx, hbm_budget_bytes=need + 4096, max_slots=1)   # one at a time
    jobs = [srv.submit(*d, p) for _ in range(4)]
    assert jobs[3].cancel()            # still waiting for memory behind the others
    with pytest.raises(fpo.FpoError) as ei:
        jobs[3].wait()
    assert ei.value.status == fpo.FPO_ERR_CANCELLED
    exp = oracle_of(c, case)
    for j in jobs[:3]:
        j.wait()
        compare(j.to_numpy(), exp, label="cancel: ")
        j.release()
    jobs[3].release()
    srv.close()


def test_batch_and_server_with_preview_variants(ctx):
    """Preview variants inside batches and served requests: the grid variant
    adds its per-cell minima to a build's workspace, which the batch
    workspace and the server's arena account for."""
    import paper_2302_05002_amd as fpo
    modes = ["grid", "stride", "hash", "grid", "grid", "stride", "hash", "grid"]
    clouds = [make(k, n, s) for (k, n, s, *_rest) in MIX]
    dev = [device_cloud(c) for c in clouds]
    params = [fpo.Params(G, C, S, L, M, None, mode) for (_, _, _, G, C, S, L, M), mode in zip(MIX, modes)]
    exp = []
    for c, (_, _, _, G, C, S, L, M), mode in zip(clouds, MIX, modes):
        r = oracle.build_octree(c.x, c.y, c.z, oracle.Params(G, C, S, L, M, None, mode))
        assert r["status"] == oracle.OK
        exp.append(r)
    print(f"[batch] {len(dev)} clouds with preview variants", flush=True)
    jobs = ctx.build_batch(dev, params)
    for j, e, case in zip(jobs, exp, MIX):
        j.wait()
        compare(j.result().to_numpy(), e, label=f"batch variants {case}: ")
        j.release()
    srv = fpo.Server(ctx, hbm_budget_bytes=6 << 30, max_slots=3)   # G=512 with grid minima: 4.7 GB
    print(f"[server] {len(dev)} requests with preview variants", flush=True)
    jobs = [srv.submit(*d, p) for d, p in zip(dev, params)]
    for j, e, case in zip(jobs, exp, MIX):
        j.wait()
        compare(j.to_numpy(), e, label=f"served variants {case}: ")
        j.release()
    srv.close()
