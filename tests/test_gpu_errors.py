"""Argument errors through the C ABI with a live context: every one is
reported with its status and a message before any work is enqueued, and the
context stays usable afterwards."""
import ctypes

import pytest

import synth
from test_gpu_parity import run_both

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2302_05002_amd as fpo
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = fpo.Context(0)
    yield c
    c.close()


def submit_raw(ctx, x, y, z, params, ws_ptr, ws_bytes):
    import paper_2302_05002_amd as fpo
    lib = fpo.load_library()
    n = int(x.shape[0])
    cloud = fpo._Cloud(n, x.data_ptr(), y.data_ptr(), z.data_ptr(), fpo.FPO_DEVICE, 0)
    h = ctypes.c_void_p()
    st = lib.fpo_build_submit(ctx._h, ctypes.byref(cloud), ctypes.byref(params.to_c()), ctypes.c_void_p(ws_ptr),
                              ws_bytes, None, ctypes.byref(h))
    return st, h, lib.fpo_last_error().decode()


def test_build_argument_errors(ctx):
    import torch
    import paper_2302_05002_amd as fpo
    c = synth.uniform(10_000, seed=3)
    x, y, z = (torch.from_numpy(a).cuda() for a in (c.x, c.y, c.z))
    p = fpo.Params(16, 1_000, 8, 100, 4)
    need = fpo.workspace_size(c.n, p)
    ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    st, h, msg = submit_raw(ctx, x, y, z, p, ws.data_ptr(), need - 1)
    assert st == fpo.FPO_ERR_OUT_OF_MEMORY and "needs" in msg and not h.value
    st, h, msg = submit_raw(ctx, x, y, z, p, ws.data_ptr() + 16, need)
    assert st == fpo.FPO_ERR_INVALID_ARG and "aligned" in msg and not h.value
    st, h, msg = submit_raw(ctx, x, y, z, p, 0, need)
    assert st == fpo.FPO_ERR_INVALID_ARG and not h.value
    st, h, msg = submit_raw(ctx, x, y, z, fpo.Params(16, 1_000, 8, 100, 0), ws.data_ptr(), need)
    assert st == fpo.FPO_ERR_INVALID_ARG and "preview_modulus" in msg
    # the context still builds correctly afterwards
    run_both(ctx, c, 16, 1_000, 8, 100, 4, label="after errors: ")


def test_gather_and_select_errors(ctx):
    import torch
    import paper_2302_05002_amd as fpo
    c = synth.planes(20_000, seed=4, num_planes=3)
    x, y, z = (torch.from_numpy(a).cuda() for a in (c.x, c.y, c.z))
    job = ctx.submit(x, y, z, fpo.Params(16, 5_000, 8, 100, 4))
    job.wait()
    with pytest.raises(fpo.FpoError) as e:
        job.gather(x[:-1].contiguous(), y[:-1].contiguous(), z[:-1].contiguous())   # wrong point count
    assert e.value.status == fpo.FPO_ERR_INVALID_ARG
    res = job.result()
    lib = fpo.load_library()
    need = ctypes.c_uint64()
    assert lib.fpo_select_workspace_size(res.num_nodes, ctypes.byref(need)) == fpo.FPO_OK
    ws = torch.empty(int(need.value), dtype=torch.uint8, device="cuda")
    out = torch.empty(res.num_nodes, dtype=torch.int32, device="cuda")
    tot = torch.zeros(2, dtype=torch.int32, device="cuda")
    view = fpo.make_view((0, 0, 0), ((0, 0, 0, 1),) * 6, 1.0, 0.0)
    lo = (ctypes.c_float * 3)(*[float(v) for v in res.bbox_min])
    args = [ctx._h, res.num_nodes, ctypes.c_void_p(res.node_depth.data_ptr()),
            ctypes.c_void_p(res.node_key.data_ptr()), ctypes.c_void_p(res.node_count.data_ptr()), lo,
            float(res.cube_size), ctypes.byref(view), ctypes.c_void_p(ws.data_ptr()), int(need.value) - 1,
            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(tot.data_ptr()), None]
    assert lib.fpo_select_nodes(*args) == fpo.FPO_ERR_INVALID_ARG            # workspace too small
    bad = fpo.make_view((0, 0, 0), ((0, 0, 0, 1),) * 6, float("nan"), 0.0)
    args[9] = int(need.value)
    args[7] = ctypes.byref(bad)
    assert lib.fpo_select_nodes(*args) == fpo.FPO_ERR_INVALID_ARG            # non-finite view
    args[7] = ctypes.byref(view)
    assert lib.fpo_select_nodes(*args) == fpo.FPO_OK
    torch.cuda.synchronize()
    assert tot.cpu().tolist() == [res.num_nodes, c.n]                        # no clipping, no limit: all
    job.release()


def test_las_decode_errors(ctx):
    import torch
    import paper_2302_05002_amd as fpo
    from synth.las import write_las
    c = synth.uniform(1000, seed=5)
    f = write_las(c.x, c.y, c.z, point_format=0)
    h = fpo.las_parse_header(f)
    recs = torch.frombuffer(bytearray(f[h.offset_to_points:]), dtype=torch.uint8).cuda()
    with pytest.raises(fpo.FpoError) as e:
        ctx.las_decode(recs, h, n=1001)                                       # one record past the buffer
    assert e.value.status == fpo.FPO_ERR_INVALID_ARG
    with pytest.raises(fpo.FpoError):
        ctx.las_decode(recs, h, rgb=True)                                     # format 0 has no colour
    with pytest.raises(fpo.FpoError):
        ctx.las_decode(recs, h, origin=(float("inf"), 0.0, 0.0))
    x, y, z, _ = ctx.las_decode(recs, h)
    torch.cuda.synchronize()
    assert x.shape[0] == 1000


def test_timer_mask(ctx):
    """Timers of a mask: the selected group records its launches, the others
    none; a bit beyond the last timer is rejected."""
    import torch
    import paper_2302_05002_amd as fpo
    lib = fpo.load_library()
    assert lib.fpo_context_set_timers(ctx._h, 1 << fpo.TIMERS["node_sort"] | 1 << 20) == fpo.FPO_ERR_INVALID_ARG
    c = synth.planes(200_000, seed=8, num_planes=20)
    x, y, z = (torch.from_numpy(a).cuda() for a in (c.x, c.y, c.z))
    p = fpo.Params(64, 100_000, 32, 10_000, 64)
    ctx.set_timing(True, ["subsample", "node_sort"])
    job = ctx.submit(x, y, z, p)
    job.wait()
    got = {k: job.timer(k) for k in fpo.TIMERS}
    job.release()
    ctx.set_timing(False)
    assert got["subsample"][1] >= 1 and got["node_sort"][1] >= 1 and got["subsample"][0] > 0
    assert all(got[k] == (0.0, 0) for k in fpo.TIMERS if k not in ("subsample", "node_sort"))
    ctx.set_timing(True)
    job = ctx.submit(x, y, z, p)
    job.wait()
    assert all(job.timer(k)[1] >= 1 for k in ("bbox", "quantize", "subsample", "node_place", "node_sort", "preview"))
    job.release()
    ctx.set_timing(False)
