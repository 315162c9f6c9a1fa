"""fpo_select_nodes_static (no workspace, the library's static scratch)
through the C ABI against fpo_select_nodes with a workspace: identical drawn
nodes and totals on two calls in a row, the second with a smaller table, and
an oversized table rejected before any work."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from oracle import view as V

pytestmark = pytest.mark.gpu


def _table(n, G, S, L, seed):
    c = synth.planes(n, seed=seed, num_planes=12)
    r = oracle.build_octree(c.x, c.y, c.z, oracle.Params(G, n // 4, S, L, 64))
    assert r["status"] == oracle.OK
    return r


def _device(r):
    import torch
    d = torch.from_numpy(r["node_depth"]).cuda()
    k = torch.from_numpy(r["node_key"].view(np.int64)).cuda()
    c = torch.from_numpy(r["node_count"].view(np.int32)).cuda()
    return d, k, c


def _call(lib, fn, ctx, r, dev, view, ws=None):
    import torch
    import paper_2302_05002_amd as fpo
    d, k, c = dev
    n = int(d.shape[0])
    out = torch.full((max(n, 1),), -1, dtype=torch.int32, device="cuda")
    tot = torch.full((2,), -1, dtype=torch.int32, device="cuda")
    lo = (ctypes.c_float * 3)(*[float(v) for v in r["bbox_min"]])
    args = [ctx._h, n, ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(k.data_ptr()), ctypes.c_void_p(c.data_ptr()),
            lo, float(r["cube_size"]), ctypes.byref(view)]
    if ws is not None:
        args += [ctypes.c_void_p(ws.data_ptr()), ws.numel()]
    args += [ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(tot.data_ptr()), None]
    st = fn(*args)
    assert st == fpo.FPO_OK, lib.fpo_last_error().decode()
    torch.cuda.synchronize()
    t = tot.cpu().tolist()
    return out[:t[0]].cpu().numpy().tolist(), t


def test_static_selection_matches_workspace_selection():
    import torch
    import paper_2302_05002_amd as fpo
    lib = fpo.load_library()
    ctx = fpo.Context(0)
    try:
        big = _table(300_000, 64, 32, 300, seed=101)
        small = _table(40_000, 32, 16, 100, seed=102)
        assert big["node_depth"].shape[0] > small["node_depth"].shape[0] > 100
        for r in (big, small):   # two calls in a row, the second smaller
            dev = _device(r)
            lo = [float(v) for v in r["bbox_min"]]
            side = float(r["cube_size"])
            eye = [lo[a] + side * f for a, f in enumerate((-0.4, 0.3, 0.6))]
            tgt = [lo[a] + side * 0.5 for a in range(3)]
            v = V.perspective_view(eye, tgt, (0.0, 0.0, 1.0), 60.0, 1.5, 0.01 * side, 8 * side, 1080.0, 60.0)
            view = fpo.make_view(v.eye, v.planes, v.proj_factor, v.min_size)
            need = ctypes.c_uint64()
            assert lib.fpo_select_workspace_size(int(dev[0].shape[0]), ctypes.byref(need)) == fpo.FPO_OK
            ws = torch.empty(int(need.value), dtype=torch.uint8, device="cuda")
            exp_nodes, exp_tot = _call(lib, lib.fpo_select_nodes, ctx, r, dev, view, ws)
            got_nodes, got_tot = _call(lib, lib.fpo_select_nodes_static, ctx, r, dev, view)
            assert got_nodes == exp_nodes and got_tot == exp_tot
            assert 0 < exp_tot[0] < dev[0].shape[0]   # the view really selects
            # and both equal the oracle's traversal
            on, op = V.select_nodes(r["node_depth"], r["node_key"], r["node_count"], r["bbox_min"], side, v)
            assert got_nodes == on and got_tot[1] == op
    finally:
        ctx.close()


def test_static_selection_rejects_oversized_table():
    import paper_2302_05002_amd as fpo
    lib = fpo.load_library()
    ctx = fpo.Context(0)
    try:
        view = fpo.make_view((0.0, 0.0, 0.0), ((0.0, 0.0, 0.0, 1.0),) * 6, 1.0, 0.0)
        lo = (ctypes.c_float * 3)(0.0, 0.0, 0.0)
        dummy = ctypes.c_void_p(8)   # never dereferenced: rejected on the host
        st = lib.fpo_select_nodes_static(ctx._h, fpo.SELECT_STATIC_MAX_NODES + 1, dummy, dummy, dummy, lo, 1.0,
                                         ctypes.byref(view), dummy, dummy, None)
        assert st == fpo.FPO_ERR_INVALID_ARG
        assert "static scratch" in lib.fpo_last_error().decode()
    finally:
        ctx.close()
