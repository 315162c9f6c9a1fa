"""The C-ABI library loads and exports every symbol include/fpo.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2302_05002_amd", "libfpo.so")
HDR = os.path.join(ROOT, "include", "fpo.h")


def declared_functions():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fpo_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import paper_2302_05002_amd.build as b
        b.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_binding_exports():
    import paper_2302_05002_amd as fpo
    assert declared_functions() == sorted(fpo.EXPORTS)


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_argument_errors_without_gpu(lib):
    """Validation runs before any GPU call: bad parameters are rejected with a
    message, on any machine."""
    import paper_2302_05002_amd as fpo
    fpo.load_library(LIB)
    for p in (fpo.Params(count_grid=3), fpo.Params(count_grid=1024), fpo.Params(subsample_grid=512),
              fpo.Params(max_points_per_chunk=0), fpo.Params(leaf_capacity=0), fpo.Params(preview_modulus=0)):
        with pytest.raises(fpo.FpoError) as e:
            fpo.workspace_size(100, p)
        assert e.value.status == fpo.FPO_ERR_INVALID_ARG and str(e.value)
    with pytest.raises(fpo.FpoError):
        fpo.workspace_size(1 << 33, fpo.Params())
    assert fpo.workspace_size(1000, fpo.Params()) > 0
    assert fpo.workspace_size(0, fpo.Params()) > 0


def test_workspace_grows_with_n(lib):
    import paper_2302_05002_amd as fpo
    fpo.load_library(LIB)
    a = fpo.workspace_size(10_000, fpo.Params())
    b = fpo.workspace_size(1_000_000, fpo.Params())
    assert b > a


def test_workspace_per_point(lib):
    """The split temporaries, the global-memory subsample path's tables and
    the node_points buffers share one region (they are live in turn), so the
    worst-case workspace stays below 150 B per point for the 20M-point planes
    parameters and below 175 B for 200M points at G = 512."""
    import paper_2302_05002_amd as fpo
    fpo.load_library(LIB)
    assert fpo.workspace_size(20_000_000, fpo.Params(128, 1_000_000, 128, 10_000, 64)) < 150 * 20_000_000
    assert fpo.workspace_size(200_000_000, fpo.Params(512, 2_000_000, 128, 10_000, 64)) < 175 * 200_000_000


def test_preview_modulus_for_a_target(lib):
    """M = max(1, ceil(n / target)); the stride preview then has ceil(n / M)
    <= target indices (the paper decimates to a fixed one million points)."""
    import paper_2302_05002_amd as fpo
    fpo.load_library(LIB)
    assert fpo.preview_modulus(100_000_000, 1_000_000) == 100
    assert fpo.preview_modulus(1_000_001, 1_000_000) == 2
    assert fpo.preview_modulus(5, 10) == 1
    assert fpo.preview_modulus(0, 1) == 1
    assert fpo.preview_modulus(0xFFFFFFFF, 1) == 0xFFFFFFFF
    rng = __import__("random").Random(4)
    for _ in range(2000):
        n, t = rng.randrange(0, 1 << 32), rng.randrange(1, 1 << 33)
        m = fpo.preview_modulus(n, t)
        assert m >= 1 and -(-n // m) <= t
        assert m == 1 or -(-n // (m - 1)) > t   # the least such M
    for n, t in ((10, 0), (1 << 32, 5)):
        with pytest.raises(fpo.FpoError) as e:
            fpo.preview_modulus(n, t)
        assert e.value.status == fpo.FPO_ERR_INVALID_ARG


def test_preview_flags(lib):
    import paper_2302_05002_amd as fpo
    fpo.load_library(LIB)
    both = fpo.Params()
    c = both.to_c()
    c.flags = fpo.FPO_PREVIEW_STRIDE | fpo.FPO_PREVIEW_GRID
    out = ctypes.c_uint64()
    assert fpo.load_library().fpo_workspace_size(100, ctypes.byref(c), ctypes.byref(out)) == fpo.FPO_ERR_INVALID_ARG
    c.flags = 8
    assert fpo.load_library().fpo_workspace_size(100, ctypes.byref(c), ctypes.byref(out)) == fpo.FPO_ERR_INVALID_ARG
    with pytest.raises(ValueError):
        fpo.Params(preview="voxel").to_c()
    # the grid preview adds its per-cell minima (8 bytes per count-grid cell)
    for G in (1, 64, 512):
        h = fpo.workspace_size(1000, fpo.Params(count_grid=G))
        assert fpo.workspace_size(1000, fpo.Params(count_grid=G, preview="stride")) == h
        assert fpo.workspace_size(1000, fpo.Params(count_grid=G, preview="grid")) >= h + 8 * G ** 3


def test_static_selection_scratch_covers_its_maximum(lib):
    """fpo_select_nodes_static's fixed scratch holds the workspace of its
    largest allowed node table (and the header and binding agree on both)."""
    import paper_2302_05002_amd as fpo
    fpo.load_library(LIB)
    src = open(HDR).read()
    max_nodes = int(re.search(r"#define FPO_SELECT_STATIC_MAX_NODES (\d+)u", src).group(1))
    nbytes = int(re.search(r"#define FPO_SELECT_STATIC_BYTES (\d+)u", src).group(1))
    assert (max_nodes, nbytes) == (fpo.SELECT_STATIC_MAX_NODES, fpo.SELECT_STATIC_BYTES)
    need = ctypes.c_uint64()
    for n in (0, 1, 4097, max_nodes - 1, max_nodes):
        assert fpo.load_library().fpo_select_workspace_size(n, ctypes.byref(need)) == fpo.FPO_OK
        assert need.value <= nbytes, n
    assert nbytes <= 1 << 20   # a modest, fixed amount per device
