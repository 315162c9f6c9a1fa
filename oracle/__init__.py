"""CPU oracle for the FastPoints (arXiv 2302.05002) octree build and preview.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, by ``__graft_entry__.smoke``
and by the ``cpu_baseline`` leg of ``bench.py``; the library under
``paper_2302_05002_amd/`` never imports it.  The arithmetic lives in plain C
(``fpo_oracle.c``), compiled here with gcc; this module only marshals numpy
arrays through ctypes.

Every function of the C file follows one step of the path in the order the
paper gives (section "Octree Construction": chunking, per-chunk indexing into
local octrees, one global tree; section "Immediate Low-Resolution Rendering":
a decimation that visits every point).  Parity is pinned for every step (see
``tests/test_oracle_*.py``); nothing here is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fpo_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, ERR_INVALID_ARG, ERR_NONFINITE, ERR_OOM = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain IEEE float: no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
             "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("count_grid", ctypes.c_uint32), ("max_points_per_chunk", ctypes.c_uint32),
                ("subsample_grid", ctypes.c_uint32), ("leaf_capacity", ctypes.c_uint32),
                ("preview_modulus", ctypes.c_uint32), ("bbox_given", ctypes.c_uint32),
                ("bbox_min", ctypes.c_float * 3), ("bbox_max", ctypes.c_float * 3),
                ("preview_mode", ctypes.c_uint32)]


PREVIEW_MODES = {"hash": 0, "stride": 1, "grid": 2}

_P = ctypes.POINTER


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("n", ctypes.c_uint64),
                ("bbox_min", ctypes.c_float * 3), ("bbox_max", ctypes.c_float * 3),
                ("cube_size", ctypes.c_float), ("scale", ctypes.c_float),
                ("n_outside", ctypes.c_uint64),
                ("u", _P(ctypes.c_uint32)), ("count_grid", _P(ctypes.c_uint32)),
                ("num_chunks", ctypes.c_uint32), ("chunk_level", _P(ctypes.c_uint8)),
                ("chunk_key", _P(ctypes.c_uint64)), ("chunk_count", _P(ctypes.c_uint32)),
                ("chunk_begin", _P(ctypes.c_uint64)), ("chunk_oversized_any", ctypes.c_uint8),
                ("perm", _P(ctypes.c_uint32)),
                ("num_nodes", ctypes.c_uint32), ("node_depth", _P(ctypes.c_uint8)),
                ("node_key", _P(ctypes.c_uint64)), ("node_child_mask", _P(ctypes.c_uint8)),
                ("node_begin", _P(ctypes.c_uint64)), ("node_count", _P(ctypes.c_uint32)),
                ("node_points", _P(ctypes.c_uint32)),
                ("preview_count", ctypes.c_uint64), ("preview_index", _P(ctypes.c_uint32))]


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        lib.oracle_build.argtypes = [ctypes.c_uint64, _P(ctypes.c_float), _P(ctypes.c_float),
                                     _P(ctypes.c_float), _P(_Params), _P(_Result)]
        lib.oracle_build.restype = ctypes.c_int
        lib.oracle_free.argtypes = [_P(_Result)]
        lib.oracle_free.restype = None
        lib.oracle_h64.argtypes = [ctypes.c_uint64]
        lib.oracle_h64.restype = ctypes.c_uint64
        _lib = lib
    return _lib


@dataclass
class Params:
    """Build parameters: G count grid, C max points per chunk, S subsample grid,
    L leaf capacity, M preview modulus; optional caller-given bounding box;
    preview variant "hash" (H64(i) mod M == 0), "stride" (i mod M == 0) or
    "grid" (least H64 of every occupied count-grid cell)."""
    count_grid: int = 64
    max_points_per_chunk: int = 100_000
    subsample_grid: int = 32
    leaf_capacity: int = 10_000
    preview_modulus: int = 64
    bbox: tuple | None = None  # ((xmin, ymin, zmin), (xmax, ymax, zmax))
    preview: str = "hash"


def h64(i: int) -> int:
    """The preview hash of one index."""
    return int(_load().oracle_h64(int(i)))


def _arr(ptr, count, dtype):
    if count == 0:
        return np.zeros(0, dtype=dtype)
    return np.ctypeslib.as_array(ptr, shape=(count,)).astype(dtype, copy=True)


def build_octree(x, y, z, params: Params) -> dict:
    """Run the whole path on the CPU.  Returns a dict of numpy arrays (status
    under key ``status``; the arrays are present only when it is OK)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    z = np.ascontiguousarray(z, dtype=np.float32)
    n = int(x.shape[0])
    assert y.shape[0] == n and z.shape[0] == n
    p = _Params(params.count_grid, params.max_points_per_chunk, params.subsample_grid,
                params.leaf_capacity, params.preview_modulus, 1 if params.bbox is not None else 0)
    p.preview_mode = PREVIEW_MODES[params.preview]
    if params.bbox is not None:
        for a in range(3):
            p.bbox_min[a] = params.bbox[0][a]
            p.bbox_max[a] = params.bbox[1][a]
    r = _Result()
    fp = _P(ctypes.c_float)
    st = lib.oracle_build(n, x.ctypes.data_as(fp), y.ctypes.data_as(fp), z.ctypes.data_as(fp),
                          ctypes.byref(p), ctypes.byref(r))
    out = {"status": int(st)}
    try:
        if st != OK:
            return out
        G = params.count_grid
        out.update(
            n=n,
            bbox_min=np.array(r.bbox_min[:], dtype=np.float32),
            bbox_max=np.array(r.bbox_max[:], dtype=np.float32),
            cube_size=np.float32(r.cube_size), scale=np.float32(r.scale),
            n_outside=int(r.n_outside),
            u=_arr(r.u, 3 * n, np.uint32).reshape(n, 3),
            count_grid=_arr(r.count_grid, G * G * G, np.uint32),
            chunk_level=_arr(r.chunk_level, r.num_chunks, np.uint8),
            chunk_key=_arr(r.chunk_key, r.num_chunks, np.uint64),
            chunk_count=_arr(r.chunk_count, r.num_chunks, np.uint32),
            chunk_begin=_arr(r.chunk_begin, r.num_chunks, np.uint64),
            chunk_oversized_any=int(r.chunk_oversized_any),
            perm=_arr(r.perm, n, np.uint32),
            node_depth=_arr(r.node_depth, r.num_nodes, np.uint8),
            node_key=_arr(r.node_key, r.num_nodes, np.uint64),
            node_child_mask=_arr(r.node_child_mask, r.num_nodes, np.uint8),
            node_begin=_arr(r.node_begin, r.num_nodes, np.uint64),
            node_count=_arr(r.node_count, r.num_nodes, np.uint32),
            node_points=_arr(r.node_points, n, np.uint32),
            preview_index=_arr(r.preview_index, r.preview_count, np.uint32),
        )
        return out
    finally:
        lib.oracle_free(ctypes.byref(r))
