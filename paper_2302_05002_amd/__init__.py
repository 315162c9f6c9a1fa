"""Python binding of libfpo: the MI355X (gfx950) octree build and decimated
preview of FastPoints (arXiv 2302.05002).

Argument marshalling only: every step runs in the HIP kernels of
``csrc/`` behind the C ABI declared in ``include/fpo.h``.  PyTorch supplies
device memory (the workspace and the inputs) and the stream.  There is no CPU
fallback: importing works anywhere, but building needs ``libfpo.so`` (built by
``paper_2302_05002_amd.build``) and a GPU, and fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfpo.so")

FPO_OK, FPO_ERR_INVALID_ARG, FPO_ERR_NONFINITE, FPO_ERR_OUT_OF_MEMORY = 0, 1, 2, 3
FPO_ERR_DEVICE, FPO_NOT_READY, FPO_ERR_REJECTED, FPO_ERR_CANCELLED = 4, 5, 6, 7
FPO_ERR_TIMEOUT = 8
FPO_BBOX_GIVEN = 1
FPO_PREVIEW_STRIDE = 2
FPO_PREVIEW_GRID = 4
PREVIEW_FLAGS = {"hash": 0, "stride": FPO_PREVIEW_STRIDE, "grid": FPO_PREVIEW_GRID}

#: every symbol include/fpo.h declares
EXPORTS = ("fpo_context_create", "fpo_context_destroy", "fpo_last_error", "fpo_workspace_size",
           "fpo_build_submit", "fpo_job_preview_ready", "fpo_job_poll", "fpo_job_wait",
           "fpo_job_result", "fpo_job_release", "fpo_workspace_size_cloud", "fpo_job_gather",
           "fpo_job_write_file", "fpo_job_export_bytes", "fpo_job_copy_to_host",
           "fpo_job_timestamps", "fpo_batch_workspace_size", "fpo_build_batch", "fpo_server_create",
           "fpo_server_submit", "fpo_job_cancel", "fpo_server_destroy", "fpo_context_set_timing", "fpo_context_set_timers", "fpo_job_timer",
           "fpo_preview_modulus", "fpo_las_parse_header", "fpo_las_header_box", "fpo_las_decode",
           "fpo_select_workspace_size", "fpo_select_nodes", "fpo_select_nodes_static",
           "fpo_job_get_stats", "fpo_context_set_batch_workers", "fpo_autotune", "fpo_autotune_batch",
           "fpo_context_force_quantize_variant", "fpo_context_set_single_block_max")
#: fpo_select_nodes_static's limits (include/fpo.h)
SELECT_STATIC_MAX_NODES = 4194304
SELECT_STATIC_BYTES = 655360

# fpo_timer values (include/fpo.h)
TIMERS = {"bbox": 0, "quantize": 1, "chunk_split": 2, "subsample": 3, "node_counts": 4, "node_place": 5,
          "preview": 6, "node_sort": 7, "cut": 8, "fused": 9}
#: quantise-pass shapes the autotuner chooses among (include/fpo.h, fpo_tuning)
QUANTIZE_VARIANTS = 5
#: largest n fpo_context_set_single_block_max accepts (include/fpo.h)
SINGLE_BLOCK_MAX_POINTS = 262143


class FpoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"fpo status {status}: {msg}")
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [("count_grid", ctypes.c_uint32), ("max_points_per_chunk", ctypes.c_uint32),
                ("subsample_grid", ctypes.c_uint32), ("leaf_capacity", ctypes.c_uint32),
                ("preview_modulus", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("bbox_min", ctypes.c_float * 3), ("bbox_max", ctypes.c_float * 3)]


FPO_DEVICE, FPO_HOST_PINNED = 0, 1


class _View(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_double * 3), ("planes", (ctypes.c_double * 4) * 6),
                ("proj_factor", ctypes.c_double), ("min_size", ctypes.c_double)]


def make_view(eye, planes, proj_factor: float, min_size: float) -> _View:
    """An fpo_view: camera position, six planes (a, b, c, e) keeping
    a*x + b*y + c*z + e >= 0, pixels per unit of radius / distance, and the
    size in pixels above which a node is refined."""
    v = _View()
    for a in range(3):
        v.eye[a] = eye[a]
    assert len(planes) == 6
    for p, q in enumerate(planes):
        for k in range(4):
            v.planes[p][k] = q[k]
    v.proj_factor = proj_factor
    v.min_size = min_size
    return v


class _LasHeader(ctypes.Structure):
    _fields_ = [("version_major", ctypes.c_uint8), ("version_minor", ctypes.c_uint8),
                ("point_format", ctypes.c_uint8), ("has_rgb", ctypes.c_uint8),
                ("record_length", ctypes.c_uint16), ("rgb_offset", ctypes.c_uint16),
                ("offset_to_points", ctypes.c_uint32), ("num_points", ctypes.c_uint64),
                ("scale", ctypes.c_double * 3), ("offset", ctypes.c_double * 3),
                ("min", ctypes.c_double * 3), ("max", ctypes.c_double * 3)]


class _Cloud(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("location", ctypes.c_uint32), ("stream_batch", ctypes.c_uint64)]


class _Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("num_chunks", ctypes.c_uint32), ("num_nodes", ctypes.c_uint32),
                ("max_depth", ctypes.c_uint32), ("chunk_oversized_any", ctypes.c_uint32),
                ("n_outside", ctypes.c_uint64), ("preview_count", ctypes.c_uint64),
                ("workspace_bytes", ctypes.c_uint64), ("submitted_ns", ctypes.c_uint64),
                ("started_ns", ctypes.c_uint64), ("completed_ns", ctypes.c_uint64),
                ("region_ms", ctypes.c_float * 16)]


class _Tuning(ctypes.Structure):
    _fields_ = [("quantize_variant", ctypes.c_uint32), ("size_class", ctypes.c_uint32),
                ("count_grid_log2", ctypes.c_uint32), ("candidates", ctypes.c_uint32),
                ("quantize_ms", ctypes.c_float * 5)]


class _Result(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("bbox_min", ctypes.c_float * 3), ("bbox_max", ctypes.c_float * 3),
                ("cube_size", ctypes.c_float), ("scale", ctypes.c_float), ("n_outside", ctypes.c_uint64),
                ("count_grid", ctypes.c_void_p), ("num_chunks", ctypes.c_uint32),
                ("chunk_level", ctypes.c_void_p), ("chunk_key", ctypes.c_void_p),
                ("chunk_count", ctypes.c_void_p), ("chunk_begin", ctypes.c_void_p),
                ("chunk_oversized_any", ctypes.c_uint8), ("perm", ctypes.c_void_p),
                ("num_nodes", ctypes.c_uint32), ("node_depth", ctypes.c_void_p), ("node_key", ctypes.c_void_p),
                ("node_child_mask", ctypes.c_void_p), ("node_begin", ctypes.c_void_p),
                ("node_count", ctypes.c_void_p), ("node_points", ctypes.c_void_p),
                ("preview_count", ctypes.c_uint64), ("preview_index", ctypes.c_void_p)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libfpo.so and declare its C signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libfpo.so is not built ({path}); run paper_2302_05002_amd.build.build()")
    lib = ctypes.CDLL(path)
    vp, P = ctypes.c_void_p, ctypes.POINTER
    lib.fpo_context_create.argtypes = [ctypes.c_int, P(vp)]
    lib.fpo_context_create.restype = ctypes.c_int
    lib.fpo_context_destroy.argtypes = [vp]
    lib.fpo_context_destroy.restype = None
    lib.fpo_last_error.argtypes = []
    lib.fpo_last_error.restype = ctypes.c_char_p
    lib.fpo_workspace_size.argtypes = [ctypes.c_uint64, P(_Params), P(ctypes.c_uint64)]
    lib.fpo_workspace_size.restype = ctypes.c_int
    lib.fpo_las_parse_header.argtypes = [vp, ctypes.c_uint64, P(_LasHeader)]
    lib.fpo_las_parse_header.restype = ctypes.c_int
    lib.fpo_las_header_box.argtypes = [P(_LasHeader), P(ctypes.c_double), P(ctypes.c_float), P(ctypes.c_float)]
    lib.fpo_las_header_box.restype = ctypes.c_int
    lib.fpo_las_decode.argtypes = [vp, P(_LasHeader), vp, ctypes.c_uint64, ctypes.c_uint64, P(ctypes.c_double), vp,
                                   vp, vp, vp, vp]
    lib.fpo_las_decode.restype = ctypes.c_int
    lib.fpo_select_workspace_size.argtypes = [ctypes.c_uint64, P(ctypes.c_uint64)]
    lib.fpo_select_workspace_size.restype = ctypes.c_int
    lib.fpo_select_nodes.argtypes = [vp, ctypes.c_uint64, vp, vp, vp, P(ctypes.c_float), ctypes.c_float, P(_View),
                                     vp, ctypes.c_uint64, vp, vp, vp]
    lib.fpo_select_nodes.restype = ctypes.c_int
    lib.fpo_select_nodes_static.argtypes = [vp, ctypes.c_uint64, vp, vp, vp, P(ctypes.c_float), ctypes.c_float,
                                            P(_View), vp, vp, vp]
    lib.fpo_select_nodes_static.restype = ctypes.c_int
    lib.fpo_preview_modulus.argtypes = [ctypes.c_uint64, ctypes.c_uint64, P(ctypes.c_uint32)]
    lib.fpo_preview_modulus.restype = ctypes.c_int
    lib.fpo_workspace_size_cloud.argtypes = [P(_Cloud), P(_Params), P(ctypes.c_uint64)]
    lib.fpo_workspace_size_cloud.restype = ctypes.c_int
    lib.fpo_build_submit.argtypes = [vp, P(_Cloud), P(_Params), vp, ctypes.c_uint64, vp, P(vp)]
    lib.fpo_build_submit.restype = ctypes.c_int
    for f in ("fpo_job_preview_ready", "fpo_job_poll", "fpo_job_wait"):
        getattr(lib, f).argtypes = [vp]
        getattr(lib, f).restype = ctypes.c_int
    lib.fpo_job_result.argtypes = [vp, P(_Result)]
    lib.fpo_job_result.restype = ctypes.c_int
    lib.fpo_job_release.argtypes = [vp]
    lib.fpo_job_release.restype = None
    u64 = ctypes.c_uint64
    lib.fpo_job_gather.argtypes = [vp, P(_Cloud), vp, ctypes.c_uint32, vp, vp, vp]
    lib.fpo_job_gather.restype = ctypes.c_int
    lib.fpo_job_write_file.argtypes = [vp, P(_Cloud), vp, ctypes.c_uint32, ctypes.c_char_p]
    lib.fpo_job_write_file.restype = ctypes.c_int
    lib.fpo_job_export_bytes.argtypes = [vp, P(u64)]
    lib.fpo_job_export_bytes.restype = ctypes.c_int
    lib.fpo_job_copy_to_host.argtypes = [vp, vp, u64]
    lib.fpo_job_copy_to_host.restype = ctypes.c_int
    lib.fpo_job_timestamps.argtypes = [vp, P(u64), P(u64), P(u64)]
    lib.fpo_job_timestamps.restype = ctypes.c_int
    lib.fpo_batch_workspace_size.argtypes = [P(_Cloud), P(_Params), ctypes.c_uint32, P(u64)]
    lib.fpo_batch_workspace_size.restype = ctypes.c_int
    lib.fpo_build_batch.argtypes = [vp, P(_Cloud), P(_Params), ctypes.c_uint32, vp, u64, vp, P(vp)]
    lib.fpo_build_batch.restype = ctypes.c_int
    lib.fpo_server_create.argtypes = [vp, u64, ctypes.c_uint32, P(vp)]
    lib.fpo_server_create.restype = ctypes.c_int
    lib.fpo_server_submit.argtypes = [vp, P(_Cloud), P(_Params), P(vp)]
    lib.fpo_server_submit.restype = ctypes.c_int
    lib.fpo_job_cancel.argtypes = [vp]
    lib.fpo_job_cancel.restype = ctypes.c_int
    lib.fpo_server_destroy.argtypes = [vp]
    lib.fpo_server_destroy.restype = None
    lib.fpo_context_set_timing.argtypes = [vp, ctypes.c_int]
    lib.fpo_context_set_timing.restype = ctypes.c_int
    lib.fpo_context_set_timers.argtypes = [vp, ctypes.c_uint32]
    lib.fpo_context_set_timers.restype = ctypes.c_int
    lib.fpo_job_timer.argtypes = [vp, ctypes.c_int, P(ctypes.c_float), P(ctypes.c_uint32)]
    lib.fpo_job_timer.restype = ctypes.c_int
    lib.fpo_job_get_stats.argtypes = [vp, P(_Stats)]
    lib.fpo_job_get_stats.restype = ctypes.c_int
    lib.fpo_context_set_batch_workers.argtypes = [vp, ctypes.c_uint32]
    lib.fpo_context_set_batch_workers.restype = ctypes.c_int
    lib.fpo_context_set_single_block_max.argtypes = [vp, ctypes.c_uint32, ctypes.c_uint32]
    lib.fpo_context_set_single_block_max.restype = ctypes.c_int
    lib.fpo_autotune.argtypes = [vp, P(_Cloud), P(_Params), vp, u64, ctypes.c_uint32, P(_Tuning)]
    lib.fpo_autotune.restype = ctypes.c_int
    lib.fpo_autotune_batch.argtypes = [vp, P(_Cloud), P(_Params), ctypes.c_uint32, vp, u64, ctypes.c_uint32,
                                       P(ctypes.c_uint32), P(ctypes.c_float)]
    lib.fpo_autotune_batch.restype = ctypes.c_int
    lib.fpo_context_force_quantize_variant.argtypes = [vp, ctypes.c_int]
    lib.fpo_context_force_quantize_variant.restype = ctypes.c_int
    _lib = lib
    return lib


def _check(st: int):
    if st != FPO_OK:
        raise FpoError(st, _lib.fpo_last_error().decode())


@dataclass
class Params:
    """G count grid, C max points per chunk, S subsample grid, L leaf capacity,
    M preview modulus; bbox = ((xmin, ymin, zmin), (xmax, ymax, zmax)) to use a
    caller-given box; preview = "hash" (H64(i) mod M == 0), "stride"
    (i mod M == 0) or "grid" (least H64 of every occupied count-grid cell)."""
    count_grid: int = 64
    max_points_per_chunk: int = 100_000
    subsample_grid: int = 32
    leaf_capacity: int = 10_000
    preview_modulus: int = 64
    bbox: tuple | None = None
    preview: str = "hash"

    def to_c(self) -> _Params:
        if self.preview not in PREVIEW_FLAGS:
            raise ValueError(f"preview must be one of {sorted(PREVIEW_FLAGS)} (got {self.preview!r})")
        flags = (FPO_BBOX_GIVEN if self.bbox is not None else 0) | PREVIEW_FLAGS[self.preview]
        p = _Params(self.count_grid, self.max_points_per_chunk, self.subsample_grid, self.leaf_capacity,
                    self.preview_modulus, flags)
        if self.bbox is not None:
            for a in range(3):
                p.bbox_min[a] = self.bbox[0][a]
                p.bbox_max[a] = self.bbox[1][a]
        return p


def workspace_size(n: int, params: Params) -> int:
    lib = load_library()
    out = ctypes.c_uint64()
    _check(lib.fpo_workspace_size(n, ctypes.byref(params.to_c()), ctypes.byref(out)))
    return int(out.value)


def preview_modulus(n: int, target: int) -> int:
    """M for a preview of about `target` points (at most `target` with preview="stride")."""
    lib = load_library()
    out = ctypes.c_uint32()
    _check(lib.fpo_preview_modulus(n, target, ctypes.byref(out)))
    return int(out.value)


_SIDE_STREAMS = {}


def _ordered_stream(dev, stream):
    """(stream to enqueue on, stream that must wait for it afterwards or None).
    The library maps a NULL stream to the context's own non-blocking stream,
    which is not ordered with torch's default (null) stream; work meant for
    that stream goes to a side stream that first waits for it instead."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    if stream.cuda_stream != 0:
        return stream, None
    side = _SIDE_STREAMS.get(dev.index)
    if side is None:
        side = _SIDE_STREAMS[dev.index] = torch.cuda.Stream(dev)
    side.wait_stream(stream)
    return side, stream


def las_parse_header(data: bytes) -> _LasHeader:
    """The public header block of a LAS file (fpo_las_parse_header)."""
    lib = load_library()
    h = _LasHeader()
    buf = ctypes.create_string_buffer(bytes(data[:4096]), min(len(data), 4096))
    _check(lib.fpo_las_parse_header(buf, min(len(data), 4096), ctypes.byref(h)))
    return h


def las_header_box(h: _LasHeader, origin=(0.0, 0.0, 0.0)):
    """((lo), (hi)) of the header's box in the decoded frame, float32 values."""
    lib = load_library()
    o = (ctypes.c_double * 3)(*origin)
    lo, hi = (ctypes.c_float * 3)(), (ctypes.c_float * 3)()
    _check(lib.fpo_las_header_box(ctypes.byref(h), o, lo, hi))
    return tuple(lo), tuple(hi)


class Context:
    """One device: its own stream and pinned staging."""

    def __init__(self, device: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: libfpo runs only on an MI355X (gfx950)")
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.fpo_context_create(device, ctypes.byref(h)))
        self._h = h
        self.device = device

    def close(self):
        if self._h:
            _lib.fpo_context_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_timing(self, enable: bool, only=None):
        """Bracket the timed kernels of later submits with HIP events: every
        timer, or only the named ones (keys of TIMERS)."""
        if only is None:
            _check(_lib.fpo_context_set_timing(self._h, 1 if enable else 0))
        else:
            mask = 0
            for name in only:
                mask |= 1 << TIMERS[name]
            _check(_lib.fpo_context_set_timers(self._h, mask if enable else 0))

    def submit(self, x, y, z, params: Params, workspace=None, stream=None, stream_batch: int = 0) -> "Job":
        """Enqueue a build of x, y, z (float32, contiguous): device tensors,
        or pinned host tensors (copied in batches of stream_batch points).
        Allocates the workspace with torch when none is given."""
        import torch
        n = int(x.shape[0])
        host = not x.is_cuda
        for t in (x, y, z):
            assert t.dtype == torch.float32 and t.is_contiguous() and t.shape[0] == n and t.is_cuda != host
            assert not host or t.is_pinned(), "host inputs must be pinned"
        cloud = _Cloud(n, x.data_ptr(), y.data_ptr(), z.data_ptr(), FPO_HOST_PINNED if host else FPO_DEVICE,
                       int(stream_batch))
        need = ctypes.c_uint64()
        _check(_lib.fpo_workspace_size_cloud(ctypes.byref(cloud), ctypes.byref(params.to_c()), ctypes.byref(need)))
        dev = torch.device("cuda", self.device)
        if workspace is None:
            workspace = torch.empty(int(need.value), dtype=torch.uint8, device=dev)
        stream, _ = _ordered_stream(dev, stream)   # inputs ready; results are read after wait()
        h = ctypes.c_void_p()
        _check(_lib.fpo_build_submit(self._h, ctypes.byref(cloud), ctypes.byref(params.to_c()),
                                     ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                     ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        return Job(h, workspace, params, (x, y, z), self)

    def las_decode(self, records, header: _LasHeader, origin=(0.0, 0.0, 0.0), rgb: bool = False, n=None,
                   stream=None):
        """Decode LAS point records (a uint8 device tensor, any alignment) into
        float32 x, y, z device tensors (and uint16 [n, 3] colours when rgb).
        Enqueued on `stream` (default: torch's current stream)."""
        import torch
        assert records.is_cuda and records.dtype == torch.uint8 and records.is_contiguous()
        if n is None:
            n = records.numel() // header.record_length
        dev = records.device
        x, y, z = (torch.empty(n, dtype=torch.float32, device=dev) for _ in range(3))
        col = torch.empty((n, 3), dtype=torch.int16, device=dev) if rgb else None
        stream, back = _ordered_stream(dev, stream)
        o = (ctypes.c_double * 3)(*origin)
        _check(_lib.fpo_las_decode(self._h, ctypes.byref(header), ctypes.c_void_p(records.data_ptr()),
                                   records.numel(), n, o,
                                   ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                   ctypes.c_void_p(z.data_ptr()),
                                   ctypes.c_void_p(col.data_ptr()) if rgb else None,
                                   ctypes.c_void_p(stream.cuda_stream)))
        if back is not None:
            back.wait_stream(stream)
        return x, y, z, col

    def select_nodes(self, node_depth, node_key, node_count, bbox_min, cube_size, view: _View, workspace=None,
                     stream=None):
        """Drawn nodes of one view (fpo_select_nodes) from device node arrays
        (uint8 depth, int64 key, int32 count tensors): (ascending int32 index
        tensor, number of drawn points).  Synchronises the stream it runs on."""
        import torch
        n = int(node_depth.shape[0])
        assert node_key.shape[0] == n and node_count.shape[0] == n
        dev = node_depth.device if n else torch.device("cuda", self.device)
        need = ctypes.c_uint64()
        _check(_lib.fpo_select_workspace_size(n, ctypes.byref(need)))
        if workspace is None:
            workspace = torch.empty(int(need.value), dtype=torch.uint8, device=dev)
        out = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        totals = torch.zeros(2, dtype=torch.int32, device=dev)
        stream, back = _ordered_stream(dev, stream)
        lo = (ctypes.c_float * 3)(*[float(v) for v in bbox_min])
        ptr = (lambda t: ctypes.c_void_p(t.data_ptr() if n else 0))
        _check(_lib.fpo_select_nodes(self._h, n, ptr(node_depth), ptr(node_key), ptr(node_count), lo,
                                     float(cube_size), ctypes.byref(view), ctypes.c_void_p(workspace.data_ptr()),
                                     workspace.numel(), ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_void_p(totals.data_ptr()), ctypes.c_void_p(stream.cuda_stream)))
        if back is not None:
            back.wait_stream(stream)
        stream.synchronize()
        t = totals.cpu().tolist()
        return out[:t[0]], t[1]

    def select_nodes_static(self, node_depth, node_key, node_count, bbox_min, cube_size, view: _View, out=None,
                            totals=None, stream=None):
        """select_nodes without a workspace (fpo_select_nodes_static: the
        library's static scratch, at most SELECT_STATIC_MAX_NODES nodes).
        Enqueues on `stream` and returns (out, totals) device tensors without
        synchronising: out[:totals[0]] are the drawn nodes, totals[1] their
        points.  Pass preallocated out / totals to allocate nothing here."""
        import torch
        n = int(node_depth.shape[0])
        dev = node_depth.device if n else torch.device("cuda", self.device)
        if out is None:
            out = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        if totals is None:
            totals = torch.empty(2, dtype=torch.int32, device=dev)
        stream, back = _ordered_stream(dev, stream)
        lo = (ctypes.c_float * 3)(*[float(v) for v in bbox_min])
        ptr = (lambda t: ctypes.c_void_p(t.data_ptr() if n else 0))
        _check(_lib.fpo_select_nodes_static(self._h, n, ptr(node_depth), ptr(node_key), ptr(node_count), lo,
                                            float(cube_size), ctypes.byref(view), ctypes.c_void_p(out.data_ptr()),
                                            ctypes.c_void_p(totals.data_ptr()), ctypes.c_void_p(stream.cuda_stream)))
        if back is not None:
            back.wait_stream(stream)
        return out, totals

    def build(self, x, y, z, params: Params, workspace=None, stream=None) -> "Result":
        job = self.submit(x, y, z, params, workspace, stream)
        try:
            job.wait()
            return job.result()
        finally:
            job.release()   # the result views the workspace, not the job

    def autotune(self, x, y, z, params: Params, workspace=None, reps: int = 5) -> dict:
        """fpo_autotune on device tensors x, y, z: the fastest quantise shape
        for clouds of this size class and count grid (kept in the context)."""
        import torch
        n = int(x.shape[0])
        for t in (x, y, z):
            assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.shape[0] == n
        cloud = _Cloud(n, x.data_ptr(), y.data_ptr(), z.data_ptr())
        if workspace is None:
            workspace = torch.empty(workspace_size(n, params), dtype=torch.uint8, device=x.device)
        torch.cuda.synchronize(x.device)   # inputs written on torch's streams are complete
        t = _Tuning()
        _check(_lib.fpo_autotune(self._h, ctypes.byref(cloud), ctypes.byref(params.to_c()),
                                 ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), int(reps),
                                 ctypes.byref(t)))
        return {"quantize_variant": int(t.quantize_variant), "size_class": int(t.size_class),
                "count_grid_log2": int(t.count_grid_log2),
                "quantize_ms": [float(t.quantize_ms[i]) for i in range(int(t.candidates))]}

    def autotune_batch(self, clouds, params, workspace=None, reps: int = 3) -> dict:
        """fpo_autotune_batch: the fastest number of batch worker streams."""
        import torch
        count = len(clouds)
        if isinstance(params, Params):
            params = [params] * count
        cs = (_Cloud * count)()
        ps = (_Params * count)()
        for i, (x, y, z) in enumerate(clouds):
            cs[i] = _Cloud(int(x.shape[0]), x.data_ptr(), y.data_ptr(), z.data_ptr())
            ps[i] = params[i].to_c()
        need = ctypes.c_uint64()
        _check(_lib.fpo_batch_workspace_size(cs, ps, count, ctypes.byref(need)))
        if workspace is None:
            workspace = torch.empty(max(int(need.value), 1), dtype=torch.uint8, device=clouds[0][0].device)
        torch.cuda.synchronize()
        w = ctypes.c_uint32()
        ms = (ctypes.c_float * 3)()
        _check(_lib.fpo_autotune_batch(self._h, cs, ps, count, ctypes.c_void_p(workspace.data_ptr()),
                                       workspace.numel(), int(reps), ctypes.byref(w), ms))
        return {"workers": int(w.value), "batch_ms": {c: float(ms[i]) for i, c in enumerate((2, 4, 8))}}

    def force_quantize_variant(self, variant: int):
        """Force the quantise shape of later builds (0..2), -1 for the tuned one."""
        _check(_lib.fpo_context_force_quantize_variant(self._h, int(variant)))

    def set_batch_workers(self, workers: int):
        """Worker streams of later build_batch calls (1..16, default 4)."""
        _check(_lib.fpo_context_set_batch_workers(self._h, int(workers)))

    def set_single_block_max(self, plain_max: int, batch_max: int | None = None):
        """Clouds up to plain_max points (plain and served builds) or batch_max
        points (build_batch; default: plain_max), within the path's other
        limits, are built by one workgroup in one launch; 0 turns that off."""
        bm = plain_max if batch_max is None else batch_max
        _check(_lib.fpo_context_set_single_block_max(self._h, int(plain_max), int(bm)))

    def build_batch(self, clouds, params, workspace=None, stream=None) -> list:
        """Enqueue one build per (x, y, z) device-tensor triple in `clouds`,
        with params[i] (one Params for all, or a list).  Returns the jobs, in
        the order of the clouds."""
        import torch
        count = len(clouds)
        if isinstance(params, Params):
            params = [params] * count
        assert len(params) == count
        cs = (_Cloud * max(count, 1))()
        ps = (_Params * max(count, 1))()
        dev = None
        for i, (x, y, z) in enumerate(clouds):
            n = int(x.shape[0])
            for t in (x, y, z):
                assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.shape[0] == n
            cs[i] = _Cloud(n, x.data_ptr(), y.data_ptr(), z.data_ptr())
            ps[i] = params[i].to_c()
            dev = x.device
        need = ctypes.c_uint64()
        _check(_lib.fpo_batch_workspace_size(cs, ps, count, ctypes.byref(need)))
        if count == 0:
            return []
        if workspace is None:
            workspace = torch.empty(max(int(need.value), 1), dtype=torch.uint8, device=dev)
        stream, _ = _ordered_stream(dev, stream)
        hs = (ctypes.c_void_p * count)()
        _check(_lib.fpo_build_batch(self._h, cs, ps, count, ctypes.c_void_p(workspace.data_ptr()),
                                    workspace.numel(), ctypes.c_void_p(stream.cuda_stream), hs))
        return [Job(ctypes.c_void_p(hs[i]), workspace, params[i], clouds[i], self) for i in range(count)]


class Server:
    """Request loop over one device: builds admitted by free slots and an HBM
    budget (the server's own arena), overlapping on the device."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_slots: int = 4):
        self.ctx = ctx
        h = ctypes.c_void_p()
        _check(_lib.fpo_server_create(ctx._h, int(hbm_budget_bytes), int(max_slots), ctypes.byref(h)))
        self._h = h

    def submit(self, x, y, z, params: Params) -> "Job":
        """Queue a build of the device tensors x, y, z (never blocks).  The
        result is read with Job.to_numpy(): it lives in the server's arena."""
        import torch
        n = int(x.shape[0])
        for t in (x, y, z):
            assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.shape[0] == n
        cloud = _Cloud(n, x.data_ptr(), y.data_ptr(), z.data_ptr())
        h = ctypes.c_void_p()
        _check(_lib.fpo_server_submit(self._h, ctypes.byref(cloud), ctypes.byref(params.to_c()), ctypes.byref(h)))
        return Job(h, None, params, (x, y, z), self)

    def close(self):
        if self._h:
            _lib.fpo_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Job:
    """One build.  It keeps its owner (the Context or Server that made it)
    alive, so whatever order handles are dropped in, a job is released before
    its owner is destroyed (the library also counts these references)."""

    def __init__(self, h, workspace, params, inputs, owner):
        self._h = h
        self.workspace = workspace
        self.params = params
        self._inputs = inputs
        self._owner = owner

    def preview_ready(self) -> bool:
        st = _lib.fpo_job_preview_ready(self._h)
        if st == FPO_NOT_READY:
            return False
        _check(st)
        return True

    def poll(self) -> bool:
        st = _lib.fpo_job_poll(self._h)
        if st == FPO_NOT_READY:
            return False
        _check(st)
        return True

    def wait(self):
        _check(_lib.fpo_job_wait(self._h))

    def result(self) -> "Result":
        r = _Result()
        _check(_lib.fpo_job_result(self._h, ctypes.byref(r)))
        return Result(r, self.workspace, self.params)

    @staticmethod
    def _cloud_and_color(x, y, z, color):
        import torch
        n = int(x.shape[0])
        for t in (x, y, z):
            assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.shape[0] == n
        stride = 0
        if color is not None:
            assert color.is_cuda and color.dtype == torch.uint8 and color.is_contiguous() and color.shape[0] == n
            stride = int(color.shape[1]) if color.dim() == 2 else 1
        return _Cloud(n, x.data_ptr(), y.data_ptr(), z.data_ptr()), stride

    def gather(self, x, y, z, color=None, stream=None):
        """Points of a completed job in node order: (xyz (n, 3) float32, colour (n, stride) uint8 or None)."""
        import torch
        cloud, stride = self._cloud_and_color(x, y, z, color)
        n = int(cloud.n)
        out_xyz = torch.empty((n, 3), dtype=torch.float32, device=x.device)
        out_col = torch.empty((n, stride), dtype=torch.uint8, device=x.device) if stride else None
        stream, back = _ordered_stream(x.device, stream)
        _check(_lib.fpo_job_gather(self._h, ctypes.byref(cloud), ctypes.c_void_p(color.data_ptr() if stride else 0),
                                   stride, ctypes.c_void_p(out_xyz.data_ptr()),
                                   ctypes.c_void_p(out_col.data_ptr() if stride else 0),
                                   ctypes.c_void_p(stream.cuda_stream)))
        if back is not None:
            back.wait_stream(stream)
        return out_xyz, out_col

    def write_file(self, path: str, x, y, z, color=None):
        """Hierarchy + node-ordered points of a completed job in one file."""
        cloud, stride = self._cloud_and_color(x, y, z, color)
        _check(_lib.fpo_job_write_file(self._h, ctypes.byref(cloud),
                                       ctypes.c_void_p(color.data_ptr() if stride else 0), stride,
                                       str(path).encode()))

    def cancel(self) -> bool:
        """Take a batch or server job that has not started out of its queue."""
        return _lib.fpo_job_cancel(self._h) == FPO_OK

    def timestamps(self):
        """(submitted, started, completed) host steady-clock ns of a completed job."""
        a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(_lib.fpo_job_timestamps(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return int(a.value), int(b.value), int(c.value)

    def to_numpy(self) -> dict:
        """Every output of a completed job as host numpy arrays (through the
        packed export of the C ABI; works for every kind of job)."""
        r = _Result()
        _check(_lib.fpo_job_result(self._h, ctypes.byref(r)))
        nbytes = ctypes.c_uint64()
        _check(_lib.fpo_job_export_bytes(self._h, ctypes.byref(nbytes)))
        buf = np.empty(max(int(nbytes.value), 8), dtype=np.uint8)
        _check(_lib.fpo_job_copy_to_host(self._h, ctypes.c_void_p(buf.ctypes.data), buf.nbytes))
        n, nc, nn, pc = int(r.n), int(r.num_chunks), int(r.num_nodes), int(r.preview_count)
        G = self.params.count_grid
        layout = [("count_grid", np.uint32, G ** 3), ("chunk_level", np.uint8, nc), ("chunk_key", np.uint64, nc),
                  ("chunk_count", np.uint32, nc), ("chunk_begin", np.uint64, nc), ("perm", np.uint32, n),
                  ("node_depth", np.uint8, nn), ("node_key", np.uint64, nn), ("node_child_mask", np.uint8, nn),
                  ("node_begin", np.uint64, nn), ("node_count", np.uint32, nn), ("node_points", np.uint32, n),
                  ("preview_index", np.uint32, pc)]
        out = dict(status=FPO_OK, n=n, bbox_min=np.array(r.bbox_min[:], dtype=np.float32),
                   bbox_max=np.array(r.bbox_max[:], dtype=np.float32), cube_size=np.float32(r.cube_size),
                   scale=np.float32(r.scale), n_outside=int(r.n_outside),
                   chunk_oversized_any=int(r.chunk_oversized_any))
        off = 0
        for name, dt, cnt in layout:
            off = (off + 7) & ~7
            nb = cnt * np.dtype(dt).itemsize
            out[name] = buf[off:off + nb].view(dt).copy()
            off += nb
        return out

    def stats(self) -> dict:
        """fpo_job_get_stats of a completed job, as a dict (region_ms by timer
        name, only the timed regions)."""
        st = _Stats()
        _check(_lib.fpo_job_get_stats(self._h, ctypes.byref(st)))
        out = {k: getattr(st, k) for k, _ in _Stats._fields_ if k != "region_ms"}
        out["region_ms"] = {name: float(st.region_ms[t]) for name, t in TIMERS.items() if st.region_ms[t] >= 0}
        return out

    def timer(self, name: str):
        """(summed device ms, launches) of a timer of a completed, timed job."""
        ms, k = ctypes.c_float(), ctypes.c_uint32()
        _check(_lib.fpo_job_timer(self._h, TIMERS[name], ctypes.byref(ms), ctypes.byref(k)))
        return float(ms.value), int(k.value)

    def release(self):
        if self._h:
            _lib.fpo_job_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


class Result:
    """Host scalars plus device tensors viewing the workspace."""

    def __init__(self, r: _Result, ws, params: Params):
        import torch
        self.n = int(r.n)
        self.bbox_min = np.array(r.bbox_min[:], dtype=np.float32)
        self.bbox_max = np.array(r.bbox_max[:], dtype=np.float32)
        self.cube_size = np.float32(r.cube_size)
        self.scale = np.float32(r.scale)
        self.n_outside = int(r.n_outside)
        self.num_chunks = int(r.num_chunks)
        self.num_nodes = int(r.num_nodes)
        self.preview_count = int(r.preview_count)
        self.chunk_oversized_any = int(r.chunk_oversized_any)
        base = ws.data_ptr()
        G = params.count_grid

        def view(ptr, count, dtype, itemsize):
            if count == 0 or not ptr:
                return torch.empty(0, dtype=dtype, device=ws.device)
            off = ptr - base
            assert 0 <= off and off + count * itemsize <= ws.numel()
            return ws[off:off + count * itemsize].view(dtype)

        u8, i32, i64 = torch.uint8, torch.int32, torch.int64
        self.count_grid = view(r.count_grid, G ** 3, i32, 4)
        self.chunk_level = view(r.chunk_level, self.num_chunks, u8, 1)
        self.chunk_key = view(r.chunk_key, self.num_chunks, i64, 8)
        self.chunk_count = view(r.chunk_count, self.num_chunks, i32, 4)
        self.chunk_begin = view(r.chunk_begin, self.num_chunks, i64, 8)
        self.perm = view(r.perm, self.n, i32, 4)
        self.node_depth = view(r.node_depth, self.num_nodes, u8, 1)
        self.node_key = view(r.node_key, self.num_nodes, i64, 8)
        self.node_child_mask = view(r.node_child_mask, self.num_nodes, u8, 1)
        self.node_begin = view(r.node_begin, self.num_nodes, i64, 8)
        self.node_count = view(r.node_count, self.num_nodes, i32, 4)
        self.node_points = view(r.node_points, self.n, i32, 4)
        self.preview_index = view(r.preview_index, self.preview_count, i32, 4)

    def to_numpy(self) -> dict:
        """Copy everything to host numpy arrays (unsigned dtypes)."""
        def cpu(t, dt):
            return t.cpu().numpy().view(dt)
        return dict(
            status=FPO_OK, n=self.n, bbox_min=self.bbox_min, bbox_max=self.bbox_max, cube_size=self.cube_size,
            scale=self.scale, n_outside=self.n_outside,
            count_grid=cpu(self.count_grid, np.uint32), chunk_level=cpu(self.chunk_level, np.uint8),
            chunk_key=cpu(self.chunk_key, np.uint64), chunk_count=cpu(self.chunk_count, np.uint32),
            chunk_begin=cpu(self.chunk_begin, np.uint64), chunk_oversized_any=self.chunk_oversized_any,
            perm=cpu(self.perm, np.uint32), node_depth=cpu(self.node_depth, np.uint8),
            node_key=cpu(self.node_key, np.uint64), node_child_mask=cpu(self.node_child_mask, np.uint8),
            node_begin=cpu(self.node_begin, np.uint64), node_count=cpu(self.node_count, np.uint32),
            node_points=cpu(self.node_points, np.uint32), preview_index=cpu(self.preview_index, np.uint32))


def read_file(path: str) -> dict:
    """Parse a file written by Job.write_file (layout in include/fpo.h)."""
    raw = np.fromfile(path, dtype=np.uint8)
    assert raw[:4].tobytes() == b"FPO1", "not an FPO1 file"
    hdr = raw[:48]
    version, = hdr[4:8].view(np.uint32)
    n, = hdr[8:16].view(np.uint64)
    num_nodes, stride = hdr[16:24].view(np.uint32)
    bbox_min = hdr[24:36].view(np.float32)
    cube_size, = hdr[36:40].view(np.float32)
    G, S = hdr[40:48].view(np.uint32)
    n, num_nodes, stride = int(n), int(num_nodes), int(stride)
    rec = raw[48:48 + 24 * num_nodes].reshape(num_nodes, 24)
    nodes = dict(depth=rec[:, 0].copy(), child_mask=rec[:, 1].copy(),
                 count=rec[:, 4:8].copy().view(np.uint32).ravel(), key=rec[:, 8:16].copy().view(np.uint64).ravel(),
                 begin=rec[:, 16:24].copy().view(np.uint64).ravel())
    off = 48 + 24 * num_nodes
    xyz = raw[off:off + 12 * n].view(np.float32).reshape(n, 3)
    off += 12 * n
    color = raw[off:off + stride * n].reshape(n, stride) if stride else None
    return dict(version=int(version), n=n, num_nodes=num_nodes, color_stride=stride, bbox_min=bbox_min.copy(),
                cube_size=np.float32(cube_size), count_grid=int(G), subsample_grid=int(S), nodes=nodes,
                xyz=xyz.copy(), color=None if color is None else color.copy())
