"""Pins of the LAS decode oracle (section "File Importing": clouds arrive as
LAS files): a hand-worked file packed byte by byte, pure-Python IEEE double
arithmetic per record on small files, the writer's round trip within half a
quantum, every record format's colour offset, and rejection of LAZ and of
short records."""
import json
import os
import struct

import numpy as np
import pytest

import synth
from oracle import las
from synth.las import write_las

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _hand_file(ex):
    """LAS 1.2, format 2, packed field by field from the fixture."""
    hdr = bytearray(227)
    hdr[0:4] = b"LASF"
    hdr[24], hdr[25] = 1, 2
    struct.pack_into("<H", hdr, 94, 227)
    struct.pack_into("<I", hdr, 96, 227 + 10)   # ten bytes standing in for VLRs
    hdr[104] = 2
    struct.pack_into("<H", hdr, 105, 26)
    struct.pack_into("<I", hdr, 107, len(ex["X"]))
    struct.pack_into("<3d", hdr, 131, *ex["scale"])
    struct.pack_into("<3d", hdr, 155, *ex["offset"])
    mn, mx = ex["min"], ex["max"]
    struct.pack_into("<6d", hdr, 179, mx[0], mn[0], mx[1], mn[1], mx[2], mn[2])
    recs = b""
    for (X, Y, Z), (r, g, b) in zip(ex["X"], ex["rgb"]):
        recs += struct.pack("<3i", X, Y, Z) + bytes(range(8)) + struct.pack("<3H", r, g, b)
    return bytes(hdr) + bytes(10) + recs


def test_worked_example():
    ex = json.load(open(os.path.join(GOLD, "las_worked_example.json")))
    f = _hand_file(ex)
    h = las.parse_header(f)
    assert h.version == (1, 2) and h.point_format == 2 and h.record_length == 26 and h.num_points == 3
    assert h.offset_to_points == 237
    assert h.scale == tuple(ex["scale"]) and h.offset == tuple(ex["offset"])
    assert h.min == tuple(ex["min"]) and h.max == tuple(ex["max"])
    x, y, z, rgb = las.decode(f[h.offset_to_points:], h, ex["origin"])
    assert x.tolist() == ex["x"] and y.tolist() == ex["y"] and z.tolist() == ex["z"]
    assert x.dtype == np.float32 and rgb.tolist() == ex["rgb"]
    lo, hi = las.header_box(h, ex["origin"])
    assert list(lo) == ex["box_lo"] and list(hi) == ex["box_hi"]


def _python_decode(records, rec_len, fmt, scale, offset, origin):
    """Record by record with struct and Python floats (IEEE doubles)."""
    xs, cols = [], []
    ro = las.FORMAT_RGB_OFFSET[fmt]
    for k in range(len(records) // rec_len):
        X = struct.unpack_from("<3i", records, k * rec_len)
        xs.append([np.float32(X[a] * scale[a] + offset[a] - origin[a]) for a in range(3)])
        if ro is not None:
            cols.append(list(struct.unpack_from("<3H", records, k * rec_len + ro)))
    return np.array(xs, dtype=np.float32).reshape(-1, 3), cols


@pytest.mark.parametrize("fmt,version,extra", [(0, (1, 2), 0), (1, (1, 2), 3), (2, (1, 2), 0), (3, (1, 3), 1),
                                               (5, (1, 3), 0), (6, (1, 4), 0), (7, (1, 4), 2), (8, (1, 4), 0),
                                               (10, (1, 4), 5), (4, (1, 3), 0), (9, (1, 4), 0)])
def test_python_brute_force(fmt, version, extra):
    c = synth.planes(3_000, seed=fmt + 1, num_planes=4)
    rng = np.random.default_rng(fmt)
    rgb = rng.integers(0, 65536, size=(c.n, 3), dtype=np.uint16)
    scale, offset = (0.001, 0.002, 0.0005), (631_000.0, 4_833_000.0, -12.5)
    f = write_las(c.x + 631_000.0, c.y + 4_833_000.0, c.z, rgb=rgb, scale=scale, offset=offset, point_format=fmt,
                  version=version, extra_bytes=extra, vlr_bytes=7, seed=fmt)
    h = las.parse_header(f)
    assert h.num_points == c.n and h.record_length == las.FORMAT_MIN_LENGTH[fmt] + extra
    recs = f[h.offset_to_points:]
    origin = (631_000.0, 4_833_000.0, 0.0)
    x, y, z, col = las.decode(recs, h, origin)
    exp, ecol = _python_decode(recs, h.record_length, fmt, scale, offset, origin)
    np.testing.assert_array_equal(np.stack([x, y, z], 1).view(np.uint32), exp.view(np.uint32))
    if las.FORMAT_RGB_OFFSET[fmt] is None:
        assert col is None
    else:
        assert col.tolist() == ecol
        np.testing.assert_array_equal(col, rgb)


def test_round_trip_within_half_a_quantum():
    c = synth.uniform(10_000, seed=5, lo=-300.0, hi=900.0)
    scale = (0.01, 0.01, 0.001)
    f = write_las(c.x, c.y, c.z, scale=scale, offset=(0.0, 0.0, 0.0), point_format=0)
    h = las.parse_header(f)
    x, y, z, _ = las.decode(f[h.offset_to_points:], h)
    for a, (got, src) in enumerate(((x, c.x), (y, c.y), (z, c.z))):
        # |decoded - source| <= scale/2 plus the two float32 roundings
        err = np.abs(got.astype(np.float64) - src.astype(np.float64))
        assert err.max() <= scale[a] / 2 + 2 * np.spacing(np.float32(900.0))
    lo, hi = las.header_box(h)
    assert lo == (float(x.min()), float(y.min()), float(z.min()))
    assert hi == (float(x.max()), float(y.max()), float(z.max()))


def test_rejections():
    c = synth.uniform(10, seed=1)
    f = bytearray(write_las(c.x, c.y, c.z, point_format=3))
    las.parse_header(bytes(f))
    g = bytearray(f)
    g[104] = 3 | 0x80          # LAZ-compressed record format
    with pytest.raises(ValueError):
        las.parse_header(bytes(g))
    g = bytearray(f)
    struct.pack_into("<H", g, 105, 33)   # shorter than format 3's 34 bytes
    with pytest.raises(ValueError):
        las.parse_header(bytes(g))
    with pytest.raises(ValueError):
        las.parse_header(b"LASG" + bytes(f[4:]))
    with pytest.raises(ValueError):
        las.parse_header(bytes(f[:200]))
