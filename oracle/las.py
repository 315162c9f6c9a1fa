"""Oracle of the LAS fixed-record decode (TEST INFRASTRUCTURE ONLY: imported
by tests/, and by nothing under paper_2302_05002_amd/).

Section "File Importing" of the paper: clouds arrive as LAS files, whose
point records are fixed-size little-endian structures holding integer
coordinates X, Y, Z that a header's scale and offset turn into real
coordinates (ASPRS LAS specification, public header block and point data
record formats 0-10).  The path works on float32 structure-of-arrays, so the
decode is:

    v = X * scale + offset        (IEEE double, two roundings)
    w = v - origin                (IEEE double, one rounding; origin chosen by the caller)
    x = float32(w)                (round to nearest even)

per axis, and R, G, B (uint16) copied where the record format has them.
LAZ (compressed) records are out of scope.  numpy float64 arithmetic is IEEE
round-to-nearest with no fused multiply-add, which is this definition.
"""
from __future__ import annotations

import struct
from dataclasses import dataclass

import numpy as np

# minimum record length and byte offset of R, G, B (None: no colour) of the
# point data record formats 0-10
FORMAT_MIN_LENGTH = {0: 20, 1: 28, 2: 26, 3: 34, 4: 57, 5: 63, 6: 30, 7: 36, 8: 38, 9: 59, 10: 67}
FORMAT_RGB_OFFSET = {0: None, 1: None, 2: 20, 3: 28, 4: None, 5: 28, 6: None, 7: 30, 8: 30, 9: None, 10: 30}


@dataclass
class LasHeader:
    version: tuple
    point_format: int
    record_length: int
    offset_to_points: int
    num_points: int
    scale: tuple
    offset: tuple
    min: tuple
    max: tuple


def parse_header(data: bytes) -> LasHeader:
    """Fields of the public header block at their specified byte offsets."""
    if len(data) < 227 or data[:4] != b"LASF":
        raise ValueError("not a LAS file")
    major, minor = data[24], data[25]
    header_size, = struct.unpack_from("<H", data, 94)
    offset_to_points, = struct.unpack_from("<I", data, 96)
    fmt = data[104]
    rec_len, = struct.unpack_from("<H", data, 105)
    legacy_count, = struct.unpack_from("<I", data, 107)
    scale = struct.unpack_from("<3d", data, 131)
    offset = struct.unpack_from("<3d", data, 155)
    mx = struct.unpack_from("<6d", data, 179)   # max x, min x, max y, min y, max z, min z
    count = legacy_count
    if (major, minor) >= (1, 4):
        if header_size < 375 or len(data) < 375:
            raise ValueError("LAS 1.4 header shorter than 375 bytes")
        count, = struct.unpack_from("<Q", data, 247)
    if fmt & 0x80:
        raise ValueError("compressed (LAZ) records are not supported")
    if fmt not in FORMAT_MIN_LENGTH or rec_len < FORMAT_MIN_LENGTH[fmt]:
        raise ValueError("bad point format or record length")
    return LasHeader((major, minor), fmt, rec_len, offset_to_points, count, scale, offset,
                     (mx[1], mx[3], mx[5]), (mx[0], mx[2], mx[4]))


def decode(records: bytes, h: LasHeader, origin=(0.0, 0.0, 0.0)):
    """x, y, z float32 arrays and rgb (uint16 [n, 3], or None) of the records."""
    n = len(records) // h.record_length
    raw = np.frombuffer(records, dtype=np.uint8, count=n * h.record_length).reshape(n, h.record_length)
    out = []
    for a in range(3):
        X = raw[:, 4 * a:4 * a + 4].copy().view("<i4").reshape(n)
        v = X.astype(np.float64) * np.float64(h.scale[a]) + np.float64(h.offset[a])
        w = v - np.float64(origin[a])
        out.append(w.astype(np.float32))
    ro = FORMAT_RGB_OFFSET[h.point_format]
    rgb = None if ro is None else raw[:, ro:ro + 6].copy().view("<u2").reshape(n, 3)
    return out[0], out[1], out[2], rgb


def header_box(h: LasHeader, origin=(0.0, 0.0, 0.0)):
    """The header's box in the decoded frame: float32(min - origin), float32(max - origin)."""
    lo = tuple(float(np.float32(np.float64(h.min[a]) - np.float64(origin[a]))) for a in range(3))
    hi = tuple(float(np.float32(np.float64(h.max[a]) - np.float64(origin[a]))) for a in range(3))
    return lo, hi
