"""Synthetic LAS files written from seeded clouds (input generation only).

A writer stores each coordinate as the integer X = round((x - offset) / scale)
of a chosen scale and offset, in little-endian point data records of a chosen
format (ASPRS LAS specification: public header block, point data record
formats 0-10), after an optional block of padding standing in for variable
length records.  The header's box is the writer's: the extreme integers
mapped back through scale and offset.
"""
from __future__ import annotations

import struct

import numpy as np

_MIN_LENGTH = {0: 20, 1: 28, 2: 26, 3: 34, 4: 57, 5: 63, 6: 30, 7: 36, 8: 38, 9: 59, 10: 67}
_RGB_AT = {2: 20, 3: 28, 5: 28, 7: 30, 8: 30, 10: 30}


def write_las(x, y, z, rgb=None, scale=(0.001, 0.001, 0.001), offset=(0.0, 0.0, 0.0), point_format=2,
              version=(1, 2), extra_bytes=0, vlr_bytes=0, seed=0) -> bytes:
    """LAS file bytes of the points.  rgb: uint16 [n, 3] or None (zeros).  The
    other record fields (intensity, return numbers, GPS time, ...) are seeded
    random bytes, so a decoder that reads the wrong offsets sees garbage."""
    n = int(np.asarray(x).shape[0])
    rec_len = _MIN_LENGTH[point_format] + extra_bytes
    rng = np.random.default_rng(seed)
    raw = rng.integers(0, 256, size=(n, rec_len), dtype=np.uint8)
    ints = []
    for a, c in enumerate((x, y, z)):
        q = np.round((np.asarray(c, dtype=np.float64) - offset[a]) / scale[a])
        assert np.all(np.abs(q) < 2 ** 31), "coordinates do not fit int32 at this scale"
        X = q.astype("<i4")
        raw[:, 4 * a:4 * a + 4] = X.view(np.uint8).reshape(n, 4)
        ints.append(X)
    if point_format in _RGB_AT:
        col = np.zeros((n, 3), dtype="<u2") if rgb is None else np.asarray(rgb, dtype="<u2")
        o = _RGB_AT[point_format]
        raw[:, o:o + 6] = np.ascontiguousarray(col).view(np.uint8).reshape(n, 6)
    header_size = 375 if version >= (1, 4) else (235 if version == (1, 3) else 227)
    hdr = bytearray(header_size)
    hdr[0:4] = b"LASF"
    hdr[24], hdr[25] = version
    hdr[26:26 + 9] = b"synthetic"
    struct.pack_into("<H", hdr, 94, header_size)
    struct.pack_into("<I", hdr, 96, header_size + vlr_bytes)
    struct.pack_into("<I", hdr, 100, 0)
    hdr[104] = point_format
    struct.pack_into("<H", hdr, 105, rec_len)
    struct.pack_into("<I", hdr, 107, n if n < 2 ** 32 and point_format < 6 else 0)
    struct.pack_into("<3d", hdr, 131, *scale)
    struct.pack_into("<3d", hdr, 155, *offset)
    box = []
    for a in range(3):
        lo = float(ints[a].min()) * scale[a] + offset[a] if n else 0.0
        hi = float(ints[a].max()) * scale[a] + offset[a] if n else 0.0
        box += [hi, lo]
    struct.pack_into("<6d", hdr, 179, *box)
    if version >= (1, 4):
        struct.pack_into("<Q", hdr, 247, n)
    return bytes(hdr) + bytes(vlr_bytes) + raw.tobytes()
