"""Host side of the LAS decode in libfpo (no GPU): the header parser against
the oracle's, the header box, and argument errors of the decode."""
import ctypes
import struct

import numpy as np
import pytest

import synth
from oracle import las
from synth.las import write_las


@pytest.fixture(scope="module")
def fpo():
    import paper_2302_05002_amd as fpo
    fpo.load_library()
    return fpo


@pytest.mark.parametrize("fmt,version,extra,vlr", [(0, (1, 0), 0, 0), (1, (1, 1), 2, 54), (2, (1, 2), 0, 0),
                                                   (3, (1, 3), 1, 10), (5, (1, 3), 0, 0), (6, (1, 4), 0, 3),
                                                   (7, (1, 4), 4, 0), (8, (1, 4), 0, 0), (10, (1, 4), 9, 1),
                                                   (4, (1, 2), 0, 0), (9, (1, 4), 0, 0), (2, (1, 4), 0, 0)])
def test_header_matches_oracle(fpo, fmt, version, extra, vlr):
    c = synth.clusters(777, seed=fmt, num_clusters=3)
    f = write_las(c.x * 3 + 1e5, c.y - 7e3, c.z, scale=(0.001, 0.01, 0.0001), offset=(1e5, -7e3, 0.5),
                  point_format=fmt, version=version, extra_bytes=extra, vlr_bytes=vlr, seed=3)
    h = fpo.las_parse_header(f)
    o = las.parse_header(f)
    assert (h.version_major, h.version_minor) == o.version
    assert h.point_format == o.point_format and h.record_length == o.record_length
    assert h.offset_to_points == o.offset_to_points and h.num_points == o.num_points == 777
    assert tuple(h.scale) == o.scale and tuple(h.offset) == o.offset
    assert tuple(h.min) == o.min and tuple(h.max) == o.max
    ro = las.FORMAT_RGB_OFFSET[fmt]
    assert bool(h.has_rgb) == (ro is not None) and (ro is None or h.rgb_offset == ro)
    origin = (1e5, -7e3, 0.0)
    lo, hi = fpo.las_header_box(h, origin)
    elo, ehi = las.header_box(o, origin)
    assert np.array(lo, np.float32).tobytes() == np.array(elo, np.float32).tobytes()
    assert np.array(hi, np.float32).tobytes() == np.array(ehi, np.float32).tobytes()


def test_header_rejections(fpo):
    c = synth.uniform(10, seed=1)
    f = bytearray(write_las(c.x, c.y, c.z, point_format=3))
    fpo.las_parse_header(bytes(f))
    cases = []
    g = bytearray(f); g[104] = 0x83; cases.append(g)                          # LAZ
    g = bytearray(f); struct.pack_into("<H", g, 105, 33); cases.append(g)     # short record
    g = bytearray(f); g[104] = 11; cases.append(g)                            # unknown format
    g = bytearray(f); g[0] = ord("X"); cases.append(g)                        # signature
    g = bytearray(f); struct.pack_into("<I", g, 96, 100); cases.append(g)     # points inside the header
    g = bytearray(f); struct.pack_into("<d", g, 131, float("nan")); cases.append(g)
    cases.append(bytearray(f[:226]))
    g = bytearray(write_las(c.x, c.y, c.z, point_format=6, version=(1, 4)))
    struct.pack_into("<H", g, 94, 300); cases.append(g)                       # 1.4 header too short
    for g in cases:
        with pytest.raises(fpo.FpoError) as e:
            fpo.las_parse_header(bytes(g))
        assert e.value.status == fpo.FPO_ERR_INVALID_ARG and str(e.value)


def test_decode_argument_errors(fpo):
    lib = fpo.load_library()
    c = synth.uniform(10, seed=1)
    h = fpo.las_parse_header(write_las(c.x, c.y, c.z, point_format=0))
    o = (ctypes.c_double * 3)(0, 0, 0)
    buf = ctypes.create_string_buffer(64)
    # no context
    assert lib.fpo_las_decode(None, ctypes.byref(h), buf, 64, 1, o, buf, buf, buf, None,
                              None) == fpo.FPO_ERR_INVALID_ARG


def test_select_argument_errors(fpo):
    lib = fpo.load_library()
    out = ctypes.c_uint64()
    assert lib.fpo_select_workspace_size(1000, ctypes.byref(out)) == fpo.FPO_OK and out.value > 0
    assert lib.fpo_select_workspace_size(1 << 33, ctypes.byref(out)) == fpo.FPO_ERR_INVALID_ARG
    v = fpo.make_view((0, 0, 0), ((0, 0, 0, 1),) * 6, 1.0, 0.0)
    lo = (ctypes.c_float * 3)(0, 0, 0)
    # no context
    assert lib.fpo_select_nodes(None, 0, None, None, None, lo, 1.0, ctypes.byref(v), None, 0, None, None,
                                None) == fpo.FPO_ERR_INVALID_ARG
