"""LAS fixed-record decode on the GPU against the oracle's numpy decode, bit
for bit: every record format, record bases at every alignment, ragged and
empty inputs, records too long for the LDS run, the 20M-point workload, and
a build from decoded records with the header's box given."""
import numpy as np
import pytest

import oracle
import synth
from oracle import las
from synth.las import write_las
from test_gpu_parity import compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2302_05002_amd as fpo
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = fpo.Context(0)
    yield c
    c.close()


def decode_both(ctx, f, origin, misalign=0, rgb=True, label=""):
    import torch
    import paper_2302_05002_amd as fpo
    h = fpo.las_parse_header(f)
    oh = las.parse_header(f)
    recs = f[h.offset_to_points:h.offset_to_points + h.num_points * h.record_length]
    print(f"[las] {label} fmt={h.point_format} R={h.record_length} n={h.num_points} misalign={misalign}", flush=True)
    dev = torch.zeros(len(recs) + misalign + 16, dtype=torch.uint8)
    dev[misalign:misalign + len(recs)] = torch.frombuffer(bytearray(recs), dtype=torch.uint8) if recs else 0
    dev = dev.cuda()
    want_rgb = rgb and bool(h.has_rgb)
    x, y, z, col = ctx.las_decode(dev[misalign:misalign + len(recs)] if recs else dev[:0], h, origin,
                                  rgb=want_rgb, n=h.num_points)
    torch.cuda.synchronize()
    ex, ey, ez, ecol = las.decode(recs, oh, origin)
    for a, b, k in ((x, ex, "x"), (y, ey, "y"), (z, ez, "z")):
        got = a.cpu().numpy()
        assert got.shape == b.shape, k
        np.testing.assert_array_equal(got.view(np.uint32), b.view(np.uint32), err_msg=f"{label} {k}")
    if want_rgb:
        np.testing.assert_array_equal(col.cpu().numpy().view(np.uint16), ecol, err_msg=f"{label} rgb")
    return x, y, z, h


FORMATS = [(0, (1, 2), 0), (1, (1, 2), 3), (2, (1, 2), 0), (3, (1, 3), 1), (4, (1, 3), 0), (5, (1, 3), 2),
           (6, (1, 4), 0), (7, (1, 4), 0), (8, (1, 4), 5), (9, (1, 4), 0), (10, (1, 4), 0)]


@pytest.mark.parametrize("fmt,version,extra", FORMATS)
def test_formats(ctx, fmt, version, extra):
    c = synth.planes(50_001, seed=fmt + 3, num_planes=6)
    rng = np.random.default_rng(fmt)
    rgb = rng.integers(0, 65536, size=(c.n, 3), dtype=np.uint16)
    f = write_las(c.x + 512_000.0, c.y + 5_400_000.0, c.z + 80.0, rgb=rgb, scale=(0.001, 0.001, 0.0005),
                  offset=(512_000.0, 5_400_000.0, 0.0), point_format=fmt, version=version, extra_bytes=extra,
                  vlr_bytes=13, seed=fmt)
    decode_both(ctx, f, (512_000.0, 5_400_000.0, 0.0), label="formats")


@pytest.mark.parametrize("misalign", range(16))
def test_alignments(ctx, misalign):
    c = synth.uniform(9_999, seed=misalign)
    f = write_las(c.x, c.y, c.z, scale=(1e-6, 1e-6, 1e-6), point_format=3 if misalign % 2 else 2)
    decode_both(ctx, f, (0.5, 0.25, 0.0), misalign=misalign, label="align")


@pytest.mark.parametrize("n", [0, 1, 2, 63, 64, 65, 1599, 1600, 1601, 4097])
def test_ragged(ctx, n):
    c = synth.uniform(max(n, 1), seed=n + 1, lo=-1000.0, hi=1000.0)
    f = write_las(c.x[:n], c.y[:n], c.z[:n], scale=(0.01, 0.02, 0.03), offset=(-3.0, 7.0, 11.0), point_format=0)
    decode_both(ctx, f, (0.0, 0.0, 0.0), misalign=n % 7, label="ragged")


def test_long_records(ctx):
    """Records longer than the LDS run takes (extra bytes): the per-thread path."""
    c = synth.clusters(20_000, seed=4, num_clusters=5)
    for extra in (400, 700):
        f = write_las(c.x, c.y, c.z, point_format=7, version=(1, 4), extra_bytes=extra, seed=extra)
        decode_both(ctx, f, (1.0, 2.0, 3.0), misalign=3, label=f"long+{extra}")


def test_extreme_integers(ctx):
    """int32 limits, scales that round, an origin far from the data."""
    import paper_2302_05002_amd as fpo  # noqa: F401
    n = 4096
    rng = np.random.default_rng(9)
    X = rng.integers(-2 ** 31, 2 ** 31, size=(n, 3), dtype=np.int64)
    X[:6] = [[-2 ** 31] * 3, [2 ** 31 - 1] * 3, [0] * 3, [1, -1, 1], [-2 ** 31, 2 ** 31 - 1, 0], [123456789] * 3]
    scale, offset = (1e-7, 3e-3, 0.1), (6e6, -1e5, 1e3)
    # records written at the offset, then their integers overwritten with X
    zero = np.full(n, offset[0]), np.full(n, offset[1]), np.full(n, offset[2])
    f = bytearray(write_las(*zero, scale=scale, offset=offset, point_format=1))
    h = las.parse_header(bytes(f))
    rec = np.frombuffer(f, dtype=np.uint8, offset=h.offset_to_points).reshape(n, h.record_length).copy()
    rec[:, :12] = X.astype("<i4").view(np.uint8).reshape(n, 12)
    f[h.offset_to_points:] = rec.tobytes()
    decode_both(ctx, bytes(f), (6.1e6, 0.0, -5e2), label="extreme")


def test_full_size_planes(ctx):
    """The 20M-point planes workload as LAS 1.2 format 3 (34-byte records)."""
    c = synth.planes_20m()
    f = write_las(c.x + 330_000.0, c.y + 4_200_000.0, c.z, scale=(0.0001, 0.0001, 0.0001),
                  offset=(330_000.0, 4_200_000.0, 0.0), point_format=3)
    decode_both(ctx, f, (330_000.0, 4_200_000.0, 0.0), misalign=5, label="planes20m")


def test_decode_then_build_with_header_box(ctx):
    """Decoded records feed a build with the header's box given (the LAS-header
    case): the result is the oracle's build of the decoded floats."""
    import torch
    import paper_2302_05002_amd as fpo
    c = synth.terrain_clusters(1_000_000, seed=12, colors=False)
    f = write_las(c.x + 500_000.0, c.y + 4_000_000.0, c.z, scale=(0.001, 0.001, 0.001),
                  offset=(500_000.0, 4_000_000.0, 0.0), point_format=6, version=(1, 4))
    origin = (500_000.0, 4_000_000.0, 0.0)
    x, y, z, h = decode_both(ctx, f, origin, label="build")
    box = fpo.las_header_box(h, origin)
    xs, ys, zs = (t.cpu().numpy() for t in (x, y, z))
    assert xs.min() == box[0][0] and zs.max() == box[1][2]
    p = fpo.Params(256, 100_000, 64, 5_000, 64, box)
    got = ctx.build(x, y, z, p).to_numpy()
    torch.cuda.synchronize()
    exp = oracle.build_octree(xs, ys, zs, oracle.Params(256, 100_000, 64, 5_000, 64, box))
    assert exp["status"] == oracle.OK
    compare(got, exp, label="las build: ")
    assert got["n_outside"] == 0
