"""The chunk and work-chunk cuts at their edges, against the oracle bit for
bit: chunk sizes just below, at and above the 4096-point work-chunk cap
(work chunks inside one chunk or across several), one chunk per occupied
finest cell (C = 1: many chunks, a multi-pass split), oversized finest cells
at opposite corners of a 512^3 grid, a one-dimensional line, and tiny clouds
on the finest grid."""
import numpy as np
import pytest

import synth
from test_gpu_parity import make, run_both

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2302_05002_amd as fpo
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = fpo.Context(0)
    yield c
    c.close()


THRESHOLD_CASES = [
    # (kind, n, seed, G, C, S, L, M)
    ("clusters", 150_000, 41, 256, 4_095, 32, 500, 16),
    ("clusters", 150_000, 42, 256, 4_096, 32, 500, 16),
    ("clusters", 150_000, 43, 256, 4_097, 32, 500, 16),
    ("planes", 200_000, 44, 512, 50_000, 64, 2_000, 64),
    ("uniform", 120_000, 45, 512, 1, 16, 100, 8),
    ("planes", 90_000, 46, 256, 7, 8, 30, 5),
]


@pytest.mark.parametrize("case", THRESHOLD_CASES, ids=[f"{c[0]}-G{c[3]}-C{c[4]}" for c in THRESHOLD_CASES])
def test_cut_thresholds(ctx, case):
    kind, n, seed, G, C, S, L, M = case
    got, exp = run_both(ctx, make(kind, n, seed), G, C, S, L, M, label=f"{case}: ")
    assert got["chunk_level"].shape[0] > 1


def test_oversized_corners(ctx):
    """Two stacks of identical points at opposite corners of the cube (plus a
    few points between): both corner cells hold more than C points."""
    k = 5_000
    xs = np.concatenate([np.zeros(k), np.ones(k), np.linspace(0.1, 0.9, 77)]).astype(np.float32)
    c = synth.Cloud(xs, xs.copy(), xs.copy())
    got, _ = run_both(ctx, c, 512, 1_000, 16, 100, 8, label="corners: ")
    assert got["chunk_oversized_any"] == 1


def test_line_along_x(ctx):
    n = 60_000
    x = np.linspace(0.0, 1.0, n, dtype=np.float32)
    z = np.zeros(n, np.float32)
    run_both(ctx, synth.Cloud(x, z, z.copy()), 256, 500, 32, 200, 16, label="line: ")


@pytest.mark.parametrize("n", [2, 3, 9])
def test_tiny_on_the_finest_grid(ctx, n):
    rng = np.random.default_rng(n)
    p = rng.random((3, n)).astype(np.float32)
    run_both(ctx, synth.Cloud(p[0].copy(), p[1].copy(), p[2].copy()), 512, 1, 8, 1, 1, label=f"n={n}: ")
