"""The benchmark's accounting, on the CPU: the per-step byte shares add up to
the whole path's algorithmic bytes (60 B per point, 48 with a given box, plus
8 B per count-grid cell and 4 B per kept preview index), every region the
library times belongs to exactly one step, and a request for more than one GPU
ends with a message before anything touches a GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("n,G,M", [(1, 1, 1), (1_000_000, 64, 64), (20_000_000, 128, 64), (200_000_000, 512, 64),
                                   (12_345, 8, 7), (0, 16, 3)])
@pytest.mark.parametrize("given", [False, True])
def test_step_bytes_add_up_to_the_path(n, G, M, given):
    total = sum(fn(n, G, M, given) for _, fn, _ in bench.GROUPS.values())
    assert total == bench.algorithmic_bytes(n, G, M, given)
    assert total == (48 if given else 60) * n + 8 * G ** 3 + 4 * ((n + M - 1) // M)


def test_every_timed_region_is_in_one_step():
    from paper_2302_05002_amd import TIMERS
    regions = [r for regs, _, _ in bench.GROUPS.values() for r in regs]
    assert len(regions) == len(set(regions))
    # the single-workgroup builds' one region is not part of a multi-kernel build
    assert set(regions) == set(TIMERS) - {"fused"}


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, env={**os.environ, "HIP_VISIBLE_DEVICES": ""})
    assert r.returncode != 0
    assert "one GPU" in r.stderr
